"""Exact entropy solutions of the Riemann problems behind the paper's verifications, and
their cell averages (test infrastructure; see ``oracle/__init__``).

They give the reference-scheme error E^{0,n} and the adaptive error e^{0,n} against the
exact solution (Sec. 5, the error definitions at the head of the verifications). Written
from the textbook theory of one-dimensional hyperbolic conservation laws:

* Burgers: a shock at the Rankine-Hugoniot speed (u_L + u_R) / 2 when u_L > u_R, else a
  centred rarefaction u = x / t between the two states.
* shallow water (h, hu): two nonlinear waves around a star state (h*, u*), each a shock
  (Rankine-Hugoniot) or a rarefaction (the Riemann invariant u +- 2 sqrt(g h) constant);
  h* is the root of the sum of the two wave functions plus the velocity jump.
* Euler (rho, rho u, E), ideal gas: the same construction on the pressure p*, with shock
  and isentropic-rarefaction wave functions; u* from the two wave functions.

Newton iterations on a monotone wave function (the star value is found to machine
precision); sampling along x / t.
"""

import math

import numpy as np


# ------------------------------------------------------------------ Burgers
def burgers_riemann(ul, ur, xi):
    """Entropy solution of u_t + (u^2 / 2)_x = 0 with u = ul (x < 0), ur (x > 0), at x / t = xi."""
    xi = np.asarray(xi, dtype=np.float64)
    if ul > ur:
        s = 0.5 * (ul + ur)
        return np.where(xi < s, ul, ur)
    return np.clip(xi, ul, ur)


# ------------------------------------------------------------------ shallow water
def _sw_wave(h, hk, g):
    """Velocity change across the wave connecting depth hk to h (and its derivative):
    rarefaction for h <= hk, shock otherwise."""
    if h <= hk:
        f = 2.0 * (math.sqrt(g * h) - math.sqrt(g * hk))
        df = math.sqrt(g / h)
    else:
        q = math.sqrt(0.5 * g * (h + hk) / (h * hk))
        f = (h - hk) * q
        df = q - 0.25 * g * (h - hk) / (q * h * h)
    return f, df


def shallow_star(hl, ul, hr, ur, g):
    """Star state (h*, u*) of the shallow-water Riemann problem (no dry bed)."""
    du = ur - ul
    if 2.0 * (math.sqrt(g * hl) + math.sqrt(g * hr)) <= -du:
        raise ValueError("dry bed forms")
    h = 0.5 * (hl + hr)
    for _ in range(100):
        fl, dfl = _sw_wave(h, hl, g)
        fr, dfr = _sw_wave(h, hr, g)
        step = (fl + fr + du) / (dfl + dfr)
        h = max(h - step, 1e-14)
        if abs(step) <= 1e-15 * h:
            break
    fl, _ = _sw_wave(h, hl, g)
    fr, _ = _sw_wave(h, hr, g)
    return h, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def shallow_riemann(hl, ul, hr, ur, g, xi):
    """(h, hu) of the shallow-water Riemann problem at x / t = xi."""
    xi = np.asarray(xi, dtype=np.float64)
    hs, us = shallow_star(hl, ul, hr, ur, g)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    cl, cr, cs = math.sqrt(g * hl), math.sqrt(g * hr), math.sqrt(g * hs)
    left = xi < us
    # left wave
    if hs > hl:  # shock
        s = ul - math.sqrt(0.5 * g * (hs + hl) * hs / hl)
        m = left & (xi < s)
        h[m], u[m] = hl, ul
        m = left & (xi >= s)
        h[m], u[m] = hs, us
    else:  # rarefaction between ul - cl and us - cs
        head, tail = ul - cl, us - cs
        m = left & (xi < head)
        h[m], u[m] = hl, ul
        m = left & (xi >= tail)
        h[m], u[m] = hs, us
        m = left & (xi >= head) & (xi < tail)
        c = (ul + 2.0 * cl - xi[m]) / 3.0
        h[m], u[m] = c * c / g, xi[m] + c
    right = ~left
    if hs > hr:
        s = ur + math.sqrt(0.5 * g * (hs + hr) * hs / hr)
        m = right & (xi > s)
        h[m], u[m] = hr, ur
        m = right & (xi <= s)
        h[m], u[m] = hs, us
    else:
        head, tail = ur + cr, us + cs
        m = right & (xi > head)
        h[m], u[m] = hr, ur
        m = right & (xi <= tail)
        h[m], u[m] = hs, us
        m = right & (xi > tail) & (xi <= head)
        c = (xi[m] - ur + 2.0 * cr) / 3.0
        h[m], u[m] = c * c / g, xi[m] - c
    return np.stack([h, h * u])


# ------------------------------------------------------------------ Euler
def _eu_wave(p, rk, pk, gam):
    """Velocity change across the wave connecting pressure pk (density rk) to p, and its
    derivative: shock for p > pk, isentropic rarefaction otherwise."""
    ck = math.sqrt(gam * pk / rk)
    if p > pk:
        a = 2.0 / ((gam + 1.0) * rk)
        b = (gam - 1.0) / (gam + 1.0) * pk
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + b))
    e = (gam - 1.0) / (2.0 * gam)
    return 2.0 * ck / (gam - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(gam + 1.0) / (2.0 * gam)) / (rk * ck)


def euler_star(rl, ul, pl, rr, ur, pr, gam):
    """Star pressure and velocity of the ideal-gas Riemann problem (no vacuum)."""
    cl, cr = math.sqrt(gam * pl / rl), math.sqrt(gam * pr / rr)
    if 2.0 * (cl + cr) / (gam - 1.0) <= ur - ul:
        raise ValueError("vacuum forms")
    p = max(1e-10, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _eu_wave(p, rl, pl, gam)
        fr, dfr = _eu_wave(p, rr, pr, gam)
        step = (fl + fr + ur - ul) / (dfl + dfr)
        p = max(p - step, 1e-14)
        if abs(step) <= 1e-15 * p:
            break
    fl, _ = _eu_wave(p, rl, pl, gam)
    fr, _ = _eu_wave(p, rr, pr, gam)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def euler_riemann(rl, ul, pl, rr, ur, pr, gam, xi):
    """(rho, rho u, E) of the Euler Riemann problem at x / t = xi, E = rho u^2 / 2 + p / (gam - 1)."""
    xi = np.asarray(xi, dtype=np.float64)
    ps, us = euler_star(rl, ul, pl, rr, ur, pr, gam)
    rho, u, p = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    g1 = (gam - 1.0) / (gam + 1.0)
    left = xi < us
    cl = math.sqrt(gam * pl / rl)
    if ps > pl:
        rs = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
        s = ul - cl * math.sqrt((gam + 1.0) / (2.0 * gam) * ps / pl + (gam - 1.0) / (2.0 * gam))
        m = left & (xi < s)
        rho[m], u[m], p[m] = rl, ul, pl
        m = left & (xi >= s)
        rho[m], u[m], p[m] = rs, us, ps
    else:
        rs = rl * (ps / pl) ** (1.0 / gam)
        cs = cl * (ps / pl) ** ((gam - 1.0) / (2.0 * gam))
        head, tail = ul - cl, us - cs
        m = left & (xi < head)
        rho[m], u[m], p[m] = rl, ul, pl
        m = left & (xi >= tail)
        rho[m], u[m], p[m] = rs, us, ps
        m = left & (xi >= head) & (xi < tail)
        uf = 2.0 / (gam + 1.0) * (cl + 0.5 * (gam - 1.0) * ul + xi[m])
        cf = uf - xi[m]
        rho[m] = rl * (cf / cl) ** (2.0 / (gam - 1.0))
        u[m], p[m] = uf, pl * (cf / cl) ** (2.0 * gam / (gam - 1.0))
    right = ~left
    cr = math.sqrt(gam * pr / rr)
    if ps > pr:
        rs = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
        s = ur + cr * math.sqrt((gam + 1.0) / (2.0 * gam) * ps / pr + (gam - 1.0) / (2.0 * gam))
        m = right & (xi > s)
        rho[m], u[m], p[m] = rr, ur, pr
        m = right & (xi <= s)
        rho[m], u[m], p[m] = rs, us, ps
    else:
        rs = rr * (ps / pr) ** (1.0 / gam)
        cs = cr * (ps / pr) ** ((gam - 1.0) / (2.0 * gam))
        head, tail = ur + cr, us + cs
        m = right & (xi > head)
        rho[m], u[m], p[m] = rr, ur, pr
        m = right & (xi <= tail)
        rho[m], u[m], p[m] = rs, us, ps
        m = right & (xi > tail) & (xi <= head)
        uf = 2.0 / (gam + 1.0) * (-cr + 0.5 * (gam - 1.0) * ur + xi[m])
        cf = xi[m] - uf
        rho[m] = rr * (cf / cr) ** (2.0 / (gam - 1.0))
        u[m], p[m] = uf, pr * (cf / cr) ** (2.0 * gam / (gam - 1.0))
    return np.stack([rho, rho * u, 0.5 * rho * u * u + p / (gam - 1.0)])


# ------------------------------------------------------------------ cell averages
def cell_averages(sample, x_min, x_max, jmax, x0, t, sub=256):
    """Cell averages on the 2^jmax cells of [x_min, x_max] of a self-similar solution
    sample(xi) (xi = (x - x0) / t, shape (..., n)) at time t > 0, by the midpoint rule with
    ``sub`` points per cell."""
    n = 2 ** jmax
    dx = (x_max - x_min) / n
    xs = x_min + (np.arange(n)[:, None] + (np.arange(sub)[None, :] + 0.5) / sub) * dx
    v = sample(((xs - x0) / t).ravel())
    v = np.atleast_2d(v)
    return v.reshape(v.shape[0], n, sub).mean(axis=2)
