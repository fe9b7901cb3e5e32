"""Seeded synthetic workloads: finest-level conserved cell averages and run parameters.

This module is shared by the oracle side and the GPU side; it holds none of the
method's arithmetic (no collision, no multiresolution operator). It only turns a seed
into the initial conserved averages of Sec. 2 (cell averages of an initial datum on the
finest lattice, computed exactly from closed-form integrals) plus the parameter set of
each workload family. The shapes follow the paper's test problems (Table 1 scalar tests,
the dam break of Sec. 5.2.2, the Riemann problems of Sec. 5.3): steps, bumps and sines
with seeded parameters; no external dataset is involved.

Workload families (sizes as used throughout the tests and the benchmark):

* ``advection``  D1Q2, V = 0.75, lambda = 1, s = 1.9, periodic [-1, 1], J 2..10,
                 gamma = 1, eps = 1e-4, 2000 steps; Gaussian bump + unit step.
* ``burgers``    D1Q3 (alpha = 0.9), lambda = 1, s in {1.5, 1.9}, periodic [-1, 1],
                 J 2..14, eps in {1e-2, 1e-3, 1e-4}, T = 0.4 (3277 steps);
                 Riemann data + sine, rescaled to max |u0| <= 0.75 lambda (larger
                 amplitudes blow up for some seeds at s = 1.9, in the uniform scheme too).
* ``shallow``    D1Q2^2 (or D1Q3, ``shallow_d1q3``), g = 1, lambda = 2, s = 1.7, clamp [-1, 1], J 2..16, eps = 1e-4,
                 T = 0.4 (26214 steps); dam break with 1% smooth noise.
* ``shallow_d1q5`` D1Q5 (Sec. 5.2: alpha = beta = 1, s3 = s4 = 1, s2 = 1.5 <= 1.6), the same
                 dam break; its stream reaches two cells (sigma = 2).
* ``batch``      D1Q2 advection/Burgers instances, J uniform in 8..14, eps in {1e-3, 1e-4}.
* ``euler``      D1Q2^3, gamma_gas = 1.4, lambda = 3, s = 1.9, clamp [-1, 1], J 2..14,
                 eps = 1e-4, T = 0.4 (9830 steps); random Riemann problems and Sod.
* ``two_d``      D2Q4 on [0, 1]^2 (the multi-D extension): Burgers (lambda = 2, s = 1.6, 1.6,
                 1.2) or advection (V = (0.4, 0.25), lambda = 1, s = 1.5), periodic, J up to
                 12, J_min = 2, eps = 1e-3; a seeded box or Gaussian bump (cell-centre
                 samples).
"""

import math

import numpy as np

# Codes (documented numbering, identical to the C header's enums).
D1Q2, D1Q3, D1Q2x2, D1Q2x3, D1Q5 = 0, 1, 2, 3, 4
ADVECTION, BURGERS, SHALLOW_WATER, EULER = 0, 1, 2, 3
PERIODIC, CLAMP = 0, 1


def edges(jmax, x_min=-1.0, x_max=1.0):
    n = 2 ** jmax
    return x_min + (x_max - x_min) * np.arange(n + 1) / n


def avg_step(e, x0, left, right):
    """Cell averages of left*1[x < x0] + right*1[x >= x0] on cells with edges e."""
    a, b = e[:-1], e[1:]
    frac_left = np.clip((x0 - a) / (b - a), 0.0, 1.0)
    return right + (left - right) * frac_left


def avg_gauss_periodic(e, amp, c, width, period=2.0, images=(-1, 0, 1)):
    """Cell averages of sum over periodic images of amp*exp(-((x - c - i P)/width)^2)."""
    a, b = e[:-1], e[1:]
    tot = np.zeros(a.size)
    k = math.sqrt(math.pi) * width / 2.0
    for i in images:
        cc = c + i * period
        tot += amp * k * (_erf((b - cc) / width) - _erf((a - cc) / width))
    return tot / (b - a)


def avg_sin(e, amp, kpi, phase):
    """Cell averages of amp*sin(kpi*x + phase)."""
    a, b = e[:-1], e[1:]
    return amp * (np.cos(kpi * a + phase) - np.cos(kpi * b + phase)) / (kpi * (b - a))


def _erf(x):
    from scipy.special import erf
    return erf(x)


def base_params(**kw):
    p = dict(scheme=D1Q2, physics=ADVECTION, bc=PERIODIC, precision=0, lam=1.0, s=[1.9],
             phys=[0.0, 1.0, 1.4, 0.9], x_min=-1.0, x_max=1.0, jmin=2, jmax=10, gamma=1,
             eps=1e-4, mu_bar=0, steps=100)
    p.update(kw)
    return p


def n_steps(T, lam, jmax, x_min=-1.0, x_max=1.0):
    """N = round(T / dt) with dt = dx_J / lambda (Sec. 2.1, acoustic scaling)."""
    dx = (x_max - x_min) / 2 ** jmax
    return int(round(T * lam / dx))


# --------------------------------------------------------------------- families
def advection(seed, jmax=10, eps=1e-4, s=1.9, steps=2000, jmin=2):
    """Gaussian bump (amplitude U(0.5,1), width U(0.05,0.2), centre U(-1,1)) plus a
    unit step at a seeded position, periodic on [-1, 1]."""
    rng = np.random.default_rng([0, seed])
    amp = rng.uniform(0.5, 1.0)
    width = rng.uniform(0.05, 0.2)
    c = rng.uniform(-1.0, 1.0)
    xs = rng.uniform(-1.0, 1.0)
    e = edges(jmax)
    u = avg_gauss_periodic(e, amp, c, width) + avg_step(e, xs, 0.0, 1.0)
    p = base_params(scheme=D1Q2, physics=ADVECTION, lam=1.0, s=[s], phys=[0.75, 1.0, 1.4, 0.9],
                    jmin=jmin, jmax=jmax, eps=eps, steps=steps, bc=PERIODIC)
    return p, u[None, :]


def burgers(seed, jmax=14, eps=1e-4, s=1.9, T=0.4, jmin=2, scheme=D1Q3, steps=None):
    """Riemann data u_L/u_R in U(-1,1) at x0 in U(-0.5,0.5) plus amp*sin(pi x + phi),
    amp in U(0.2,1), rescaled so that max |u0| <= 0.75 lambda; periodic on [-1, 1]."""
    rng = np.random.default_rng([1, seed])
    ul, ur = rng.uniform(-1.0, 1.0, size=2)
    x0 = rng.uniform(-0.5, 0.5)
    amp = rng.uniform(0.2, 1.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    lam = 1.0
    e = edges(jmax)
    u = avg_step(e, x0, ul, ur) + avg_sin(e, amp, math.pi, phi)
    m = np.max(np.abs(u))
    if m > 0.75 * lam:
        u = u * (0.75 * lam / m)
    if steps is None:
        steps = n_steps(T, lam, jmax)
    p = base_params(scheme=scheme, physics=BURGERS, lam=lam, s=[s], phys=[0.0, 1.0, 1.4, 0.9],
                    jmin=jmin, jmax=jmax, eps=eps, steps=steps, bc=PERIODIC)
    return p, u[None, :]


def shallow(seed, jmax=16, eps=1e-4, s=1.7, T=0.4, jmin=2, steps=None, scheme=D1Q2x2):
    """Dam break: h = h_L (x < 0) or h_R, times (1 + 0.01 xi(x)) with xi a normalised sum of
    8 random-phase sines; hu = 0. h_L in U(1.5,3), h_R in U(0.5,1), redrawn until the
    initial states satisfy |u| + sqrt(g h) <= 0.8 lambda. Clamp boundaries on [-1, 1].
    scheme: D1Q2x2 (vectorial, the default) or D1Q3 (one relaxation rate s)."""
    rng = np.random.default_rng([2, seed])
    g, lam = 1.0, 2.0
    while True:
        hl = rng.uniform(1.5, 3.0)
        hr = rng.uniform(0.5, 1.0)
        if math.sqrt(g * hl) <= 0.8 * lam and math.sqrt(g * hr) <= 0.8 * lam:
            break
    ks = np.arange(1, 9)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=8)
    xx = np.linspace(-1.0, 1.0, 4097)
    norm = np.max(np.abs(sum(np.sin(k * math.pi * xx + ph) for k, ph in zip(ks, phases))))
    e = edges(jmax)
    xi = sum(avg_sin(e, 1.0, k * math.pi, ph) for k, ph in zip(ks, phases)) / norm
    base = avg_step(e, 0.0, hl, hr)
    h = base * (1.0 + 0.01 * xi)
    hu = np.zeros_like(h)
    if steps is None:
        steps = n_steps(T, lam, jmax)
    if scheme == D1Q5:
        # rates of M2, M3, M4 and phys = [beta, g, -, alpha] with alpha = beta = 1 (Sec. 5.2)
        p = base_params(scheme=scheme, physics=SHALLOW_WATER, lam=lam, s=[s, 1.0, 1.0], phys=[1.0, g, 1.4, 1.0],
                        jmin=jmin, jmax=jmax, eps=eps, steps=steps, bc=CLAMP)
    else:
        p = base_params(scheme=scheme, physics=SHALLOW_WATER, lam=lam, s=[s], phys=[0.0, g, 1.4, 0.9],
                        jmin=jmin, jmax=jmax, eps=eps, steps=steps, bc=CLAMP)
    return p, np.stack([h, hu])


def euler(seed, jmax=14, eps=1e-4, s=1.9, T=0.4, jmin=2, sod=False, steps=None):
    """Riemann problem at x = 0 with rho, p in U(0.1,1), u in U(-0.5,0.5) on each side,
    redrawn until |u| + c <= 0.8 lambda on both sides (c = sqrt(gamma p / rho));
    E = rho u^2 / 2 + p / (gamma - 1) (Sec. 5.3). ``sod`` gives the Sod data of Sec. 5.3."""
    gam, lam = 1.4, 3.0
    if sod:
        rl, ul, pl, rr, ur, pr = 1.0, 0.0, 1.0, 0.125, 0.0, 0.1
    else:
        rng = np.random.default_rng([4, seed])
        while True:
            rl, rr = rng.uniform(0.1, 1.0, size=2)
            pl, pr = rng.uniform(0.1, 1.0, size=2)
            ul, ur = rng.uniform(-0.5, 0.5, size=2)
            cl, cr = math.sqrt(gam * pl / rl), math.sqrt(gam * pr / rr)
            if abs(ul) + cl <= 0.8 * lam and abs(ur) + cr <= 0.8 * lam:
                break
    El = 0.5 * rl * ul * ul + pl / (gam - 1.0)
    Er = 0.5 * rr * ur * ur + pr / (gam - 1.0)
    e = edges(jmax)
    rho = avg_step(e, 0.0, rl, rr)
    mom = avg_step(e, 0.0, rl * ul, rr * ur)
    ene = avg_step(e, 0.0, El, Er)
    if steps is None:
        steps = n_steps(T, lam, jmax)
    p = base_params(scheme=D1Q2x3, physics=EULER, lam=lam, s=[s], phys=[0.0, 1.0, gam, 0.9],
                    jmin=jmin, jmax=jmax, eps=eps, steps=steps, bc=CLAMP)
    return p, np.stack([rho, mom, ene])


def batch_instance(seed, steps=512):
    """One instance of the batched ensemble: D1Q2 advection (V=0.75, s=1.9) or Burgers
    (s in {1.5, 1.9}) with probability 1/2, J uniform in 8..14, eps in {1e-3, 1e-4}; the
    advection generator's data, rescaled to max |u0| <= 0.75 for Burgers."""
    rng = np.random.default_rng([3, seed])
    jmax = int(rng.integers(8, 15))
    eps = float(rng.choice([1e-3, 1e-4]))
    is_burgers = bool(rng.integers(0, 2))
    s = float(rng.choice([1.5, 1.9])) if is_burgers else 1.9
    p, u = advection(seed + 100000, jmax=jmax, eps=eps, s=s, steps=steps)
    if is_burgers:
        m = np.max(np.abs(u))
        if m > 0.75:
            u = u * (0.75 / m)
        p["physics"] = BURGERS
        p["phys"] = [0.0, 1.0, 1.4, 0.9]
    return p, u


def small_case(kind="advection", seed=0, jmax=7, **kw):
    """Reduced-size versions used by the fast tests."""
    if kind == "advection":
        return advection(seed, jmax=jmax, **kw)
    if kind == "burgers":
        return burgers(seed, jmax=jmax, **kw)
    if kind == "burgers_d1q2":
        return burgers(seed, jmax=jmax, scheme=D1Q2, **kw)
    if kind == "shallow":
        return shallow(seed, jmax=jmax, **kw)
    if kind == "shallow_d1q3":
        return shallow(seed, jmax=jmax, scheme=D1Q3, **kw)
    if kind == "shallow_d1q5":
        kw.setdefault("s", 1.5)
        return shallow(seed, jmax=jmax, scheme=D1Q5, **kw)
    if kind == "euler":
        return euler(seed, jmax=jmax, **kw)
    raise ValueError(kind)


def mlp_init(seed, nin=32, hidden=64):
    """Seeded initial parameters of the refinement predictor's network (He-uniform weights,
    zero biases), flat float32 in the order W1[64][32], b1, W2[64][64], b2, w3, b3."""
    rng = np.random.default_rng([5, seed])
    a1 = math.sqrt(6.0 / nin)
    a2 = math.sqrt(6.0 / hidden)
    W1 = rng.uniform(-a1, a1, size=(hidden, nin))
    W1[:, nin - 1] = 0.0
    W2 = rng.uniform(-a2, a2, size=(hidden, hidden))
    w3 = rng.uniform(-a2, a2, size=hidden)
    return np.concatenate([W1.ravel(), np.zeros(hidden), W2.ravel(), np.zeros(hidden), w3, np.zeros(1)]).astype(np.float32)


def mlp_constant_bits(logit):
    """bfloat16 parameter bits of a network whose every weight is zero and whose output bias is
    ``logit`` (a constant decision: refine everything for logit >= 0, decline every gated pair
    otherwise). ``logit`` must be exactly representable in bfloat16."""
    t = np.zeros(6337, dtype=np.float32)
    t[-1] = logit
    u = t.view(np.uint32)
    if np.any(u & 0xFFFF):
        raise ValueError("logit is not a bfloat16 value")
    return (u >> 16).astype(np.uint16)


def two_d(seed, jmax=12, kind="box", physics=BURGERS, eps=1e-3, jmin=2, bc=PERIODIC):
    """Parameters (the dict ``mrlbm.make_params2d`` takes) and the 2^J x 2^J datum of a seeded
    2D run: 0.2 plus 0.5 times a box or a Gaussian bump, sampled at cell centres."""
    rng = np.random.default_rng([20, seed])
    x = (np.arange(2 ** jmax) + 0.5) / 2 ** jmax - 0.5
    X, Y = np.meshgrid(x, x, indexing="ij")
    cx, cy = rng.uniform(-0.15, 0.15, 2)
    if kind == "box":
        a, b = rng.uniform(0.1, 0.25, 2)
        u0 = 0.2 + 0.5 * ((np.abs(X - cx) < a) & (np.abs(Y - cy) < b))
    else:
        w = rng.uniform(0.01, 0.04)
        u0 = 0.2 + 0.5 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / w)
    adv = physics == ADVECTION
    p = dict(physics=physics, bc=bc, gamma=1, lam=1.0 if adv else 2.0, s=[1.5] * 3 if adv else [1.6, 1.6, 1.2],
             V=(0.4, 0.25), jmin=jmin, jmax=jmax, mu_bar=0, eps=eps)
    return p, u0
