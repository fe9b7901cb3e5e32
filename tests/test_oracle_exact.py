"""Pins of the exact Riemann solutions (oracle/exact.py) against what the theory fixes
independently of how they are computed: the jump conditions across every sampled shock,
the Riemann invariants and entropy inside every sampled fan, global conservation with the
boundary fluxes, the textbook Sod star state; then the reference scheme's error against
them (E, Sec. 5) decreasing as the finest level grows, and the adaptive perturbation staying
well below it (delta << E, the paper's design target)."""

import numpy as np
import pytest

import workloads as W
from oracle import exact, metrics
from oracle.adaptive import AdaptiveMRLBM
from oracle.lattice import scheme_from_params
from oracle.reference import UniformLBM

GAM = 1.4
SOD = (1.0, 0.0, 1.0, 0.125, 0.0, 0.1)


def euler_flux(U):
    rho, mom, ene = U
    u = mom / rho
    p = (GAM - 1.0) * (ene - 0.5 * rho * u * u)
    return np.stack([mom, mom * u + p, (ene + p) * u])


def sw_flux(U, g):
    h, hu = U
    return np.stack([hu, hu * hu / h + 0.5 * g * h * h])


def jumps(sample, xi_lo, xi_hi, n=20001):
    """Every jump of a sampled self-similar solution on [xi_lo, xi_hi]: (speed, U-, U+)."""
    xi = np.linspace(xi_lo, xi_hi, n)
    U = sample(xi)
    d = np.max(np.abs(np.diff(U, axis=1)), axis=0)
    out = []
    for k in np.nonzero(d > 1e-3)[0]:
        out.append((0.5 * (xi[k] + xi[k + 1]), U[:, k], U[:, k + 1]))
    return out


def euler_data(seed, jmax=8):
    """The Riemann data of the Euler workload: its end cells hold the two pure states (the
    jump sits on a cell edge)."""
    _, mc = W.euler(seed, jmax=jmax)
    rl, rr = mc[0][0], mc[0][-1]
    ul, ur = mc[1][0] / rl, mc[1][-1] / rr
    pl = (GAM - 1.0) * (mc[2][0] - 0.5 * rl * ul * ul)
    pr = (GAM - 1.0) * (mc[2][-1] - 0.5 * rr * ur * ur)
    return rl, ul, pl, rr, ur, pr


def test_sod_star_state():
    """Sod's problem (rho, u, p = 1, 0, 1 | 0.125, 0, 0.1; gamma 1.4): star pressure, velocity
    and densities as tabulated in the textbook literature (0.30313, 0.92745, 0.42632, 0.26557)."""
    ps, us = exact.euler_star(*SOD, GAM)
    assert abs(ps - 0.30313) < 5e-6 and abs(us - 0.92745) < 5e-6
    U = exact.euler_riemann(*SOD, GAM, np.array([us - 1e-6, us + 1e-6]))
    assert abs(U[0, 0] - 0.42632) < 5e-6 and abs(U[0, 1] - 0.26557) < 5e-6


@pytest.mark.parametrize("seed", range(6))
def test_euler_jump_conditions_and_fans(seed):
    """Across every discontinuity F(U+) - F(U-) = s (U+ - U-) (the contact included: its
    speed is u*, pressure and velocity continuous); inside a fan the entropy p / rho^gamma and
    the Riemann invariant of the other family are constant."""
    rl, ul, pl, rr, ur, pr = euler_data(seed)
    sample = lambda xi: exact.euler_riemann(rl, ul, pl, rr, ur, pr, GAM, xi)
    for s, um, up in jumps(sample, -4.0, 4.0):
        lhs = euler_flux(up[:, None])[:, 0] - euler_flux(um[:, None])[:, 0]
        assert np.allclose(lhs, s * (up - um), atol=2e-3 * (1 + np.abs(lhs).max())), (seed, s)
    xi = np.linspace(-4.0, 4.0, 20001)
    U = sample(xi)
    rho, u = U[0], U[1] / U[0]
    pres = (GAM - 1.0) * (U[2] - 0.5 * rho * u * u)
    c = np.sqrt(GAM * pres / rho)
    ps, us = exact.euler_star(rl, ul, pl, rr, ur, pr, GAM)
    checked = 0
    for k in fan_pairs(u, xi, us):
        inv = u + 2 * c / (GAM - 1) if xi[k] < us else u - 2 * c / (GAM - 1)
        assert abs(inv[k + 1] - inv[k]) < 1e-9
        s_ent = pres / rho ** GAM
        assert abs(s_ent[k + 1] - s_ent[k]) < 1e-9 * s_ent[k]
        checked += 1
    assert checked > 0 or (ps > pl and ps > pr)  # no fan only when both waves are shocks


def fan_pairs(u, xi, us):
    """Indices k where (xi[k], xi[k+1]) lies inside a fan: u varies smoothly there and on the
    neighbouring intervals, and the pair does not cross the contact x / t = u*."""
    du = np.abs(np.diff(u))
    smooth = (du > 0) & (du < 1e-3)
    inner = smooth[1:-1] & smooth[:-2] & smooth[2:]
    ks = np.nonzero(inner)[0] + 1
    return [k for k in ks if (xi[k] - us) * (xi[k + 1] - us) > 0]


@pytest.mark.parametrize("hl,ul,hr,ur", [(2.0, 0.0, 1.0, 0.0), (1.0, 0.5, 2.0, -0.3), (1.5, -0.6, 1.0, 0.8)])
def test_shallow_jump_conditions_and_fans(hl, ul, hr, ur):
    g = 1.0
    sample = lambda xi: exact.shallow_riemann(hl, ul, hr, ur, g, xi)
    for s, um, up in jumps(sample, -4.0, 4.0):
        lhs = sw_flux(up[:, None], g)[:, 0] - sw_flux(um[:, None], g)[:, 0]
        assert np.allclose(lhs, s * (up - um), atol=2e-3 * (1 + np.abs(lhs).max())), s
    xi = np.linspace(-4.0, 4.0, 20001)
    U = sample(xi)
    h, u = U[0], U[1] / U[0]
    hs, us = exact.shallow_star(hl, ul, hr, ur, g)
    checked = 0
    for k in fan_pairs(u, xi, us):
        inv = u + 2 * np.sqrt(g * h) if xi[k] < us else u - 2 * np.sqrt(g * h)
        assert abs(inv[k + 1] - inv[k]) < 1e-9
        checked += 1
    assert checked > 0 or (hs > hl and hs > hr)


def test_burgers_shock_speed_and_fan():
    assert np.all(exact.burgers_riemann(1.0, 0.0, np.array([0.49, 0.51])) == np.array([1.0, 0.0]))
    xi = np.linspace(-0.5, 0.5, 11)
    assert np.allclose(exact.burgers_riemann(-0.2, 0.3, xi), np.clip(xi, -0.2, 0.3))


@pytest.mark.parametrize("which", ["euler", "shallow"])
def test_cell_averages_conserve_with_boundary_fluxes(which):
    """d/dt of the integral of U over [-1, 1] is F(U_L) - F(U_R) while the waves stay inside:
    the cell averages of the exact solution at t reproduce it to the midpoint rule's accuracy."""
    t = 0.2
    if which == "euler":
        UL = np.array([1.0, 0.0, 1.0 / (GAM - 1.0)])
        UR = np.array([0.125, 0.0, 0.1 / (GAM - 1.0)])
        sample = lambda xi: exact.euler_riemann(*SOD, GAM, xi)
        F = euler_flux
    else:
        g = 1.0
        UL, UR = np.array([2.0, 0.0]), np.array([1.0, 0.0])
        sample = lambda xi: exact.shallow_riemann(2.0, 0.0, 1.0, 0.0, g, xi)
        F = lambda U: sw_flux(U, g)
    avg = exact.cell_averages(sample, -1.0, 1.0, 10, 0.0, t)
    total = avg.sum(axis=1) * (2.0 / 2 ** 10)
    want = UL + UR + t * (F(UL[:, None])[:, 0] - F(UR[:, None])[:, 0])
    assert np.allclose(total, want, atol=1e-6), (total, want)


def euler_errors(seed, jmax, eps, steps_at_j9=60):
    p, mc = W.euler(seed, jmax=jmax, eps=eps)
    n = steps_at_j9 * 2 ** (jmax - 9)
    t = n * (p["x_max"] - p["x_min"]) / 2 ** jmax / p["lam"]
    rl, ul, pl, rr, ur, pr = euler_data(seed, jmax)
    ex = exact.cell_averages(lambda xi: exact.euler_riemann(rl, ul, pl, rr, ur, pr, GAM, xi),
                             p["x_min"], p["x_max"], jmax, 0.0, t)
    sch = scheme_from_params(p)
    ref = UniformLBM(sch, jmax, p["bc"], mc).step(n)
    E = metrics.delta(ex, ref.conserved(), p["x_min"], p["x_max"])[0]
    if eps is None:
        return E, None
    a = AdaptiveMRLBM(sch, p["jmin"], jmax, p["gamma"], eps, p["mu_bar"], p["bc"], mc).step(n)
    d = metrics.delta(ref.conserved(), a.finest_conserved(), p["x_min"], p["x_max"])[0]
    return E, d


def test_reference_scheme_converges_to_the_exact_solution():
    """E (density, Sec. 5) of the uniform D1Q2^3 scheme against the exact Riemann solution at
    the same physical time decreases as J grows (first order at best across discontinuities,
    so at least a factor 2^0.4 per level here)."""
    Es = [euler_errors(2, j, None)[0] for j in (8, 9, 10)]
    assert Es[0] > Es[1] > Es[2], Es
    assert Es[0] / Es[2] > 2 ** 0.8, Es


def test_adaptive_perturbation_is_far_below_the_scheme_error():
    """delta << E at eps = 1e-4 (the paper's design target for eps): below a tenth of E."""
    E, d = euler_errors(2, 10, 1e-4)
    assert d < 0.1 * E, (d, E)
