"""Pins of the oracle's lattice schemes.

Paper passages: Sec. 2.1 (d'Humieres formalism: conserved moments unchanged, the
others relaxed), Sec. 5.1.1 (D1Q2, its l1 continuity constant in the Example), Sec. 5.2.1
(D1Q3 and D1Q5 for shallow water), Sec. 5.3 (vectorial D1Q2^3 equilibria consistent with
the Euler fluxes).
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle.reference import UniformLBM

SCHEMES = [
    dict(scheme=L.D1Q2, physics=L.ADVECTION, lam=1.0, s=1.9, V=0.75),
    dict(scheme=L.D1Q2, physics=L.BURGERS, lam=1.0, s=1.5),
    dict(scheme=L.D1Q3, physics=L.BURGERS, lam=1.0, s=1.9, alpha=0.9),
    dict(scheme=L.D1Q3, physics=L.SHALLOW_WATER, lam=2.0, s=1.3, g=1.0),
    dict(scheme=L.D1Q2x2, physics=L.SHALLOW_WATER, lam=2.0, s=1.7, g=1.0),
    dict(scheme=L.D1Q2x3, physics=L.EULER, lam=3.0, s=1.9, gamma_gas=1.4),
    dict(scheme=L.D1Q5, physics=L.SHALLOW_WATER, lam=2.0, s=[1.5, 1.0, 1.0], g=1.0, alpha=1.0, beta=1.0),
    # lambda not a power of two, every rate and coefficient different: the divisions round
    dict(scheme=L.D1Q5, physics=L.SHALLOW_WATER, lam=3.0, s=[1.3, 0.8, 1.7], g=0.7, alpha=0.6, beta=1.3),
]


def make(d):
    d = dict(d)
    return L.Scheme(d.pop("scheme"), d.pop("physics"), d.pop("lam"), d.pop("s"), **d)


def random_state(sch, rng, n=200):
    """Positive densities so that the nonlinear equilibria are defined."""
    mc = rng.uniform(0.5, 1.5, size=(sch.qc, n))
    if sch.physics in (L.SHALLOW_WATER, L.EULER):
        mc[1] = rng.uniform(-0.3, 0.3, size=n) * mc[0]
    if sch.physics == L.EULER:
        mc[2] = 0.5 * mc[1] ** 2 / mc[0] + rng.uniform(0.3, 1.0, size=n) / 0.4
    f = sch.equilibrium(mc) + 0.05 * rng.standard_normal((sch.q, n))
    return f


@pytest.mark.parametrize("cfg", SCHEMES)
def test_explicit_collision_matches_definition(cfg):
    """The fixed-order collision equals m -> relax -> M^-1 m* of Sec. 2.1.1."""
    sch = make(cfg)
    f = random_state(sch, np.random.default_rng(5))
    a = sch.collide(f)
    b = sch.collide_by_definition(f)
    assert np.max(np.abs(a - b)) <= 1e-14 * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("cfg", SCHEMES)
def test_collision_keeps_conserved_moments(cfg):
    sch = make(cfg)
    f = random_state(sch, np.random.default_rng(6))
    assert np.allclose(sch.conserved(sch.collide(f)), sch.conserved(f), rtol=0, atol=1e-14)


@pytest.mark.parametrize("cfg", SCHEMES)
def test_equilibrium_is_fixed_point(cfg):
    """Populations at equilibrium are not changed by the collision, and they carry the
    requested conserved moments."""
    sch = make(cfg)
    rng = np.random.default_rng(8)
    mc = random_state(sch, rng)
    mc = sch.conserved(mc)
    f = sch.equilibrium(mc)
    assert np.allclose(sch.conserved(f), mc, rtol=0, atol=1e-14)
    assert np.allclose(sch.collide(f), f, rtol=0, atol=1e-14)


def test_euler_equilibria_are_the_fluxes():
    """Sec. 5.3: m1^eq = rho u, m3^eq = rho u^2 + p, m5^eq = (E + p) u with
    p = (gamma - 1)(E - rho u^2 / 2)."""
    sch = make(SCHEMES[5])
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.2, 2.0, 50)
    u = rng.uniform(-1, 1, 50)
    p = rng.uniform(0.1, 2.0, 50)
    gam = 1.4
    E = 0.5 * rho * u * u + p / (gam - 1)
    eq = sch._eq_vectorial([rho, rho * u, E])
    assert np.allclose(eq[0], rho * u, rtol=1e-14)
    assert np.allclose(eq[1], rho * u * u + p, rtol=1e-13)
    assert np.allclose(eq[2], (E + p) * u, rtol=1e-13, atol=1e-14)


def test_shallow_water_equilibria_are_the_fluxes():
    for cfg in (SCHEMES[3], SCHEMES[4]):
        sch = make(cfg)
        h = np.array([0.5, 1.0, 2.0])
        hu = np.array([0.1, -0.3, 0.2])
        if sch.scheme == L.D1Q2x2:
            eq = sch._eq_vectorial([h, hu])
            assert np.allclose(eq[0], hu)
            assert np.allclose(eq[1], hu ** 2 / h + 0.5 * h ** 2)
        else:
            m = np.stack([h, hu, np.zeros(3)])
            assert np.allclose(sch.equilibria_by_definition(m)[2], hu ** 2 / h + 0.5 * h ** 2)


def l1_operator_norm(s, c_over_lam, n=16):
    sch = L.Scheme(L.D1Q2, L.ADVECTION, 1.0, s, V=c_over_lam)
    cols = []
    for i in range(2 * n):
        e = np.zeros(2 * n)
        e[i] = 1.0
        ref = UniformLBM(sch, 4, 0, np.zeros((1, n)))
        ref.F = e.reshape(2, n)
        ref.step(1)
        cols.append(np.abs(ref.F).sum())
    return max(cols)


@pytest.mark.parametrize("s,expected", [(1.0, 1.0), (8.0 / 7.0, 1.0), (1.5, 1.625), (1.9, 2.325)])
def test_d1q2_l1_continuity_constant(s, expected):
    """Example of Sec. 5.1.1: C_L = 1 if s <= 2/(1 + c/lambda), else s (1 + c/lambda) - 1,
    for c/lambda = 0.75. The operator is linear, so C_L is its l1 operator norm."""
    assert abs(l1_operator_norm(s, 0.75) - expected) < 1e-12


def test_d1q2_advection_at_lattice_speed_is_a_shift():
    """c = lambda and s = 1: the collision lands on equilibrium f+ = u, f- = 0, and the
    stream moves u one cell to the right: the exact upwind shift."""
    sch = L.Scheme(L.D1Q2, L.ADVECTION, 1.0, 1.0, V=1.0)
    rng = np.random.default_rng(0)
    u0 = rng.uniform(size=(1, 64))
    ref = UniformLBM(sch, 6, 0, u0).step(5)
    assert np.allclose(ref.conserved()[0], np.roll(u0[0], 5), rtol=0, atol=1e-15)


def test_d1q5_moments_and_equilibria_are_the_shallow_water_fluxes():
    """Sec. 5.2.1, D1Q5: at equilibrium the first moment is hu (the flux of h), the second is
    hu^2 + g h^2 / 2 (the flux of hu), and the higher ones are alpha lambda^2 hu and
    beta lambda^2 (hu^2 + g h^2 / 2); all read through the paper's M."""
    sch = make(SCHEMES[7])
    rng = np.random.default_rng(3)
    h = rng.uniform(0.3, 2.5, 40)
    hu = rng.uniform(-0.5, 0.5, 40) * h
    m = sch.moment_matrix() @ sch.equilibrium(np.stack([h, hu]))
    flux = hu ** 2 / h + 0.7 / 2 * h ** 2
    lam2 = 9.0
    assert np.allclose(m[0], h, rtol=1e-14)
    assert np.allclose(m[1], hu, rtol=1e-13, atol=1e-14)
    assert np.allclose(m[2], flux, rtol=1e-13)
    assert np.allclose(m[3], 0.6 * lam2 * hu, rtol=1e-13, atol=1e-13)
    assert np.allclose(m[4], 1.3 * lam2 * flux, rtol=1e-13)
    # the velocities of Sec. 5.2.1: M's second row is lambda (0, 1, -1, 2, -2)
    assert np.array_equal(sch.moment_matrix()[1], 3.0 * np.array([0.0, 1.0, -1.0, 2.0, -2.0]))
    assert sch.sigma == 2


def test_d1q5_acoustic_pulse_travels_at_the_wave_speed():
    """A small hump on water at rest (h = 1 + 1e-3 bump, u = 0, g = 1) splits into two pulses
    moving at -+ sqrt(g h) in the uniform D1Q5 scheme: after time t the right-moving pulse's
    centre of mass sits at sqrt(g) t (g = 1 with lambda = 2; g = 0.7 with lambda = 3). Pins the two-cell stencil (w = +-2) and the moments
    together against the shallow-water wave speed, not against the formulas above."""
    for sch in (make(SCHEMES[6]), make(SCHEMES[7])):
        J = 10
        n = 2 ** J
        x = -1.0 + (np.arange(n) + 0.5) * 2.0 / n
        h = 1.0 + 1e-3 * np.exp(-(x / 0.05) ** 2)
        ref = UniformLBM(sch, J, 0, np.stack([h, np.zeros(n)]))
        steps = 200
        ref.step(steps)
        t = steps * (2.0 / n) / sch.lam  # dt = dx / lambda
        d = ref.conserved()[0] - 1.0
        right = x > 0
        centre = np.sum(x[right] * d[right]) / np.sum(d[right])
        want = np.sqrt(sch.g * 1.0) * t
        assert abs(centre - want) < 0.02 * want, (sch.lam, centre, want)
