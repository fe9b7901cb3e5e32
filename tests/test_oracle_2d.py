"""Pins of the two-dimensional oracle (the multi-dimensional extension of the paper's
conclusion: tensor-product prediction, eps_l = 2^{d (l - J)} eps, rule (b) at 2^{mu_bar + d}
eps_l). None of them restates the oracle's formulas: exactness on tensor polynomials (and
its loss one degree above), the reduction to the pinned one-dimensional transform, exact
inversion on dyadic data, eps = 0 against the uniform scheme, the compact stream against
the plain mean over the leaf, conservation, tree invariants and the scaling of delta."""

import numpy as np
import pytest

from oracle import adaptive2d as A
from oracle import mr


def poly_averages(J, p, q):
    """Exact cell averages of x^p y^q on the unit square's 2^J x 2^J cells."""
    e = np.arange(2 ** J + 1) / 2 ** J
    ax = (e[1:] ** (p + 1) - e[:-1] ** (p + 1)) / ((p + 1) * (e[1:] - e[:-1]))
    ay = (e[1:] ** (q + 1) - e[:-1] ** (q + 1)) / ((q + 1) * (e[1:] - e[:-1]))
    return np.outer(ax, ay)


@pytest.mark.parametrize("gamma", [1, 2, 3])
def test_tensor_prediction_is_exact_on_tensor_polynomials(gamma):
    """The tensor product of the centered prediction reproduces the children's averages of
    x^p y^q for p, q <= 2 gamma away from the boundary (Sec. 3.1 exactness, in each variable);
    a degree 2 gamma + 1 in x leaves nonzero details."""
    J = 5
    inner = slice(2 * (gamma + 1), 2 ** J - 2 * (gamma + 1))
    for p in range(2 * gamma + 1):
        for q in range(2 * gamma + 1):
            fine = poly_averages(J, p, q)
            coarse = poly_averages(J - 1, p, q)
            d = A.details(fine, coarse, gamma, A.CLAMP)
            assert np.max(np.abs(d[inner, inner])) <= 1e-13, (p, q)
    fine = poly_averages(J, 2 * gamma + 1, 0)
    d = A.details(fine, poly_averages(J - 1, 2 * gamma + 1, 0), gamma, A.CLAMP)
    assert np.max(np.abs(d[inner, inner])) > 1e-9


@pytest.mark.parametrize("gamma", [1, 2])
def test_two_dimensional_transform_reduces_to_the_one_dimensional_one(gamma):
    """Data constant in y: every child of (i, j) is predicted as the one-dimensional child of
    i (the y and cross terms vanish), so the 2D details are the pinned 1D details in each row."""
    rng = np.random.default_rng(3)
    J = 6
    c1 = rng.standard_normal(2 ** (J - 1))
    f1 = rng.standard_normal(2 ** J)
    coarse = np.repeat(c1[:, None], 2 ** (J - 1), axis=1)
    fine = np.repeat(f1[:, None], 2 ** J, axis=1)
    for bc in (A.PERIODIC, A.CLAMP):
        pred2 = A.predict(coarse, gamma, bc)
        pred1 = mr.predict_level(c1[None, :], gamma, bc)[0]
        assert np.array_equal(pred2, np.repeat(pred1[:, None], 2 ** J, axis=1)), bc
        d1 = f1 - pred1
        assert np.array_equal(A.details(fine, coarse, gamma, bc), np.repeat(d1[:, None], 2 ** J, axis=1)), bc


def test_projection_of_prediction_and_exact_inversion():
    """Projection of the four predicted children returns the parent (consistency of the
    prediction, Sec. 3.1); on dyadic data, projection then prediction plus details gives the
    children back bit for bit."""
    rng = np.random.default_rng(4)
    for gamma in (1, 2, 3):
        for bc in (A.PERIODIC, A.CLAMP):
            coarse = rng.integers(-512, 512, size=(16, 16)) * 2.0 ** -10
            assert np.max(np.abs(A.project(A.predict(coarse, gamma, bc)) - coarse)) <= 1e-15
            fine = rng.integers(-512, 512, size=(32, 32)) * 2.0 ** -10
            c = A.project(fine)
            assert np.array_equal(A.predict(c, gamma, bc) + A.details(fine, c, gamma, bc), fine)


def bump(J, kind="smooth"):
    x = (np.arange(2 ** J) + 0.5) / 2 ** J - 0.5
    X, Y = np.meshgrid(x, x, indexing="ij")
    if kind == "smooth":
        return 0.2 + 0.5 * np.exp(-((X - 0.1) ** 2 + (Y + 0.05) ** 2) / 0.02)
    return 0.2 + 0.5 * ((np.abs(X) < 0.2) & (np.abs(Y) < 0.15))


# stable settings of the uniform D2Q4 scheme on these data (Burgers needs lambda = 2: the flux
# speed u along both axes reaches 0.7 + 0.7 > 1)
SCH = [A.D2Q4(A.ADVECTION, 1.0, 1.5, V=(0.4, 0.25)), A.D2Q4(A.BURGERS, 2.0, [1.6, 1.6, 1.2])]


@pytest.mark.parametrize("sch", SCH, ids=["advection", "burgers"])
def test_eps_zero_is_the_uniform_scheme_bitwise(sch):
    J = 5
    u0 = bump(J, "box")
    a = A.Adaptive2D(sch, 2, J, 1, 0.0, 0, A.PERIODIC, u0).step(12)
    r = A.Uniform2D(sch, J, A.PERIODIC, u0).step(12)
    assert a.n_leaves() == 4 ** J
    assert np.array_equal(a.finest_conserved(), r.conserved())


def test_eps_zero_with_a_one_cell_coarsest_level():
    """J_min = 0 under clamp: eps = 0 keeps the full tree and equals the uniform 2D scheme bit
    for bit."""
    J = 5
    u0 = bump(J, "box")
    a = A.Adaptive2D(SCH[1], 0, J, 1, 0.0, 0, A.CLAMP, u0).step(10)
    r = A.Uniform2D(SCH[1], J, A.CLAMP, u0).step(10)
    assert a.n_leaves() == 4 ** J
    assert np.array_equal(a.finest_conserved(), r.conserved())


@pytest.mark.parametrize("bc", [A.PERIODIC, A.CLAMP])
def test_compact_stream_equals_the_mean_over_the_leaf(bc):
    """The strip form of the stream equals the mean of the shifted reconstruction over the
    leaf (Sec. 4.3.2 carried to 2D) up to rounding: same trees, values within 1e-13."""
    J = 5
    u0 = bump(J, "box")
    a = A.Adaptive2D(SCH[1], 2, J, 1, 1e-3, 0, bc, u0)
    b = A.Adaptive2D(SCH[1], 2, J, 1, 1e-3, 0, bc, u0, compact=False)
    for _ in range(6):
        a.step(1)
        b.step(1)
        for l in a.split:
            assert np.array_equal(a.split[l], b.split[l])
        assert np.max(np.abs(a.finest_conserved() - b.finest_conserved())) <= 1e-13
    assert a.n_leaves() < 4 ** J


def test_mass_is_conserved_with_periodic_boundaries():
    J = 5
    u0 = bump(J, "box")
    a = A.Adaptive2D(SCH[1], 2, J, 1, 1e-3, 0, A.PERIODIC, u0)
    m0 = u0.mean()
    for _ in range(5):
        a.step(2)
        total = sum(np.sum(a.F[l][:, mask].sum(axis=0)) * 4.0 ** (-l) for l, mask in a.leaves().items())
        assert abs(total - m0) <= 1e-13


def test_graded_tree_invariants():
    """Along a run: split cells have split parents, the gamma-box of every split cell at its
    own level lies in R, the complete leaves tile the finest lattice once, and edge-adjacent
    leaves differ by at most one level."""
    J, g = 6, 1
    a = A.Adaptive2D(SCH[1], 2, J, g, 1e-3, 0, A.CLAMP, bump(J, "box"))
    for _ in range(4):
        a.step(2)
        R = a.complete_tree()
        for l in range(a.jmin + 1, J):
            p = np.argwhere(a.split[l])
            assert np.all(a.split[l - 1][p[:, 0] // 2, p[:, 1] // 2])
            for di in range(-g, g + 1):
                for dj in range(-g, g + 1):
                    ii = A.bc_index(p[:, 0] + di, 2 ** l, A.CLAMP)
                    jj = A.bc_index(p[:, 1] + dj, 2 ** l, A.CLAMP)
                    assert np.all(R[l][ii, jj])
        level = np.full((2 ** J, 2 ** J), -1)
        for l, mask in a.leaves().items():
            L = 2 ** (J - l)
            for i, j in np.argwhere(mask):
                assert np.all(level[i * L:(i + 1) * L, j * L:(j + 1) * L] == -1)
                level[i * L:(i + 1) * L, j * L:(j + 1) * L] = l
        assert np.all(level >= 0)
        assert np.max(np.abs(np.diff(level, axis=0))) <= 1 and np.max(np.abs(np.diff(level, axis=1))) <= 1


def test_delta_scales_with_eps():
    """Sec. 4.4 carried to 2D: delta = ||M_ref - m_hathat||_1 decreases with eps, with a log-log
    slope near one, and stays of the order of eps."""
    J = 6
    sch = SCH[0]
    u0 = bump(J, "smooth")
    n = 16
    ref = A.Uniform2D(sch, J, A.PERIODIC, u0).step(n).conserved()
    ds = []
    epss = [1e-2, 1e-3, 1e-4]
    for eps in epss:
        a = A.Adaptive2D(sch, 2, J, 1, eps, 0, A.PERIODIC, u0).step(n)
        ds.append(float(np.sum(np.abs(a.finest_conserved() - ref))) / 4 ** J)
    assert ds[0] > ds[1] > ds[2] > 0, ds
    slopes = np.diff(np.log10(ds)) / np.diff(np.log10(epss))
    assert np.all((slopes > 0.5) & (slopes < 1.5)), (ds, slopes)
    assert all(d <= 5 * e for d, e in zip(ds, epss)), ds


def test_d2q4_collision_is_the_moment_relaxation():
    """D2Q4: the fixed-order collision equals m = M f, relaxation of m1, m2, m3 towards
    (phi_x(u), phi_y(u), 0), f* = M^-1 m* (Sec. 2.1.1 in two dimensions); the equilibrium
    populations carry the fluxes as their first moments."""
    rng = np.random.default_rng(7)
    for sch in SCH:
        lam = sch.lam
        M = np.array([[1.0, 1.0, 1.0, 1.0], [lam, -lam, 0.0, 0.0], [0.0, 0.0, lam, -lam],
                      [lam * lam, lam * lam, -lam * lam, -lam * lam]])
        f = rng.uniform(0.0, 0.5, size=(4, 50))
        m = M @ f
        px, py = (sch.V[0] * m[0], sch.V[1] * m[0]) if sch.physics == A.ADVECTION else (m[0] ** 2 / 2, m[0] ** 2 / 2)
        ms = m.copy()
        for k, eq in ((1, px), (2, py), (3, 0.0)):
            ms[k] = (1 - sch.s[k - 1]) * m[k] + sch.s[k - 1] * eq
        assert np.max(np.abs(sch.collide(f) - np.linalg.solve(M, ms))) <= 1e-14
        u = rng.uniform(0.1, 1.0, 50)
        me = M @ sch.equilibrium(u)
        fx, fy = (sch.V[0] * u, sch.V[1] * u) if sch.physics == A.ADVECTION else (u ** 2 / 2, u ** 2 / 2)
        assert np.allclose(me, np.stack([u, fx, fy, np.zeros_like(u)]), rtol=0, atol=1e-15)
