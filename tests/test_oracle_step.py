"""Pins of the oracle's adaptive step: tree operators, data transfer, stream, error bound.

Paper passages: Sec. 3.3 (tree, complete leaves partition the domain, graded tree and the
smallest graded tree), Sec. 3.4 (T_eps, Proposition ErrorControl), Sec. 4.1-4.2 (mesh
adaptation, H_eps rules), Sec. 4.3.2 (uncompacted and compact stream; sigma = 0 gives the
identity), Sec. 4.4 (Proposition Additional error estimate: delta <= C eps), and the
eps = 0 special case where the adaptive scheme is the uniform scheme L.
"""

import numpy as np
import pytest

import workloads as W
from oracle.adaptive import AdaptiveMRLBM
from oracle.brute import BruteMRLBM
from oracle.lattice import scheme_from_params
from oracle.reference import UniformLBM
from oracle import metrics, mr

KINDS = ["advection", "burgers", "burgers_d1q2", "shallow", "shallow_d1q3", "shallow_d1q5", "euler"]


def build(p, mc, eps=None, cls=AdaptiveMRLBM, **kw):
    sch = scheme_from_params(p)
    e = p["eps"] if eps is None else eps
    return cls(sch, p["jmin"], p["jmax"], p["gamma"], e, p["mu_bar"], p["bc"], mc, **kw)


@pytest.mark.parametrize("kind", KINDS)
def test_eps_zero_is_uniform_scheme_bitwise(kind):
    """eps = 0 keeps every detail (the test is >=), so Lambda stays full and the adaptive
    step is the reference scheme L on the finest lattice, bit for bit."""
    p, mc = W.small_case(kind, seed=1, jmax=8)
    a = build(p, mc, eps=0.0).step(40)
    r = UniformLBM(scheme_from_params(p), p["jmax"], p["bc"], mc).step(40)
    assert a.n_leaves() == 2 ** p["jmax"]
    assert np.array_equal(a.finest_populations(), r.F)


@pytest.mark.parametrize("kind", ["advection", "burgers", "shallow", "euler", "shallow_d1q5"])
@pytest.mark.parametrize("seed", [0, 1])
def test_dense_oracle_matches_set_twin(kind, seed):
    """Dense-level oracle vs the literal set twin on J = 6: identical leaf sets at every
    step; values differ only by rounding (compact vs uncompacted stream)."""
    for eps in (1e-2, 1e-3):
        p, mc = W.small_case(kind, seed=seed, jmax=6)
        a = build(p, mc, eps=eps)
        b = build(p, mc, eps=eps, cls=BruteMRLBM)
        for _ in range(15):
            a.step(1)
            b.step()
            la = {l: list(np.nonzero(m)[0]) for l, m in a.leaves().items() if m.any()}
            assert la == b.leaf_levels()
            fa, fb = a.finest_populations(), b.finest_populations()
            assert np.max(np.abs(fa - fb)) <= 1e-13 * max(1.0, np.max(np.abs(fb)))


@pytest.mark.parametrize("kind", ["advection", "burgers", "shallow_d1q5"])
def test_coarsest_level_zero_matches_set_twin(kind):
    """J_min = 0 (a one-cell coarsest level, clamped): the dense oracle against the literal set
    twin at every step (identical leaf sets, values within rounding), and eps = 0 equal to the
    reference scheme bit for bit."""
    p, mc = W.small_case(kind, seed=2, jmax=6)
    p["jmin"], p["bc"] = 0, 1
    a = build(p, mc, eps=1e-3)
    b = build(p, mc, eps=1e-3, cls=BruteMRLBM)
    for _ in range(15):
        a.step(1)
        b.step()
        la = {l: list(np.nonzero(m)[0]) for l, m in a.leaves().items() if m.any()}
        assert la == b.leaf_levels()
        fa, fb = a.finest_populations(), b.finest_populations()
        assert np.max(np.abs(fa - fb)) <= 1e-13 * max(1.0, np.max(np.abs(fb)))
    z = build(p, mc, eps=0.0).step(20)
    r = UniformLBM(scheme_from_params(p), p["jmax"], p["bc"], mc).step(20)
    assert np.array_equal(z.finest_populations(), r.F)


def check_tree_invariants(a):
    J, jmin, g = a.jmax, a.jmin, a.gamma
    R = a.complete_tree()
    S = a.leaves()
    # tree: split cells below J_min+1 have split parents (no orphans)
    for l in range(jmin + 1, J):
        p = np.nonzero(a.split[l])[0]
        assert np.all(a.split[l - 1][p // 2])
    # graded: split (l, p) => (l, p + delta) in R, |delta| <= gamma
    for l in range(jmin + 1, J):
        p = np.nonzero(a.split[l])[0]
        for dl in range(-g, g + 1):
            assert np.all(R[l][mr.bc_index(p + dl, 2 ** l, a.bc)])
    # complete leaves partition the finest lattice
    cover = np.zeros(2 ** J, dtype=int)
    for l, m in S.items():
        for k in np.nonzero(m)[0]:
            L = 2 ** (J - l)
            cover[k * L:(k + 1) * L] += 1
    assert np.all(cover == 1)
    # 2:1 balance between spatially adjacent leaves (a consequence of grading, gamma >= 1)
    lv, ix = a.leaf_list()
    d = np.abs(np.diff(lv))
    assert np.all(d <= 1)


@pytest.mark.parametrize("kind", ["advection", "burgers", "euler"])
def test_tree_invariants_along_a_run(kind):
    p, mc = W.small_case(kind, seed=2, jmax=9)
    a = build(p, mc)
    for _ in range(30):
        a.step(1)
        check_tree_invariants(a)


def random_split(rng, jmin, J, density):
    split = {}
    for l in range(jmin, J):
        split[l] = rng.uniform(size=2 ** l) < density
    return split


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("gamma", [1, 2])
def test_grading_sweep_is_smallest_graded_tree(bc, gamma):
    """One fine-to-coarse sweep equals the fixed point of the graded-tree condition
    (set twin), on random split patterns."""
    rng = np.random.default_rng(10 + bc + 3 * gamma)
    p, mc = W.small_case("advection", seed=0, jmax=7)
    p["bc"] = bc
    p["gamma"] = gamma
    jmin = 3 if gamma == 2 else 2
    p["jmin"] = jmin
    for trial in range(20):
        a = build(p, mc)
        b = build(p, mc, cls=BruteMRLBM)
        sp = random_split(rng, jmin, 7, 0.08)
        got = a.grade({l: v.copy() for l, v in sp.items()})
        lam = {(jmin, k) for k in range(2 ** jmin)}
        for l, v in sp.items():
            for k in np.nonzero(v)[0]:
                lam.add((l + 1, 2 * int(k)))
        want = b.grade(lam)
        want_split = {l: np.zeros(2 ** l, dtype=bool) for l in range(jmin, 7)}
        for (l, k) in want:
            if l > jmin:
                want_split[l - 1][k // 2] = True
        for l in range(jmin, 7):
            assert np.array_equal(got[l], want_split[l]), (trial, l)


def test_stream_identity_for_resting_population():
    """sigma^h = 0: the reconstructed stream returns the collided value itself (Sec. 4.3.2)."""
    p, mc = W.small_case("burgers", seed=4, jmax=8)
    a = build(p, mc).step(5)
    a.adapt()
    a.collide_leaves()
    before = {l: a.F[l][0].copy() for l in a.F}
    a.project_up()
    a.stream()
    for l, m in a.leaves().items():
        k = np.nonzero(m)[0]
        assert np.array_equal(a.F[l][0, k], before[l][k])


@pytest.mark.parametrize("kind", ["advection", "burgers_d1q2", "burgers", "shallow_d1q5"])
def test_mass_conserved_periodic(kind):
    """With periodic boundaries the interface terms of the compact stream telescope and
    collision keeps the conserved moments: sum over leaves of dx_l m_c is constant (for
    D1Q5 both h and hu, with the two-cell stream terms)."""
    p, mc = W.small_case(kind, seed=5, jmax=9)
    p = dict(p, bc=W.PERIODIC)
    a = build(p, mc)
    m0 = np.sum(mc, axis=1) / 2 ** p["jmax"]
    for _ in range(8):
        a.step(10)
        lv, _ = a.leaf_list()
        for c in range(mc.shape[0]):
            u = a.leaf_conserved()[c]
            m = np.sum(u * 2.0 ** -lv.astype(float))
            assert abs(m - m0[c]) <= 1e-13 * max(1.0, abs(m0[c])), (c, m, m0[c])


def test_static_compression_error_bounded_independently_of_J():
    """Proposition ErrorControl: thresholding then grading then reconstructing loses at
    most C_MR eps in l1, with C_MR not growing with the number of levels."""
    eps = 1e-4
    ratios = []
    for J in (8, 10, 12):
        p, mc = W.advection(3, jmax=J, eps=eps)
        a = build(p, mc)
        f0 = a.F[J].copy()
        a.project_up()
        D = a.details()
        keep = a.threshold(D)
        new = a.grade({l: keep[l].copy() for l in keep})
        # leaves of the compressed tree hold projections of the original data
        a.split = new
        a.project_up()
        rec = a.reconstruct()[J]
        err = metrics.l1(rec - f0, 2.0 / 2 ** J)
        ratios.append(err / eps)
    assert max(ratios) < 4.0, ratios
    assert max(ratios) / max(min(ratios), 1e-30) < 10.0, ratios


def test_delta_scales_linearly_with_eps():
    """Sec. 4.4: delta <= C eps; the measured delta is monotone in eps with a log-log slope
    near one."""
    p, mc = W.advection(1, jmax=9)
    ref = UniformLBM(scheme_from_params(p), 9, p["bc"], mc).step(150)
    ds = []
    epss = [1e-3, 1e-4, 1e-5]
    for eps in epss:
        a = build(p, mc, eps=eps).step(150)
        ds.append(metrics.delta(ref.conserved(), a.finest_conserved(), -1.0, 1.0)[0])
    assert ds[0] > ds[1] > ds[2] > 0
    slopes = np.diff(np.log10(ds)) / np.diff(np.log10(epss))
    assert np.all((slopes > 0.6) & (slopes < 1.4)), slopes
    assert max(d / e for d, e in zip(ds, epss)) < 20.0


def test_compression_reported():
    p, mc = W.advection(0, jmax=9)
    a = build(p, mc).step(20)
    cr = a.compression()
    assert 50.0 < cr < 100.0
    assert abs(metrics.average_compression(a.leaf_history, 9) - metrics.compression(np.mean(a.leaf_history), 9)) < 1e-12
