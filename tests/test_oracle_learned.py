"""Pins of the oracle's refinement predictor (not a method of the paper; parity with the
paper is unpinned, so these pin the network and the judge against closed forms, finite
differences and the plain rule (b) of Sec. 4.2)."""

import numpy as np
import pytest

import workloads as W
from oracle import learned as Lr
from oracle import metrics
from oracle.adaptive import AdaptiveMRLBM
from oracle.lattice import scheme_from_params
from oracle.reference import UniformLBM


def test_bf16_rounding_ties_to_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7 + 2 ** -10, -2.5, 3.0e-3], dtype=np.float32)
    got = Lr.bf16_round(x)
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, np.float32(3.0e-3)], dtype=np.float32)
    assert got[:5].tolist() == want[:5].tolist()
    assert abs(got[5] - 3e-3) <= 3e-3 * 2 ** -8
    assert Lr.NPARAM == 6337


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = W.mlp_init(1).astype(np.float64) + 0.05 * rng.standard_normal(Lr.NPARAM)
    X = rng.standard_normal((40, Lr.NIN)) * 0.5
    y = (rng.uniform(size=40) < 0.4).astype(float)
    loss, g = Lr.loss_and_grad64(theta, X, y, 2.0, quantize=False)
    idx = rng.choice(Lr.NPARAM, size=60, replace=False)
    idx = np.concatenate([idx, [Lr.NPARAM - 1, 64 * 32 + 3, 64 * 32 + 64 + 5]])  # b3, b1, W2 entries
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (Lr.loss_and_grad64(tp, X, y, 2.0, quantize=False)[0]
              - Lr.loss_and_grad64(tm, X, y, 2.0, quantize=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_deployment_sums_match_float64():
    rng = np.random.default_rng(2)
    wbf = Lr.bf16_round(W.mlp_init(3) + 0.1 * rng.standard_normal(Lr.NPARAM).astype(np.float32))
    X = rng.uniform(-1, 1, size=(30, Lr.NIN)).astype(np.float32)
    X[:, -1] = 0
    got = Lr.logits32(wbf, X)
    P = Lr.unpack(wbf.astype(np.float64))
    h1 = np.maximum(X.astype(np.float64) @ P["W1"].T + P["b1"], 0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0)
    ref = h2 @ P["w3"] + P["b3"][0]
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-5)


def constant_network(logit):
    t = np.zeros(Lr.NPARAM, dtype=np.float32)
    t[-1] = logit
    return Lr.bf16_round(t)


def build(p, mc):
    return AdaptiveMRLBM(scheme_from_params(p), p["jmin"], p["jmax"], p["gamma"], p["eps"], p["mu_bar"], p["bc"], mc)


def test_features_of_a_step():
    """A unit step: the pair straddling the jump has a large detail; its feature is
    d / (|d| + eps) computed from the closed-form detail of the step averages."""
    p, mc = W.advection(0, jmax=7)
    mc = np.where(np.arange(128) < 64, 0.0, 1.0)[None, :]
    a = build(p, mc)
    a.project_up()
    l = 5
    X = Lr.features(a, l, np.array([16]))
    # level 6 cells 32 and 33 straddle... cell (6, 32) is 1, its parent (5, 16) averages (6, 32),(6, 33)
    d = Lr.pair_details(a, l, np.array([14, 15, 16, 17, 18]))
    eps_l1 = np.ldexp(p["eps"], l + 1 - p["jmax"])
    q = a.sch.q
    for di in range(5):
        for h in range(q):
            assert X[0, di * q + h] == np.float32(d[h, di] / (abs(d[h, di]) + eps_l1))
    assert X[0, 5 * q] == np.float32((l + 1) / p["jmax"])
    assert np.all(X[0, 5 * q + 1:] == 0)
    assert np.all(np.abs(X) < 1)


@pytest.mark.parametrize("kind", ["euler", "burgers"])
def test_always_refining_network_is_the_plain_method(kind):
    p, mc = W.small_case(kind, seed=1, jmax=8, eps=1e-4)
    plain = build(p, mc).step(25)
    a = build(p, mc)
    Lr.LearnedRefinement(a, constant_network(1.0)).step(25)
    assert {l: v.tolist() for l, v in a.split.items()} == {l: v.tolist() for l, v in plain.split.items()}
    assert np.array_equal(a.finest_populations(), plain.finest_populations())


def test_never_refining_network_is_caught_by_the_judge():
    p, mc = W.euler(2, jmax=8, eps=1e-4)
    ref = UniformLBM(scheme_from_params(p), p["jmax"], p["bc"], mc).step(40)
    plain = build(p, mc).step(40)
    a = build(p, mc)
    lr = Lr.LearnedRefinement(a, constant_network(-1.0))
    lr.step(40)
    assert lr.misses > 0 and lr.redos > 0
    d_plain = metrics.delta(ref.conserved(), plain.finest_conserved(), -1, 1)
    d_lrn = metrics.delta(ref.conserved(), a.finest_conserved(), -1, 1)
    for c in range(3):
        assert d_lrn[c] <= 2 * d_plain[c] + p["eps"]


def test_record_mode_labels():
    p, mc = W.euler(3, jmax=8, eps=1e-4)
    a = build(p, mc)
    lr = Lr.LearnedRefinement(a, None, mode="record")
    lr.step(10)
    X = np.concatenate(lr.samples_X)
    y = np.concatenate(lr.samples_y)
    assert X.shape[1] == Lr.NIN and X.shape[0] == y.shape[0] > 0
    assert set(np.unique(y)).issubset({0.0, 1.0})
    # record mode runs the plain rule (b)
    plain = build(p, mc).step(10)
    assert np.array_equal(a.finest_populations(), plain.finest_populations())
