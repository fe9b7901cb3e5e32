"""Pins of the oracle's multiresolution operators against closed forms and invariants.

Paper passages: Sec. 3.1 (projection, centered prediction exact on averages of
polynomials of degree <= 2 gamma), Sec. 3.2 (details, eq. DetailRedundancy, the MR
transform and its inverse, vanishing moments of the dual wavelet, Proposition Details
decay).
"""

import numpy as np
import pytest

from oracle import mr


def poly_avgs_unit(k, d):
    """Averages of (d+1) x^d over [k, k+1]: an integer."""
    k = np.asarray(k, dtype=np.float64)
    return (k + 1) ** (d + 1) - k ** (d + 1)


def poly_avgs_half(k, d, delta):
    """Averages of (d+1) x^d over the child half-cells of [k, k+1]; dyadic rationals."""
    k = np.asarray(k, dtype=np.float64)
    a = k + 0.5 * delta
    return 2.0 * ((a + 0.5) ** (d + 1) - a ** (d + 1))


@pytest.mark.parametrize("gamma", [1, 2, 3])
def test_prediction_exact_on_polynomials(gamma):
    """Prediction reproduces the children's averages exactly for degree <= 2 gamma and not
    for degree 2 gamma + 1 (Sec. 3.1). All values are dyadic, so equality is exact."""
    n = 40
    k = np.arange(n) - n // 2
    interior = np.arange(gamma, n - gamma)
    for d in range(0, 2 * gamma + 2):
        coarse = poly_avgs_unit(k, d)[None, :]
        for delta in (0, 1):
            c = 2 * interior + delta
            pred = mr.predict_cells(coarse, c, gamma, mr.CLAMP)[0]
            exact = poly_avgs_half(k[interior], d, delta)
            if d <= 2 * gamma:
                assert np.array_equal(pred, exact), (gamma, d, delta)
            else:
                assert not np.allclose(pred, exact), (gamma, d, delta)


def test_gamma3_coefficient_sign_reading():
    """The printed c_3 = +5/1024 breaks exactness on degree 1; the read sign restores it."""
    k = np.arange(30) - 15
    coarse = poly_avgs_unit(k, 1)
    p = np.arange(3, 27)
    c1, c2, _ = mr.PRED_COEFFS[3]
    printed = coarse[p] + (c1 * (coarse[p + 1] - coarse[p - 1]) + c2 * (coarse[p + 2] - coarse[p - 2])
                           + (5 / 1024) * (coarse[p + 3] - coarse[p - 3]))
    assert not np.array_equal(printed, poly_avgs_half(k[p], 1, 0))
    assert mr.PRED_COEFFS[3][2] == -5 / 1024


def dyadic_random(rng, shape, bits=10):
    return rng.integers(-2 ** 12, 2 ** 12, size=shape).astype(np.float64) * 2.0 ** -bits


@pytest.mark.parametrize("gamma", [1, 2, 3])
@pytest.mark.parametrize("bc", [mr.PERIODIC, mr.CLAMP])
def test_consistency_and_redundancy(gamma, bc):
    """P_v o P_^ = identity (Definition Prediction operator) and d_{2k} = -d_{2k+1}
    (eq. DetailRedundancy), exact on dyadic data."""
    rng = np.random.default_rng(7)
    coarse = dyadic_random(rng, (3, 32))
    pred = mr.predict_level(coarse, gamma, bc)
    assert np.array_equal(mr.project(pred), coarse)
    fine = dyadic_random(rng, (3, 64))
    parent = mr.project(fine)
    pred = mr.predict_level(parent, gamma, bc)
    d = fine - pred
    assert np.array_equal(d[:, 0::2], -d[:, 1::2])


@pytest.mark.parametrize("gamma", [1, 2, 3])
def test_mr_transform_roundtrip_bitwise(gamma):
    """M_R maps f_J to (f_Jmin, details of even children) with the same cardinality, and the
    inverse (prediction plus details, level by level) returns f_J bit for bit on dyadic
    data (Sec. 3.2, eq. actionMultiresolutionTransform)."""
    rng = np.random.default_rng(11)
    J, jmin = 8, 3
    fJ = dyadic_random(rng, (2, 2 ** J))
    levels = {J: fJ}
    for l in range(J - 1, jmin - 1, -1):
        levels[l] = mr.project(levels[l + 1])
    dets = {}
    for l in range(jmin, J):
        p = np.arange(2 ** l)
        dets[l + 1] = mr.details_even(levels[l + 1], levels[l], p, gamma, mr.PERIODIC)
    count = levels[jmin].shape[1] + sum(v.shape[1] for v in dets.values())
    assert count == 2 ** J
    f = levels[jmin]
    for l in range(jmin, J):
        pred = mr.predict_level(f, gamma, mr.PERIODIC)
        nxt = pred.copy()
        nxt[:, 0::2] = pred[:, 0::2] + dets[l + 1]
        nxt[:, 1::2] = pred[:, 1::2] - dets[l + 1]
        f = nxt
    assert np.array_equal(f, fJ)


def test_projection_conserves_level_averages():
    """sum_k 2^-j f_{j,k} is the same on every level (exact on dyadic data)."""
    rng = np.random.default_rng(3)
    f = dyadic_random(rng, (1, 1024))
    tot = f.sum() / 1024
    for _ in range(8):
        f = mr.project(f)
        assert f.sum() / f.shape[1] == tot


def test_details_vanish_on_polynomials_periodic_free():
    """Details of averages of a degree-2 polynomial are zero away from the boundary for
    gamma = 1 (dual wavelet vanishing moments, Sec. 3.2)."""
    k = np.arange(64) - 32
    fine = poly_avgs_half(np.repeat(k, 1), 2, 0)
    # fine level with cells of width 1/2: build children of unit cells
    kids = np.empty(128)
    kids[0::2] = poly_avgs_half(k, 2, 0)
    kids[1::2] = poly_avgs_half(k, 2, 1)
    parent = mr.project(kids[None, :])
    assert np.array_equal(parent[0], poly_avgs_unit(k, 2))
    p = np.arange(2, 62)
    d = mr.details_even(kids[None, :], parent, p, 1, mr.CLAMP)
    assert np.all(d == 0.0)
    del fine


def _avg_sin(n):
    e = np.linspace(0.0, 1.0, n + 1)
    w = 2 * np.pi
    return (np.cos(w * e[:-1]) - np.cos(w * e[1:])) / (w * (e[1:] - e[:-1]))


@pytest.mark.parametrize("gamma,rate", [(1, 3.0), (2, 5.0)])
def test_detail_decay_rates(gamma, rate):
    """Smooth data: max |d_j| decays like 2^{-j mu} with mu = 2 gamma + 1; a jump keeps
    O(1) details at every level (Proposition Details decay)."""
    mx = []
    for j in range(5, 10):
        fine = _avg_sin(2 ** (j + 1))[None, :]
        d = mr.details_even(fine, mr.project(fine), np.arange(2 ** j), gamma, mr.PERIODIC)
        mx.append(np.max(np.abs(d)))
    slopes = -np.diff(np.log2(mx))
    assert np.all(np.abs(slopes - rate) < 0.35), slopes
    jumps = []
    for j in range(5, 10):
        n = 2 ** (j + 1)
        fine = np.where(np.arange(n) < n // 3, 1.0, 0.0)[None, :]
        d = mr.details_even(fine, mr.project(fine), np.arange(2 ** j), gamma, mr.PERIODIC)
        jumps.append(np.max(np.abs(d)))
    assert min(jumps) > 0.05


def test_level_thresholds_exact():
    assert mr.level_threshold(1e-4, 10, 10) == 1e-4
    assert mr.level_threshold(1e-4, 7, 10) == 1e-4 / 8
    assert mr.level_threshold(0.0, 3, 10) == 0.0
