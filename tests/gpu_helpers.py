"""Shared helpers of the GPU parity tests: oracle construction and comparisons.

Leaf sets must agree exactly; a differing decision is tolerated only when the oracle's
detail at that decision lies within 1e-12 (relative) of its threshold, in which case the
flip is reported and the comparison of that run stops. Moments must agree to 1e-12
relative (max-norm over max(|m|, 1)) on the FP64 path.
"""

import numpy as np

from oracle.adaptive import AdaptiveMRLBM
from oracle.lattice import scheme_from_params

MOMENT_TOL = 1e-12
FLIP_MARGIN = 1e-12


def make_oracle(p, mc, eps=None):
    e = p["eps"] if eps is None else eps
    return AdaptiveMRLBM(scheme_from_params(p), p["jmin"], p["jmax"], p["gamma"], e, p["mu_bar"], p["bc"], mc,
                         collision=p.get("collision", "leaves"))


def threshold_margin(ora):
    """Smallest |D / thr - 1| over the decisions of the oracle's last adaptation."""
    if ora.last_D is None:
        return np.inf
    J = ora.jmax
    best = np.inf
    for l, D in ora.last_D.items():
        m = D >= 0
        if not m.any():
            continue
        thr = np.ldexp(ora.eps, l + 1 - J)
        thrb = np.ldexp(ora.eps, ora.mu_bar + 1 + l + 1 - J)
        for t in (thr, thrb):
            if t > 0:
                best = min(best, float(np.min(np.abs(D[m] / t - 1.0))))
    return best


def rel_err(got, want):
    return float(np.max(np.abs(got - want)) / max(1.0, float(np.max(np.abs(want)))))


def compare_leaves(run, ora, label=""):
    """Returns (same, flip_report). Raises on a difference that is not a near-threshold flip."""
    lv, ix = run.leaves()
    olv, oix = ora.leaf_list()
    if lv.shape == olv.shape and np.array_equal(lv, olv) and np.array_equal(ix, oix):
        return True, None
    margin = threshold_margin(ora)
    msg = f"{label}: leaf sets differ (gpu {lv.size}, oracle {olv.size}); closest threshold margin {margin:.3e}"
    if margin <= FLIP_MARGIN:
        print("reported flip:", msg)
        return False, msg
    raise AssertionError(msg)


def compare_run(run, ora, label="", tol=MOMENT_TOL):
    same, flip = compare_leaves(run, ora, label)
    if not same:
        return False
    got = run.moments()
    want = ora.leaf_conserved()
    err = rel_err(got, want)
    assert err <= tol, f"{label}: leaf moments differ by {err:.3e}"
    return True
