"""Shared helpers of the GPU parity tests: oracle construction and comparisons.

Leaf sets must agree exactly on the FP64 path: any differing leaf fails the test. When
they differ, the failure message locates the first time step at which the trees
diverged (both sides are re-run one step at a time from t = 0) and gives the closest
threshold margin |D / thr - 1| over the decisions the oracle took at that step, so that
a decision within 1e-12 of its threshold (rounding order) is told apart from a real
error; neither is accepted. Moments must agree to 1e-12 relative (max-norm over
max(|m|, 1)) on the FP64 path.

FP32 storage is held to 1e-5 relative plus the eps bound (``fp32_bound``), with the two
parts reported separately.
"""

import numpy as np

from oracle import metrics
from oracle.adaptive import AdaptiveMRLBM
from oracle.lattice import scheme_from_params
from oracle.reference import UniformLBM

MOMENT_TOL = 1e-12
FLIP_MARGIN = 1e-12
FP32_REL = 1e-5


def make_oracle(p, mc, eps=None):
    e = p["eps"] if eps is None else eps
    return AdaptiveMRLBM(scheme_from_params(p), p["jmin"], p["jmax"], p["gamma"], e, p["mu_bar"], p["bc"], mc,
                         collision=p.get("collision", "leaves"))


def threshold_margin(ora):
    """Smallest |D / thr - 1| over the decisions (T_eps and rule (b)) of the oracle's most
    recent adaptation."""
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


def same_leaves(run_leaves, ora):
    lv, ix = run_leaves
    olv, oix = ora.leaf_list()
    return lv.shape == olv.shape and np.array_equal(lv, olv) and np.array_equal(ix, oix)


def first_divergence(make_run, p, mc, upto):
    """Re-run a fresh GPU run (``make_run()``, an object with step() and leaves()) and a
    fresh oracle one step at a time from t = 0; return (step, margin) for the first step
    after which their leaf sets differ (margin: the closest threshold margin of the
    oracle's adaptation at that step), or (None, inf) if none does within ``upto`` steps."""
    run = make_run()
    ora = make_oracle(p, mc)
    try:
        for s in range(1, upto + 1):
            run.step(1)
            ora.step(1)
            if not same_leaves(run.leaves(), ora):
                return s, threshold_margin(ora)
        return None, np.inf
    finally:
        run.close()


def leaf_mismatch(label, gpu_leaves, ora, locate=None):
    """AssertionError describing a leaf-set difference; ``locate`` () -> (step, margin)
    finds where the trees diverged."""
    lv = gpu_leaves[0]
    msg = f"{label}: leaf sets differ (gpu {lv.size}, oracle {ora.n_leaves()})"
    if locate is not None:
        step, margin = locate()
        near = "within" if margin <= FLIP_MARGIN else "not within"
        msg += (f"; first differing step {step}, closest threshold margin there {margin:.3e} "
                f"({near} {FLIP_MARGIN:g} of a threshold)")
    return AssertionError(msg)


def compare_run(run, ora, label="", tol=MOMENT_TOL, locate=None):
    """Leaf sets bit-exact (a difference raises, located by ``locate`` when given) and leaf
    moments within ``tol``."""
    lvs = run.leaves()
    if not same_leaves(lvs, ora):
        raise leaf_mismatch(label, lvs, ora, locate)
    got = run.moments()
    want = ora.leaf_conserved()
    err = rel_err(got, want)
    assert err <= tol, f"{label}: leaf moments differ by {err:.3e}"
    return True


def fp32_bound(p, mc, m32, m64, nsteps, ref=None):
    """FP32-storage bound against the FP64 oracle: the FP32 run m32 (finest conserved
    moments) stays within 1e-5 relative plus the eps bound of the uniform reference scheme,

        delta32 = ||ref - m32||_1 <= 1e-5 ||ref||_1 + C eps,   C = max(2 delta64 / eps, 1),

    where delta64 = ||ref - m64||_1 is the FP64 oracle's own perturbation (the eps bound's
    constant is pinned by the oracle's recorded run, as every eps bound here). Returns a dict
    of the parts per conserved moment; ``ok`` is True when every moment passes."""
    if ref is None:
        ref = UniformLBM(scheme_from_params(p), p["jmax"], p["bc"], mc).step(nsteps).conserved()
    x0, x1 = p["x_min"], p["x_max"]
    d32 = np.asarray(metrics.delta(ref, m32, x0, x1))
    d64 = np.asarray(metrics.delta(ref, m64, x0, x1))
    d3264 = np.asarray(metrics.delta(m64, m32, x0, x1))
    norm = np.asarray(metrics.delta(np.zeros_like(ref), ref, x0, x1))
    eps = p["eps"]
    out = {"delta32": d32.tolist(), "delta64": d64.tolist(), "fp32_vs_fp64": d3264.tolist(),
           "rel_part": (FP32_REL * norm).tolist(), "eps_part": [], "ok": True}
    for c in range(ref.shape[0]):
        C = max(2.0 * d64[c] / eps, 1.0) if eps > 0 else 0.0
        out["eps_part"].append(C * eps)
        if not d32[c] <= FP32_REL * norm[c] + C * eps:
            out["ok"] = False
    return out
