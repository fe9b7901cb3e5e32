"""Multiresolution operators on dense level arrays (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed
-----------------------
* Sec. 3, nested lattices: level j has N_j = 2^j cells; cell (j, k) has children
  (j+1, 2k) and (j+1, 2k+1).
* Sec. 3.1, Definition (Projection operator): the parent average is half the sum of
  the two children.
* Sec. 3.1, centered polynomial prediction: the child (j+1, 2k+delta) is predicted as
  f_{j,k} + (-1)^delta * sum_{alpha=1..gamma} c_alpha (f_{j,k+alpha} - f_{j,k-alpha}),
  exact on averages of polynomials of degree <= 2 gamma.
* Sec. 3.2, Definition (Detail): d = f - f_hat; siblings carry opposite details
  (eq. DetailRedundancy), so only the even child's detail is kept.
* Sec. 3.4, Proposition (ErrorControl): level thresholds eps_j = 2^(j - J) eps.

Readings
--------
* gamma = 3: the paper prints c_3 = +5/1024; the moment conditions for exactness on
  degrees 1, 3, 5 force c_3 = -5/1024, which is what is used here.
* Boundary handling, which the paper leaves open: an index outside [0, N_j) at level j
  is either wrapped (periodic) or mapped to the nearest in-range cell (clamp), in
  every stencil at every level.

The prediction sum is accumulated alpha = 1, 2, ... in order and the parent value is
added last (f + acc for the even child, f - acc for the odd child). The GPU side must
use the same order so that details, and thus leaf sets, agree bit for bit.
"""

import numpy as np

PERIODIC, CLAMP = 0, 1

# Prediction coefficients c_alpha, Sec. 3.1 (gamma = 3 with the sign reading above).
PRED_COEFFS = {
    1: (-1.0 / 8.0,),
    2: (-22.0 / 128.0, 3.0 / 128.0),
    3: (-201.0 / 1024.0, 11.0 / 256.0, -5.0 / 1024.0),
}


def bc_index(idx, n, bc):
    """Map (possibly out-of-range) integer indices at a level with n cells."""
    idx = np.asarray(idx)
    if bc == PERIODIC:
        return np.mod(idx, n)
    return np.clip(idx, 0, n - 1)


def project(fine):
    """Projection of a whole fine level (q, 2n) onto its parent level (q, n)."""
    return 0.5 * (fine[:, 0::2] + fine[:, 1::2])


def project_cells(fine, p):
    """Projection at parent indices p only."""
    p = np.asarray(p)
    return 0.5 * (fine[:, 2 * p] + fine[:, 2 * p + 1])


def predict_cells(coarse, c, gamma, bc):
    """Predicted values of the children c (indices at level j+1) from the parent level
    array ``coarse`` (q, N_j)."""
    c = np.asarray(c)
    n = coarse.shape[1]
    p = c // 2
    odd = (c % 2).astype(bool)
    coeffs = PRED_COEFFS[gamma]
    acc = None
    for a, ca in enumerate(coeffs, start=1):
        term = ca * (coarse[:, bc_index(p + a, n, bc)] - coarse[:, bc_index(p - a, n, bc)])
        acc = term if acc is None else acc + term
    f0 = coarse[:, p]
    return np.where(odd[None, :], f0 - acc, f0 + acc)


def predict_level(coarse, gamma, bc):
    """Predicted values on the whole finer level (q, 2 N_j)."""
    n = coarse.shape[1]
    return predict_cells(coarse, np.arange(2 * n), gamma, bc)


def details_even(fine, coarse, p, gamma, bc):
    """Details of the even children (j+1, 2p) for parent indices p: d = f - f_hat."""
    p = np.asarray(p)
    return fine[:, 2 * p] - predict_cells(coarse, 2 * p, gamma, bc)


def level_threshold(eps, level, jmax):
    """eps_level = 2^(level - J) eps, computed exactly with ldexp."""
    return float(np.ldexp(eps, level - jmax))
