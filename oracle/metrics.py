"""Error and compression metrics (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2: the l^p norms are weighted by dx_J = 2^-J (b - a). Sec. 5: delta is the l^1
distance between the reference scheme's conserved moments and the reconstruction of the
adaptive ones on the finest level; CR^n = 100 (1 - #S(Lambda^n) / N_J) and
ACR^N = 100 (1 - (1/N) sum_n #S(Lambda^n) / N_J).
"""

import numpy as np


def l1(a, dx):
    return float(dx * np.sum(np.abs(a)))


def delta(ref_conserved, adaptive_finest_conserved, x_min, x_max):
    """Per conserved moment: || M_ref - m_hathat ||_{l1, dx_J}."""
    ref = np.atleast_2d(ref_conserved)
    ada = np.atleast_2d(adaptive_finest_conserved)
    dx = (x_max - x_min) / ref.shape[1]
    return [l1(ref[i] - ada[i], dx) for i in range(ref.shape[0])]


def compression(n_leaves, jmax):
    return 100.0 * (1.0 - n_leaves / 2.0 ** jmax)


def average_compression(leaf_history, jmax):
    h = np.asarray(leaf_history, dtype=np.float64)
    return 100.0 * (1.0 - h.mean() / 2.0 ** jmax)
