"""The oracle against the only numbers the paper prints for its method: Table 2 of Sec. 5.1
(ratio E^{0,N} / delta^{0,N} of the reference scheme's error against the exact solution to
the adaptive method's perturbation error, D1Q2, J = 9, eps = 1e-4).

Column I (advection of a Gaussian) has a closed-form exact solution and no rule-(b) or
shock sensitivity, so it is the column compared here. The paper leaves the boundary
treatment, the sampling of the initial datum and the rounding of T / dt unstated; the
readings below are clamp boundaries (the datum vanishes near x = +-3), cell averages and
N = round(T / dt).

What the paper fixes, and this test pins:
* the dependence on the relaxation rate s: each ratio normalised by the one at s = 0.75
  follows the printed column within 15 % (printed 99.7 -> 8.34, a factor 12 over s);
* the order of magnitude the text states for test I (the perturbation error 10 to 100
  times below the reference error): every ratio within a factor 10 of the printed one.
The absolute level is an open gap, not pinned: the oracle's ratios sit at 1.8-1.95 times
the printed ones at every s (delta / eps is 1.3-1.6 here where the printed ratios imply
about twice that). The alternative readings of the setup move the level by less than 5 %
(mu_bar = infinity as 30 or as "no rule (b)"; an initial compression T_eps then G of the
datum; one more adaptation at the final time; N rounded up or down; point-sampled data;
periodic boundaries), and the changes that do move it do so by other factors and are not
readings of the text (thresholds doubled: 0.66 times printed; rule (a) dropped: 0.13)."""

import math
import os

import numpy as np

import workloads as W
from oracle import metrics
from oracle.adaptive import AdaptiveMRLBM
from oracle.lattice import scheme_from_params
from oracle.reference import UniformLBM

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_ratio_errors.txt")
J, JMIN, EPS, XMIN, XMAX, T = 9, 2, 1e-4, -3.0, 3.0, 0.4
WIDTH = 1.0 / math.sqrt(20.0)  # exp(-20 x^2) = exp(-(x / WIDTH)^2)


def printed_column_I():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return {float(r[0]): float(r[1]) for r in rows}


def gauss_averages(e, centre):
    """Exact cell averages of exp(-((x - centre) / WIDTH)^2), no periodic images."""
    return W.avg_gauss_periodic(e, 1.0, centre, WIDTH, period=XMAX - XMIN, images=(0,))


def ratio_test_I(s):
    p = W.base_params(scheme=W.D1Q2, physics=W.ADVECTION, lam=1.0, s=[s], phys=[0.75, 1.0, 1.4, 0.9])
    sch = scheme_from_params(p)
    e = W.edges(J, XMIN, XMAX)
    u0 = gauss_averages(e, 0.0)
    n_steps = W.n_steps(T, 1.0, J, XMIN, XMAX)
    t = n_steps * (XMAX - XMIN) / 2 ** J
    # mu_bar = 30 stands for the paper's infinity: 2^31 eps_l exceeds every detail of this datum
    ada = AdaptiveMRLBM(sch, JMIN, J, 1, EPS, 30, W.CLAMP, u0[None, :]).step(n_steps)
    ref = UniformLBM(sch, J, W.CLAMP, u0[None, :]).step(n_steps)
    exact = gauss_averages(e, 0.75 * t)
    E = metrics.delta(exact[None, :], ref.conserved(), XMIN, XMAX)[0]
    d = metrics.delta(ref.conserved(), ada.finest_conserved(), XMIN, XMAX)[0]
    return E / d, d / EPS


def test_table2_column_I():
    printed = printed_column_I()
    ss = sorted(printed)
    got = {s: ratio_test_I(s) for s in ss}
    for s in ss:
        ratio, d_over_eps = got[s]
        # the perturbation error stays of the order of eps (Sec. 4.4 error estimate)
        assert 0.5 < d_over_eps < 3.0, (s, d_over_eps)
        # order of magnitude (the text: delta 10 to 100 times below E for test I); the level
        # itself is an open gap (module docstring)
        assert 0.1 < ratio / printed[s] < 10.0, (s, ratio, printed[s])
        # dependence on s: normalised by s = 0.75, within 15 % of the printed column
        ours = ratio / got[ss[0]][0]
        paper = printed[s] / printed[ss[0]]
        assert abs(ours / paper - 1.0) < 0.15, (s, ours, paper)
