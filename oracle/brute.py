"""Literal set-based twin of the adaptive MR-LBM step, for tiny J only (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

This version follows the paper's set definitions instead of the dense-level arrays of
``oracle.adaptive``, so that the two can be checked against each other:

* Lambda is a set of detail indices: all of (J_min, k), and (l, k) with k even for
  l > J_min (Sec. 3.2, index sets nabla_j).
* R(Lambda) adds the odd sibling of every detail index (Sec. 3.3, complete tree); the
  complete leaves are the cells of R(Lambda) with no child in R(Lambda) (reading of the
  partition property of Sec. 3.3).
* T_eps per Sec. 3.4; H_eps per Sec. 4.2, rules (a) and (b); G per Sec. 3.3 computed as
  a fixed point: keep adding the detail indices that the graded-tree condition asks for
  until nothing changes.
* Values on R(Lambda) are the stored leaf values or, for split cells, the recursive
  projection; the reconstruction f-double-hat at any cell is the stored/projected value
  on R(Lambda) and the prediction from the level above elsewhere (Sec. 3.3), memoized.
* Data transfer evaluates the old reconstruction at the new complete leaves
  (equivalently M_R^-1 T_Lambda M_R, Sec. 3.4).
* The stream is the uncompacted mean over the finest sub-cells
  (eq. StreamUncompacted); the compact form of the dense oracle must agree with it up
  to rounding.
"""

import numpy as np

PERIODIC, CLAMP = 0, 1
_COEFFS = {1: [-1 / 8], 2: [-22 / 128, 3 / 128], 3: [-201 / 1024, 11 / 256, -5 / 1024]}


def _bc(i, n, bc):
    return i % n if bc == PERIODIC else min(max(i, 0), n - 1)


class BruteMRLBM:
    def __init__(self, scheme, jmin, jmax, gamma, eps, mu_bar, bc, mc0):
        if jmax > 8:
            raise ValueError("the brute-force twin is for tiny J only")
        self.sch, self.jmin, self.J = scheme, jmin, jmax
        self.gamma, self.eps, self.mu, self.bc = gamma, eps, mu_bar, bc
        f0 = scheme.equilibrium(np.asarray(mc0, dtype=np.float64).reshape(scheme.qc, -1))
        self.lam_set = self.full_set()
        self.vals = {(jmax, k): f0[:, k].copy() for k in range(2 ** jmax)}

    # ---------------------------------------------------------------- sets
    def full_set(self):
        s = {(self.jmin, k) for k in range(2 ** self.jmin)}
        for l in range(self.jmin + 1, self.J + 1):
            s |= {(l, k) for k in range(0, 2 ** l, 2)}
        return s

    def R(self, lam):
        out = {(self.jmin, k) for k in range(2 ** self.jmin)}
        for (l, k) in lam:
            if l > self.jmin:
                out.add((l, k))
                out.add((l, k + 1))
        return out

    def S(self, lam):
        r = self.R(lam)
        return {(l, k) for (l, k) in r if (l + 1, 2 * k) not in r and (l + 1, 2 * k + 1) not in r}

    def detail_index(self, l, k):
        return (l, k) if l == self.jmin else (l, k - k % 2)

    # ---------------------------------------------------------------- values
    def _valuer(self, lam, leafvals):
        r = self.R(lam)
        memo = {}

        def val(l, k):
            if (l, k) in memo:
                return memo[(l, k)]
            if (l, k) in leafvals:
                v = leafvals[(l, k)]
            else:
                v = 0.5 * (val(l + 1, 2 * k) + val(l + 1, 2 * k + 1))
            memo[(l, k)] = v
            return v

        rmemo = {}

        def recon(l, k):
            k = _bc(k, 2 ** l, self.bc)
            if (l, k) in rmemo:
                return rmemo[(l, k)]
            if (l, k) in r:
                v = val(l, k)
            else:
                p = k // 2
                acc = 0.0
                for a, c in enumerate(_COEFFS[self.gamma], start=1):
                    acc = acc + c * (recon(l - 1, p + a) - recon(l - 1, p - a))
                v = recon(l - 1, p) + (acc if k % 2 == 0 else -acc)
            rmemo[(l, k)] = v
            return v

        return val, recon

    def detail(self, val, l, k):
        """d_{l,k} for a detail index (l, k), l > J_min."""
        n = 2 ** (l - 1)
        p = k // 2
        acc = 0.0
        for a, c in enumerate(_COEFFS[self.gamma], start=1):
            acc = acc + c * (val(l - 1, _bc(p + a, n, self.bc)) - val(l - 1, _bc(p - a, n, self.bc)))
        pred = val(l - 1, p) + (acc if k % 2 == 0 else -acc)
        return val(l, k) - pred

    # ---------------------------------------------------------------- operators
    def threshold(self, lam, val):
        out = {(self.jmin, k) for k in range(2 ** self.jmin)}
        D = {}
        for (l, k) in lam:
            if l == self.jmin:
                continue
            D[(l, k)] = float(np.max(np.abs(self.detail(val, l, k))))
            if D[(l, k)] >= np.ldexp(self.eps, l - self.J):
                out.add((l, k))
        return out, D

    def enlarge(self, T, D):
        out = set(T)
        sig = self.sch.sigma
        for (l, k) in self.R(T):
            if l == self.jmin:
                continue
            for dl in range(-sig, sig + 1):
                out.add(self.detail_index(l, _bc(k + dl, 2 ** l, self.bc)))
        for (l, k) in T:
            if self.jmin < l < self.J and D[(l, k)] >= np.ldexp(self.eps, self.mu + 1 + l - self.J):
                out.add((l + 1, 2 * k))
                out.add((l + 1, 2 * k + 2))
        return out

    def grade(self, lam):
        lam = set(lam)
        changed = True
        while changed:
            changed = False
            for (l, k) in list(lam):
                if l == self.jmin:
                    continue
                for dl in range(-self.gamma, self.gamma + 1):
                    c = _bc(k // 2 + dl, 2 ** (l - 1), self.bc)
                    if l - 1 == self.jmin:
                        continue
                    di = self.detail_index(l - 1, c)
                    if di not in lam:
                        lam.add(di)
                        changed = True
        return lam

    # ---------------------------------------------------------------- step
    def step(self):
        val, recon = self._valuer(self.lam_set, self.vals)
        T, D = self.threshold(self.lam_set, val)
        new = self.grade(self.enlarge(T, D))
        S_new = self.S(new)
        moved = {c: np.array(recon(*c), dtype=np.float64) for c in S_new}
        keys = sorted(moved)
        fs = self.sch.collide(np.stack([moved[c] for c in keys], axis=1))
        star = {c: fs[:, i] for i, c in enumerate(keys)}
        _, rstar = self._valuer(new, star)
        NJ = 2 ** self.J
        G = np.stack([rstar(self.J, m) for m in range(NJ)], axis=1)
        out = {}
        for (l, k) in keys:
            L = 2 ** (self.J - l)
            v = np.empty(self.sch.q)
            for h in range(self.sch.q):
                wh = int(self.sch.w[h])
                idx = [_bc(k * L + d - wh, NJ, self.bc) for d in range(L)]
                v[h] = np.sum(G[h, idx]) / L
            out[(l, k)] = v
        self.lam_set, self.vals = new, out
        return self

    def leaf_levels(self):
        """Dict level -> sorted list of leaf indices."""
        d = {}
        for (l, k) in self.vals:
            d.setdefault(l, []).append(k)
        return {l: sorted(v) for l, v in d.items()}

    def finest_populations(self):
        _, recon = self._valuer(self.lam_set, self.vals)
        return np.stack([recon(self.J, m) for m in range(2 ** self.J)], axis=1)
