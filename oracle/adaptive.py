"""Dense-level adaptive MR-LBM (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Every level j = J_min..J is held as a full array F[j] of shape (q, 2^j); only the
cells of the complete tree R(Lambda) carry meaningful values. The tree itself is held
as one boolean array per level, ``split[j][p]`` = "cell (j, p) has children", for
j = J_min..J-1. The paper's detail index (j+1, 2p) belongs to Lambda exactly when
split[j][p] is set (Sec. 3.3, with the reading that a tree's parent condition means
"the parent is in R(Lambda)").

One time step (Sec. 4.1: adapt with the details of t^n, then the scheme on the new
complete leaves) is, in the paper's order:

  1. projection up the tree of the leaf values (Sec. 3.1 Projection; Sec. 4.1.1),
  2. details of every kept pair (Sec. 3.2) and their max over populations,
  3. thresholding T_eps with eps_j = 2^(j-J) eps (Sec. 3.4),
  4. enlargement H_eps: rule (a) finite speed, rule (b) regularity loss
     (Sec. 4.2, eq. HartenLossOfRegularity),
  5. grading G: smallest graded tree (Sec. 3.3, Definition Graded tree),
  6. data transfer: coarsened cells keep their projections, added cells are predicted
     from their parents, coarse to fine (Sec. 4.1.1),
  7. leaves collision on S(Lambda^{n+1}) (Sec. 4.5, eq. LeavesCollision), or with
     collision="reconstructed" the reconstructed collision (Sec. 4.3.1,
     eq. reconstructedCollision),
  8. projection of the collided values up the new tree, reconstruction f-double-hat to
     the finest level by level-by-level prediction (Sec. 3.3), and the compact
     reconstructed stream (Sec. 4.3.2, eq. AdaptiveStreamPhase). Leaves already at the
     finest level take the reconstructed finest neighbour directly (the same value in
     exact arithmetic, and the uniform scheme's value when eps = 0).

Readings: complete leaves are the cells of R(Lambda) without children;
rule (a) is applied once to every cell of R(T_eps(Lambda^n)); rules (a) and (b) both read
T_eps(Lambda^n) and their results are united; a tie with a threshold keeps/refines.
"""

import numpy as np

from . import mr


class AdaptiveMRLBM:
    """State of one adaptive MR-LBM run on [J_min, J].

    ``refine_rule`` optionally replaces enlargement rule (b): a callable
    (state, level, keep_parents, D) -> boolean array over the parents at ``level``
    saying which kept pairs get both children refined. ``None`` uses the paper's rule.
    """

    def __init__(self, scheme, jmin, jmax, gamma, eps, mu_bar, bc, mc0, refine_rule=None,
                 collision="leaves"):
        if not (0 <= jmin <= jmax):
            raise ValueError("need 0 <= J_min <= J")
        if collision not in ("leaves", "reconstructed"):
            raise ValueError("collision is 'leaves' or 'reconstructed'")
        self.collision = collision
        self.sch = scheme
        self.jmin, self.jmax = int(jmin), int(jmax)
        self.gamma, self.eps, self.mu_bar, self.bc = int(gamma), float(eps), int(mu_bar), int(bc)
        self.refine_rule = refine_rule
        q = scheme.q
        self.F = {l: np.zeros((q, 2 ** l)) for l in range(self.jmin, self.jmax + 1)}
        mc0 = np.asarray(mc0, dtype=np.float64).reshape(scheme.qc, 2 ** self.jmax)
        self.F[self.jmax] = scheme.equilibrium(mc0)
        # Lambda^0 is the full tree: every cell below J is split.
        self.split = {l: np.ones(2 ** l, dtype=bool) for l in range(self.jmin, self.jmax)}
        self.steps = 0
        self.leaf_updates = 0
        self.leaf_history = []
        self.last_D = None

    # ------------------------------------------------------------- tree views
    def complete_tree(self, split=None):
        """R(Lambda) per level: all of level J_min, then the children of split cells."""
        split = self.split if split is None else split
        R = {self.jmin: np.ones(2 ** self.jmin, dtype=bool)}
        for l in range(self.jmin, self.jmax):
            R[l + 1] = np.repeat(split[l], 2)
        return R

    def leaves(self, split=None):
        """S(Lambda): cells of R(Lambda) that have no children."""
        split = self.split if split is None else split
        R = self.complete_tree(split)
        out = {}
        for l in range(self.jmin, self.jmax + 1):
            s = split[l] if l < self.jmax else np.zeros(2 ** l, dtype=bool)
            out[l] = R[l] & ~s
        return out

    def n_leaves(self, split=None):
        return int(sum(v.sum() for v in self.leaves(split).values()))

    # ------------------------------------------------------------- operators
    def project_up(self):
        """Projection of leaf values onto every split cell, finest to coarsest."""
        for l in range(self.jmax - 1, self.jmin - 1, -1):
            p = np.nonzero(self.split[l])[0]
            if p.size:
                self.F[l][:, p] = mr.project_cells(self.F[l + 1], p)

    def details(self):
        """D[l][p] = max over populations of |d_{l+1, 2p}| for split (l, p); -1 elsewhere."""
        D = {}
        for l in range(self.jmin, self.jmax):
            Dl = np.full(2 ** l, -1.0)
            p = np.nonzero(self.split[l])[0]
            if p.size:
                d = mr.details_even(self.F[l + 1], self.F[l], p, self.gamma, self.bc)
                Dl[p] = np.max(np.abs(d), axis=0)
            D[l] = Dl
        return D

    def threshold(self, D):
        """T_eps: keep the pair under (l, p) iff it is in Lambda and D >= eps_{l+1}."""
        keep = {}
        for l in range(self.jmin, self.jmax):
            thr = mr.level_threshold(self.eps, l + 1, self.jmax)
            keep[l] = self.split[l] & (D[l] >= thr)
        return keep

    def rule_b(self, keep, D):
        """Pairs flagged by enlargement rule (b): kept detail (l+1, 2p) with J_min < l+1 < J and
        D >= 2^(mu+1) eps_{l+1}, per parent level l (Sec. 4.2, eq. HartenLossOfRegularity)."""
        J = self.jmax
        out = {}
        for l in range(self.jmin, J):
            if l + 1 < J:
                thr_b = float(np.ldexp(self.eps, self.mu_bar + 1 + (l + 1) - J))
                out[l] = keep[l] & (D[l] >= thr_b)
            else:
                out[l] = np.zeros_like(keep[l])
        return out

    def enlarge(self, keep, D, rule_b=None):
        """H_eps applied to T_eps(Lambda^n), rules (a) and (b) united. ``rule_b`` overrides the
        cells where rule (b) refines (default: the paper's rule, or ``refine_rule``)."""
        J, jmin = self.jmax, self.jmin
        new = {l: keep[l].copy() for l in range(jmin, J)}
        sig = self.sch.sigma
        # Rule (a): every cell (l+1, k) of R(T) puts (l+1, k+delta), |delta| <= sigma, into R.
        for l in range(jmin, J):
            n1 = 2 ** (l + 1)
            kids = np.nonzero(np.repeat(keep[l], 2))[0]
            if kids.size == 0:
                continue
            for dl in range(-sig, sig + 1):
                idx = mr.bc_index(kids + dl, n1, self.bc)
                new[l][idx // 2] = True
        # Rule (b): kept detail (l+1, 2p) with J_min < l+1 < J and D >= 2^(mu+1) eps_{l+1}
        # puts (l+2, 4p + delta), delta = 0..3, into R: both children of (l, p) split.
        if rule_b is None and self.refine_rule is None:
            rule_b = self.rule_b(keep, D)
        for l in range(jmin, J - 1):
            if rule_b is not None:
                hit = rule_b[l]
            else:
                hit = keep[l] & self.refine_rule(self, l, keep[l], D[l])
            p = np.nonzero(hit)[0]
            new[l + 1][2 * p] = True
            new[l + 1][2 * p + 1] = True
        return new

    def grade(self, new):
        """Smallest graded tree containing ``new``: one sweep from fine to coarse. A split
        cell (a, p) needs (a, p+delta), |delta| <= gamma, in R, i.e. their parents split;
        delta = 0 also restores the tree (no orphans)."""
        for a in range(self.jmax - 1, self.jmin, -1):
            p = np.nonzero(new[a])[0]
            if p.size == 0:
                continue
            n = 2 ** a
            for dl in range(-self.gamma, self.gamma + 1):
                idx = mr.bc_index(p + dl, n, self.bc)
                new[a - 1][idx // 2] = True
        return new

    def transfer(self, new):
        """Move data from R(Lambda^n) to R(Lambda^{n+1}): added cells are predicted from
        their parent level, coarse to fine; every other cell keeps its value."""
        Ro = self.complete_tree(self.split)
        Rn = self.complete_tree(new)
        for l in range(self.jmin, self.jmax):
            c = np.nonzero(Rn[l + 1] & ~Ro[l + 1])[0]
            if c.size:
                self.F[l + 1][:, c] = mr.predict_cells(self.F[l], c, self.gamma, self.bc)
        self.split = new

    def adapt(self):
        """Lambda^{n+1} = G(H_eps(T_eps(Lambda^n))) and the data transfer (Sec. 4.1.1)."""
        self.project_up()
        D = self.details()
        self.last_D = D
        keep = self.threshold(D)
        new = self.enlarge(keep, D)
        new = self.grade(new)
        self.transfer(new)

    def collide_leaves(self):
        for l, mask in self.leaves().items():
            k = np.nonzero(mask)[0]
            if k.size:
                self.F[l][:, k] = self.sch.collide(self.F[l][:, k])

    def leaf_mean_equilibria(self):
        """Per complete leaf (l, k): the mean over its finest cells (J, k 2^(J-l) + delta),
        delta = 0 .. 2^(J-l) - 1, of the equilibria of the reconstructed conserved moments
        (those of the reconstructed populations, equal in exact arithmetic) (Sec. 4.3.1,
        eq. reconstructedCollision). The leaf values are projected up the tree first; the sum
        runs over delta in increasing order and is scaled by 2^-(J-l) (exact). Returns
        {l: (k, eqbar)} with eqbar of shape (q - qc, #k)."""
        J = self.jmax
        self.project_up()
        eqJ = self.sch.equilibria(self.reconstruct()[J])  # (q - qc, 2^J)
        out = {}
        for l, mask in self.leaves().items():
            k = np.nonzero(mask)[0]
            if k.size == 0:
                continue
            d = J - l
            acc = eqJ[:, k << d].copy()
            for delta in range(1, 2 ** d):
                acc = acc + eqJ[:, (k << d) + delta]
            out[l] = (k, np.ldexp(acc, -d))
        return out

    def collide_reconstructed(self):
        """Reconstructed collision on S(Lambda^{n+1}) (Sec. 4.3.1, eq. reconstructedCollision):
        every non-conserved moment of a leaf relaxes towards the leaf's mean equilibrium over
        its finest cells; the conserved moments stay."""
        for l, (k, eqbar) in self.leaf_mean_equilibria().items():
            self.F[l][:, k] = self.sch.collide_with_equilibria(self.F[l][:, k], eqbar)

    def reconstruct(self):
        """f-double-hat on every level: G[J_min] = F[J_min]; G[l+1] = prediction of G[l],
        overwritten by F on R(Lambda). Returns the dict of levels."""
        R = self.complete_tree()
        G = {self.jmin: self.F[self.jmin].copy()}
        for l in range(self.jmin, self.jmax):
            g = mr.predict_level(G[l], self.gamma, self.bc)
            m = R[l + 1]
            g[:, m] = self.F[l + 1][:, m]
            G[l + 1] = g
        return G

    def stream(self):
        """Compact reconstructed stream on every complete leaf (eq. AdaptiveStreamPhase)."""
        J = self.jmax
        NJ = 2 ** J
        G = self.reconstruct()[J]
        w = self.sch.w
        newF = {}
        for l, mask in self.leaves().items():
            k = np.nonzero(mask)[0]
            if k.size == 0:
                continue
            fs = self.F[l][:, k]
            out = fs.copy()
            for h in range(self.sch.q):
                wh = int(w[h])
                if wh == 0:
                    continue
                if l == J:
                    out[h] = G[h, mr.bc_index(k - wh, NJ, self.bc)]
                    continue
                sg = 1 if wh > 0 else -1
                L = 2 ** (J - l)
                acc = None
                for dl in range(1, abs(wh) + 1):
                    eta = -dl if sg > 0 else dl - 1
                    a = G[h, mr.bc_index(k * L + eta, NJ, self.bc)]
                    b = G[h, mr.bc_index((k + 1) * L + eta, NJ, self.bc)]
                    t = a - b
                    acc = t if acc is None else acc + t
                out[h] = fs[h] + np.ldexp(sg * acc, -(J - l))
            newF[l] = (k, out)
        for l, (k, out) in newF.items():
            self.F[l][:, k] = out

    def step(self, nsteps=1):
        for _ in range(int(nsteps)):
            self.adapt()
            if self.collision == "reconstructed":
                self.collide_reconstructed()
            else:
                self.collide_leaves()
            self.project_up()
            self.stream()
            nl = self.n_leaves()
            self.leaf_history.append(nl)
            self.leaf_updates += nl
            self.steps += 1
        return self

    # ------------------------------------------------------------- observables
    def finest_populations(self):
        """Reconstruction of the current populations on the finest level (q, N_J)."""
        self.project_up()
        return self.reconstruct()[self.jmax]

    def finest_conserved(self):
        return self.sch.conserved(self.finest_populations())

    def leaf_list(self):
        """Complete leaves in spatial order as (level, index) arrays."""
        lv, ix, left = [], [], []
        for l, mask in self.leaves().items():
            k = np.nonzero(mask)[0]
            lv.append(np.full(k.size, l))
            ix.append(k)
            left.append(k * 2 ** (self.jmax - l))
        lv, ix, left = np.concatenate(lv), np.concatenate(ix), np.concatenate(left)
        o = np.argsort(left, kind="stable")
        return lv[o], ix[o]

    def leaf_conserved(self):
        """Conserved moments on the complete leaves, spatial order, shape (qc, n_leaves)."""
        lv, ix = self.leaf_list()
        f = np.stack([self.F[int(l)][:, int(k)] for l, k in zip(lv, ix)], axis=1)
        return self.sch.conserved(f)

    def leaf_populations(self):
        lv, ix = self.leaf_list()
        return np.stack([self.F[int(l)][:, int(k)] for l, k in zip(lv, ix)], axis=1)

    def compression(self):
        """CR = 100 (1 - #S / N_J) (Sec. 5)."""
        return 100.0 * (1.0 - self.n_leaves() / 2 ** self.jmax)
