"""Two-dimensional adaptive MR-LBM (oracle side): the multi-dimensional extension the paper
outlines in its conclusion.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed (Sec. 6, conclusions and perspectives, the points listed for the
generalisation to dimension d; and the one-dimensional definitions they extend):
* projection: the mean over the 2^d children (Sec. 3.1 Definition Projection, generalised);
* prediction: the tensor product of the one-dimensional centered prediction of Sec. 3.1
  (Bihari and Harten): child (2i + a, 2j + b) of (i, j) is
      f_ij + s_a Qx + s_b Qy + s_a s_b Qxy,     s_0 = +1, s_1 = -1,
      Qx  = sum_al c_al (f_{i+al, j} - f_{i-al, j}),
      Qy  = sum_be c_be (f_{i, j+be} - f_{i, j-be}),
      Qxy = sum_al sum_be c_al c_be ((f_{i+al, j+be} - f_{i+al, j-be}) - (f_{i-al, j+be} - f_{i-al, j-be}));
  the details are child minus prediction, four per parent (siblings no longer share a modulus);
* level thresholds eps_l = 2^{d (l - J)} eps (d = 2) in T_eps (Sec. 3.4), and enlargement rule
  (b) with the threshold 2^{mu_bar + d} eps_l (Sec. 4.2, eq. HartenLossOfRegularity, as the
  conclusion modifies it);
* enlargement rule (a) (Sec. 4.2) with the sigma-box of neighbours; grading (Sec. 3.3) with the
  gamma-box of the prediction stencil;
* collision on the complete leaves (Sec. 4.5) and the compact stream (Sec. 4.3.2), which the
  conclusion says carries over: for a leaf (l, i, j) of side L = 2^{J-l} finest cells and a
  velocity w, the mean of the reconstructed f* over the leaf shifted by -w is the leaf's own
  value plus the difference of the strips entering and leaving it, divided by L^2.

Readings where the paper is silent (it defers multi-D schemes to a companion paper):
* the lattice scheme is D2Q4 for a scalar law u_t + phi_x(u)_x + phi_y(u)_y = 0:
  velocities lambda (1, 0), (-1, 0), (0, 1), (0, -1); moments u = f0+f1+f2+f3,
  m1 = lambda (f0 - f1), m2 = lambda (f2 - f3), m3 = lambda^2 (f0 + f1 - f2 - f3); equilibria
  m1 = phi_x(u), m2 = phi_y(u), m3 = 0 (advection phi = (Vx u, Vy u); Burgers phi = (u^2/2, u^2/2));
* the tree is held as per-level boolean arrays split[l][i, j] ("cell has four children"),
  the two-dimensional form of the one-dimensional oracle's split bits;
* rule (b) refines the four children of the parent of a flagged detail (the 1D rule refines
  both children), and the grading box has half-width gamma in each direction;
* boundaries: periodic or clamp in each direction, at every level, as in 1D;
* the strip sums of the compact stream run over the strip's cells in increasing order.

Arrays: F[l] has shape (q, N_l, N_l) with N_l = 2^l, index [h, i, j], i along x.
"""

import numpy as np

PERIODIC, CLAMP = 0, 1
ADVECTION, BURGERS = 0, 1
D = 2  # spatial dimension


def bc_index(i, n, bc):
    i = np.asarray(i)
    if bc == PERIODIC:
        return np.mod(i, n)
    return np.clip(i, 0, n - 1)


def pred_coeffs(gamma):
    """Centered prediction coefficients of Sec. 3.1 (gamma = 3 with c3 = -5/1024, the sign that
    makes the stencil exact on degree 5)."""
    return {1: [-1.0 / 8.0], 2: [-22.0 / 128.0, 3.0 / 128.0], 3: [-201.0 / 1024.0, 11.0 / 256.0, -5.0 / 1024.0]}[gamma]


def level_threshold(eps, l, J):
    """eps_l = 2^{d (l - J)} eps (exact scaling)."""
    return float(np.ldexp(eps, D * (l - J)))


# ------------------------------------------------------------------ multiresolution operators
def project(fine):
    """Mean over the four children of every coarse cell: fine (..., 2N, 2N) -> (..., N, N)."""
    a = fine[..., 0::2, 0::2]
    b = fine[..., 1::2, 0::2]
    c = fine[..., 0::2, 1::2]
    d = fine[..., 1::2, 1::2]
    return (((a + b) + c) + d) * 0.25


def _shift(f, di, dj, bc):
    """f[..., bc(i + di), bc(j + dj)] for every (i, j)."""
    n = f.shape[-1]
    ii = bc_index(np.arange(n) + di, n, bc)
    jj = bc_index(np.arange(n) + dj, n, bc)
    return f[..., ii, :][..., :, jj]


def predict(coarse, gamma, bc):
    """Tensor-product prediction of every child of every coarse cell: (..., N, N) -> (..., 2N, 2N)."""
    c = pred_coeffs(gamma)
    Qx = None
    Qy = None
    Qxy = None
    for a in range(1, gamma + 1):
        tx = c[a - 1] * (_shift(coarse, a, 0, bc) - _shift(coarse, -a, 0, bc))
        ty = c[a - 1] * (_shift(coarse, 0, a, bc) - _shift(coarse, 0, -a, bc))
        Qx = tx if Qx is None else Qx + tx
        Qy = ty if Qy is None else Qy + ty
    for a in range(1, gamma + 1):
        for b in range(1, gamma + 1):
            t = (c[a - 1] * c[b - 1]) * ((_shift(coarse, a, b, bc) - _shift(coarse, a, -b, bc))
                                         - (_shift(coarse, -a, b, bc) - _shift(coarse, -a, -b, bc)))
            Qxy = t if Qxy is None else Qxy + t
    shape = coarse.shape[:-2] + (2 * coarse.shape[-2], 2 * coarse.shape[-1])
    out = np.empty(shape)
    for sa, ia in ((1.0, 0), (-1.0, 1)):
        for sb, jb in ((1.0, 0), (-1.0, 1)):
            out[..., ia::2, jb::2] = ((coarse + sa * Qx) + sb * Qy) + (sa * sb) * Qxy
    return out


def details(fine, coarse, gamma, bc):
    """d = child - prediction for every child: shape of fine."""
    return fine - predict(coarse, gamma, bc)


def max_detail(fine, coarse, gamma, bc):
    """Per coarse cell: max over its four children and the leading axes of |d|."""
    d = np.abs(details(fine, coarse, gamma, bc))
    d = d.reshape((-1,) + d.shape[-2:]).max(axis=0)
    n = d.shape[-1] // 2
    return np.maximum(np.maximum(d[0::2, 0::2], d[1::2, 0::2]), np.maximum(d[0::2, 1::2], d[1::2, 1::2])).reshape(n, n)


# ------------------------------------------------------------------ D2Q4 scheme (reading)
class D2Q4:
    """D2Q4 for a scalar conservation law (reading above); populations ordered
    (+x, -x, +y, -y)."""

    def __init__(self, physics, lam, s, V=(0.0, 0.0)):
        self.physics, self.lam = int(physics), float(lam)
        s = np.atleast_1d(np.asarray(s, dtype=np.float64))
        self.s = np.repeat(s, 3) if s.size == 1 else s
        if self.s.size != 3:
            raise ValueError("need one rate or three (m1, m2, m3)")
        self.V = (float(V[0]), float(V[1]))
        self.q, self.qc = 4, 1
        self.w = np.array([[1, 0], [-1, 0], [0, 1], [0, -1]])
        self.sigma = 1

    def flux(self, u):
        if self.physics == ADVECTION:
            return self.V[0] * u, self.V[1] * u
        return (u * u) * 0.5, (u * u) * 0.5

    def _from_moments(self, u, m1, m2, m3):
        lam = self.lam
        a = m1 / lam
        b = m2 / lam
        c = m3 / (lam * lam)
        e = 0.5 * (u + c)
        o = 0.5 * (u - c)
        return np.stack([0.5 * (e + a), 0.5 * (e - a), 0.5 * (o + b), 0.5 * (o - b)])

    def collide(self, f):
        lam = self.lam
        u = ((f[0] + f[1]) + f[2]) + f[3]
        m1 = lam * (f[0] - f[1])
        m2 = lam * (f[2] - f[3])
        m3 = (lam * lam) * ((f[0] + f[1]) - (f[2] + f[3]))
        px, py = self.flux(u)
        s1, s2, s3 = self.s
        m1s = (1.0 - s1) * m1 + s1 * px
        m2s = (1.0 - s2) * m2 + s2 * py
        m3s = (1.0 - s3) * m3
        return self._from_moments(u, m1s, m2s, m3s)

    def equilibrium(self, u):
        px, py = self.flux(u)
        return self._from_moments(u, px, py, np.zeros_like(u))

    def conserved(self, f):
        return (((f[0] + f[1]) + f[2]) + f[3])[None]


class Uniform2D:
    """Reference scheme on the finest lattice: collide every cell, then F_h(x) = F*_h(x - w_h)."""

    def __init__(self, scheme, J, bc, u0):
        self.sch, self.J, self.bc = scheme, int(J), int(bc)
        self.F = scheme.equilibrium(np.asarray(u0, dtype=np.float64).reshape(2 ** J, 2 ** J))

    def step(self, n=1):
        for _ in range(int(n)):
            fs = self.sch.collide(self.F)
            self.F = np.stack([_shift(fs[h], -int(self.sch.w[h][0]), -int(self.sch.w[h][1]), self.bc)
                               for h in range(self.sch.q)])
        return self

    def conserved(self):
        return self.sch.conserved(self.F)


# ------------------------------------------------------------------ adaptive scheme
class Adaptive2D:
    """Dense-level adaptive MR-LBM in 2D; one step = adapt (project, details, T_eps, H_eps, G,
    transfer) then collide on the complete leaves and the compact stream (the order of Sec. 4.1)."""

    def __init__(self, scheme, jmin, jmax, gamma, eps, mu_bar, bc, u0, compact=True):
        self.sch = scheme
        self.jmin, self.J = int(jmin), int(jmax)
        self.gamma, self.eps, self.mu_bar, self.bc = int(gamma), float(eps), int(mu_bar), int(bc)
        self.compact = compact
        q = scheme.q
        self.F = {l: np.zeros((q, 2 ** l, 2 ** l)) for l in range(self.jmin, self.J + 1)}
        self.F[self.J] = scheme.equilibrium(np.asarray(u0, dtype=np.float64).reshape(2 ** self.J, 2 ** self.J))
        self.split = {l: np.ones((2 ** l, 2 ** l), dtype=bool) for l in range(self.jmin, self.J)}
        self.steps = 0
        self.leaf_updates = 0

    # tree views
    def complete_tree(self, split=None):
        split = self.split if split is None else split
        R = {self.jmin: np.ones((2 ** self.jmin,) * 2, dtype=bool)}
        for l in range(self.jmin, self.J):
            R[l + 1] = np.repeat(np.repeat(split[l], 2, axis=0), 2, axis=1)
        return R

    def leaves(self, split=None):
        split = self.split if split is None else split
        R = self.complete_tree(split)
        return {l: R[l] & ~(split[l] if l < self.J else np.zeros_like(R[l])) for l in range(self.jmin, self.J + 1)}

    def n_leaves(self):
        return int(sum(v.sum() for v in self.leaves().values()))

    # operators
    def project_up(self):
        for l in range(self.J - 1, self.jmin - 1, -1):
            m = self.split[l]
            if m.any():
                p = project(self.F[l + 1])
                self.F[l][:, m] = p[:, m]

    def details(self):
        """D[l][i, j]: max over children and populations of |d| for split (l, i, j); -1 elsewhere."""
        out = {}
        for l in range(self.jmin, self.J):
            Dl = np.full((2 ** l, 2 ** l), -1.0)
            m = self.split[l]
            if m.any():
                Dl[m] = max_detail(self.F[l + 1], self.F[l], self.gamma, self.bc)[m]
            out[l] = Dl
        return out

    def threshold(self, Dd):
        return {l: self.split[l] & (Dd[l] >= level_threshold(self.eps, l + 1, self.J)) for l in range(self.jmin, self.J)}

    def enlarge(self, keep, Dd):
        J, jmin, sig = self.J, self.jmin, self.sch.sigma
        new = {l: keep[l].copy() for l in range(jmin, J)}
        # rule (a): every cell (l + 1, k) of R(T) puts its sigma-box neighbours into R
        for l in range(jmin, J):
            kids = np.argwhere(np.repeat(np.repeat(keep[l], 2, axis=0), 2, axis=1))
            if kids.size == 0:
                continue
            n1 = 2 ** (l + 1)
            for di in range(-sig, sig + 1):
                for dj in range(-sig, sig + 1):
                    ii = bc_index(kids[:, 0] + di, n1, self.bc)
                    jj = bc_index(kids[:, 1] + dj, n1, self.bc)
                    new[l][ii // 2, jj // 2] = True
        # rule (b): a kept detail at level l + 1, J_min < l + 1 < J, with
        # D >= 2^{mu_bar + d} eps_{l+1} refines the four children of its parent
        for l in range(jmin, J - 1):
            thr = float(np.ldexp(level_threshold(self.eps, l + 1, J), self.mu_bar + D))
            hit = keep[l] & (Dd[l] >= thr)
            if hit.any():
                new[l + 1] |= np.repeat(np.repeat(hit, 2, axis=0), 2, axis=1)
        return new

    def grade(self, new):
        """Smallest graded tree: a split (a, p) needs its gamma-box at level a in R (the
        parents of those cells split); one sweep from fine to coarse."""
        for a in range(self.J - 1, self.jmin, -1):
            p = np.argwhere(new[a])
            if p.size == 0:
                continue
            n = 2 ** a
            for di in range(-self.gamma, self.gamma + 1):
                for dj in range(-self.gamma, self.gamma + 1):
                    ii = bc_index(p[:, 0] + di, n, self.bc)
                    jj = bc_index(p[:, 1] + dj, n, self.bc)
                    new[a - 1][ii // 2, jj // 2] = True
        return new

    def transfer(self, new):
        Ro = self.complete_tree(self.split)
        Rn = self.complete_tree(new)
        for l in range(self.jmin, self.J):
            add = Rn[l + 1] & ~Ro[l + 1]
            if add.any():
                pr = predict(self.F[l], self.gamma, self.bc)
                self.F[l + 1][:, add] = pr[:, add]
        self.split = new

    def adapt(self):
        self.project_up()
        Dd = self.details()
        keep = self.threshold(Dd)
        self.transfer(self.grade(self.enlarge(keep, Dd)))

    def reconstruct(self):
        """f-double-hat on the finest level: level-by-level prediction, stored values on R."""
        R = self.complete_tree()
        G = self.F[self.jmin].copy()
        for l in range(self.jmin, self.J):
            g = predict(G, self.gamma, self.bc)
            m = R[l + 1]
            g[:, m] = self.F[l + 1][:, m]
            G = g
        return G

    def stream(self):
        J = self.J
        NJ = 2 ** J
        G = self.reconstruct()
        newF = {}
        for l, mask in self.leaves().items():
            cells = np.argwhere(mask)
            if cells.size == 0:
                continue
            L = 2 ** (J - l)
            fs = self.F[l][:, mask]
            out = fs.copy()
            for h in range(self.sch.q):
                wx, wy = (int(v) for v in self.sch.w[h])
                for c, (i, j) in enumerate(cells):
                    x0, y0 = i * L, j * L
                    if l == J:
                        out[h, c] = G[h, bc_index(x0 - wx, NJ, self.bc), bc_index(y0 - wy, NJ, self.bc)]
                    elif self.compact:
                        out[h, c] = fs[h, c] + np.ldexp(self._strip(G[h], x0, y0, L, wx, wy), -D * (J - l))
                    else:
                        xs = bc_index(np.arange(x0, x0 + L) - wx, NJ, self.bc)
                        ys = bc_index(np.arange(y0, y0 + L) - wy, NJ, self.bc)
                        out[h, c] = np.sum(G[h][np.ix_(xs, ys)]) / (L * L)
            newF[l] = (mask, out)
        for l, (mask, out) in newF.items():
            self.F[l][:, mask] = out

    def _strip(self, g, x0, y0, L, wx, wy):
        """Entering minus leaving strip of a leaf for a unit velocity (wx, wy): for w = (1, 0) the
        column x0 - 1 minus the column x0 + L - 1 over the leaf's rows, and alike."""
        NJ = g.shape[-1]
        bc = self.bc
        acc = 0.0
        for t in range(L):
            if wx != 0:
                y = bc_index(y0 + t, NJ, bc)
                a = g[bc_index(x0 - 1 if wx > 0 else x0, NJ, bc), y]
                b = g[bc_index(x0 + L - 1 if wx > 0 else x0 + L, NJ, bc), y]
                term = (a - b) if wx > 0 else -(a - b)
            else:
                x = bc_index(x0 + t, NJ, bc)
                a = g[x, bc_index(y0 - 1 if wy > 0 else y0, NJ, bc)]
                b = g[x, bc_index(y0 + L - 1 if wy > 0 else y0 + L, NJ, bc)]
                term = (a - b) if wy > 0 else -(a - b)
            acc = term if t == 0 else acc + term
        return acc

    def collide_leaves(self):
        for l, mask in self.leaves().items():
            if mask.any():
                self.F[l][:, mask] = self.sch.collide(self.F[l][:, mask])

    def step(self, n=1):
        for _ in range(int(n)):
            self.adapt()
            self.collide_leaves()
            self.project_up()
            self.stream()
            nl = self.n_leaves()
            self.leaf_updates += nl
            self.steps += 1
        return self

    def finest_conserved(self):
        self.project_up()
        return self.sch.conserved(self.reconstruct())
