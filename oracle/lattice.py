"""Lattice Boltzmann schemes in the d'Humieres formalism (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed
-----------------------
* Sec. 2.1: velocities v^h = lambda * w^h with integer w^h, moments m = M f with an
  invertible M, acoustic scaling dt = dx_J / lambda.
* Sec. 2.1.1 (collision): conserved moments unchanged, the others relaxed
  m*_h = (1 - s_h) m_h + s_h m^eq_h(conserved moments).
* Sec. 5.1.1: D1Q2, M = [[1, 1], [lambda, -lambda]], m^eq = phi(u) with
  phi(u) = V u (advection) or u^2/2 (Burgers).
* Sec. 5.2.1: D1Q3 lattice with velocities (0, lambda, -lambda) and
  M rows (1,1,1), (0,lambda,-lambda), (0,lambda^2,lambda^2); shallow-water
  equilibrium of the third moment (hu)^2/h + g h^2/2.
* Sec. 5.3: vectorial D1Q2^3 for Euler, three juxtaposed D1Q2 blocks coupled
  through the equilibria of the odd moments.
* Sec. 5.2.1: D1Q5 for shallow water, velocities (0, lambda, -lambda, 2 lambda,
  -2 lambda), M rows (1,1,1,1,1), lambda (0,1,-1,2,-2), lambda^2 (0,1,1,4,4),
  lambda^3 (0,1,-1,8,-8), lambda^4 (0,1,1,16,16); conserved h, hu; equilibria
  M2 = (hu)^2/h + g h^2/2, M3 = alpha lambda^2 hu, M4 = beta lambda^2 M2 (the paper's
  runs: alpha = beta = 1, s3 = s4 = 1). Its stencil reaches two cells (sigma = 2).

Readings where the paper is silent
----------------------------------------------------------------
* D1Q3 for Burgers (one conserved moment): m1^eq = u^2/2, m2^eq = alpha lambda^2 u.
* Vectorial D1Q2^2 for shallow water: blocks (h, hu) with m1^eq = hu and
  m3^eq = (hu)^2/h + g h^2/2, by analogy with the Euler blocks.
* One relaxation rate given is broadcast to every non-conserved moment.
* D1Q5's M^-1 is written through the even and odd parts of the moving populations:
  a = f1 + f2, b = f3 + f4 from M2 / lambda^2 = a + 4 b and M4 / lambda^4 = a + 16 b, and
  c = f1 - f2, d = f3 - f4 from M1 / lambda = c + 2 d and M3 / lambda^3 = c + 8 d.

Two forms of the collision live here. ``collide`` spells the arithmetic out in a
fixed order (the order the GPU kernels must reproduce for bit-exact leaf sets);
``collide_by_definition`` is the literal matrix statement m -> relax -> M^{-1}
and exists so that a test can pin the explicit form to the definition.
"""

import numpy as np

# Scheme and physics codes (shared numbering with the C header by documentation only).
D1Q2, D1Q3, D1Q2x2, D1Q2x3, D1Q5 = 0, 1, 2, 3, 4
ADVECTION, BURGERS, SHALLOW_WATER, EULER = 0, 1, 2, 3

VALID_PAIRS = {
    (D1Q2, ADVECTION), (D1Q2, BURGERS),
    (D1Q3, BURGERS), (D1Q3, SHALLOW_WATER),
    (D1Q2x2, SHALLOW_WATER),
    (D1Q2x3, EULER),
    (D1Q5, SHALLOW_WATER),
}


class Scheme:
    """One DdQq scheme with its equilibria.

    Parameters
    ----------
    scheme, physics : int codes above.
    lam : lattice velocity lambda > 0.
    s : relaxation rate(s) of the non-conserved moments, each in (0, 2].
        A scalar (or length-1 sequence) is broadcast.
    V : advection velocity (advection only).
    g : gravity (shallow water).
    gamma_gas : ratio of specific heats (Euler).
    alpha : coefficient of the D1Q3 Burgers third-moment equilibrium, or of the D1Q5
        fourth-moment equilibrium alpha lambda^2 hu.
    beta : coefficient of the D1Q5 fifth-moment equilibrium beta lambda^2 M2eq.
    """

    def __init__(self, scheme, physics, lam, s, V=0.0, g=1.0, gamma_gas=1.4, alpha=0.9, beta=1.0):
        if (scheme, physics) not in VALID_PAIRS:
            raise ValueError("unsupported scheme/physics pair")
        self.scheme, self.physics = scheme, physics
        self.lam = float(lam)
        self.V, self.g, self.gamma_gas, self.alpha = float(V), float(g), float(gamma_gas), float(alpha)
        self.beta = float(beta)
        if scheme == D1Q5:
            self.q, self.qc, self.w = 5, 2, np.array([0, 1, -1, 2, -2])
        elif scheme == D1Q2:
            self.q, self.qc, self.w = 2, 1, np.array([1, -1])
        elif scheme == D1Q3:
            self.q = 3
            self.qc = 1 if physics == BURGERS else 2
            self.w = np.array([0, 1, -1])
        elif scheme == D1Q2x2:
            self.q, self.qc, self.w = 4, 2, np.array([1, -1, 1, -1])
        else:
            self.q, self.qc, self.w = 6, 3, np.array([1, -1, 1, -1, 1, -1])
        nn = self.q - self.qc
        s_arr = np.atleast_1d(np.asarray(s, dtype=np.float64))
        if s_arr.size == 1:
            s_arr = np.repeat(s_arr, nn)
        if s_arr.size != nn:
            raise ValueError("need one relaxation rate per non-conserved moment")
        self.s = s_arr
        self.sigma = int(np.max(np.abs(self.w)))

    # ------------------------------------------------------------------ explicit
    def _eq_vectorial(self, c):
        """Equilibria of the odd moments of the vectorial schemes (Sec. 5.3)."""
        if self.physics == SHALLOW_WATER:
            c0, c1 = c
            g2 = 0.5 * self.g
            return [c1, (c1 * c1) / c0 + g2 * (c0 * c0)]
        gam = self.gamma_gas
        k3 = 0.5 * (3.0 - gam)
        gm1 = gam - 1.0
        k5 = 0.5 * (1.0 - gam)
        c0, c1, c2 = c
        e1 = c1
        e3 = k3 * ((c1 * c1) / c0) + gm1 * c2
        e5 = gam * ((c2 * c1) / c0) + k5 * (((c1 * c1) * c1) / (c0 * c0))
        return [e1, e3, e5]

    # D1Q5 (Sec. 5.2.1): moments, equilibria and the way back, in a fixed order
    def _q5_moments(self, f):
        lam = self.lam
        lam2 = lam * lam
        lam3 = lam2 * lam
        lam4 = lam2 * lam2
        m0 = (((f[0] + f[1]) + f[2]) + f[3]) + f[4]
        m1 = lam * ((f[1] - f[2]) + 2.0 * (f[3] - f[4]))
        m2 = lam2 * ((f[1] + f[2]) + 4.0 * (f[3] + f[4]))
        m3 = lam3 * ((f[1] - f[2]) + 8.0 * (f[3] - f[4]))
        m4 = lam4 * ((f[1] + f[2]) + 16.0 * (f[3] + f[4]))
        return m0, m1, m2, m3, m4

    def _q5_equilibria(self, m0, m1):
        lam2 = self.lam * self.lam
        eq2 = (m1 * m1) / m0 + (0.5 * self.g) * (m0 * m0)
        eq3 = (self.alpha * lam2) * m1
        eq4 = (self.beta * lam2) * eq2
        return eq2, eq3, eq4

    def _q5_populations(self, m0, m1, m2, m3, m4):
        lam = self.lam
        lam2 = lam * lam
        lam3 = lam2 * lam
        lam4 = lam2 * lam2
        p1, p2, p3, p4 = m1 / lam, m2 / lam2, m3 / lam3, m4 / lam4
        b = (p4 - p2) / 12.0
        a = p2 - 4.0 * b
        d = (p3 - p1) / 6.0
        c = p1 - 2.0 * d
        return np.stack([(m0 - a) - b, 0.5 * (a + c), 0.5 * (a - c), 0.5 * (b + d), 0.5 * (b - d)])

    def _q5_relax(self, f, eqs):
        m0, m1, m2, m3, m4 = self._q5_moments(f)
        s2, s3, s4 = self.s
        m2s = (1.0 - s2) * m2 + s2 * eqs[0]
        m3s = (1.0 - s3) * m3 + s3 * eqs[1]
        m4s = (1.0 - s4) * m4 + s4 * eqs[2]
        return self._q5_populations(m0, m1, m2s, m3s, m4s)

    def collide(self, f):
        """Local relaxation of the non-conserved moments; f has shape (q, n)."""
        f = np.asarray(f, dtype=np.float64)
        lam = self.lam
        out = np.empty_like(f)
        if self.scheme == D1Q5:
            m0, m1 = self._q5_moments(f)[:2]
            return self._q5_relax(f, self._q5_equilibria(m0, m1))
        if self.scheme == D1Q2:
            u = f[0] + f[1]
            m1 = lam * (f[0] - f[1])
            eq = self.V * u if self.physics == ADVECTION else (u * u) * 0.5
            s = self.s[0]
            m1s = (1.0 - s) * m1 + s * eq
            r = m1s / lam
            out[0] = 0.5 * (u + r)
            out[1] = 0.5 * (u - r)
        elif self.scheme == D1Q3:
            lam2 = lam * lam
            m0 = (f[0] + f[1]) + f[2]
            m1 = lam * (f[1] - f[2])
            m2 = lam2 * (f[1] + f[2])
            if self.physics == BURGERS:
                s1, s2 = self.s
                eq1 = (m0 * m0) * 0.5
                eq2 = (self.alpha * lam2) * m0
                m1s = (1.0 - s1) * m1 + s1 * eq1
                m2s = (1.0 - s2) * m2 + s2 * eq2
            else:
                s2 = self.s[0]
                g2 = 0.5 * self.g
                eq2 = (m1 * m1) / m0 + g2 * (m0 * m0)
                m1s = m1
                m2s = (1.0 - s2) * m2 + s2 * eq2
            a = m2s / lam2
            b = m1s / lam
            out[0] = m0 - a
            out[1] = 0.5 * (a + b)
            out[2] = 0.5 * (a - b)
        else:
            nb = self.q // 2
            c = [f[2 * b] + f[2 * b + 1] for b in range(nb)]
            eqs = self._eq_vectorial(c)
            for b in range(nb):
                s = self.s[b]
                n = lam * (f[2 * b] - f[2 * b + 1])
                ns = (1.0 - s) * n + s * eqs[b]
                r = ns / lam
                out[2 * b] = 0.5 * (c[b] + r)
                out[2 * b + 1] = 0.5 * (c[b] - r)
        return out

    def equilibria(self, f):
        """Equilibria of the non-conserved moments, shape (q - qc, n), from the conserved
        moments of populations f (q, n): the expressions ``collide`` uses (Sec. 5)."""
        f = np.asarray(f, dtype=np.float64)
        lam = self.lam
        if self.scheme == D1Q5:
            m0, m1 = self._q5_moments(f)[:2]
            return np.array(self._q5_equilibria(m0, m1))
        if self.scheme == D1Q2:
            u = f[0] + f[1]
            return np.array([self.V * u if self.physics == ADVECTION else (u * u) * 0.5])
        if self.scheme == D1Q3:
            lam2 = lam * lam
            m0 = (f[0] + f[1]) + f[2]
            if self.physics == BURGERS:
                return np.array([(m0 * m0) * 0.5, (self.alpha * lam2) * m0])
            m1 = lam * (f[1] - f[2])
            g2 = 0.5 * self.g
            return np.array([(m1 * m1) / m0 + g2 * (m0 * m0)])
        nb = self.q // 2
        return np.array(self._eq_vectorial([f[2 * b] + f[2 * b + 1] for b in range(nb)]))

    def collide_with_equilibria(self, f, eq):
        """``collide`` with the non-conserved moments relaxed towards the given equilibria eq
        (q - qc, n) instead of those of f itself; the conserved moments stay (Sec. 4.3.1,
        eq. reconstructedCollision, where eq is the mean over a leaf's finest cells).
        collide_with_equilibria(f, equilibria(f)) is collide(f)."""
        f = np.asarray(f, dtype=np.float64)
        eq = np.asarray(eq, dtype=np.float64)
        lam = self.lam
        out = np.empty_like(f)
        if self.scheme == D1Q5:
            return self._q5_relax(f, eq)
        if self.scheme == D1Q2:
            u = f[0] + f[1]
            m1 = lam * (f[0] - f[1])
            s = self.s[0]
            m1s = (1.0 - s) * m1 + s * eq[0]
            r = m1s / lam
            out[0] = 0.5 * (u + r)
            out[1] = 0.5 * (u - r)
        elif self.scheme == D1Q3:
            lam2 = lam * lam
            m0 = (f[0] + f[1]) + f[2]
            m1 = lam * (f[1] - f[2])
            m2 = lam2 * (f[1] + f[2])
            if self.physics == BURGERS:
                s1, s2 = self.s
                m1s = (1.0 - s1) * m1 + s1 * eq[0]
                m2s = (1.0 - s2) * m2 + s2 * eq[1]
            else:
                s2 = self.s[0]
                m1s = m1
                m2s = (1.0 - s2) * m2 + s2 * eq[0]
            a = m2s / lam2
            b = m1s / lam
            out[0] = m0 - a
            out[1] = 0.5 * (a + b)
            out[2] = 0.5 * (a - b)
        else:
            nb = self.q // 2
            for b in range(nb):
                c = f[2 * b] + f[2 * b + 1]
                s = self.s[b]
                n = lam * (f[2 * b] - f[2 * b + 1])
                ns = (1.0 - s) * n + s * eq[b]
                r = ns / lam
                out[2 * b] = 0.5 * (c + r)
                out[2 * b + 1] = 0.5 * (c - r)
        return out

    def equilibrium(self, mc):
        """Populations at equilibrium for conserved moments mc of shape (qc, n) (Sec. 2.1.1:
        the initial datum is taken at equilibrium)."""
        mc = np.asarray(mc, dtype=np.float64).reshape(self.qc, -1)
        lam = self.lam
        n = mc.shape[1]
        out = np.empty((self.q, n))
        if self.scheme == D1Q5:
            eq2, eq3, eq4 = self._q5_equilibria(mc[0], mc[1])
            return self._q5_populations(mc[0], mc[1], eq2, eq3, eq4)
        if self.scheme == D1Q2:
            u = mc[0]
            eq = self.V * u if self.physics == ADVECTION else (u * u) * 0.5
            r = eq / lam
            out[0] = 0.5 * (u + r)
            out[1] = 0.5 * (u - r)
        elif self.scheme == D1Q3:
            lam2 = lam * lam
            m0 = mc[0]
            if self.physics == BURGERS:
                eq1 = (m0 * m0) * 0.5
                eq2 = (self.alpha * lam2) * m0
            else:
                eq1 = mc[1]
                g2 = 0.5 * self.g
                eq2 = (eq1 * eq1) / m0 + g2 * (m0 * m0)
            a = eq2 / lam2
            b = eq1 / lam
            out[0] = m0 - a
            out[1] = 0.5 * (a + b)
            out[2] = 0.5 * (a - b)
        else:
            nb = self.q // 2
            c = [mc[b] for b in range(nb)]
            eqs = self._eq_vectorial(c)
            for b in range(nb):
                r = eqs[b] / lam
                out[2 * b] = 0.5 * (c[b] + r)
                out[2 * b + 1] = 0.5 * (c[b] - r)
        return out

    def conserved(self, f):
        """Conserved moments (qc, n) of populations f (q, n)."""
        f = np.asarray(f, dtype=np.float64)
        if self.scheme == D1Q5:
            m0, m1 = self._q5_moments(f)[:2]
            return np.stack([m0, m1])
        if self.scheme == D1Q2:
            return (f[0] + f[1])[None, :]
        if self.scheme == D1Q3:
            m0 = (f[0] + f[1]) + f[2]
            if self.qc == 1:
                return m0[None, :]
            return np.stack([m0, self.lam * (f[1] - f[2])])
        nb = self.q // 2
        return np.stack([f[2 * b] + f[2 * b + 1] for b in range(nb)])

    # ---------------------------------------------------------- by definition
    def moment_matrix(self):
        """The change of basis M of Sec. 2.1 / 5.1.1 / 5.2.1 / 5.3, moments ordered as in the paper."""
        lam = self.lam
        if self.scheme == D1Q5:
            w = np.array([0.0, 1.0, -1.0, 2.0, -2.0])
            return np.stack([(lam * w) ** k for k in range(5)])
        if self.scheme == D1Q2:
            return np.array([[1.0, 1.0], [lam, -lam]])
        if self.scheme == D1Q3:
            return np.array([[1.0, 1.0, 1.0], [0.0, lam, -lam], [0.0, lam * lam, lam * lam]])
        nb = self.q // 2
        M = np.zeros((self.q, self.q))
        for b in range(nb):
            M[2 * b, 2 * b:2 * b + 2] = [1.0, 1.0]
            M[2 * b + 1, 2 * b:2 * b + 2] = [lam, -lam]
        return M

    def conserved_indices(self):
        if self.scheme in (D1Q2, D1Q3, D1Q5):
            return list(range(self.qc))
        return [2 * b for b in range(self.q // 2)]

    def equilibria_by_definition(self, m):
        """Dict {moment index: equilibrium value} from the moment vector m (q, n), written as
        the paper prints the formulas (Sec. 5.1.1, 5.2.1, 5.3)."""
        if self.scheme == D1Q5:
            m2 = m[1] ** 2 / m[0] + self.g * m[0] ** 2 / 2
            return {2: m2, 3: self.alpha * self.lam ** 2 * m[1], 4: self.beta * self.lam ** 2 * m2}
        if self.scheme == D1Q2:
            u = m[0]
            return {1: self.V * u if self.physics == ADVECTION else u ** 2 / 2}
        if self.scheme == D1Q3:
            if self.physics == BURGERS:
                return {1: m[0] ** 2 / 2, 2: self.alpha * self.lam ** 2 * m[0]}
            return {2: m[1] ** 2 / m[0] + self.g * m[0] ** 2 / 2}
        if self.physics == SHALLOW_WATER:
            return {1: m[2], 3: m[2] ** 2 / m[0] + self.g * m[0] ** 2 / 2}
        gam = self.gamma_gas
        return {1: m[2],
                3: (3 / 2 - gam / 2) * m[2] ** 2 / m[0] + (gam - 1) * m[4],
                5: gam * m[4] * m[2] / m[0] + (1 - gam) / 2 * m[2] ** 3 / m[0] ** 2}

    def collide_by_definition(self, f):
        M = self.moment_matrix()
        m = M @ np.asarray(f, dtype=np.float64)
        eq = self.equilibria_by_definition(m)
        ms = m.copy()
        for i, (idx, val) in enumerate(sorted(eq.items())):
            ms[idx] = (1 - self.s[i]) * m[idx] + self.s[i] * val
        return np.linalg.solve(M, ms)


def scheme_from_params(p):
    """Build a Scheme from a params dict with keys scheme, physics, lam, s, phys (V, g, gamma_gas, alpha)."""
    phys = list(p.get("phys", [0.0, 1.0, 1.4, 0.9])) + [0.0] * 4
    if p["scheme"] == D1Q5:  # phys[0] carries beta (no advection velocity in shallow water)
        return Scheme(p["scheme"], p["physics"], p["lam"], p["s"], g=phys[1], alpha=phys[3], beta=phys[0])
    return Scheme(p["scheme"], p["physics"], p["lam"], p["s"],
                  V=phys[0], g=phys[1], gamma_gas=phys[2], alpha=phys[3])
