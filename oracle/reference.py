"""Uniform finest-grid lattice Boltzmann scheme L (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2.1: collision (Sec. 2.1.1) on every cell of the lattice L_J, then the stream
(Sec. 2.1.2) F^{n+1}_k = F*_{k - w^h}; the out-of-range index is wrapped (periodic) or
clamped, the same boundary reading as the multiresolution operators.
"""

import numpy as np

from . import mr


class UniformLBM:
    def __init__(self, scheme, jmax, bc, mc0):
        self.sch, self.jmax, self.bc = scheme, int(jmax), int(bc)
        mc0 = np.asarray(mc0, dtype=np.float64).reshape(scheme.qc, 2 ** self.jmax)
        self.F = scheme.equilibrium(mc0)
        self.steps = 0

    def step(self, nsteps=1):
        n = 2 ** self.jmax
        k = np.arange(n)
        for _ in range(int(nsteps)):
            fs = self.sch.collide(self.F)
            out = np.empty_like(fs)
            for h in range(self.sch.q):
                out[h] = fs[h, mr.bc_index(k - int(self.sch.w[h]), n, self.bc)]
            self.F = out
            self.steps += 1
        return self

    def conserved(self):
        return self.sch.conserved(self.F)
