"""Plain FP64 CPU oracle for the multiresolution-adapted lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously correct reference
that the HIP path is checked against. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product package
never does, and nothing here imports the product package.

Modules
-------
lattice    d'Humieres schemes: velocities, moments, equilibria, collision (Sec. 2.1,
           Sec. 5.1.1, Sec. 5.2.1, Sec. 5.3).
mr         projection, prediction, details, level thresholds (Sec. 3.1, 3.2, 3.4).
adaptive   dense-level adaptive MR-LBM step: T_eps, H_eps, G, transfer, leaves
           collision, compact reconstructed stream (Sec. 3.3, 4.1, 4.2, 4.3.2, 4.5).
brute      literal set-based twin of the tree operators and of the uncompacted
           stream, for tiny J only (Sec. 3.3, 3.4, 4.2, eq. StreamUncompacted).
reference  the uniform finest-grid scheme L (Sec. 2.1).
metrics    delta, E-style l1 norms and compression factors (Sec. 5).
exact      exact Riemann solutions (Burgers, shallow water, Euler) and their cell averages,
           for the errors E and e against the exact solution (Sec. 5).
"""
