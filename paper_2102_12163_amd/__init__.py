"""MI355X-native multiresolution-adapted lattice Boltzmann (MR-LBM) hot path.

The compute path is the HIP library ``libmrlbm.so`` (C ABI in ``include/mrlbm.h``);
``paper_2102_12163_amd.mrlbm`` is its ctypes binding. ``build`` compiles the library.
"""

from .build import build_library  # noqa: F401
