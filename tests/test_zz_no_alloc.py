"""The allocation-free entry point (mrlbm_run_noalloc) against the entry points it stands
for (mrlbm_create + mrlbm_step + mrlbm_moments(FINEST)): the same bits on the finest-level
conserved moments, on two calls in a row (the second one smaller), and its refusals."""

import ctypes
import sys

import numpy as np
import pytest

import workloads as W
from paper_2102_12163_amd import mrlbm

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


class Hip:
    """Device buffers for the test through the HIP runtime the library uses."""

    def __init__(self):
        mrlbm.lib()
        self.h = ctypes.CDLL("libamdhip64.so")
        self.bufs = []

    def alloc(self, nbytes):
        p = ctypes.c_void_p()
        assert self.h.hipMalloc(ctypes.byref(p), ctypes.c_size_t(nbytes)) == 0
        self.bufs.append(p)
        return p.value

    def put(self, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        d = self.alloc(a.nbytes)
        assert self.h.hipMemcpy(ctypes.c_void_p(d), a.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(a.nbytes), 1) == 0
        return d

    def get(self, d, shape):
        out = np.empty(shape, dtype=np.float64)
        assert self.h.hipDeviceSynchronize() == 0
        assert self.h.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(d), ctypes.c_size_t(out.nbytes),
                                2) == 0
        return out

    def close(self):
        for p in self.bufs:
            self.h.hipFree(p)
        self.bufs = []


def reference(p, mc, n):
    run = mrlbm.MRLBM(p, mc)
    try:
        run.step(n)
        return run.moments(mrlbm.FINEST)
    finally:
        run.close()


def test_noalloc_equals_create_step_moments():
    """Two calls in a row, the second on a smaller run, each against the handle-based path:
    bit for bit. The Euler run at J = 14 uses most of the scratch array; the second call must
    not see anything of the first."""
    hip = Hip()
    try:
        cases = [(W.euler(2, jmax=14, eps=1e-4), 300), (W.burgers(1, jmax=9, eps=1e-3), 60),
                 (dict(W.small_case("burgers_d1q2", seed=4, jmax=10, eps=1e-3)[0], collision="reconstructed",
                       precision=mrlbm.FP32_STORAGE), W.small_case("burgers_d1q2", seed=4, jmax=10, eps=1e-3)[1], 40)]
        cases = [(c[0][0], c[0][1], c[1]) if len(c) == 2 else c for c in cases]
        for p, mc, n in cases:
            announce("noalloc", p["scheme"], "J", p["jmax"], "steps", n)
            d_in = hip.put(mc)
            d_out = hip.alloc(mc.nbytes)
            assert mrlbm.run_noalloc(p, d_in, n, d_out) == mrlbm.OK
            got = hip.get(d_out, mc.shape)
            want = reference(p, mc, n)
            assert np.array_equal(got, want), (p["jmax"], float(np.max(np.abs(got - want))))
        # zero steps: the equilibrium initial data, reconstructed on the finest level
        p, mc = W.advection(3, jmax=8)
        d_in, d_out = hip.put(mc), hip.alloc(mc.nbytes)
        assert mrlbm.run_noalloc(p, d_in, 0, d_out) == mrlbm.OK
        assert np.array_equal(hip.get(d_out, mc.shape), reference(p, mc, 0))
    finally:
        hip.close()


def test_noalloc_refusals():
    """Invalid parameters, NULL pointers and negative step counts are refused on the host; a
    run whose state exceeds the scratch array returns MRLBM_ECAPACITY."""
    hip = Hip()
    try:
        p, mc = W.burgers(0, jmax=8)
        d_in, d_out = hip.put(mc), hip.alloc(mc.nbytes)
        assert mrlbm.run_noalloc(dict(p, eps=-1.0), d_in, 5, d_out) == mrlbm.EINVAL
        assert mrlbm.run_noalloc(p, 0, 5, d_out) == mrlbm.EINVAL
        assert mrlbm.run_noalloc(p, d_in, 5, 0) == mrlbm.EINVAL
        assert mrlbm.run_noalloc(p, d_in, -1, d_out) == mrlbm.EINVAL
        ps, ms = W.shallow(0, jmax=16)  # 65536 cells, four populations: beyond the scratch array
        d_big, d_bout = hip.put(ms), hip.alloc(ms.nbytes)
        assert mrlbm.run_noalloc(ps, d_big, 5, d_bout) == mrlbm.ECAPACITY
        # a refused call leaves the next one unaffected
        assert mrlbm.run_noalloc(p, d_in, 7, d_out) == mrlbm.OK
        assert np.array_equal(hip.get(d_out, mc.shape), reference(p, mc, 7))
    finally:
        hip.close()
