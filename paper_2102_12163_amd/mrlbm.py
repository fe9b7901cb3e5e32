"""ctypes binding of the C ABI in include/mrlbm.h (argument marshalling only).

Every step of the method runs in the HIP kernels of ``libmrlbm.so``; this module only
converts Python parameters and numpy arrays to the ABI's structs and pointers. Importing
it does not load the library; the first call does, and raises if it is not built.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrlbm.so")

ABI_VERSION = 1
OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, ECAPACITY, ESTATE = 0, -1, -2, -3, -4, -5, -6
D1Q2, D1Q3, D1Q2x2, D1Q2x3, D1Q5 = 0, 1, 2, 3, 4
ADVECTION, BURGERS, SHALLOW_WATER, EULER = 0, 1, 2, 3
PERIODIC, CLAMP = 0, 1
FP64, FP32_STORAGE = 0, 1
FLAG_RECONSTRUCTED_COLLISION = 1  # mrlbm_params.flags: reconstructed collision (Sec. 4.3.1)
LEAVES, FINEST = 0, 1
MAX_J = 24
ONCHIP_MAX_J = 16
PRED_OFF, PRED_LEARNED, PRED_RECORD = 0, 1, 2
MLP_INPUTS, MLP_PARAMS = 32, 6337

_STATUS = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENUMERIC: "ENUMERIC",
           ECAPACITY: "ECAPACITY", ESTATE: "ESTATE"}

c_int32, c_int64, c_uint32, c_double, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                                   ctypes.c_double, ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [("abi_version", c_int32), ("scheme", c_int32), ("physics", c_int32), ("bc", c_int32),
                ("precision", c_int32), ("n_s", c_int32), ("lam", c_double), ("s", c_double * 8),
                ("phys", c_double * 4), ("x_min", c_double), ("x_max", c_double), ("j_min", c_int32),
                ("j_max", c_int32), ("gamma", c_int32), ("mu_bar", c_int32), ("eps", c_double),
                ("flags", c_uint32), ("reserved", c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("steps", c_int64), ("leaves", c_int64), ("leaf_updates", c_int64),
                ("numeric_error", c_int32), ("q", c_int32), ("q_cons", c_int32), ("j_max", c_int32),
                ("tree_cells", c_int64), ("misses", c_int64), ("redos", c_int64)]


class Params2D(ctypes.Structure):
    _fields_ = [("abi_version", c_int32), ("physics", c_int32), ("bc", c_int32), ("gamma", c_int32),
                ("lam", c_double), ("s", c_double * 3), ("V", c_double * 2), ("j_min", c_int32), ("j_max", c_int32),
                ("mu_bar", c_int32), ("reserved", c_int32), ("eps", c_double)]


class MRLBMError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


# Names and signatures of every exported entry point (also used by the export test).
_P, _PP = ctypes.POINTER, ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "mrlbm_validate": (c_int32, [_P(Params)]),
    "mrlbm_create": (c_int32, [_P(Params), _P(c_double), c_void_p, _PP]),
    "mrlbm_adapt": (c_int32, [c_void_p]),
    "mrlbm_step": (c_int32, [c_void_p, c_int32]),
    "mrlbm_moments": (c_int32, [c_void_p, c_int32, _P(c_double), c_int64, _P(c_int64)]),
    "mrlbm_populations": (c_int32, [c_void_p, _P(c_double), c_int64, _P(c_int64)]),
    "mrlbm_leaves": (c_int32, [c_void_p, _P(c_int32), _P(c_int64), c_int64, _P(c_int64)]),
    "mrlbm_stats": (c_int32, [c_void_p, _P(Stats)]),
    "mrlbm_step_timed": (c_int32, [c_void_p, c_int32, _P(c_double)]),
    "mrlbm_destroy": (None, [c_void_p]),
    "mrlbm_last_error": (ctypes.c_char_p, [c_void_p]),
    "mrlbm_batch_create": (c_int32, [_P(Params), c_int32, _P(_P(c_double)), c_void_p, _PP]),
    "mrlbm_batch_step": (c_int32, [c_void_p, c_int32]),
    "mrlbm_batch_step_timed": (c_int32, [c_void_p, c_int32, _P(c_double)]),
    "mrlbm_batch_moments": (c_int32, [c_void_p, c_int32, c_int32, _P(c_double), c_int64, _P(c_int64)]),
    "mrlbm_batch_leaves": (c_int32, [c_void_p, c_int32, _P(c_int32), _P(c_int64), c_int64, _P(c_int64)]),
    "mrlbm_batch_stats": (c_int32, [c_void_p, c_int32, _P(Stats)]),
    "mrlbm_batch_total_updates": (c_int32, [c_void_p, _P(c_int64)]),
    "mrlbm_batch_set_block": (c_int32, [c_void_p, c_int32]),
    "mrlbm_batch_get_block": (c_int32, [c_void_p, _P(c_int32)]),
    "mrlbm_batch_set_capacity": (c_int32, [c_void_p, c_int32]),
    "mrlbm_batch_get_capacity": (c_int32, [c_void_p, _P(c_int32)]),
    "mrlbm_batch_tune": (c_int32, [c_void_p, c_int32, _P(c_int32), _P(c_int32)]),
    "mrlbm_batch_set_schedule": (c_int32, [c_void_p, c_int32]),
    "mrlbm_batch_get_schedule": (c_int32, [c_void_p, _P(c_int32)]),
    "mrlbm_batch_set_launch_steps": (c_int32, [c_void_p, c_int32]),
    "mrlbm_batch_set_classes": (c_int32, [c_void_p, c_int32, _P(c_int32), _P(c_int32), _P(c_int32)]),
    "mrlbm_batch_get_classes": (c_int32, [c_void_p, c_int32, _P(c_int32), _P(c_int32), _P(c_int32)]),
    "mrlbm_batch_checkpoint": (c_int32, [c_void_p]),
    "mrlbm_batch_restore": (c_int32, [c_void_p]),
    "mrlbm_set_predictor": (c_int32, [c_void_p, _P(ctypes.c_uint16), c_int32, c_double, c_int64]),
    "mrlbm_batch_set_predictor": (c_int32, [c_void_p, _P(ctypes.c_uint16), c_int32, c_double, c_int64]),
    "mrlbm_samples": (c_int32, [c_void_p, _P(ctypes.c_float), _P(ctypes.c_float), c_int64, _P(c_int64)]),
    "mrlbm_batch_samples": (c_int32, [c_void_p, _P(ctypes.c_float), _P(ctypes.c_float), c_int64, _P(c_int64)]),
    "mrlbm_mlp_create": (c_int32, [_P(ctypes.c_float), _PP]),
    "mrlbm_mlp_loss_grad": (c_int32, [c_void_p, _P(ctypes.c_float), _P(ctypes.c_float), c_int64, ctypes.c_float,
                                      _P(ctypes.c_float), _P(ctypes.c_float)]),
    "mrlbm_mlp_train": (c_int32, [c_void_p, _P(ctypes.c_float), _P(ctypes.c_float), c_int64, c_int32, c_int32,
                                  ctypes.c_float, ctypes.c_float, ctypes.c_uint64, _P(ctypes.c_float)]),
    "mrlbm_mlp_params": (c_int32, [c_void_p, _P(ctypes.c_float), _P(ctypes.c_uint16)]),
    "mrlbm_mlp_logits": (c_int32, [c_void_p, _P(ctypes.c_float), c_int64, _P(ctypes.c_float)]),
    "mrlbm_mlp_destroy": (None, [c_void_p]),
    "mrlbm_mlp_last_error": (ctypes.c_char_p, [c_void_p]),
    "mrlbm_run_noalloc": (c_int32, [_P(Params), c_void_p, c_int32, c_void_p, c_void_p]),
    "mrlbm2d_validate": (c_int32, [_P(Params2D)]),
    "mrlbm2d_create": (c_int32, [_P(Params2D), _P(c_double), c_void_p, _PP]),
    "mrlbm2d_step": (c_int32, [c_void_p, c_int32]),
    "mrlbm2d_step_timed": (c_int32, [c_void_p, c_int32, _P(ctypes.c_float)]),
    "mrlbm2d_moments": (c_int32, [c_void_p, _P(c_double), c_int64]),
    "mrlbm2d_split": (c_int32, [c_void_p, c_int32, _P(ctypes.c_uint8), c_int64]),
    "mrlbm2d_stats": (c_int32, [c_void_p, _P(c_int64), _P(c_int64), _P(c_int64)]),
    "mrlbm2d_destroy": (None, [c_void_p]),
    "mrlbm2d_last_error": (ctypes.c_char_p, [c_void_p]),
    "mrlbm_batch_destroy": (None, [c_void_p]),
    "mrlbm_batch_last_error": (ctypes.c_char_p, [c_void_p]),
}

_lib = None


def lib():
    """Load libmrlbm.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(c_double))


def make_params(p):
    """Params struct from a dict with keys scheme, physics, bc, precision, lam, s, phys,
    x_min, x_max, jmin, jmax, gamma, mu_bar, eps (the workload dictionaries), and optionally
    collision = "leaves" (default) or "reconstructed"."""
    s = list(np.atleast_1d(np.asarray(p.get("s", [1.0]), dtype=np.float64)))
    phys = list(p.get("phys", [0.0, 1.0, 1.4, 0.9])) + [0.0] * 4
    P = Params()
    P.abi_version = p.get("abi_version", ABI_VERSION)
    P.scheme = p["scheme"]
    P.physics = p["physics"]
    P.bc = p.get("bc", PERIODIC)
    P.precision = p.get("precision", FP64)
    P.n_s = len(s)
    P.lam = p["lam"]
    for i, v in enumerate(s[:8]):
        P.s[i] = v
    for i in range(4):
        P.phys[i] = phys[i]
    P.x_min = p.get("x_min", -1.0)
    P.x_max = p.get("x_max", 1.0)
    P.j_min = p["jmin"]
    P.j_max = p["jmax"]
    P.gamma = p.get("gamma", 1)
    P.mu_bar = p.get("mu_bar", 0)
    P.eps = p["eps"]
    P.flags = p.get("flags", 0) | (FLAG_RECONSTRUCTED_COLLISION if p.get("collision", "leaves") == "reconstructed" else 0)
    return P


# Conserved moments per (scheme, physics) pair (the valid pairs of the C ABI).
_Q_CONS = {(D1Q2, ADVECTION): 1, (D1Q2, BURGERS): 1, (D1Q3, BURGERS): 1, (D1Q3, SHALLOW_WATER): 2,
           (D1Q2x2, SHALLOW_WATER): 2, (D1Q2x3, EULER): 3, (D1Q5, SHALLOW_WATER): 2}


def _initial_moments(P, m_cons0):
    """m_cons0 as a contiguous float64 array of shape (q_cons, 2^j_max): the C side reads
    exactly q_cons 2^j_max doubles from it."""
    m = np.ascontiguousarray(m_cons0, dtype=np.float64)
    qc = _Q_CONS.get((P.scheme, P.physics))
    if qc is not None and 0 <= P.j_max <= 30:
        want = (qc, 1 << P.j_max)
        if m.shape != want and not (qc == 1 and m.shape == (want[1],)):
            raise ValueError(f"initial moments have shape {m.shape}, need {want}")
    return m


def validate(p):
    P = p if isinstance(p, Params) else make_params(p)
    return lib().mrlbm_validate(ctypes.byref(P))


NOALLOC_SCRATCH_BYTES = 5 << 20


def run_noalloc(params, d_m_cons0, nsteps, d_m_out, stream=None):
    """mrlbm_run_noalloc: device addresses (ints) of the initial finest conserved averages
    [q_cons][2^J] and of the output [q_cons][2^J]; returns the status code (nothing is
    allocated; the call is enqueued on ``stream`` and does not synchronize)."""
    P = params if isinstance(params, Params) else make_params(params)
    return lib().mrlbm_run_noalloc(ctypes.byref(P), c_void_p(d_m_cons0), int(nsteps), c_void_p(d_m_out), stream)


def _check(rc, msgfn):
    if rc != OK:
        raise MRLBMError(rc, msgfn())


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _u16ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))


def _samples(fn, h, err):
    n = c_int64()
    rc = fn(h, None, None, 0, ctypes.byref(n))
    if rc not in (OK, ECAPACITY):
        _check(rc, err)
    X = np.zeros((max(n.value, 1), MLP_INPUTS), dtype=np.float32)
    y = np.zeros(max(n.value, 1), dtype=np.float32)
    _check(fn(h, _fptr(X), _fptr(y), X.shape[0], ctypes.byref(n)), err)
    return X[: n.value], y[: n.value]


class MLP:
    """The refinement predictor's network on the GPU (training and deployment logits)."""

    def __init__(self, theta0):
        t = np.ascontiguousarray(theta0, dtype=np.float32)
        if t.size != MLP_PARAMS:
            raise ValueError("need MLP_PARAMS parameters")
        h = ctypes.c_void_p()
        _check(lib().mrlbm_mlp_create(_fptr(t), ctypes.byref(h)), lambda: lib().mrlbm_mlp_last_error(None).decode())
        self.h = h

    def _err(self):
        return lib().mrlbm_mlp_last_error(self.h).decode()

    def loss_grad(self, X, y, pos_weight=1.0):
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        loss = ctypes.c_float()
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(lib().mrlbm_mlp_loss_grad(self.h, _fptr(X), _fptr(y), X.shape[0], float(pos_weight), ctypes.byref(loss),
                                         _fptr(g)), self._err)
        return loss.value, g

    def train(self, X, y, epochs=20, batch=512, lr=1e-3, pos_weight=1.0, seed=0):
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        loss = ctypes.c_float()
        _check(lib().mrlbm_mlp_train(self.h, _fptr(X), _fptr(y), X.shape[0], int(epochs), int(batch), float(lr),
                                     float(pos_weight), int(seed), ctypes.byref(loss)), self._err)
        return loss.value

    def params(self):
        t = np.zeros(MLP_PARAMS, dtype=np.float32)
        b = np.zeros(MLP_PARAMS, dtype=np.uint16)
        _check(lib().mrlbm_mlp_params(self.h, _fptr(t), _u16ptr(b)), self._err)
        return t, b

    def logits(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.zeros(X.shape[0], dtype=np.float32)
        _check(lib().mrlbm_mlp_logits(self.h, _fptr(X), X.shape[0], _fptr(out)), self._err)
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().mrlbm_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MRLBM:
    """One adaptive run on the GPU."""

    def __init__(self, params, m_cons0, stream=None):
        L = lib()
        self.P = params if isinstance(params, Params) else make_params(params)
        m = _initial_moments(self.P, m_cons0)
        h = ctypes.c_void_p()
        rc = L.mrlbm_create(ctypes.byref(self.P), _dptr(m), stream, ctypes.byref(h))
        _check(rc, lambda: L.mrlbm_last_error(None).decode())
        self.h = h
        st = self.stats()
        self.q, self.qc, self.jmax = st["q"], st["q_cons"], st["j_max"]

    def _err(self):
        return lib().mrlbm_last_error(self.h).decode()

    def adapt(self):
        _check(lib().mrlbm_adapt(self.h), self._err)

    def step(self, n=1):
        _check(lib().mrlbm_step(self.h, int(n)), self._err)

    def step_timed(self, n):
        ms = c_double()
        _check(lib().mrlbm_step_timed(self.h, int(n), ctypes.byref(ms)), self._err)
        return ms.value

    def moments(self, where=LEAVES):
        n = c_int64()
        rc = lib().mrlbm_moments(self.h, where, None, 0, ctypes.byref(n))
        if rc not in (OK, ECAPACITY):
            _check(rc, self._err)
        out = np.empty(self.qc * max(n.value, 1))
        _check(lib().mrlbm_moments(self.h, where, _dptr(out), out.size, ctypes.byref(n)), self._err)
        return out[: self.qc * n.value].reshape(self.qc, n.value)

    def populations(self):
        n = c_int64()
        rc = lib().mrlbm_populations(self.h, None, 0, ctypes.byref(n))
        if rc not in (OK, ECAPACITY):
            _check(rc, self._err)
        out = np.empty(self.q * max(n.value, 1))
        _check(lib().mrlbm_populations(self.h, _dptr(out), out.size, ctypes.byref(n)), self._err)
        return out[: self.q * n.value].reshape(self.q, n.value)

    def leaves(self):
        n = c_int64()
        rc = lib().mrlbm_leaves(self.h, None, None, 0, ctypes.byref(n))
        if rc not in (OK, ECAPACITY):
            _check(rc, self._err)
        lv = np.empty(max(n.value, 1), dtype=np.int32)
        ix = np.empty(max(n.value, 1), dtype=np.int64)
        _check(lib().mrlbm_leaves(self.h, lv.ctypes.data_as(ctypes.POINTER(c_int32)),
                                  ix.ctypes.data_as(ctypes.POINTER(c_int64)), lv.size, ctypes.byref(n)), self._err)
        return lv[: n.value], ix[: n.value]

    def stats(self):
        s = Stats()
        _check(lib().mrlbm_stats(self.h, ctypes.byref(s)), self._err)
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def set_predictor(self, bf16_params=None, mode=PRED_LEARNED, gate=8.0, sample_capacity=0):
        ptr = None
        if bf16_params is not None:
            self._pw = np.ascontiguousarray(bf16_params, dtype=np.uint16)
            ptr = _u16ptr(self._pw)
        _check(lib().mrlbm_set_predictor(self.h, ptr, int(mode), float(gate), int(sample_capacity)), self._err)

    def samples(self):
        return _samples(lib().mrlbm_samples, self.h, self._err)

    def close(self):
        if getattr(self, "h", None):
            lib().mrlbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent runs advanced by one launch per step call."""

    def __init__(self, params_list, m_cons_list, stream=None):
        L = lib()
        n = len(params_list)
        arr = (Params * n)()
        for i, p in enumerate(params_list):
            arr[i] = p if isinstance(p, Params) else make_params(p)
        if len(m_cons_list) != n:
            raise ValueError("need one initial moment array per run")
        self._m = [_initial_moments(arr[i], m) for i, m in enumerate(m_cons_list)]
        ptrs = (ctypes.POINTER(c_double) * n)(*[_dptr(m) for m in self._m])
        h = ctypes.c_void_p()
        rc = L.mrlbm_batch_create(arr, n, ptrs, stream, ctypes.byref(h))
        _check(rc, lambda: L.mrlbm_batch_last_error(None).decode())
        self.h = h
        self.n = n
        self._qc = []
        for i in range(n):
            self._qc.append(self.stats(i)["q_cons"])

    def _err(self):
        return lib().mrlbm_batch_last_error(self.h).decode()

    def step(self, nsteps=1):
        _check(lib().mrlbm_batch_step(self.h, int(nsteps)), self._err)

    def step_timed(self, nsteps):
        ms = c_double()
        _check(lib().mrlbm_batch_step_timed(self.h, int(nsteps), ctypes.byref(ms)), self._err)
        return ms.value

    def moments(self, inst, where=LEAVES):
        n = c_int64()
        qc = self._qc[inst]
        rc = lib().mrlbm_batch_moments(self.h, inst, where, None, 0, ctypes.byref(n))
        if rc not in (OK, ECAPACITY):
            _check(rc, self._err)
        out = np.empty(qc * max(n.value, 1))
        _check(lib().mrlbm_batch_moments(self.h, inst, where, _dptr(out), out.size, ctypes.byref(n)), self._err)
        return out[: qc * n.value].reshape(qc, n.value)

    def leaves(self, inst):
        n = c_int64()
        rc = lib().mrlbm_batch_leaves(self.h, inst, None, None, 0, ctypes.byref(n))
        if rc not in (OK, ECAPACITY):
            _check(rc, self._err)
        lv = np.empty(max(n.value, 1), dtype=np.int32)
        ix = np.empty(max(n.value, 1), dtype=np.int64)
        _check(lib().mrlbm_batch_leaves(self.h, inst, lv.ctypes.data_as(ctypes.POINTER(c_int32)),
                                        ix.ctypes.data_as(ctypes.POINTER(c_int64)), lv.size, ctypes.byref(n)),
               self._err)
        return lv[: n.value], ix[: n.value]

    def stats(self, inst):
        s = Stats()
        _check(lib().mrlbm_batch_stats(self.h, inst, ctypes.byref(s)), self._err)
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def set_predictor(self, bf16_params=None, mode=PRED_LEARNED, gate=8.0, sample_capacity=0):
        ptr = None
        if bf16_params is not None:
            self._pw = np.ascontiguousarray(bf16_params, dtype=np.uint16)
            ptr = _u16ptr(self._pw)
        _check(lib().mrlbm_batch_set_predictor(self.h, ptr, int(mode), float(gate), int(sample_capacity)), self._err)

    def samples(self):
        return _samples(lib().mrlbm_batch_samples, self.h, self._err)

    def total_updates(self):
        t = c_int64()
        _check(lib().mrlbm_batch_total_updates(self.h, ctypes.byref(t)), self._err)
        return t.value

    def set_block(self, threads):
        _check(lib().mrlbm_batch_set_block(self.h, int(threads)), self._err)

    def set_capacity(self, cells):
        _check(lib().mrlbm_batch_set_capacity(self.h, int(cells)), self._err)

    def tune(self, trial_steps=20):
        t, c = c_int32(), c_int32()
        _check(lib().mrlbm_batch_tune(self.h, int(trial_steps), ctypes.byref(t), ctypes.byref(c)), self._err)
        return t.value, c.value

    def set_schedule(self, stride):
        _check(lib().mrlbm_batch_set_schedule(self.h, int(stride)), self._err)

    def set_launch_steps(self, steps):
        _check(lib().mrlbm_batch_set_launch_steps(self.h, int(steps)), self._err)

    def set_classes(self, j_upper=(), threads=(), runs_per_cu=()):
        """Launch classes by j_max (see mrlbm_batch_set_classes); empty: one launch."""
        n = len(j_upper)
        arr = lambda v: (c_int32 * max(n, 1))(*[int(x) for x in v])  # noqa: E731
        _check(lib().mrlbm_batch_set_classes(self.h, n, arr(j_upper), arr(threads), arr(runs_per_cu)), self._err)

    def get_classes(self):
        """[(runs, on-chip capacity)] per class; empty for a single launch."""
        n = c_int32()
        counts = (c_int32 * 4)()
        cells = (c_int32 * 4)()
        _check(lib().mrlbm_batch_get_classes(self.h, 4, ctypes.byref(n), counts, cells), self._err)
        return [(counts[i], cells[i]) for i in range(n.value)]

    def checkpoint(self):
        """Keep every run's state on the device (one copy, overwritten by the next call)."""
        _check(lib().mrlbm_batch_checkpoint(self.h), self._err)

    def restore(self):
        """Put every run back to the last checkpoint."""
        _check(lib().mrlbm_batch_restore(self.h), self._err)

    def get_schedule(self):
        t = c_int32()
        _check(lib().mrlbm_batch_get_schedule(self.h, ctypes.byref(t)), self._err)
        return t.value

    def get_capacity(self):
        t = c_int32()
        _check(lib().mrlbm_batch_get_capacity(self.h, ctypes.byref(t)), self._err)
        return t.value

    def get_block(self):
        t = c_int32()
        _check(lib().mrlbm_batch_get_block(self.h, ctypes.byref(t)), self._err)
        return t.value

    def close(self):
        if getattr(self, "h", None):
            lib().mrlbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params2d(p):
    """Params2D from a dict with keys physics, bc, gamma, lam, s (three rates or one), V, jmin,
    jmax, mu_bar, eps."""
    P = Params2D()
    P.abi_version = p.get("abi_version", ABI_VERSION)
    P.physics = p["physics"]
    P.bc = p.get("bc", PERIODIC)
    P.gamma = p.get("gamma", 1)
    P.lam = p["lam"]
    s = list(np.atleast_1d(np.asarray(p["s"], dtype=np.float64)))
    s = s * 3 if len(s) == 1 else s
    for i in range(3):
        P.s[i] = s[i]
    V = list(p.get("V", (0.0, 0.0)))
    P.V[0], P.V[1] = V[0], V[1]
    P.j_min = p["jmin"]
    P.j_max = p["jmax"]
    P.mu_bar = p.get("mu_bar", 0)
    P.eps = p["eps"]
    return P


class MRLBM2D:
    """One two-dimensional adaptive run on the GPU (D2Q4, quadtree)."""

    def __init__(self, params, u0, stream=None):
        L = lib()
        self.P = params if isinstance(params, Params2D) else make_params2d(params)
        n = 1 << self.P.j_max if 0 <= self.P.j_max <= 30 else 0
        u = np.ascontiguousarray(u0, dtype=np.float64)
        if u.shape != (n, n):
            raise ValueError(f"initial data have shape {u.shape}, need {(n, n)}")
        h = ctypes.c_void_p()
        _check(L.mrlbm2d_create(ctypes.byref(self.P), _dptr(u), stream, ctypes.byref(h)),
               lambda: L.mrlbm2d_last_error(None).decode())
        self.h = h
        self.n = n

    def _err(self):
        return lib().mrlbm2d_last_error(self.h).decode()

    def step(self, n=1):
        _check(lib().mrlbm2d_step(self.h, int(n)), self._err)

    def step_timed(self, n=1):
        """n steps; returns the milliseconds between HIP events around them."""
        ms = ctypes.c_float()
        _check(lib().mrlbm2d_step_timed(self.h, int(n), ctypes.byref(ms)), self._err)
        return ms.value

    def moments(self):
        out = np.empty((self.n, self.n))
        _check(lib().mrlbm2d_moments(self.h, _dptr(out), out.size), self._err)
        return out

    def split(self, level):
        m = 1 << level
        out = np.empty((m, m), dtype=np.uint8)
        _check(lib().mrlbm2d_split(self.h, int(level), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), out.size),
               self._err)
        return out.astype(bool)

    def stats(self):
        a, b, c = c_int64(), c_int64(), c_int64()
        _check(lib().mrlbm2d_stats(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), self._err)
        return {"steps": a.value, "leaves": b.value, "leaf_updates": c.value}

    def close(self):
        if getattr(self, "h", None):
            lib().mrlbm2d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
