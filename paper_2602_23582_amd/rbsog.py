"""Thin ctypes binding of the RBSOG C ABI (include/rbsog.h).

Argument marshalling only: every step of the evaluation runs in the HIP
library ``librbsog.so``.  Position and force arrays may be torch tensors on
the GPU (fast path: their device pointers are passed) or numpy arrays on the
host; small outputs come back as numpy arrays.  Importing this module does
not load the library; the first use does, and raises if it is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RBSOG_LIBRARY") or os.path.join(HERE, "librbsog.so")

PREC_FP64 = 0
PREC_FP32C = 1
RECAL_PRINTED = 0
RECAL_EXCHANGE = 1
MAX_P = 1024
MAX_MODES = MAX_P + 1

ERRORS = {0: "RBSOG_OK", -1: "RBSOG_EINVAL", -2: "RBSOG_ENEUTRAL", -3: "RBSOG_EBOX", -4: "RBSOG_ENOMEM",
          -5: "RBSOG_EDEVICE", -6: "RBSOG_ESTATE", -7: "RBSOG_EAGAIN"}

EXPORTS = ["rbsog_params_init", "rbsog_setup", "rbsog_sample_modes", "rbsog_force_virial", "rbsog_pressure",
           "rbsog_rescale", "rbsog_destroy", "rbsog_strerror", "rbsog_last_error", "rbsog_debug_cells",
           "rbsog_debug_modes", "rbsog_step_info", "rbsog_set_timing", "rbsog_get_timing", "rbsog_version"]


class rbsog_params(C.Structure):
    _fields_ = [("b", C.c_double), ("sigma", C.c_double), ("omega", C.c_double), ("M", C.c_int32),
                ("rc", C.c_double), ("P", C.c_int32), ("seed", C.c_uint64), ("system_id", C.c_uint64),
                ("coulomb_k", C.c_double), ("precision", C.c_int32), ("recalibration", C.c_int32),
                ("reserved", C.c_int32 * 6)]


class RBSOGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str | None = None):
    """Load librbsog.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (__graft_entry__.build())")
    L = C.CDLL(path)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pd, pi32, pi64 = C.POINTER(d), C.POINTER(i32), C.POINTER(i64)
    sig = {
        "rbsog_params_init": (C.c_int, [C.POINTER(rbsog_params), d]),
        "rbsog_setup": (C.c_int, [C.POINTER(rbsog_params), i64, pd, pd, vp, C.POINTER(vp)]),
        "rbsog_sample_modes": (C.c_int, [vp, i64, pd, pi32, pi32, pd]),
        "rbsog_force_virial": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, pd, pd]),
        "rbsog_pressure": (C.c_int, [vp, pd, pd]),
        "rbsog_rescale": (C.c_int, [vp, pd, vp, vp, vp, pd]),
        "rbsog_destroy": (C.c_int, [vp]),
        "rbsog_strerror": (C.c_char_p, [C.c_int]),
        "rbsog_last_error": (C.c_char_p, [vp]),
        "rbsog_debug_cells": (C.c_int, [vp, pi32, pi32]),
        "rbsog_debug_modes": (C.c_int, [vp, i32, pi32, pi32, pi32, pd]),
        "rbsog_step_info": (C.c_int, [vp, pi64]),
        "rbsog_set_timing": (C.c_int, [vp, C.c_int]),
        "rbsog_get_timing": (C.c_int, [vp, i32, pi32, C.c_char_p, pd, pi64]),
        "rbsog_version": (C.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pi32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _ptr(a):
    """Device pointer of a torch tensor or host pointer of a numpy array (float64, contiguous)."""
    if hasattr(a, "data_ptr"):
        import torch
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError("position/force tensors must be contiguous float64")
        return C.c_void_p(a.data_ptr())
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
        raise TypeError("position/force arrays must be contiguous float64")
    return C.c_void_p(a.ctypes.data)


def default_params(rc: float) -> rbsog_params:
    p = rbsog_params()
    rc_ = load().rbsog_params_init(C.byref(p), rc)
    if rc_ != 0:
        raise RBSOGError(rc_, "rbsog_params_init")
    return p


class Context:
    """One system: wraps rbsog_setup .. rbsog_destroy."""

    def __init__(self, q, box, rc, P=100, seed=0, system_id=0, precision=PREC_FP32C, recalibration=RECAL_PRINTED,
                 M=10, b=None, sigma=None, omega=None, coulomb_k=1.0, stream=None):
        L = load()
        p = default_params(rc)
        p.P, p.seed, p.system_id, p.M = int(P), int(seed), int(system_id), int(M)
        p.precision, p.recalibration, p.coulomb_k = int(precision), int(recalibration), float(coulomb_k)
        if b is not None:
            p.b = b
        if sigma is not None:
            p.sigma = sigma
        if omega is not None:
            p.omega = omega
        self.params = p
        self.n = len(q)
        q = np.ascontiguousarray(q, dtype=np.float64)
        box = np.ascontiguousarray(box, dtype=np.float64)
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
            except ImportError:
                stream = None
        self._stream = stream
        h = C.c_void_p()
        rc_ = L.rbsog_setup(C.byref(p), self.n, _pd(q), _pd(box), C.c_void_p(stream) if stream else None,
                            C.byref(h))
        if rc_ != 0:
            raise RBSOGError(rc_, "rbsog_setup")
        self._h = h
        self.box = box.copy()

    def _check(self, rc_, what):
        if rc_ != 0:
            msg = load().rbsog_last_error(self._h)
            raise RBSOGError(rc_, f"{what}: {msg.decode() if msg else ''}")

    def sample_modes(self, step, box=None, return_modes=False):
        if box is not None:
            self.box = np.ascontiguousarray(box, dtype=np.float64).copy()
        S = np.zeros(2)
        P = self.params.P
        if return_modes:
            m_r = np.zeros((P, 3), dtype=np.int32)
            m_nr = np.zeros((P, 3), dtype=np.int32)
            self._check(load().rbsog_sample_modes(self._h, int(step), _pd(self.box), _pi32(m_r), _pi32(m_nr),
                                                  _pd(S)), "rbsog_sample_modes")
            return m_r, m_nr, S
        self._check(load().rbsog_sample_modes(self._h, int(step), _pd(self.box), None, None, _pd(S)),
                    "rbsog_sample_modes")
        return None, None, S

    def force_virial(self, x, y, z, fx, fy, fz, energy=True):
        e = np.zeros(3)
        v = np.zeros(6)
        self._check(load().rbsog_force_virial(self._h, _ptr(x), _ptr(y), _ptr(z), _ptr(fx), _ptr(fy), _ptr(fz),
                                              _pd(e) if energy else None, _pd(v) if energy else None),
                    "rbsog_force_virial")
        return (e, v) if energy else (None, None)

    def pressure(self):
        P = np.zeros(9)
        parts = np.zeros(27)
        self._check(load().rbsog_pressure(self._h, _pd(P), _pd(parts)), "rbsog_pressure")
        return P.reshape(3, 3), parts.reshape(3, 3, 3)

    def rescale(self, mu, x, y, z):
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        self._check(load().rbsog_rescale(self._h, _pd(mu), _ptr(x), _ptr(y), _ptr(z), _pd(self.box)),
                    "rbsog_rescale")
        return self.box

    def debug_cells(self):
        cell = np.zeros(self.n, dtype=np.int32)
        nc = np.zeros(3, dtype=np.int32)
        self._check(load().rbsog_debug_cells(self._h, _pi32(cell), _pi32(nc)), "rbsog_debug_cells")
        return cell, nc

    def debug_modes(self, with_rho=True):
        nd = np.zeros(1, dtype=np.int32)
        modes = np.zeros((MAX_MODES, 3), dtype=np.int32)
        counts = np.zeros((MAX_MODES, 2), dtype=np.int32)
        rho = np.zeros((MAX_MODES, 2))
        self._check(load().rbsog_debug_modes(self._h, MAX_MODES, _pi32(nd), _pi32(modes), _pi32(counts),
                                             _pd(rho) if with_rho else None), "rbsog_debug_modes")
        k = int(nd[0])
        return modes[:k], counts[:k], (rho[:k, 0] + 1j * rho[:k, 1]) if with_rho else None

    def step_info(self):
        """(distinct modes, r-chain accepts, recalibration accepts, unordered in-cutoff pairs)."""
        info = np.zeros(4, dtype=np.int64)
        self._check(load().rbsog_step_info(self._h, info.ctypes.data_as(C.POINTER(C.c_int64))), "rbsog_step_info")
        return dict(nd=int(info[0]), acc_r=int(info[1]), acc_nr=int(info[2]), npairs=int(info[3]))

    def set_timing(self, on=True):
        self._check(load().rbsog_set_timing(self._h, 1 if on else 0), "rbsog_set_timing")

    def get_timing(self):
        cap = 32
        nk = np.zeros(1, dtype=np.int32)
        names = C.create_string_buffer(32 * cap)
        ms = np.zeros(cap)
        cnt = np.zeros(cap, dtype=np.int64)
        self._check(load().rbsog_get_timing(self._h, cap, _pi32(nk), names, _pd(ms),
                                            cnt.ctypes.data_as(C.POINTER(C.c_int64))), "rbsog_get_timing")
        out = {}
        raw = names.raw
        for k in range(int(nk[0])):
            nm = raw[32 * k: 32 * k + 32].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[k]), int(cnt[k]))
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().rbsog_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
