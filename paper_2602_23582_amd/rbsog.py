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
RECAL_SHARED = 2
RECAL_INDEPENDENT = 3
FLAG_EXP_FORM = 1
FLAG_FULL_SHELL = 2
FLAG_HALF_SHELL = 4
MAX_P = 1024
MAX_MODES = MAX_P + 2

ERRORS = {0: "RBSOG_OK", -1: "RBSOG_EINVAL", -2: "RBSOG_ENEUTRAL", -3: "RBSOG_EBOX", -4: "RBSOG_ENOMEM",
          -5: "RBSOG_EDEVICE", -6: "RBSOG_ESTATE", -7: "RBSOG_EAGAIN"}

SCHED_STATIC = 0
SCHED_PERSISTENT = 1
AUTOTUNE_CANDIDATES = [("static", 1), ("persistent", 4), ("persistent", 8), ("persistent", 16), ("persistent", 32)]
# rbsog_batch_autotune_cached: the same schedules without, then with graph replay
TUNE_CANDIDATES = [(s, w, g) for g in (False, True) for s, w in AUTOTUNE_CANDIDATES]

EXPORTS = ["rbsog_params_init", "rbsog_setup", "rbsog_sample_modes", "rbsog_force_virial", "rbsog_pressure",
           "rbsog_rescale", "rbsog_destroy", "rbsog_strerror", "rbsog_last_error", "rbsog_debug_cells",
           "rbsog_debug_modes", "rbsog_step_info", "rbsog_set_timing", "rbsog_get_timing", "rbsog_version",
           "rbsog_batch_setup", "rbsog_batch_step", "rbsog_batch_rescale", "rbsog_batch_set_options",
           "rbsog_batch_autotune", "rbsog_batch_set_timing", "rbsog_batch_get_timing", "rbsog_batch_destroy",
           "rbsog_batch_last_error", "rbsog_server_create", "rbsog_server_submit", "rbsog_server_wait",
           "rbsog_server_stats", "rbsog_server_destroy", "rbsog_server_set_energy", "rbsog_server_last_error",
           "rbsog_npt_init", "rbsog_npt_run", "rbsog_batch_create", "rbsog_batch_admit", "rbsog_stage",
           "rbsog_batch_release", "rbsog_debug_long_range_force", "rbsog_force_virial_noalloc",
           "rbsog_batch_autotune_cached", "rbsog_sample_modes_cell", "rbsog_step",
           "rbsog_step_async", "rbsog_step_wait"]

COUPLE_ANISO = 0
COUPLE_SEMI = 1
COUPLE_ISO = 2


class rbsog_npt_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("kT", C.c_double), ("gamma", C.c_double), ("gamma_box", C.c_double),
                ("box_mass", C.c_double), ("p_ext", C.c_double), ("coupling", C.c_int32),
                ("reserved", C.c_int32 * 7)]


class rbsog_params(C.Structure):
    _fields_ = [("b", C.c_double), ("sigma", C.c_double), ("omega", C.c_double), ("M", C.c_int32),
                ("rc", C.c_double), ("P", C.c_int32), ("seed", C.c_uint64), ("system_id", C.c_uint64),
                ("coulomb_k", C.c_double), ("precision", C.c_int32), ("recalibration", C.c_int32),
                ("flags", C.c_int32), ("M_energy", C.c_int32), ("reserved", C.c_int32 * 4)]


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
        "rbsog_step": (C.c_int, [vp, i64, pd, pd, vp, vp, vp, vp, vp, vp, pd, pd]),
        "rbsog_step_async": (C.c_int, [vp, i64, pd, pd, vp, vp, vp, vp, vp, vp, i32, C.POINTER(C.c_int64)]),
        "rbsog_step_wait": (C.c_int, [vp, i64, pd, pd]),
        "rbsog_destroy": (C.c_int, [vp]),
        "rbsog_strerror": (C.c_char_p, [C.c_int]),
        "rbsog_last_error": (C.c_char_p, [vp]),
        "rbsog_debug_cells": (C.c_int, [vp, pi32, pi32]),
        "rbsog_debug_modes": (C.c_int, [vp, i32, pi32, pi32, pi32, pd]),
        "rbsog_step_info": (C.c_int, [vp, pi64]),
        "rbsog_set_timing": (C.c_int, [vp, C.c_int]),
        "rbsog_get_timing": (C.c_int, [vp, i32, pi32, C.c_char_p, pd, pi64]),
        "rbsog_version": (C.c_int, []),
        "rbsog_batch_setup": (C.c_int, [C.POINTER(rbsog_params), i32, pi64, pd, pd, vp, C.POINTER(vp)]),
        "rbsog_batch_step": (C.c_int, [vp, pi64, pd, vp, vp, vp, vp, vp, vp, pd, pd, pi64]),
        "rbsog_batch_rescale": (C.c_int, [vp, pd, vp, vp, vp, pd]),
        "rbsog_batch_set_options": (C.c_int, [vp, i32, i32, i32]),
        "rbsog_batch_autotune": (C.c_int, [vp, pi64, pd, vp, vp, vp, vp, vp, vp, i32, pd, pi32]),
        "rbsog_batch_set_timing": (C.c_int, [vp, C.c_int]),
        "rbsog_batch_get_timing": (C.c_int, [vp, i32, pi32, C.c_char_p, pd, pi64]),
        "rbsog_batch_destroy": (C.c_int, [vp]),
        "rbsog_batch_last_error": (C.c_char_p, [vp]),
        "rbsog_server_create": (C.c_int, [i32, i64, i32, vp, C.POINTER(vp)]),
        "rbsog_server_submit": (C.c_int, [vp, C.POINTER(rbsog_params), i64, pd, pd, pd, pd, pd, i32, d, pi64]),
        "rbsog_server_wait": (C.c_int, [vp, i64, d, pd, pd, pd, pd, pd, pd]),
        "rbsog_server_stats": (C.c_int, [vp, pd]),
        "rbsog_server_set_energy": (C.c_int, [vp, C.c_int32]),
        "rbsog_server_destroy": (C.c_int, [vp]),
        "rbsog_server_last_error": (C.c_char_p, [vp]),
        "rbsog_npt_init": (C.c_int, [vp, C.POINTER(rbsog_npt_params), pd]),
        "rbsog_npt_run": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, i64, i32, pd, pd, pd, pd]),
        "rbsog_batch_create": (C.c_int, [i64, vp, C.POINTER(vp)]),
        "rbsog_batch_admit": (C.c_int, [vp, vp]),
        "rbsog_stage": (C.c_int, [vp, i64, pd, vp, vp, vp, vp, vp, vp]),
        "rbsog_batch_release": (C.c_int, [vp, vp]),
        "rbsog_debug_long_range_force": (C.c_int, [vp, vp, vp, vp]),
        "rbsog_force_virial_noalloc": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, pd, pd]),
        "rbsog_sample_modes_cell": (C.c_int, [vp, i64, pd, pi32, pi32, pd]),
        "rbsog_batch_autotune_cached": (C.c_int, [vp, C.c_char_p, i32, pi64, pd, vp, vp, vp, vp, vp, vp, i32, pd,
                                                  pi32, pi32]),
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


def _ptr(a, n=None, device=None):
    """Device pointer of a torch tensor or host pointer of a numpy array
    (float64, contiguous).  With n, the array must hold exactly n entries;
    with device (a CUDA device index), a tensor must live on that device.  The
    C ABI sees only pointers and cannot check either."""
    if hasattr(a, "data_ptr"):
        import torch
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError("position/force tensors must be contiguous float64")
        if n is not None and a.numel() != n:
            raise ValueError(f"position/force tensor has {a.numel()} entries, expected {n}")
        if device is not None and a.is_cuda and a.device.index != device:
            raise ValueError(f"tensor on cuda:{a.device.index}, the library's work runs on cuda:{device}")
        return C.c_void_p(a.data_ptr())
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
        raise TypeError("position/force arrays must be contiguous float64")
    if n is not None and a.size != n:
        raise ValueError(f"position/force array has {a.size} entries, expected {n}")
    return C.c_void_p(a.ctypes.data)


def _ptrs(arrs, n, device):
    return [_ptr(a, n, device) for a in arrs]


def _current_device():
    try:
        import torch
        return torch.cuda.current_device() if torch.cuda.is_available() else None
    except ImportError:
        return None


def default_params(rc: float) -> rbsog_params:
    p = rbsog_params()
    rc_ = load().rbsog_params_init(C.byref(p), rc)
    if rc_ != 0:
        raise RBSOGError(rc_, "rbsog_params_init")
    return p


class Context:
    """One system: wraps rbsog_setup .. rbsog_destroy."""

    def __init__(self, q, box, rc, P=100, seed=0, system_id=0, precision=PREC_FP32C, recalibration=RECAL_EXCHANGE,
                 M=10, b=None, sigma=None, omega=None, coulomb_k=1.0, stream=None, flags=0, M_energy=0):
        L = load()
        p = default_params(rc)
        p.P, p.seed, p.system_id, p.M = int(P), int(seed), int(system_id), int(M)
        p.precision, p.recalibration, p.coulomb_k = int(precision), int(recalibration), float(coulomb_k)
        p.flags, p.M_energy = int(flags), int(M_energy)
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
        self.device = _current_device()

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

    def sample_modes_cell(self, step, h, return_modes=False):
        """rbsog_sample_modes_cell: sampling on a general cell h (3 x 3, columns the cell vectors)."""
        self.cell = np.ascontiguousarray(h, dtype=np.float64).reshape(3, 3).copy()
        S = np.zeros(2)
        P = self.params.P
        m_r = np.zeros((P, 3), dtype=np.int32) if return_modes else None
        m_nr = np.zeros((P, 3), dtype=np.int32) if return_modes else None
        self._check(load().rbsog_sample_modes_cell(self._h, int(step), _pd(self.cell),
                                                   _pi32(m_r) if return_modes else None,
                                                   _pi32(m_nr) if return_modes else None, _pd(S)),
                    "rbsog_sample_modes_cell")
        return m_r, m_nr, S

    def force_virial(self, x, y, z, fx, fy, fz, energy=True):
        e = np.zeros(3)
        v = np.zeros(6)
        px = _ptrs((x, y, z, fx, fy, fz), self.n, self.device)
        self._check(load().rbsog_force_virial(self._h, *px, _pd(e) if energy else None, _pd(v) if energy else None),
                    "rbsog_force_virial")
        return (e, v) if energy else (None, None)

    def force_virial_noalloc(self, x, y, z, fx, fy, fz, energy=True):
        """rbsog_force_virial_noalloc: force_virial with the step's partial
        results in the library's fixed per-GPU array; device arrays only."""
        e = np.zeros(3)
        v = np.zeros(6)
        px = _ptrs((x, y, z, fx, fy, fz), self.n, self.device)
        self._check(load().rbsog_force_virial_noalloc(self._h, *px, _pd(e) if energy else None,
                                                      _pd(v) if energy else None),
                    "rbsog_force_virial_noalloc")
        return (e, v) if energy else (None, None)

    def pressure(self):
        P = np.zeros(9)
        parts = np.zeros(27)
        self._check(load().rbsog_pressure(self._h, _pd(P), _pd(parts)), "rbsog_pressure")
        return P.reshape(3, 3), parts.reshape(3, 3, 3)

    def rescale(self, mu, x, y, z):
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        self._check(load().rbsog_rescale(self._h, _pd(mu), *_ptrs((x, y, z), self.n, self.device), _pd(self.box)),
                    "rbsog_rescale")
        return self.box

    def step(self, step, mu, x, y, z, fx, fy, fz, pressure=True, energy=False):
        """rbsog_step: rescale by mu (None: no rescale), sample at the new box,
        forces and pressure in one call (device tensors).  Returns the
        pressure tensor (3, 3) or None, and the energies or None."""
        box = self.box.copy()
        P = np.zeros(9) if pressure else None
        e = np.zeros(3) if energy else None
        m = None if mu is None else np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (3,)))
        self._check(load().rbsog_step(self._h, int(step), _pd(m) if m is not None else None, _pd(box),
                                      *_ptrs((x, y, z, fx, fy, fz), self.n, self.device),
                                      _pd(P) if pressure else None, _pd(e) if energy else None), "rbsog_step")
        self.box = box
        return (P.reshape(3, 3) if pressure else None), e

    def step_async(self, step, mu, x, y, z, fx, fy, fz, energy=False):
        """rbsog_step_async: queue the step and the copy of its results;
        returns the ticket for step_wait."""
        box = self.box.copy()
        m = None if mu is None else np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (3,)))
        t = C.c_int64(-1)
        self._check(load().rbsog_step_async(self._h, int(step), _pd(m) if m is not None else None, _pd(box),
                                            *_ptrs((x, y, z, fx, fy, fz), self.n, self.device), 1 if energy else 0,
                                            C.byref(t)), "rbsog_step_async")
        self.box = box
        return t.value

    def step_wait(self, ticket, energy=False):
        """rbsog_step_wait: the pressure tensor (3, 3) of a queued step, and
        its energies when asked for."""
        P = np.zeros(9)
        e = np.zeros(3) if energy else None
        self._check(load().rbsog_step_wait(self._h, int(ticket), _pd(P), _pd(e) if energy else None),
                    "rbsog_step_wait")
        return P.reshape(3, 3), e

    def stage(self, step, box, x, y, z, fx, fy, fz):
        """Inputs of the next step of a batch of contexts (device tensors)."""
        self.box = np.ascontiguousarray(box, dtype=np.float64).copy()
        self._check(load().rbsog_stage(self._h, int(step), _pd(self.box), *_ptrs((x, y, z, fx, fy, fz), self.n,
                                                                                  self.device)), "rbsog_stage")

    def debug_cells(self):
        cell = np.zeros(self.n, dtype=np.int32)
        nc = np.zeros(3, dtype=np.int32)
        self._check(load().rbsog_debug_cells(self._h, _pi32(cell), _pi32(nc)), "rbsog_debug_cells")
        return cell, nc

    def debug_long_range_force(self, fx, fy, fz):
        """F^{F*} of the last evaluation alone into device tensors (caller order)."""
        self._check(load().rbsog_debug_long_range_force(self._h, *_ptrs((fx, fy, fz), self.n, self.device)),
                    "rbsog_debug_long_range_force")

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
        """rbsog_set_timing: True or 1 every kernel group, 2 the pair kernel only, False off."""
        self._check(load().rbsog_set_timing(self._h, int(on)), "rbsog_set_timing")

    def get_timing(self):
        rc_, out = _timing_table(load().rbsog_get_timing, self._h)
        self._check(rc_, "rbsog_get_timing")
        return out

    def npt_init(self, mass, dt, kT, gamma, gamma_box, box_mass, p_ext, coupling=COUPLE_ANISO):
        """Attach the Langevin NPT integrator (rbsog_npt_init)."""
        p = rbsog_npt_params(dt=dt, kT=kT, gamma=gamma, gamma_box=gamma_box, box_mass=box_mass, p_ext=p_ext,
                             coupling=coupling)
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        if mass.shape != (self.n,):
            raise ValueError("one mass per atom")
        self._check(load().rbsog_npt_init(self._h, C.byref(p), _pd(mass)), "rbsog_npt_init")

    def npt_run(self, x, y, z, px, py, pz, first_step, nsteps, pbox):
        """Advance nsteps NPT steps in place (device tensors); returns (box, pbox, P_ins, P_kin)."""
        box = np.ascontiguousarray(self.box, dtype=np.float64).copy()
        pbox = np.ascontiguousarray(pbox, dtype=np.float64).copy()
        Pi = np.zeros(9)
        Pk = np.zeros(9)
        self._check(load().rbsog_npt_run(self._h, *_ptrs((x, y, z, px, py, pz), self.n, self.device),
                                         int(first_step), int(nsteps), _pd(box), _pd(pbox), _pd(Pi), _pd(Pk)),
                    "rbsog_npt_run")
        self.box = box.copy()
        return box, pbox, Pi.reshape(3, 3), Pk.reshape(3, 3)

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


def _pi64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _timing_table(getter, handle):
    cap = 32
    nk = np.zeros(1, dtype=np.int32)
    names = C.create_string_buffer(32 * cap)
    ms = np.zeros(cap)
    cnt = np.zeros(cap, dtype=np.int64)
    rc = getter(handle, cap, _pi32(nk), names, _pd(ms), _pi64(cnt))
    out = {}
    raw = names.raw
    for k in range(int(nk[0])):
        nm = raw[32 * k: 32 * k + 32].split(b"\0", 1)[0].decode()
        out[nm] = (float(ms[k]), int(cnt[k]))
    return rc, out


def make_params(rc, P=100, seed=0, system_id=0, precision=PREC_FP32C, recalibration=RECAL_EXCHANGE, M=10,
                coulomb_k=1.0, flags=0, M_energy=0):
    p = default_params(rc)
    p.P, p.seed, p.system_id, p.M = int(P), int(seed), int(system_id), int(M)
    p.precision, p.recalibration, p.coulomb_k = int(precision), int(recalibration), float(coulomb_k)
    p.flags, p.M_energy = int(flags), int(M_energy)
    return p


def _stream_or_default(stream):
    if stream is not None:
        return stream
    try:
        import torch
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    except ImportError:
        return None


class Batch:
    """Many systems per launch: wraps rbsog_batch_setup .. rbsog_batch_destroy.

    systems: list of dicts with keys q, box, rc and optionally P, seed,
    system_id, M, recalibration.  Positions and forces are device tensors of
    sum(n) float64 entries, system after system."""

    def __init__(self, systems, precision=PREC_FP32C, stream=None):
        L = load()
        S = len(systems)
        arr = (rbsog_params * S)()
        n = np.zeros(S, dtype=np.int64)
        qs, boxes = [], np.zeros((S, 3))
        for s, spec in enumerate(systems):
            arr[s] = make_params(spec["rc"], P=spec.get("P", 100), seed=spec.get("seed", 0),
                                 system_id=spec.get("system_id", 0), precision=precision,
                                 recalibration=spec.get("recalibration", RECAL_EXCHANGE), M=spec.get("M", 10),
                                 flags=spec.get("flags", 0), M_energy=spec.get("M_energy", 0))
            n[s] = len(spec["q"])
            qs.append(np.asarray(spec["q"], dtype=np.float64))
            boxes[s] = spec["box"]
        q = np.ascontiguousarray(np.concatenate(qs))
        self.n = n
        self.offsets = np.concatenate([[0], np.cumsum(n)])
        self.nsys = S
        self.boxes = np.ascontiguousarray(boxes)
        stream = _stream_or_default(stream)
        h = C.c_void_p()
        rc_ = L.rbsog_batch_setup(arr, S, _pi64(n), _pd(q), _pd(self.boxes), C.c_void_p(stream) if stream else None,
                                  C.byref(h))
        if rc_ != 0:
            raise RBSOGError(rc_, "rbsog_batch_setup")
        self._h = h
        self.device = _current_device()

    def _check(self, rc_, what):
        if rc_ != 0:
            msg = load().rbsog_batch_last_error(self._h)
            raise RBSOGError(rc_, f"{what}: {msg.decode() if msg else ''}")

    def _arrays(self, arrs):
        return _ptrs(arrs, int(self.offsets[-1]), self.device)

    def step(self, steps, boxes, x, y, z, fx, fy, fz, results=True, energy=True):
        """One step of every system.  With results, returns the pressure
        tensors, the energies (zeros unless energy) and the counters of
        rbsog_step_info per system; the energy sum runs only when asked for."""
        steps = np.ascontiguousarray(np.broadcast_to(np.asarray(steps, dtype=np.int64), (self.nsys,)))
        boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(self.nsys, 3)
        if not results:
            self._check(load().rbsog_batch_step(self._h, _pi64(steps), _pd(boxes), *self._arrays((x, y, z, fx, fy, fz)),
                                                None, None, None), "rbsog_batch_step")
            return None
        P = np.zeros((self.nsys, 9))
        U = np.zeros((self.nsys, 3))
        info = np.zeros((self.nsys, 4), dtype=np.int64)
        self._check(load().rbsog_batch_step(self._h, _pi64(steps), _pd(boxes), *self._arrays((x, y, z, fx, fy, fz)),
                                            _pd(P), _pd(U) if energy else None, _pi64(info)),
                    "rbsog_batch_step")
        return P.reshape(self.nsys, 3, 3), U, info

    def rescale(self, mu, x, y, z):
        mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (self.nsys, 3)))
        self._check(load().rbsog_batch_rescale(self._h, _pd(mu), *self._arrays((x, y, z)), _pd(self.boxes)),
                    "rbsog_batch_rescale")
        return self.boxes

    def set_options(self, schedule=SCHED_STATIC, wg_per_cu=16, graph=False):
        self._check(load().rbsog_batch_set_options(self._h, int(schedule), int(wg_per_cu), 1 if graph else 0),
                    "rbsog_batch_set_options")

    def autotune(self, steps, boxes, x, y, z, fx, fy, fz, reps=3):
        steps = np.ascontiguousarray(np.broadcast_to(np.asarray(steps, dtype=np.int64), (self.nsys,)))
        boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(self.nsys, 3)
        ms = np.zeros(len(AUTOTUNE_CANDIDATES))
        choice = np.zeros(1, dtype=np.int32)
        self._check(load().rbsog_batch_autotune(self._h, _pi64(steps), _pd(boxes), *self._arrays((x, y, z, fx, fy, fz)),
                                                int(reps), _pd(ms), _pi32(choice)),
                    "rbsog_batch_autotune")
        return int(choice[0]), ms

    def autotune_cached(self, cache_path, steps, boxes, x, y, z, fx, fy, fz, reps=3, force=False):
        """rbsog_batch_autotune_cached: (index into TUNE_CANDIDATES, per-candidate ms, found in the cache)."""
        steps = np.ascontiguousarray(np.broadcast_to(np.asarray(steps, dtype=np.int64), (self.nsys,)))
        boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(self.nsys, 3)
        ms = np.zeros(len(TUNE_CANDIDATES))
        choice = np.zeros(1, dtype=np.int32)
        cached = np.zeros(1, dtype=np.int32)
        self._check(load().rbsog_batch_autotune_cached(self._h, os.fsencode(cache_path), 1 if force else 0,
                                                       _pi64(steps), _pd(boxes),
                                                       *self._arrays((x, y, z, fx, fy, fz)), int(reps), _pd(ms),
                                                       _pi32(choice), _pi32(cached)),
                    "rbsog_batch_autotune_cached")
        return int(choice[0]), ms, bool(cached[0])

    def set_timing(self, on=True):
        self._check(load().rbsog_batch_set_timing(self._h, int(on)), "rbsog_batch_set_timing")

    def get_timing(self):
        rc_, out = _timing_table(load().rbsog_batch_get_timing, self._h)
        self._check(rc_, "rbsog_batch_get_timing")
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().rbsog_batch_destroy(self._h)
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


class ContextBatch:
    """A batch of existing contexts admitted by device memory: wraps
    rbsog_batch_create, rbsog_batch_admit, rbsog_batch_release and the
    context form of rbsog_batch_step."""

    def __init__(self, mem_budget, stream=None):
        stream = _stream_or_default(stream)
        h = C.c_void_p()
        rc_ = load().rbsog_batch_create(int(mem_budget), C.c_void_p(stream) if stream else None, C.byref(h))
        if rc_ != 0:
            raise RBSOGError(rc_, "rbsog_batch_create")
        self._h = h
        self.members = []

    def _check(self, rc_, what):
        if rc_ != 0:
            msg = load().rbsog_batch_last_error(self._h)
            raise RBSOGError(rc_, f"{what}: {msg.decode() if msg else ''}")

    def admit(self, ctx):
        """Admit a Context; returns False (RBSOG_EAGAIN) when the budget or the slots are full."""
        rc_ = load().rbsog_batch_admit(self._h, ctx._h)
        if rc_ == -7:
            return False
        self._check(rc_, "rbsog_batch_admit")
        self.members.append(ctx)
        return True

    def release(self, ctx):
        self._check(load().rbsog_batch_release(self._h, ctx._h), "rbsog_batch_release")
        self.members.remove(ctx)

    def step(self, energy=True):
        """One step of every admitted context from its staged inputs; returns
        pressures (S, 3, 3), energies (S, 3) and counters (S, 4) in admission order."""
        S = len(self.members)
        P = np.zeros((max(S, 1), 9))
        U = np.zeros((max(S, 1), 3))
        info = np.zeros((max(S, 1), 4), dtype=np.int64)
        self._check(load().rbsog_batch_step(self._h, None, None, None, None, None, None, None, None, _pd(P),
                                            _pd(U) if energy else None, _pi64(info)), "rbsog_batch_step")
        return P[:S].reshape(S, 3, 3), U[:S], info[:S]

    def close(self):
        if getattr(self, "_h", None):
            load().rbsog_batch_destroy(self._h)
            self._h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """The served form: wraps rbsog_server_create .. rbsog_server_destroy."""

    def __init__(self, precision=PREC_FP32C, pool_bytes=1 << 30, max_active=4096, stream=None, energy=True):
        L = load()
        stream = _stream_or_default(stream)
        h = C.c_void_p()
        rc_ = L.rbsog_server_create(int(precision), int(pool_bytes), int(max_active),
                                    C.c_void_p(stream) if stream else None, C.byref(h))
        if rc_ != 0:
            raise RBSOGError(rc_, "rbsog_server_create")
        self._h = h
        self.precision = precision
        self._n = {}
        self._steps = {}
        if not energy:
            self.set_energy(False)

    def set_energy(self, on):
        self._check(load().rbsog_server_set_energy(self._h, 1 if on else 0), "rbsog_server_set_energy")

    def _check(self, rc_, what):
        if rc_ != 0:
            msg = load().rbsog_server_last_error(self._h)
            raise RBSOGError(rc_, f"{what}: {msg.decode() if msg else ''}")

    def submit(self, q, pos, box, rc, nsteps=10, growth=0.001, P=100, seed=0, system_id=0, M=10,
               recalibration=RECAL_EXCHANGE):
        """Queue one request; pos is (n, 3).  Returns its ticket."""
        p = make_params(rc, P=P, seed=seed, system_id=system_id, precision=self.precision, M=M,
                        recalibration=recalibration)
        q = np.ascontiguousarray(q, dtype=np.float64)
        pos = np.asarray(pos, dtype=np.float64)
        x, y, z = (np.ascontiguousarray(pos[:, k]) for k in range(3))
        box = np.ascontiguousarray(box, dtype=np.float64)
        t = np.zeros(1, dtype=np.int64)
        self._check(load().rbsog_server_submit(self._h, C.byref(p), len(q), _pd(q), _pd(x), _pd(y), _pd(z), _pd(box),
                                               int(nsteps), float(growth), _pi64(t)), "rbsog_server_submit")
        ticket = int(t[0])
        self._n[ticket] = len(q)
        self._steps[ticket] = int(nsteps)
        return ticket

    def wait(self, ticket, timeout=-1.0):
        """Block until the request completes; returns dict(forces (n, 3), P (nsteps, 3, 3),
        U (nsteps, 3), queue_s, latency_s, shared_ticks), or None on timeout."""
        n, ns = self._n[ticket], self._steps[ticket]
        fx, fy, fz = np.zeros(n), np.zeros(n), np.zeros(n)
        P = np.zeros((ns, 9))
        U = np.zeros((ns, 3))
        tm = np.zeros(3)
        rc_ = load().rbsog_server_wait(self._h, int(ticket), float(timeout), _pd(fx), _pd(fy), _pd(fz), _pd(P), _pd(U),
                                       _pd(tm))
        if rc_ == -7:
            return None
        del self._n[ticket], self._steps[ticket]
        self._check(rc_, "rbsog_server_wait")
        return dict(forces=np.stack([fx, fy, fz], axis=1), P=P.reshape(ns, 3, 3), U=U, queue_s=float(tm[0]),
                    latency_s=float(tm[1]), shared_ticks=int(tm[2]))

    def stats(self):
        st = np.zeros(11)
        self._check(load().rbsog_server_stats(self._h, _pd(st)), "rbsog_server_stats")
        keys = ["submitted", "completed", "ticks", "atom_steps", "busy_s", "peak_active", "peak_pool_bytes",
                "waiting", "admit_s", "launch_s", "wait_s"]
        return dict(zip(keys, st.tolist()))

    def close(self):
        if getattr(self, "_h", None):
            load().rbsog_server_destroy(self._h)
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
