"""Python binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this module.  It wraps the C functions of
``rbsog_oracle.c`` with numpy arrays and composes them into the per-step
evaluation of Algorithm 1 (steps 2-6) of the paper:

    sample modes -> short-range force/virial/energy -> structure factors ->
    random-batch estimators -> totals.

Nothing here is shared with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None

# Table 1 of the paper (parameter sets at r_c = 9 Angstrom):
# (b~, sigma~, omega~, M energy, M force, M~ pressure), rows 1..4.
TABLE1 = {
    1: (2.0, 4.524309831775139, 0.994446492762232, 12, 4, 4),
    2: (1.62976708826776469, 3.270345668108471, 1.007806979343806, 25, 7, 10),
    3: (1.32070036405934420, 2.049434420796892, 1.001889141148119, 64, 20, 27),
    4: (1.21812525709410644, 1.597010732309955, 1.000901461560333, 124, 40, 69),
}
TABLE1_RC = 9.0


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build_oracle()
        L = C.CDLL(_build.LIB)
        d, i32, i64, u32, u64 = C.c_double, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        P = C.POINTER
        pd, pi32, pi64, pu32 = P(d), P(i32), P(i64), P(u32)
        sig = {
            "orc_sog_params": (None, [d, d, d, C.c_int, pd, pd, pd]),
            "orc_F": (d, [C.c_int, pd, pd, d]),
            "orc_Ft": (d, [C.c_int, pd, pd, d]),
            "orc_omega_c0": (d, [d, d, d, C.c_int]),
            "orc_bsa": (d, [d, d, d, d, C.c_int, C.c_int]),
            "orc_bsa_bound": (d, [d, d]),
            "orc_H_direct": (None, [pd, d, d, pd, pd]),
            "orc_H_poisson": (None, [pd, d, d, pd, pd]),
            "orc_norm_consts": (None, [pd, C.c_int, pd, pd, C.c_int, pd, pd]),
            "orc_philox4x32_10": (None, [pu32, pu32, pu32]),
            "orc_draw_proposal": (None, [u64, u64, u64, u32, u32, u32, pd, pd]),
            "orc_npt_normals": (None, [u64, u64, u64, i64, pd, pd]),
            "orc_target_r": (d, [pi32, pd, C.c_int, pd, pd]),
            "orc_ratio_nr": (d, [pi32, pd, C.c_int, pd, pd]),
            "orc_proposal_pmf": (d, [pi32, pd, d]),
            "orc_sample_modes": (C.c_int, [pd, C.c_int, pd, pd, C.c_int, u64, u64, u64, C.c_int,
                                           pi32, pi32, pi64]),
            "orc_recalibrate": (None, [C.c_int, pi32, pd, pd, C.c_int, pd, pd, pi32, pi64]),
            "orc_start_bound": (d, [pd, C.c_int, pd, pd, C.c_int]),
            "orc_start_states": (C.c_int, [pd, C.c_int, pd, pd, u64, u64, u64, pi32, pi32]),
            "orc_cell_ids": (None, [i64, pd, pd, pd, pd, pi32, pi32]),
            "orc_short_range_brute": (None, [i64, pd, pd, pd, pd, pd, d, C.c_int, pd, pd, pd,
                                             pd, pd, pd, pd, pd]),
            "orc_short_range_cells": (None, [i64, pd, pd, pd, pd, pd, d, C.c_int, pd, pd, pd,
                                             i64, pi64, pd, pd, pd, pd, pd]),
            "orc_rho": (None, [i64, pd, pd, pd, pd, pd, i64, pi32, pd, pd]),
            "orc_long_range_rb": (None, [i64, pd, pd, pd, pd, pd, C.c_int, pi32, pi32, d, d,
                                         i64, pi64, pd, pd, pd, pd, pd, pd]),
            "orc_sog_kspace_full": (None, [i64, pd, pd, pd, pd, pd, C.c_int, pd, pd, pd,
                                           pd, pd, pd, pd, pd]),
            "orc_self_energy": (d, [d, d, d, C.c_int, i64, pd]),
            "orc_ewald": (None, [i64, pd, pd, pd, pd, pd, d, d, d, pd, pd, pd, pd, pd]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_num_threads": (None, [C.c_int]),
            "orc_tri_H_direct": (None, [pd, d, d, pd, pd]),
            "orc_tri_H_poisson": (None, [pd, d, d, pd, pd]),
            "orc_tri_norm_consts": (None, [pd, C.c_int, pd, pd, C.c_int, pd, pd]),
            "orc_tri_target_r": (d, [pi32, pd, C.c_int, pd, pd]),
            "orc_tri_ratio_nr": (d, [pi32, pd, C.c_int, pd, pd]),
            "orc_tri_proposal_pmf": (d, [pi32, pd, d]),
            "orc_tri_round": (None, [pd, pd, d, pi32]),
            "orc_tri_start_bound": (d, [pd, C.c_int, pd, pd, C.c_int]),
            "orc_tri_start_states": (C.c_int, [pd, C.c_int, pd, pd, u64, u64, u64, pi32, pi32]),
            "orc_tri_sample_modes": (C.c_int, [pd, C.c_int, pd, pd, C.c_int, u64, u64, u64, C.c_int,
                                               pi32, pi32, pi64]),
            "orc_tri_chains": (None, [pd, C.c_int, pd, pd, C.c_int, u64, u64, u64, C.c_int, pi32, pi32,
                                      pi32, pi32, pi64]),
            "orc_tri_rho": (None, [i64, pd, pd, pd, pd, pd, i64, pi32, pd, pd]),
            "orc_tri_long_range_rb": (None, [i64, pd, pd, pd, pd, pd, C.c_int, pi32, pi32, d, d,
                                             pd, pd, pd, pd, pd, pd]),
            "orc_tri_short_range": (None, [i64, pd, pd, pd, pd, pd, d, C.c_int, pd, pd, pd,
                                           pd, pd, pd, pd, pd]),
            "orc_tri_sog_kspace_full": (None, [i64, pd, pd, pd, pd, pd, C.c_int, pd, pd, pd,
                                               pd, pd, pd, pd, pd]),
            "orc_tri_ewald": (None, [i64, pd, pd, pd, pd, pd, d, d, d, pd, pd, pd, pd, pd]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _pi32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def _pi64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class SOG:
    """SOG splitting at cutoff rc: Table 1 row scaled to rc (sigma = sigma9 * rc / 9)."""
    b: float
    sigma: float
    omega: float
    M: int
    rc: float
    w: np.ndarray
    wt: np.ndarray
    s: np.ndarray


def sog(rc: float, row: int = 2, M: int = 10, omega: float | None = None, b: float | None = None,
        sigma: float | None = None) -> SOG:
    """SOG weights (Sec. 2.2 and 3.1).  Defaults: Table 1 row, sigma scaled by rc/9."""
    b0, s9, om, *_ = TABLE1[row]
    b = b0 if b is None else b
    sigma = s9 * rc / TABLE1_RC if sigma is None else sigma
    omega = om if omega is None else omega
    w = np.zeros(M); wt = np.zeros(M); s = np.zeros(M)
    lib().orc_sog_params(b, sigma, omega, M, _pd(w), _pd(wt), _pd(s))
    return SOG(b, sigma, omega, M, rc, w, wt, s)


def omega_c0(b, sigma, rc, M):
    return lib().orc_omega_c0(b, sigma, rc, M)


def F(p: SOG, r):
    return lib().orc_F(p.M, _pd(p.w), _pd(p.s), float(r))


def Ft(p: SOG, r):
    return lib().orc_Ft(p.M, _pd(p.wt), _pd(p.s), float(r))


def bsa(beta, b, sigma, r, lmin, lmax):
    return lib().orc_bsa(beta, b, sigma, r, lmin, lmax)


def bsa_bound(beta, b):
    return lib().orc_bsa_bound(beta, b)


def H(L, wt, s, form):
    L = _f64(L); hr = C.c_double(); hnr = C.c_double()
    f = lib().orc_H_direct if form == "direct" else lib().orc_H_poisson
    f(_pd(L), wt, s, C.byref(hr), C.byref(hnr))
    return hr.value, hnr.value


def norm_consts(L, p: SOG, form: int = 0):
    """(S^r, S^nr) of eqs. Sr, Snr.  form 0 = per-Gaussian choice, 1 = direct, 2 = Poisson."""
    L = _f64(L); sr = C.c_double(); snr = C.c_double()
    lib().orc_norm_consts(_pd(L), p.M, _pd(p.wt), _pd(p.s), form, C.byref(sr), C.byref(snr))
    return sr.value, snr.value


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    P = C.POINTER(C.c_uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(P), k.ctypes.data_as(P), o.ctypes.data_as(P))
    return o


def draw_proposal(seed, sys, step, t, sxy=0, sz=1):
    z = np.zeros(3); u = np.zeros(2)
    lib().orc_draw_proposal(seed, sys, step, t, sxy, sz, _pd(z), _pd(u))
    return z, u


def target_r(m, L, p: SOG):
    m = np.ascontiguousarray(m, dtype=np.int32)
    return lib().orc_target_r(_pi32(m), _pd(_f64(L)), p.M, _pd(p.wt), _pd(p.s))


def ratio_nr(m, L, p: SOG):
    m = np.ascontiguousarray(m, dtype=np.int32)
    return lib().orc_ratio_nr(_pi32(m), _pd(_f64(L)), p.M, _pd(p.wt), _pd(p.s))


def proposal_pmf(m, L, s0):
    m = np.ascontiguousarray(m, dtype=np.int32)
    return lib().orc_proposal_pmf(_pi32(m), _pd(_f64(L)), s0)


RECAL_PRINTED = 0
RECAL_EXCHANGE = 1
RECAL_SHARED = 2        # no recalibration: the r-chain's modes, weighted by P^nr/P^r
RECAL_INDEPENDENT = 3   # a second MH chain with target P^nr (2P structure factors)


def sample_modes(L, p: SOG, P, seed, system_id, step, variant=RECAL_EXCHANGE):
    """r-chain and nr-chain modes (P x 3 int32 each) and accepted-move counts.
    variant 0: recalibration chain as printed; 1: exchange form (the default);
    2: shared proposal (m_nr = m_r); 3: an independent chain for P^nr."""
    m_r = np.zeros((P, 3), dtype=np.int32)
    m_nr = np.zeros((P, 3), dtype=np.int32)
    acc = np.zeros(2, dtype=np.int64)
    rc = lib().orc_sample_modes(_pd(_f64(L)), p.M, _pd(p.wt), _pd(p.s), P, seed, system_id, step, variant,
                                _pi32(m_r), _pi32(m_nr), _pi64(acc))
    if rc != 0:
        raise RuntimeError("oracle sampler: no start draw accepted")
    return m_r, m_nr, acc


def start_bound(L, p: SOG, power):
    """Upper bound of g_p / q' (power 2: radial target, 4: non-radial) used by
    the rejection draw of a chain's start state."""
    return lib().orc_start_bound(_pd(_f64(L)), p.M, _pd(p.wt), _pd(p.s), power)


def start_states(L, p: SOG, seed, system_id, step):
    """The exact start draws of both chains of one step (radial, non-radial)."""
    a = np.zeros(3, dtype=np.int32); b = np.zeros(3, dtype=np.int32)
    rc = lib().orc_start_states(_pd(_f64(L)), p.M, _pd(p.wt), _pd(p.s), seed, system_id, step, _pi32(a), _pi32(b))
    if rc != 0:
        raise RuntimeError("oracle sampler: no start draw accepted")
    return a, b


def recalibrate(props, u, L, p: SOG):
    """The Sec. 3.2 recalibration chain on given proposals and uniforms."""
    props = np.ascontiguousarray(props, dtype=np.int32)
    u = _f64(u)
    out = np.zeros_like(props)
    acc = np.zeros(1, dtype=np.int64)
    lib().orc_recalibrate(props.shape[0], _pi32(props), _pd(u), _pd(_f64(L)), p.M, _pd(p.wt), _pd(p.s),
                          _pi32(out), _pi64(acc))
    return out, int(acc[0])


def cell_ids(pos, L, ncell):
    pos = _f64(pos)
    n = pos.shape[0]
    x, y, z = (_f64(pos[:, k]) for k in range(3))
    nc = np.ascontiguousarray(ncell, dtype=np.int32)
    out = np.zeros(n, dtype=np.int32)
    lib().orc_cell_ids(n, _pd(x), _pd(y), _pd(z), _pd(_f64(L)), _pi32(nc), _pi32(out))
    return out


def _xyz(pos):
    pos = _f64(pos)
    return tuple(_f64(pos[:, k]) for k in range(3))


def short_range(q, pos, L, p: SOG, method="cells", sample=None):
    """Short-range force (n x 3, or len(sample) x 3), virial sum (6) and U^N."""
    q = _f64(q); x, y, z = _xyz(pos); n = q.shape[0]
    vir = np.zeros(6); U = C.c_double()
    if method == "brute":
        f = [np.zeros(n) for _ in range(3)]
        lib().orc_short_range_brute(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(_f64(L)), p.rc, p.M,
                                    _pd(p.w), _pd(p.wt), _pd(p.s), *map(_pd, f), _pd(vir), C.byref(U))
    else:
        smp = None if sample is None else np.ascontiguousarray(sample, dtype=np.int64)
        ni = n if smp is None else smp.shape[0]
        f = [np.zeros(ni) for _ in range(3)]
        lib().orc_short_range_cells(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(_f64(L)), p.rc, p.M,
                                    _pd(p.w), _pd(p.wt), _pd(p.s), 0 if smp is None else ni,
                                    _pi64(smp), *map(_pd, f), _pd(vir), C.byref(U))
    return np.stack(f, axis=1), vir, U.value


def rho(q, pos, L, modes):
    q = _f64(q); x, y, z = _xyz(pos)
    m = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, 3)
    re = np.zeros(m.shape[0]); im = np.zeros(m.shape[0])
    lib().orc_rho(q.shape[0], _pd(q), _pd(x), _pd(y), _pd(z), _pd(_f64(L)), m.shape[0], _pi32(m),
                  _pd(re), _pd(im))
    return re + 1j * im


def long_range_rb(q, pos, L, m_r, m_nr, Sr, Snr, forces=True, sample=None):
    q = _f64(q); x, y, z = _xyz(pos); n = q.shape[0]
    m_r = np.ascontiguousarray(m_r, dtype=np.int32); m_nr = np.ascontiguousarray(m_nr, dtype=np.int32)
    P = m_r.shape[0]
    smp = None if sample is None else np.ascontiguousarray(sample, dtype=np.int64)
    ni = n if smp is None else smp.shape[0]
    f = [np.zeros(ni) for _ in range(3)] if forces else [None, None, None]
    Pr = np.zeros(9); Pnr = np.zeros(9); UF = C.c_double()
    lib().orc_long_range_rb(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(_f64(L)), P, _pi32(m_r), _pi32(m_nr),
                            Sr, Snr, 0 if smp is None else ni, _pi64(smp), *map(_pd, f),
                            _pd(Pr), _pd(Pnr), C.byref(UF))
    F = np.stack(f, axis=1) if forces else None
    return F, Pr.reshape(3, 3), Pnr.reshape(3, 3), UF.value


def nonradial_shared(q, pos, L, p: SOG, m_r, Sr):
    """Non-radial pressure from the r-chain's modes without recalibration
    (the shared-proposal estimator the recalibration of Sec. 3.2 replaces):
    importance sampling of eq. P_approx_nr's sum under P^r instead of P^nr,
        -S^r/(8 V^2 P) sum_p R(k_p) |rho_p|^2 k_p k_p^T / |k_p|^4,
    R = P^nr S^nr / (P^r S^r) = |k|^2 sum_l wt_l s_l^7 e_l / sum_l wt_l s_l^5 e_l.
    Each sample's rho is evaluated on its own."""
    L = _f64(L); V = float(np.prod(L))
    m = np.ascontiguousarray(m_r, dtype=np.int32).reshape(-1, 3)
    P = m.shape[0]
    r = rho(q, pos, L, m)
    acc = np.zeros((3, 3))
    for t in range(P):
        k = 2.0 * np.pi * m[t] / L
        k2 = float(k @ k)
        acc += ratio_nr(m[t], L, p) * abs(r[t]) ** 2 * np.outer(k, k) / (k2 * k2)
    return -Sr / (8.0 * V * V * P) * acc


def uf_rb_energy(q, pos, L, m_r, Sr, p_force: SOG, p_energy: SOG):
    """Random-batch long-range energy when the energy kernel keeps more
    Gaussians than the force (Table 1 gives the energy its own, larger M):
    the importance-sampling estimate of eq. U_long under the radial proposal,
        U^{F*} = (1/P) sum_p Fhat_e(k_p) |rho_p|^2 / (2 V P^r(k_p)),
        Fhat_e(k) = pi^(3/2) sum_{l < M_e} w_l s_l^3 exp(-s_l^2 k^2 / 4)   (energy kernel),
        P^r(k)    = pi^(3/2) |k|^2 sum_{l < M} wt_l s_l^5 exp(-s_l^2 k^2 / 4) / S^r   (eq. samplingP).
    With M_e = M it is the U^{F*} of long_range_rb."""
    L = _f64(L); V = float(np.prod(L))
    m = np.ascontiguousarray(m_r, dtype=np.int32).reshape(-1, 3)
    P = m.shape[0]
    r = rho(q, pos, L, m)
    tot = 0.0
    for t in range(P):
        k = 2.0 * np.pi * m[t] / L
        k2 = float(k @ k)
        Fe = np.pi ** 1.5 * np.sum(p_energy.w * p_energy.s ** 3 * np.exp(-p_energy.s ** 2 * k2 / 4.0))
        Pr = np.pi ** 1.5 * k2 * np.sum(p_force.wt * p_force.s ** 5 * np.exp(-p_force.s ** 2 * k2 / 4.0)) / Sr
        tot += Fe * abs(r[t]) ** 2 / (2.0 * V * Pr)
    return tot / P


def sog_kspace_full(q, pos, L, p: SOG, forces=True):
    q = _f64(q); x, y, z = _xyz(pos); n = q.shape[0]
    f = [np.zeros(n) for _ in range(3)] if forces else [None, None, None]
    Pf = np.zeros(9); UF = C.c_double()
    lib().orc_sog_kspace_full(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(_f64(L)), p.M, _pd(p.w), _pd(p.wt),
                              _pd(p.s), *map(_pd, f), _pd(Pf), C.byref(UF))
    return (np.stack(f, axis=1) if forces else None), Pf.reshape(3, 3), UF.value


def self_energy(p: SOG, q):
    q = _f64(q)
    return lib().orc_self_energy(p.b, p.sigma, p.omega, p.M, q.shape[0], _pd(q))


def ewald(q, pos, L, beta=None, forces=True):
    """Exact Ewald energy, forces and pressure tensor (remainders below ~1e-17)."""
    q = _f64(q); x, y, z = _xyz(pos); n = q.shape[0]
    L = _f64(L)
    if beta is None:
        beta = 6.5 / (0.9 * float(np.min(L)))
    rcut = 6.5 / beta
    kcut = 2.0 * beta * 6.7
    f = [np.zeros(n) for _ in range(3)] if forces else [None, None, None]
    Pt = np.zeros(9); U = C.c_double()
    lib().orc_ewald(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(L), beta, rcut, kcut, *map(_pd, f),
                    _pd(Pt), C.byref(U))
    return (np.stack(f, axis=1) if forces else None), Pt.reshape(3, 3), U.value


def vir_to_tensor(v):
    xx, yy, zz, xy, xz, yz = v
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def sog_deterministic(q, pos, L, p: SOG, forces=True):
    """Deterministic SOG total: U = U^N + U^F - U_self (eq. couldecomp), F = F^N + F^F,
    P = P^N + P^F (eq. SOGDecomp with Theorem 1)."""
    L = _f64(L); V = float(np.prod(L))
    n = len(q)
    method = "brute" if n <= 4000 else "cells"
    FN, vir, UN = short_range(q, pos, L, p, method=method)
    FF, PF, UF = sog_kspace_full(q, pos, L, p, forces=forces)
    US = self_energy(p, q)
    PN = vir_to_tensor(vir) / V
    F = FN + FF if forces else None
    return dict(F=F, P=PN + PF, U=UN + UF - US, PN=PN, PF=PF, UN=UN, UF=UF, Uself=US)


def rbsog_step(q, pos, L, p: SOG, P, seed, system_id, step, modes=None, sample=None,
               variant=RECAL_EXCHANGE):
    """One evaluation of Algorithm 1 steps 2-6 (Algorithm O): returns forces,
    energy parts, pressure parts and the sampled modes.

    modes: optional (m_r, m_nr) to skip sampling (parity conditional on modes).
    sample: optional atom indices; forces are then returned for those atoms only
    and the short-range virial/energy are their partial shares.
    """
    L = _f64(L); V = float(np.prod(L))
    if modes is None:
        m_r, m_nr, acc = sample_modes(L, p, P, seed, system_id, step, variant)
    else:
        m_r, m_nr = modes
        acc = None
    Sr, Snr = norm_consts(L, p)
    FN, vir, UN = short_range(q, pos, L, p, method="cells", sample=sample)
    FF, Pr, Pnr, UF = long_range_rb(q, pos, L, m_r, m_nr, Sr, Snr, forces=True, sample=sample)
    if variant == RECAL_SHARED:
        Pnr = nonradial_shared(q, pos, L, p, m_r, Sr)
    US = self_energy(p, q)
    PN = vir_to_tensor(vir) / V
    return dict(F=FN + FF, FN=FN, FF=FF, UN=UN, UF=UF, Uself=US, U=UN + UF - US,
                PN=PN, Pr=Pr, Pnr=Pnr, P=PN + Pr + Pnr, vir=vir, Sr=Sr, Snr=Snr,
                m_r=m_r, m_nr=m_nr, acc=acc)


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# NPT integration (Algorithm 1 step 7; eq. Langevin_NPT for a diagonal h)
# ---------------------------------------------------------------------------

def npt_normals(seed, system_id, step, n):
    """Standard normals of one step's Langevin noise: (n, 3) for the atoms, 3 for the box."""
    z = np.zeros((n, 3)); zb = np.zeros(3)
    lib().orc_npt_normals(seed, system_id, step, n, _pd(z), _pd(zb))
    return z, zb


COUPLINGS = {0: [[0], [1], [2]], 1: [[0, 1], [2]], 2: [[0, 1, 2]]}   # box degrees of freedom per coupling


def npt_kinetic(mom, mass, L):
    """Kinetic pressure sum_i p_i p_i^T / (m_i V) (eq. K_U_Pins_re), 3x3."""
    return (mom[:, :, None] * mom[:, None, :] / mass[:, None, None]).sum(axis=0) / np.prod(L)


def npt_kick_box(ph, L, Pi, groups, p_ext, kT, t):
    """B_h over t: dp^h/dt = det(h) [(P_ins - p_ext - kT/det h) h^-T]_mumu (eq.
    Langevin_NPT, diagonal h); a coupled group of n_g axes sharing p^h and L_g
    takes the sum over its axes, (V/L_g) sum_mu (P_mumu - p_ext) - n_g kT/L_g."""
    V = np.prod(L)
    for k, g in enumerate(groups):
        Lg = L[g[0]]
        ph[k] += t * ((V / Lg) * sum(Pi[d, d] - p_ext for d in g) - len(g) * kT / Lg)


def npt_drift(pos, mom, mass, L, ph, groups, M, t):
    """A over t, in place: dL_g/dt = p^h_g/(n_g M) with p^h fixed (L linear in
    t), and for each atom dr/dt = p/m + (dL/dt / L) r, dp/dt = -(dL/dt / L) p.
    The exact flow: p(t) = p0 L0/L(t), and d(r/L)/dt = p0 L0/(m L^2) integrates
    to r(t) = (L(t)/L0) r0 + t p0/m."""
    a = np.ones(3)
    for k, g in enumerate(groups):
        Lnew = L[g[0]] + t * ph[k] / (len(g) * M)
        for d in g:
            a[d] = Lnew / L[d]
            L[d] = Lnew
    pos[:] = a * pos + t * mom / mass[:, None]
    mom[:] = mom / a


def npt_ou(mom, mass, ph, groups, M, kT, c1, ch, z, zb):
    """O over dt, in place: the exact Ornstein-Uhlenbeck update of dp = -gamma p
    dt + sqrt(2 gamma kT m) dW, p <- c p + sqrt((1 - c^2) kT m) xi with
    c = exp(-gamma dt); the box with its own friction and mass n_g M."""
    mom[:] = c1 * mom + np.sqrt((1.0 - c1 * c1) * kT * mass)[:, None] * z
    for k, g in enumerate(groups):
        ph[k] = ch * ph[k] + np.sqrt((1.0 - ch * ch) * kT * len(g) * M) * zb[k]


def npt_run(q, pos, mom, mass, L, pbox, prm, p: SOG, P, seed, system_id, first_step, nsteps, evaluate=None):
    """Langevin NPT steps of eq. Langevin_NPT for h = diag(L), advanced by the
    splitting B_h B A O A [evaluate] B B_h (prm: dt, kT, gamma, gamma_box,
    box_mass, p_ext, coupling); B is dp_i/dt = F_i.  P_ins = P_coul + the
    kinetic pressure.  evaluate(pos, L, step) -> (F, P_coul); default: the
    random-batch step of this oracle with modes sampled at that step.  The
    evaluation after step k and the noise of step k use step index
    first_step + k.  Returns (pos, mom, L, pbox, P_ins, P_kin)."""
    pos = _f64(pos).copy(); mom = _f64(mom).copy(); mass = _f64(mass)
    L = _f64(L).copy(); groups = COUPLINGS[prm["coupling"]]
    ph = np.array([pbox[g[0]] for g in groups], dtype=np.float64)
    dt = prm["dt"]; kT = prm["kT"]; M = prm["box_mass"]; tau = 0.5 * dt
    n = len(mass)
    if evaluate is None:
        def evaluate(x, box, step):
            o = rbsog_step(q, x, box, p, P, seed, system_id, step)
            return o["F"], o["P"]
    F, PC = evaluate(pos, L.copy(), first_step)
    Pk = npt_kinetic(mom, mass, L); Pi = PC + Pk
    c1 = np.exp(-prm["gamma"] * dt); ch = np.exp(-prm["gamma_box"] * dt)
    for s in range(1, nsteps + 1):
        step = first_step + s
        npt_kick_box(ph, L, Pi, groups, prm["p_ext"], kT, tau)
        mom += tau * F
        npt_drift(pos, mom, mass, L, ph, groups, M, tau)
        z, zb = npt_normals(seed, system_id, step, n)
        npt_ou(mom, mass, ph, groups, M, kT, c1, ch, z, zb)
        npt_drift(pos, mom, mass, L, ph, groups, M, tau)
        F, PC = evaluate(pos, L.copy(), step)
        mom += tau * F
        Pk = npt_kinetic(mom, mass, L); Pi = PC + Pk
        npt_kick_box(ph, L, Pi, groups, prm["p_ext"], kT, tau)
    pbox_out = np.array([ph[next(k for k, g in enumerate(groups) if d in g)] for d in range(3)])
    return pos, mom, L, pbox_out, Pi, Pk


# ---------------------------------------------------------------------------
# General (triclinic) cells: h = [h_1, h_2, h_3] (columns are the cell
# vectors), r = h s (Sec. 2.1), k = 2 pi h^-T m.  h is a 3 x 3 array.
# ---------------------------------------------------------------------------

def _h(h):
    h = np.ascontiguousarray(h, dtype=np.float64).reshape(3, 3)
    return h


def tri_H(h, wt, s, form):
    """(H^r_l, H^nr_l) of one Gaussian: form 1 direct sums (eqs. Sr, Snr), 2 Poisson forms (Prop. 1)."""
    hr = C.c_double(); hnr = C.c_double()
    f = lib().orc_tri_H_direct if form == 1 else lib().orc_tri_H_poisson
    f(_pd(_h(h)), float(wt), float(s), C.byref(hr), C.byref(hnr))
    return hr.value, hnr.value


def tri_norm_consts(h, p: SOG, form: int = 0):
    sr = C.c_double(); snr = C.c_double()
    lib().orc_tri_norm_consts(_pd(_h(h)), p.M, _pd(p.wt), _pd(p.s), form, C.byref(sr), C.byref(snr))
    return sr.value, snr.value


def tri_target_r(m, h, p: SOG):
    return lib().orc_tri_target_r(_pi32(np.ascontiguousarray(m, dtype=np.int32)), _pd(_h(h)), p.M, _pd(p.wt), _pd(p.s))


def tri_ratio_nr(m, h, p: SOG):
    return lib().orc_tri_ratio_nr(_pi32(np.ascontiguousarray(m, dtype=np.int32)), _pd(_h(h)), p.M, _pd(p.wt), _pd(p.s))


def tri_proposal_pmf(m, h, s0):
    """q(m) of eq. proposal for a general cell (Gauss-Legendre over the unit cube)."""
    return lib().orc_tri_proposal_pmf(_pi32(np.ascontiguousarray(m, dtype=np.int32)), _pd(_h(h)), float(s0))


def tri_round(z, h, s0):
    """round(h^T u) for u = z / (sqrt2 pi s0)."""
    m = np.zeros(3, dtype=np.int32)
    lib().orc_tri_round(_pd(_f64(z)), _pd(_h(h)), float(s0), _pi32(m))
    return m


def tri_start_bound(h, p: SOG, power):
    return lib().orc_tri_start_bound(_pd(_h(h)), p.M, _pd(p.wt), _pd(p.s), power)


def tri_start_states(h, p: SOG, seed, system_id, step):
    a = np.zeros(3, dtype=np.int32); b = np.zeros(3, dtype=np.int32)
    rc = lib().orc_tri_start_states(_pd(_h(h)), p.M, _pd(p.wt), _pd(p.s), seed, system_id, step, _pi32(a), _pi32(b))
    if rc != 0:
        raise RuntimeError("oracle sampler: no start draw accepted")
    return a, b


def tri_sample_modes(h, p: SOG, P, seed, system_id, step, variant=RECAL_EXCHANGE):
    m_r = np.zeros((P, 3), dtype=np.int32)
    m_nr = np.zeros((P, 3), dtype=np.int32)
    acc = np.zeros(2, dtype=np.int64)
    rc = lib().orc_tri_sample_modes(_pd(_h(h)), p.M, _pd(p.wt), _pd(p.s), P, seed, system_id, step, variant,
                                    _pi32(m_r), _pi32(m_nr), _pi64(acc))
    if rc != 0:
        raise RuntimeError("oracle sampler: no start draw accepted")
    return m_r, m_nr, acc


def tri_chains(h, p: SOG, P, seed, system_id, step, variant, start_r, start_nr):
    """The chains of one step on a general cell from given start states."""
    m_r = np.zeros((P, 3), dtype=np.int32)
    m_nr = np.zeros((P, 3), dtype=np.int32)
    acc = np.zeros(2, dtype=np.int64)
    lib().orc_tri_chains(_pd(_h(h)), p.M, _pd(p.wt), _pd(p.s), P, seed, system_id, step, variant,
                         _pi32(np.ascontiguousarray(start_r, dtype=np.int32)),
                         _pi32(np.ascontiguousarray(start_nr, dtype=np.int32)), _pi32(m_r), _pi32(m_nr), _pi64(acc))
    return m_r, m_nr, acc


def tri_rho(q, pos, h, modes):
    q = _f64(q); x, y, z = _xyz(pos)
    m = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, 3)
    re = np.zeros(m.shape[0]); im = np.zeros(m.shape[0])
    lib().orc_tri_rho(q.shape[0], _pd(q), _pd(x), _pd(y), _pd(z), _pd(_h(h)), m.shape[0], _pi32(m), _pd(re), _pd(im))
    return re + 1j * im


def tri_long_range_rb(q, pos, h, m_r, m_nr, Sr, Snr, forces=True):
    q = _f64(q); x, y, z = _xyz(pos); n = q.shape[0]
    m_r = np.ascontiguousarray(m_r, dtype=np.int32); m_nr = np.ascontiguousarray(m_nr, dtype=np.int32)
    f = [np.zeros(n) for _ in range(3)] if forces else [None, None, None]
    Pr = np.zeros(9); Pnr = np.zeros(9); UF = C.c_double()
    lib().orc_tri_long_range_rb(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(_h(h)), m_r.shape[0], _pi32(m_r), _pi32(m_nr),
                                Sr, Snr, *map(_pd, f), _pd(Pr), _pd(Pnr), C.byref(UF))
    return (np.stack(f, axis=1) if forces else None), Pr.reshape(3, 3), Pnr.reshape(3, 3), UF.value


def tri_short_range(q, pos, h, p: SOG):
    """Short-range force (n x 3), virial sum (6) and U^N over every image inside rc."""
    q = _f64(q); x, y, z = _xyz(pos); n = q.shape[0]
    vir = np.zeros(6); U = C.c_double()
    f = [np.zeros(n) for _ in range(3)]
    lib().orc_tri_short_range(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(_h(h)), p.rc, p.M, _pd(p.w), _pd(p.wt), _pd(p.s),
                              *map(_pd, f), _pd(vir), C.byref(U))
    return np.stack(f, axis=1), vir, U.value


def tri_sog_kspace_full(q, pos, h, p: SOG, forces=True):
    q = _f64(q); x, y, z = _xyz(pos); n = q.shape[0]
    f = [np.zeros(n) for _ in range(3)] if forces else [None, None, None]
    Pf = np.zeros(9); UF = C.c_double()
    lib().orc_tri_sog_kspace_full(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(_h(h)), p.M, _pd(p.w), _pd(p.wt), _pd(p.s),
                                  *map(_pd, f), _pd(Pf), C.byref(UF))
    return (np.stack(f, axis=1) if forces else None), Pf.reshape(3, 3), UF.value


def tri_ewald(q, pos, h, beta, rcut, kcut, forces=True):
    q = _f64(q); x, y, z = _xyz(pos); n = q.shape[0]
    f = [np.zeros(n) for _ in range(3)] if forces else [None, None, None]
    Pt = np.zeros(9); U = C.c_double()
    lib().orc_tri_ewald(n, _pd(q), _pd(x), _pd(y), _pd(z), _pd(_h(h)), beta, rcut, kcut, *map(_pd, f), _pd(Pt),
                        C.byref(U))
    return (np.stack(f, axis=1) if forces else None), Pt.reshape(3, 3), U.value


def tri_rbsog_step(q, pos, h, p: SOG, P, seed, system_id, step, variant=RECAL_EXCHANGE, modes=None):
    """One evaluation of Algorithm 1 steps 2-6 on a general cell (as rbsog_step)."""
    h = _h(h); V = abs(float(np.linalg.det(h)))
    if modes is None:
        m_r, m_nr, acc = tri_sample_modes(h, p, P, seed, system_id, step, variant)
    else:
        (m_r, m_nr), acc = modes, None
    Sr, Snr = tri_norm_consts(h, p)
    FN, vir, UN = tri_short_range(q, pos, h, p)
    FF, Pr, Pnr, UF = tri_long_range_rb(q, pos, h, m_r, m_nr, Sr, Snr, forces=True)
    US = self_energy(p, q)
    PN = vir_to_tensor(vir) / V
    return dict(F=FN + FF, FN=FN, FF=FF, UN=UN, UF=UF, Uself=US, U=UN + UF - US, PN=PN, Pr=Pr, Pnr=Pnr,
                P=PN + Pr + Pnr, vir=vir, Sr=Sr, Snr=Snr, m_r=m_r, m_nr=m_nr, acc=acc)
