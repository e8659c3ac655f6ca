"""CPU FP64 oracle of the coupled enthalpy / flow lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  The compute
lives in lbpc_oracle.cpp (plain C++, FP64, OpenMP over z planes); this module
marshals numpy arrays.  Public arrays use the layout [q][z][y][x] (x fastest);
the C side stores cell-major [cell][q] and the conversion happens here.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build as _build

_c_double_p = ctypes.POINTER(ctypes.c_double)


class OrCfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("flow", ctypes.c_int32), ("enth_model", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("face_bc", ctypes.c_int32 * 6),
        ("face_T", ctypes.c_double * 6),
        ("omega_T", ctypes.c_double), ("cp_s", ctypes.c_double), ("cp_l", ctypes.c_double),
        ("cp_ref", ctypes.c_double), ("lambda_s", ctypes.c_double),
        ("lambda_l", ctypes.c_double), ("latent", ctypes.c_double), ("T_m", ctypes.c_double),
        ("rho0", ctypes.c_double), ("nu", ctypes.c_double), ("s_e", ctypes.c_double),
        ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double), ("s_pi", ctypes.c_double),
        ("s_t", ctypes.c_double), ("g_beta", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("sigma_override", ctypes.c_double * 7),
    ]


def _cfg(cfg: dict) -> OrCfg:
    c = OrCfg()
    for name, typ in OrCfg._fields_:
        v = cfg[name]
        if hasattr(typ, "_length_"):
            arr = getattr(c, name)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(c, name, v)
    for d in range(3):
        lo, hi = cfg["face_bc"][2 * d], cfg["face_bc"][2 * d + 1]
        if (lo == 0) != (hi == 0):
            raise ValueError("a periodic face needs a periodic partner")
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            _build()
        L = ctypes.CDLL(LIB_PATH)
        P = _c_double_p
        L.or_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_tables.argtypes = [P] * 6
        L.or_g_eq.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, P, P]
        L.or_n_eq.argtypes = L.or_g_eq.argtypes
        L.or_m_eq.argtypes = [ctypes.c_double, P, P]
        L.or_force_moments.argtypes = [P, P, P]
        L.or_phase.argtypes = [ctypes.c_void_p, ctypes.c_double, P, P]
        L.or_collide_cell.argtypes = [ctypes.c_void_p, P, P, P, P, P]
        L.or_init.argtypes = [ctypes.c_void_p, P, P, P]
        L.or_run.argtypes = [ctypes.c_void_p, P, P, P, ctypes.c_int64, P]
        L.or_fields.argtypes = [ctypes.c_void_p, P, P, P]
        L.or_loss.argtypes = [ctypes.c_void_p, P, ctypes.c_int]
        L.or_loss.restype = ctypes.c_double
        L.or_run_tangent.argtypes = [ctypes.c_void_p, P, P, P, P, P, P, ctypes.c_int64,
                                     ctypes.c_int, P, P]
        L.or_init_tangent.argtypes = [ctypes.c_void_p, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_c_double_p)


def threads() -> int:
    return lib().or_threads()


def set_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls (for timing)."""
    lib().or_set_threads(int(n))


# --------------------------------------------------------------------------- #
# Tables and cell-level building blocks
# --------------------------------------------------------------------------- #
def tables():
    e7, e19 = np.zeros((7, 3)), np.zeros((19, 3))
    N, Ninv, M, Minv = np.zeros((7, 7)), np.zeros((7, 7)), np.zeros((19, 19)), np.zeros((19, 19))
    lib().or_tables(_p(e7), _p(e19), _p(N), _p(Ninv), _p(M), _p(Minv))
    return dict(e7=e7, e19=e19, N=N, Ninv=Ninv, M=M, Minv=Minv)


def g_eq(cfg, h, T, cp, u):
    out = np.zeros(7)
    lib().or_g_eq(ctypes.byref(_cfg(cfg)), h, T, cp, _p(np.asarray(u, float)), _p(out))
    return out


def n_eq(cfg, h, T, cp, u):
    out = np.zeros(7)
    lib().or_n_eq(ctypes.byref(_cfg(cfg)), h, T, cp, _p(np.asarray(u, float)), _p(out))
    return out


def m_eq(rho, u):
    out = np.zeros(19)
    lib().or_m_eq(rho, _p(np.asarray(u, float)), _p(out))
    return out


def force_moments(F, u):
    out = np.zeros(19)
    lib().or_force_moments(_p(np.asarray(F, float)), _p(np.asarray(u, float)), _p(out))
    return out


def phase(cfg, h):
    T, fl = ctypes.c_double(), ctypes.c_double()
    lib().or_phase(ctypes.byref(_cfg(cfg)), h, ctypes.byref(T), ctypes.byref(fl))
    return T.value, fl.value


AUX = ("h", "T", "fl", "cp", "rho", "ux", "uy", "uz", "Fx", "Fy", "Fz")


def collide_cell(cfg, f, g):
    f = np.ascontiguousarray(f, dtype=np.float64) if f is not None else np.zeros(19)
    g = np.ascontiguousarray(g, dtype=np.float64)
    fs, gs, aux = np.zeros(19), np.zeros(7), np.zeros(11)
    lib().or_collide_cell(ctypes.byref(_cfg(cfg)), _p(f), _p(g), _p(fs), _p(gs), _p(aux))
    return fs, gs, dict(zip(AUX, aux))


# --------------------------------------------------------------------------- #
# Lattice-level runs.  State = (f, g) in SoA [q][z][y][x]; f is None without flow.
# --------------------------------------------------------------------------- #
def _to_aos(a, q):
    return np.ascontiguousarray(a.reshape(q, -1).T)


def _to_soa(a, q, cfg):
    return np.ascontiguousarray(a.reshape(-1, q).T).reshape(q, cfg["nz"], cfg["ny"], cfg["nx"])


def _ncell(cfg):
    return cfg["nx"] * cfg["ny"] * cfg["nz"]


def init_state(cfg, T0=None):
    n = _ncell(cfg)
    f = np.zeros(n * 19) if cfg["flow"] else None
    g = np.zeros(n * 7)
    T0a = None if T0 is None else np.ascontiguousarray(np.asarray(T0, float).reshape(-1))
    lib().or_init(ctypes.byref(_cfg(cfg)), _p(T0a), _p(f), _p(g))
    return (_to_soa(f, 19, cfg) if f is not None else None), _to_soa(g, 7, cfg)


def _wall(cfg, tw):
    from workloads import wall_fields
    if tw is None:
        tw = wall_fields(cfg)
    tw = np.ascontiguousarray(np.asarray(tw, dtype=np.float64).reshape(-1))
    if tw.size != wall_fields(cfg).size:
        raise ValueError("wall field has the wrong length")
    return tw


def run(cfg, state, nsteps, tw=None, history=False):
    """Advance `state` by nsteps.  Returns the new state (and, with history=True,
    an (nsteps, 4) array of H, mass, sum f_l, wall flux per step)."""
    f, g = state
    fa = _to_aos(np.asarray(f, float), 19) if cfg["flow"] else None
    ga = _to_aos(np.asarray(g, float), 7)
    hist = np.zeros((nsteps, 4)) if history else None
    lib().or_run(ctypes.byref(_cfg(cfg)), _p(fa), _p(ga), _p(_wall(cfg, tw)),
                 int(nsteps), _p(hist))
    new = ((_to_soa(fa, 19, cfg) if fa is not None else None), _to_soa(ga, 7, cfg))
    return (new, hist) if history else new


FIELDS = ("h", "T", "fl", "rho", "ux", "uy", "uz")


def fields(cfg, state):
    f, g = state
    fa = _to_aos(np.asarray(f, float), 19) if cfg["flow"] else None
    ga = _to_aos(np.asarray(g, float), 7)
    out = np.zeros(_ncell(cfg) * 7)
    lib().or_fields(ctypes.byref(_cfg(cfg)), _p(fa), _p(ga), _p(out))
    o = _to_soa(out, 7, cfg)
    return {k: o[i] for i, k in enumerate(FIELDS)}


def loss(cfg, state, kind=0):
    ga = _to_aos(np.asarray(state[1], float), 7)
    return lib().or_loss(ctypes.byref(_cfg(cfg)), _p(ga), int(kind))


def run_tangent(cfg, state, nsteps, tw=None, dtw=None, dstate=None, loss_kind=0):
    """Loss after nsteps and its derivative along (dstate, dtw)."""
    f, g = state
    fa = _to_aos(np.asarray(f, float), 19) if cfg["flow"] else None
    ga = _to_aos(np.asarray(g, float), 7)
    dfa = dga = None
    if dstate is not None:
        if cfg["flow"] and dstate[0] is not None:
            dfa = _to_aos(np.asarray(dstate[0], float), 19)
        if dstate[1] is not None:
            dga = _to_aos(np.asarray(dstate[1], float), 7)
    dtwa = None if dtw is None else np.ascontiguousarray(np.asarray(dtw, float).reshape(-1))
    L, dL = ctypes.c_double(), ctypes.c_double()
    lib().or_run_tangent(ctypes.byref(_cfg(cfg)), _p(fa), _p(ga), _p(dfa), _p(dga),
                         _p(_wall(cfg, tw)), _p(dtwa), int(nsteps), int(loss_kind),
                         ctypes.byref(L), ctypes.byref(dL))
    return L.value, dL.value


def init_tangent(cfg, T0, dT0):
    n = _ncell(cfg)
    f = np.zeros(n * 19) if cfg["flow"] else None
    df = np.zeros(n * 19) if cfg["flow"] else None
    g, dg = np.zeros(n * 7), np.zeros(n * 7)
    T0a = np.ascontiguousarray(np.asarray(T0, float).reshape(-1))
    dT0a = np.ascontiguousarray(np.asarray(dT0, float).reshape(-1))
    lib().or_init_tangent(ctypes.byref(_cfg(cfg)), _p(T0a), _p(dT0a), _p(f), _p(g),
                          _p(df), _p(dg))
    st = ((_to_soa(f, 19, cfg) if f is not None else None), _to_soa(g, 7, cfg))
    dst = ((_to_soa(df, 19, cfg) if df is not None else None), _to_soa(dg, 7, cfg))
    return st, dst
