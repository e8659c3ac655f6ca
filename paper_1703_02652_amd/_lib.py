"""ctypes binding of liblbpc.so (the C ABI of include/lbpc.h).

Argument marshalling only: every computation runs in the HIP library.  The
library must have been built (paper_1703_02652_amd/build.py); a missing
library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbpc.so")

LBPC_OK, LBPC_EINVAL, LBPC_EHIP, LBPC_ENOSPACE, LBPC_EUNSTABLE = 0, -1, -2, -3, -4
FIELD_BITS = {"h": 1, "T": 2, "fl": 4, "rho": 8, "u": 16}

# every entry point declared in include/lbpc.h
EXPORTS = (
    "lbpc_workspace_bytes", "lbpc_create", "lbpc_set_wall_T", "lbpc_step", "lbpc_fields",
    "lbpc_budgets", "lbpc_budgets_noalloc", "lbpc_status", "lbpc_get_state", "lbpc_set_state", "lbpc_state_bytes",
    "lbpc_save", "lbpc_load", "lbpc_set_launch", "lbpc_get_launch", "lbpc_autotune",
    "lbpc_time_step_kernel", "lbpc_adjoint_workspace_bytes", "lbpc_adjoint_forward",
    "lbpc_adjoint_backward", "lbpc_adjoint", "lbpc_destroy", "lbpc_last_error", "lbpc_version",
)


class LbpcConfig(ctypes.Structure):
    """Mirror of lbpc_config."""
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
        ("sigma_override", ctypes.c_double * 7), ("T_shift", ctypes.c_double),
    ]


class LbpcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbpc error {code}: {msg}")
        self.code = code


def make_configs(cfgs):
    arr = (LbpcConfig * len(cfgs))()
    for i, cfg in enumerate(cfgs):
        for name, typ in LbpcConfig._fields_:
            v = cfg[name]
            if hasattr(typ, "_length_"):
                a = getattr(arr[i], name)
                for j, x in enumerate(v):
                    a[j] = x
            else:
                setattr(arr[i], name, v)
    return arr


_lib = None


def lib():
    """Load liblbpc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1703_02652_amd/build.py "
                           "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                             ctypes.c_size_t)
    dp = ctypes.POINTER(ctypes.c_double)
    L.lbpc_workspace_bytes.argtypes = [vp, i32]
    L.lbpc_workspace_bytes.restype = sz
    L.lbpc_create.argtypes = [vp, i32, vp, sz, vp, vp, ctypes.POINTER(vp)]
    L.lbpc_set_wall_T.argtypes = [vp, i32, i32, vp]
    L.lbpc_step.argtypes = [vp, i64]
    L.lbpc_fields.argtypes = [vp, i32, u32, vp]
    L.lbpc_budgets.argtypes = [vp, dp]
    L.lbpc_budgets_noalloc.argtypes = [vp, dp]
    L.lbpc_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.lbpc_get_state.argtypes = [vp, i32, vp, vp]
    L.lbpc_set_state.argtypes = [vp, i32, vp, vp]
    L.lbpc_state_bytes.argtypes = [vp]
    L.lbpc_state_bytes.restype = sz
    L.lbpc_save.argtypes = [vp, vp, sz]
    L.lbpc_load.argtypes = [vp, vp, sz]
    L.lbpc_set_launch.argtypes = [vp, i32, i32, i32, i32]
    L.lbpc_get_launch.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.lbpc_autotune.argtypes = [vp, i32, dp]
    L.lbpc_time_step_kernel.argtypes = [vp, i32, dp]
    L.lbpc_adjoint_workspace_bytes.argtypes = [vp, i64, i32]
    L.lbpc_adjoint_workspace_bytes.restype = sz
    L.lbpc_adjoint_forward.argtypes = [vp, i64, i32, i32, vp, sz, dp]
    L.lbpc_adjoint_backward.argtypes = [vp, ctypes.c_double, vp, vp]
    L.lbpc_adjoint.argtypes = [vp, i64, i32, i32, vp, sz, vp, vp, dp]
    L.lbpc_destroy.argtypes = [vp]
    L.lbpc_destroy.restype = None
    L.lbpc_last_error.argtypes = [vp]
    L.lbpc_last_error.restype = ctypes.c_char_p
    L.lbpc_version.restype = ctypes.c_char_p
    for name in ("lbpc_create", "lbpc_set_wall_T", "lbpc_step", "lbpc_fields", "lbpc_budgets",
                 "lbpc_budgets_noalloc",
                 "lbpc_status", "lbpc_get_state", "lbpc_set_state", "lbpc_save", "lbpc_load",
                 "lbpc_set_launch", "lbpc_get_launch", "lbpc_autotune", "lbpc_time_step_kernel",
                 "lbpc_adjoint_forward", "lbpc_adjoint_backward", "lbpc_adjoint"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L
