"""ctypes declarations of the C ABI in include/dsbt.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsbt.so")

DSBT_OK = 0
DSBT_ERR_OOM, DSBT_ERR_NONFINITE = -3, -6
DSBT_C64, DSBT_C128, DSBT_C64_FP64 = 0, 1, 2
DSBT_K_PLAIN, DSBT_K_CORRECTED = 0, 1
DSBT_SIGN_C, DSBT_SIGN_PRINTED_F = 0, 1
DSBT_MODE_BATCHED, DSBT_MODE_PLAIN = 0, 1
DSBT_PLAN_ON_DEVICE, DSBT_PLAN_ON_HOST = 0, 1
DSBT_STEP_ADJOINT, DSBT_STEP_GRAPH, DSBT_STEP_RESIDENT = 1, 2, 4
DSBT_TIME_IMAGINARY = 1
DSBT_ALG_TILED, DSBT_ALG_MONOMIAL = 0, 1

STATUS_NAMES = {
    0: "DSBT_OK", -1: "DSBT_ERR_INVALID_ARG", -2: "DSBT_ERR_UNSUPPORTED", -3: "DSBT_ERR_OOM",
    -4: "DSBT_ERR_HIP", -5: "DSBT_ERR_PLAN_MISMATCH", -6: "DSBT_ERR_NONFINITE", -7: "DSBT_ERR_NO_DEVICE",
}

# every symbol include/dsbt.h declares
EXPORTED = [
    "dsbt_plan_opts_default", "dsbt_plan_create", "dsbt_plan_create_uniform", "dsbt_plan_destroy",
    "dsbt_plan_info", "dsbt_forward", "dsbt_inverse", "dsbt_set_potential", "dsbt_set_potential_ex",
    "dsbt_kinetic_step", "dsbt_step_grad_s", "dsbt_step_grad_s_noalloc", "dsbt_adjoint_segment", "dsbt_energy", "dsbt_orthonormalize", "dsbt_profile_enable",
    "dsbt_profile_read", "dsbt_host_ftb_tables", "dsbt_host_monomial_tables", "dsbt_device_ftb_tables",
    "dsbt_kinetic_momenta", "dsbt_autotune", "dsbt_sht_grid", "dsbt_sht_host_tables", "dsbt_sht_create",
    "dsbt_sht_destroy", "dsbt_sht_forward", "dsbt_sht_inverse", "dsbt_sht_potential_phase",
    "dsbt_sht_momentum_order", "dsbt_sht_kinetic", "dsbt_sht_momentum_pz", "dsbt_step3d", "dsbt_step3d_velocity",
    "dsbt_status_string", "dsbt_last_error",
]


class Channel(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("ell", ctypes.c_int32), ("rmax", ctypes.c_double),
                ("offset", ctypes.c_int64)]


# dsbt_plan_opts.dev_alloc / dev_free
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class PlanOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("kinetic", ctypes.c_int32), ("sign", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("plan_where", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("chans_per_block", ctypes.c_int32), ("algorithm", ctypes.c_int32),
                ("check_finite", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
                ("reserved", ctypes.c_int32 * 4)]


class DsbtError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {detail}")


_lib = None


def load() -> ctypes.CDLL:
    """Load libdsbt.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1509_07115_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    proto = {
        "dsbt_plan_opts_default": (None, [ctypes.POINTER(PlanOpts)]),
        "dsbt_plan_create": (i32, [ctypes.POINTER(P), ctypes.POINTER(Channel), i32, ctypes.POINTER(PlanOpts), P]),
        "dsbt_plan_create_uniform": (i32, [ctypes.POINTER(P), i32, dbl, ctypes.POINTER(i32), i32, i32,
                                           ctypes.POINTER(PlanOpts), P]),
        "dsbt_plan_destroy": (i32, [P]),
        "dsbt_plan_info": (i32, [P, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                 ctypes.POINTER(i64)]),
        "dsbt_forward": (i32, [P, P, P, P]),
        "dsbt_inverse": (i32, [P, P, P, P]),
        "dsbt_set_potential": (i32, [P, ctypes.POINTER(dbl), dbl]),
        "dsbt_set_potential_ex": (i32, [P, ctypes.POINTER(dbl), dbl, i32]),
        "dsbt_energy": (i32, [P, P, P, P, P]),
        "dsbt_orthonormalize": (i32, [P, P, ctypes.POINTER(i32), i32, P]),
        "dsbt_kinetic_step": (i32, [P, P, i32, P, i32, P]),
        "dsbt_step_grad_s": (i32, [P, P, P, P, P, P, P]),
        "dsbt_step_grad_s_noalloc": (i32, [P, P, P, P, P, P, P]),
        "dsbt_adjoint_segment": (i32, [P, P, i32, P, P, P, i32, P]),
        "dsbt_profile_enable": (i32, [P, i32]),
        "dsbt_profile_read": (i32, [P, ctypes.POINTER(dbl), ctypes.POINTER(i64), i32]),
        "dsbt_host_ftb_tables": (i32, [i32, i32, i32, ctypes.POINTER(dbl), i64, ctypes.POINTER(i64)]),
        "dsbt_host_monomial_tables": (i32, [i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                            ctypes.POINTER(i64)]),
        "dsbt_device_ftb_tables": (i32, [i32, i32, i32, ctypes.POINTER(dbl), i64, ctypes.POINTER(i64), P]),
        "dsbt_kinetic_momenta": (i32, [i32, i32, dbl, i32, ctypes.POINTER(dbl)]),
        "dsbt_autotune": (i32, [ctypes.POINTER(Channel), i32, ctypes.POINTER(PlanOpts), i32, ctypes.c_char_p,
                                ctypes.POINTER(PlanOpts), ctypes.POINTER(dbl), P]),
        "dsbt_sht_grid": (i32, [i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
        "dsbt_sht_host_tables": (i32, [i32, i32, ctypes.POINTER(dbl)]),
        "dsbt_sht_create": (i32, [ctypes.POINTER(P), i32, i32, i32, i32]),
        "dsbt_sht_destroy": (i32, [P]),
        "dsbt_sht_forward": (i32, [P, P, P, P]),
        "dsbt_sht_inverse": (i32, [P, P, P, P]),
        "dsbt_sht_potential_phase": (i32, [P, P, P, P, dbl, dbl, P]),
        "dsbt_sht_momentum_order": (i32, [P, P, P, i32, P]),
        "dsbt_sht_kinetic": (i32, [P, dbl, i32, P, P]),
        "dsbt_sht_momentum_pz": (i32, [P, dbl, P, P]),
        "dsbt_step3d": (i32, [P, P, P, P, P, P, dbl, dbl, P]),
        "dsbt_step3d_velocity": (i32, [P, P, P, P, P, P, P, P, dbl, dbl, P]),
        "dsbt_status_string": (ctypes.c_char_p, [i32]),
        "dsbt_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in proto.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != DSBT_OK:
        lib = load()
        raise DsbtError(status, where, lib.dsbt_last_error().decode(errors="replace"))
