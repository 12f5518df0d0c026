"""ctypes binding of libmgshell.so (include/mg.h). Argument marshalling only.

Loading fails loudly (ImportError) when the library is missing: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgshell.so")

MG_MAX_LEVELS = 32
MG_MAX_NLEV = 128
MG_HIST = 128
MG_NK = 8
KERNEL_CLASSES = ["residual64", "smooth", "restrict", "prolong", "coarse", "adjoint", "other",
                  "smooth0"]

MG_OK, MG_ERR_NOT_CONVERGED = 0, 1
MG_ERR_ARG, MG_ERR_HIP, MG_ERR_OOM, MG_ERR_BREAKDOWN = -1, -2, -3, -4
MG_PREC_MIXED, MG_PREC_FP64, MG_PREC_FP32 = 0, 1, 2


class mg_grid(C.Structure):
    _fields_ = [("nlon", C.c_int32), ("nlat", C.c_int32), ("nlev", C.c_int32),
                ("radius", C.c_double), ("thickness", C.c_double),
                ("stretch", C.c_double), ("K", C.c_double)]


class mg_coeffs(C.Structure):
    _fields_ = [("alpha", C.c_void_p)]


class mg_options(C.Structure):
    _fields_ = [("levels", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("coarse_sweeps", C.c_int32), ("max_iters", C.c_int32),
                ("omega", C.c_double), ("semi_threshold", C.c_double),
                ("precision", C.c_int32), ("stream", C.c_void_p), ("profile", C.c_int32),
                ("smooth_lo", C.c_double), ("smooth_hi", C.c_double),
                ("staged_columns", C.c_int32), ("stall_factor", C.c_double),
                ("stall_iters", C.c_int32), ("graphs", C.c_int32),
                ("zero_guess", C.c_int32), ("poison", C.c_int32)]


class mg_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("relres", C.c_double),
                ("res_hist", C.c_double * MG_HIST), ("ms_total", C.c_double),
                ("levels_used", C.c_int32), ("alg_bytes", C.c_double),
                ("kern_ms", C.c_double * MG_NK), ("kern_launches", C.c_int64 * MG_NK),
                ("kern_bytes", C.c_double * MG_NK),
                ("kern_fine_ms", C.c_double * MG_NK),
                ("kern_fine_launches", C.c_int64 * MG_NK),
                ("kern_fine_bytes", C.c_double * MG_NK),
                ("ms_vcycle", C.c_double), ("ms_residual", C.c_double),
                ("fell_back_fp64", C.c_int32)]


_P = C.c_void_p
_I = C.c_int32
_D = C.c_double
_H = C.c_void_p   # mg_handle*

_SIGS = {
    "mg_options_default": (None, [C.POINTER(mg_options)]),
    "mg_setup": (_I, [C.POINTER(mg_grid), C.POINTER(mg_coeffs), C.POINTER(mg_options),
                      C.POINTER(C.c_void_p)]),
    "mg_update_coeffs": (_I, [_H, C.POINTER(mg_coeffs)]),
    "mg_set_options": (_I, [_H, C.POINTER(mg_options)]),
    "mg_solve": (_I, [_H, _P, _P, _D, C.POINTER(mg_stats)]),
    "mg_solve_adjoint": (_I, [_H, _P, _P, _D, C.POINTER(mg_stats)]),
    "mg_solve_noalloc": (_I, [_H, _P, _P, _D, C.POINTER(mg_stats)]),
    "mg_grad_alpha": (_I, [_H, _P, _P, _P]),
    "mg_apply": (_I, [_H, _P, _P]),
    "mg_cell_volumes": (_I, [_H, _P]),
    "mg_vcycle": (_I, [_H, _P, _P, _I]),
    "mg_level_shape": (_I, [_H, _I, C.POINTER(C.c_int32)]),
    "mg_level_sweep": (_I, [_H, _I, _P, _P, _P]),
    "mg_level_residual_restrict": (_I, [_H, _I, _P, _P, _P]),
    "mg_level_prolong_add": (_I, [_H, _I, _P, _P]),
    "mg_plan": (_I, [C.POINTER(mg_grid), C.POINTER(mg_options), C.POINTER(C.c_int32),
                     C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                     C.POINTER(C.c_int32), C.c_int32]),
    "mg_plan_tables": (_I, [C.POINTER(mg_grid), C.POINTER(mg_options), C.c_int32,
                            C.POINTER(C.c_double), C.POINTER(C.c_double),
                            C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mg_destroy": (None, [_H]),
    "mg_status_string": (C.c_char_p, [_I]),
    "mg_last_error": (C.c_char_p, [_H]),
}

EXPORTED = tuple(_SIGS)


def load(path: str | None = None) -> C.CDLL:
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2307_04528_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib: C.CDLL | None = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


class MGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status: int, handle=None, what: str = "") -> int:
    if status < 0:
        detail = ""
        if handle is not None:
            detail = (lib().mg_last_error(handle) or b"").decode()
        name = (lib().mg_status_string(status) or b"").decode()
        raise MGError(status, f"{what}: {name}" + (f": {detail}" if detail else ""))
    return status
