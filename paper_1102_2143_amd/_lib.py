"""ctypes declarations of the C ABI in ``include/msc.h``.

Only argument marshalling lives here: every numerical step runs in the HIP library.
torch is imported before the library is loaded so that both share one HIP runtime.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the process's HIP runtime first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MSC_LIB", os.path.join(HERE, "libmsc.so"))

MSC_OK, MSC_ENOTCONV, MSC_EINVAL, MSC_ENOMEM, MSC_EHIP, MSC_EBREAKDOWN = 0, 1, -1, -2, -3, -4
MSC_A_MHM, MSC_A_HERM, MSC_A_GENERAL = 0, 1, 2
MSC_PREC_FP64, MSC_PREC_MIXED = 0, 1
MSC_FORMAT_AUTO, MSC_FORMAT_CSR, MSC_FORMAT_SELL, MSC_FORMAT_SELL32, MSC_FORMAT_STENCIL = 0, 1, 2, 3, 4

STATUS_NAMES = {0: "ok", 1: "notconv", -1: "einval", -2: "enomem", -3: "ehip", -4: "breakdown"}

EXPORTED = (
    "msc_params_default", "msc_version", "msc_last_error", "msc_op_create_csr",
    "msc_op_create_staggered", "msc_op_update_links", "msc_op_update_values",
    "msc_op_set_shifts", "msc_op_query", "msc_op_storage", "msc_op_apply",
    "msc_op_apply_noalloc", "msc_solve", "msc_solve_adjoint", "msc_solve_bicgstab",
    "msc_solve_multi_rhs", "msc_solve_real", "msc_solve_batched",
    "msc_op_destroy",
)


class Params(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("reliable_every", ctypes.c_int32),
        ("freeze", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("poll_every", ctypes.c_int32),
        ("switch_tol", ctypes.c_double),
        ("refine_max_iter", ctypes.c_int32),
        ("lanes", ctypes.c_int32),
        ("verify", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("max_grid", ctypes.c_int32),
        ("format", ctypes.c_int32),
        ("mixed_margin", ctypes.c_double),
        ("update_steps", ctypes.c_int32),
        ("sweep", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32),
        ("n_reliable", ctypes.c_int32),
        ("n_refined", ctypes.c_int32),
        ("true_rel_res", ctypes.POINTER(ctypes.c_double)),
        ("freeze_iter", ctypes.POINTER(ctypes.c_int32)),
        ("seconds", ctypes.c_double),
        ("alg_bytes", ctypes.c_double),
        ("kernel_ms", ctypes.c_double * 3),
        ("kernel_samples", ctypes.c_int32),
        ("iters_fp64", ctypes.c_int32),
        ("kernel_bytes", ctypes.c_double * 3),
        ("fp64_kernel_ms", ctypes.c_double * 3),
        ("fp64_kernel_bytes", ctypes.c_double * 3),
        ("fp64_kernel_samples", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_lib = None


def load():
    """Load ``libmsc.so``; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library not found at {LIB_PATH}; build it with "
            "`python -m paper_1102_2143_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.msc_params_default.argtypes = [ctypes.POINTER(Params)]
    lib.msc_params_default.restype = None
    lib.msc_version.restype = ctypes.c_char_p
    lib.msc_last_error.restype = ctypes.c_char_p
    lib.msc_op_create_csr.argtypes = [ctypes.POINTER(vp), i32, i64, i64, vp, vp, vp, vp]
    lib.msc_op_create_csr.restype = i32
    lib.msc_op_create_staggered.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i32), dbl, vp, vp]
    lib.msc_op_create_staggered.restype = i32
    lib.msc_op_update_links.argtypes = [vp, vp, vp]
    lib.msc_op_update_links.restype = i32
    lib.msc_op_update_values.argtypes = [vp, vp, vp]
    lib.msc_op_update_values.restype = i32
    lib.msc_op_set_shifts.argtypes = [vp, ctypes.POINTER(dbl), i32]
    lib.msc_op_set_shifts.restype = i32
    lib.msc_op_query.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                 ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.msc_op_query.restype = i32
    lib.msc_op_storage.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.msc_op_storage.restype = i32
    lib.msc_op_apply.argtypes = [vp, i32, vp, vp, dbl, vp]
    lib.msc_op_apply.restype = i32
    lib.msc_op_apply_noalloc.argtypes = [vp, i32, vp, vp, dbl, vp]
    lib.msc_op_apply_noalloc.restype = i32
    lib.msc_solve.argtypes = [vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(Info), vp]
    lib.msc_solve.restype = i32
    lib.msc_solve_bicgstab.argtypes = [vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(Info), vp]
    lib.msc_solve_bicgstab.restype = i32
    lib.msc_solve_multi_rhs.argtypes = [vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(Info), vp]
    lib.msc_solve_multi_rhs.restype = i32
    lib.msc_solve_real.argtypes = [vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(Info), vp]
    lib.msc_solve_real.restype = i32
    lib.msc_solve_adjoint.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(Params),
                                      ctypes.POINTER(Info), vp]
    lib.msc_solve_adjoint.restype = i32
    lib.msc_solve_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i32),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(Params), ctypes.POINTER(Info), vp]
    lib.msc_solve_batched.restype = i32
    lib.msc_op_destroy.argtypes = [vp]
    lib.msc_op_destroy.restype = None
    _lib = lib
    return lib


def last_error() -> str:
    return load().msc_last_error().decode()


class MscError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {last_error()}")
