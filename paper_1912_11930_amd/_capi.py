"""ctypes declarations of the C ABI in include/bcg.h (argument marshalling only).

The shared library must have been built (``paper_1912_11930_amd.build``);
importing this module without it raises, so no code path can run without the
HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbcg.so")

BCG_OK = 0
BCG_NOT_CONVERGED = 1
BCG_EINVAL = -1
BCG_EBREAKDOWN = -2
BCG_ENOMEM = -3
BCG_EHIP = -4

SUBALGEBRA = {"block": 0, "global": 1, "parallel": 2, "hybrid": 3}
PRECISION = {"fp64": 0, "fp32_refine": 1, "fp32_reliable": 2}
PRECOND = {"none": 0, "jacobi": 1}
STATUS_NAME = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "EBREAKDOWN", -3: "ENOMEM", -4: "EHIP"}


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("values", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("outer_iterations", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("fp64_fallback", ctypes.c_int32), ("k", ctypes.c_int32),
                ("max_rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelTime(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


KERNEL_CLASSES = ["spmm", "update_r", "update_xp", "reduce", "small", "residual", "product"]

# (name, restype, argtypes) for every function declared in include/bcg.h
SIGNATURES = [
    ("bcg_create", ctypes.c_int, [ctypes.POINTER(Csr), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_void_p)]),
    ("bcg_destroy", None, [ctypes.c_void_p]),
    ("bcg_set_stream", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("bcg_set_precision", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int]),
    ("bcg_solve", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                 ctypes.c_int]),
    ("bcg_solve_noalloc", ctypes.c_int, [ctypes.POINTER(Csr), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.POINTER(Info)]),
    ("bcg_update_values", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("bcg_set_preconditioner", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("bcg_csr_outer", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                     ctypes.c_void_p]),
    ("bcg_get_info", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    ("bcg_get_column_ratios", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
    ("bcg_set_row_schedule", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("bcg_set_sell", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    ("bcg_sell_layout", ctypes.c_int64, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    ("bcg_set_profiling", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("bcg_get_kernel_times", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelTime), ctypes.c_int]),
    ("bcg_last_error", ctypes.c_char_p, []),
    ("bcg_stencil_nnz", ctypes.c_int64, [ctypes.c_int, ctypes.c_int]),
    ("bcg_stencil_build", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("bcg_stencil_schedule", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    ("bcg_stencil_brick_schedule", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_int), ctypes.c_void_p, ctypes.c_void_p]),
    ("bcg_stencil_kappa_vjp", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
]

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1912_11930_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class BCGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAME.get(status, status)}: {msg}")
        self.status = status


def check(status: int) -> int:
    """Raise BCGError for argument / runtime errors; pass solver outcomes through."""
    if status in (BCG_EINVAL, BCG_ENOMEM, BCG_EHIP):
        raise BCGError(status, lib().bcg_last_error().decode(errors="replace"))
    return status
