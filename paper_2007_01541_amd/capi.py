"""ctypes declarations of the C ABI in include/wcs.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libwcs.so")

c_i32 = C.c_int32
c_i64 = C.c_int64
c_p = C.c_void_p


class AnalyzeOpts(C.Structure):
    _fields_ = [
        ("leaf_size", c_i32),
        ("dense_degree_frac", C.c_double),
        ("dense_degree_min", C.c_double),
        ("coords", c_p),
        ("coord_dim", c_i32),
        ("user_perm", c_p),
        ("relax", c_i32),
    ]


class SymbolicInfo(C.Structure):
    _fields_ = [
        ("n", c_i32),
        ("nnz_lower", c_i64),
        ("nnz_l", c_i64),
        ("flops", c_i64),
        ("flops_padded", c_i64),
        ("nsuper_fund", c_i32),
        ("nsuper", c_i32),
        ("nlevels", c_i32),
        ("max_front", c_i32),
        ("nsep_nodes", c_i32),
        ("npeeled", c_i32),
        ("front_elems", c_i64),
        ("nnz_l_padded", c_i64),
        ("nseg", c_i32),
    ]


class KernelStat(C.Structure):
    _fields_ = [("launches", c_i32), ("ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


KERNEL_CLASSES = ["fill", "scatter", "extend_add", "panel", "panel_fp64diag", "update"]


class IRReport(C.Structure):
    _fields_ = [("iterations", c_i32), ("raw_residual", C.c_double), ("final_residual", C.c_double)]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("wcs_status_string", C.c_char_p, [C.c_int]),
    ("wcs_last_error", C.c_char_p, []),
    ("wcs_analyze", C.c_int, [c_i32, c_p, c_p, C.POINTER(AnalyzeOpts), C.POINTER(c_p)]),
    ("wcs_symbolic_info", C.c_int, [c_p, C.POINTER(SymbolicInfo)]),
    ("wcs_symbolic_export", C.c_int, [c_p, c_p, c_p, c_p, c_p, c_p]),
    ("wcs_symbolic_fronts", C.c_int, [c_p, c_p, c_p]),
    ("wcs_symbolic_batch", C.c_int, [c_i32, c_p, C.POINTER(c_p)]),
    ("wcs_symbolic_segments", C.c_int, [c_p, c_p]),
    ("wcs_symbolic_free", None, [c_p]),
    ("wcs_workspace_size", C.c_int, [c_p, C.c_int, c_i32, C.POINTER(C.c_size_t)]),
    ("wcs_factor_create", C.c_int, [c_p, C.c_int, c_i32, c_p, C.c_size_t, c_p, C.POINTER(c_p)]),
    ("wcs_factor_create_static", C.c_int, [c_p, C.c_int, c_i32, c_p, C.POINTER(c_p)]),
    ("wcs_factor_numeric", C.c_int, [c_p, c_p, c_p, C.POINTER(c_i32)]),
    ("wcs_factor_numeric_lu", C.c_int, [c_p, c_p, c_p, c_p, C.POINTER(c_i32)]),
    ("wcs_factor_export_upper", C.c_int, [c_p, c_i32, c_i32, c_p, c_p, c_p, c_p]),
    ("wcs_factor_check", C.c_int, [c_p, c_p, C.POINTER(c_i32)]),
    ("wcs_factor_free", None, [c_p]),
    ("wcs_factor_residuals", C.c_int, [c_p, c_p, c_i64]),
    ("wcs_factor_use_graphs", C.c_int, [c_p, C.c_int]),
    ("wcs_factor_autotune", C.c_int, [c_p, c_p, c_p, c_p, c_p]),
    ("wcs_factor_set_tiles", C.c_int, [c_p, c_p]),
    ("wcs_factor_profile", C.c_int, [c_p, c_p, c_p, c_p]),
    ("wcs_factor_profile_levels", C.c_int, [c_p, c_p, c_p, c_p]),
    ("wcs_factor_export", C.c_int, [c_p, c_i32, c_i32, c_p, c_p, c_p, c_p]),
    ("wcs_solve", C.c_int, [c_p, C.c_int, c_i32, c_p, c_i64, c_p]),
    ("wcs_apply", C.c_int, [c_p, C.c_int, c_i32, c_p, c_i64, c_p]),
    ("wcs_solve_refined", C.c_int, [c_p, c_p, c_i32, c_p, c_p, c_i64, C.c_double, c_i32,
                                    C.POINTER(IRReport), c_p]),
    ("wcs_spmv", C.c_int, [c_p, c_p, c_i32, c_p, c_p, c_i64, c_p]),
    ("wcs_grad_pattern", C.c_int, [c_p, c_p, c_p, c_p, c_p]),
    ("wcs_field_sample", C.c_int, [c_p, c_p, c_i32, c_p, c_i64, c_p, c_i64, c_p, c_i64, c_p]),
    ("wcs_theta_matrix", C.c_int, [c_p, c_p, C.c_double, C.c_double, c_p, c_p]),
    ("wcs_theta_steps", C.c_int, [c_p, c_p, C.c_double, C.c_double, c_i32, c_p, c_i64, c_p, c_i64, C.c_double,
                                  C.POINTER(IRReport), c_p]),
]

_lib: Optional[C.CDLL] = None


class WcsError(RuntimeError):
    def __init__(self, code: int, call: str, detail: str = "", bad_col: int = -1):
        msg = f"{call} failed: {status_string(code)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)
        self.code = code
        self.bad_col = bad_col


def lib() -> C.CDLL:
    """Load the compiled library; raise if it was not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2007_01541_amd.build.build()")
    h = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(h, name)
        fn.restype = res
        fn.argtypes = args
    _lib = h
    return h


def status_string(code: int) -> str:
    try:
        return lib().wcs_status_string(code).decode()
    except ImportError:
        return str(code)


def check(code: int, call: str, bad_col: int = -1) -> None:
    if code != 0:
        detail = lib().wcs_last_error().decode(errors="replace")
        raise WcsError(code, call, detail, bad_col)
