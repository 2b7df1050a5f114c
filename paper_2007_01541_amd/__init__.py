"""MI355X-native sparse Cholesky for compressed wavelet Galerkin matrices.

Host ordering/symbolic analysis and gfx950 numeric kernels live in the
compiled library _lib/libwcs.so (see build.py); this package only binds it.
"""
from .solver import (APPLY_L, APPLY_LT, FP32, FP64, LU64, SOLVE_FULL, SOLVE_L, SOLVE_LT, Factor, Symbolic,  # noqa: F401
                     cholesky_solve, field_sample)
