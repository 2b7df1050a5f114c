"""CPU oracle for the sparse Cholesky path — test infrastructure only.

Plain FP64 C code (``oracle.c``) behind ctypes.  Only the tests, the smoke
check and the benchmark's CPU baseline use it; the GPU library never does.
"""
from .oracle import (  # noqa: F401
    OracleError,
    build,
    load,
    symbolic,
    pattern,
    factor,
    solve,
    apply,
    symv,
    residual,
    grad,
    check_nd,
    check_perm,
    Factor,
    factorize,
    theta_steps,
    lu,
    lu_solve,
    gemv,
    gemv_residual,
    LUFactor,
    lu_factorize,
    field_sample,
)
