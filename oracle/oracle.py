"""ctypes binding of the CPU oracle (oracle.c).  Test infrastructure only.

Every function here marshals NumPy arrays into the C oracle and back; the
arithmetic lives in oracle.c, where each routine cites the part of the paper
it follows.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lib: Optional[C.CDLL] = None


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str, bad_col: int = -1):
        super().__init__(f"oracle {what} failed with code {code}" + (f" (column {bad_col})" if bad_col >= 0 else ""))
        self.code = code
        self.bad_col = bad_col


def build() -> str:
    """Compile oracle.c with gcc (plain -O2, no fast-math) into _build/liboracle.so."""
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_P = C.c_void_p


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def load() -> C.CDLL:
    """The compiled oracle; ORACLE_LIB names another build of oracle.c (the
    sanitizer test runs the pins against an instrumented one)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIB", _LIB)
    if path == _LIB and not os.path.exists(_LIB):
        build()
    lib = C.CDLL(path)
    i32, i64 = C.c_int32, C.c_int64
    lib.orc_check_perm.argtypes = [i32, _P]
    lib.orc_symbolic.argtypes = [i32, _P, _P, _P, _P, _P, _P, _P]
    lib.orc_pattern.argtypes = [i32, _P, _P, _P, _P, _P, _P, _P]
    lib.orc_factor.argtypes = [i32, _P, _P, _P, _P, _P, _P, _P, i32, _P]
    lib.orc_solve.argtypes = [i32, _P, _P, _P, _P, i32, i32, _P, _P, i64]
    lib.orc_apply.argtypes = [i32, _P, _P, _P, _P, i32, i32, _P, _P, i64]
    lib.orc_symv.argtypes = [i32, _P, _P, _P, i32, _P, _P, i64]
    lib.orc_grad.argtypes = [i32, _P, _P, _P, _P, _P]
    lib.orc_lu.argtypes = [i32, _P, _P, _P, _P, _P, _P, _P, _P, _P, i32, _P]
    lib.orc_lu_solve.argtypes = [i32, _P, _P, _P, _P, _P, i32, i32, _P, _P, i64]
    lib.orc_gemv.argtypes = [i32, _P, _P, _P, _P, i32, _P, _P, i64]
    lib.orc_check_nd.argtypes = [i32, _P, _P, _P, i32, _P]
    lib.orc_check_nd.restype = i64
    for f in ("orc_check_perm", "orc_symbolic", "orc_pattern", "orc_factor", "orc_solve", "orc_apply", "orc_symv",
              "orc_grad", "orc_lu", "orc_lu_solve", "orc_gemv"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _csc(colptr, rowind, values=None):
    cp = np.ascontiguousarray(colptr, np.int64)
    ri = np.ascontiguousarray(rowind, np.int32)
    if values is None:
        return cp, ri
    return cp, ri, np.ascontiguousarray(values, np.float64)


def check_perm(perm: np.ndarray) -> bool:
    p = np.ascontiguousarray(perm, np.int32)
    return load().orc_check_perm(p.size, _ptr(p)) == 0


def symbolic(n: int, colptr, rowind, perm) -> Tuple[np.ndarray, np.ndarray, int, int]:
    """(parent, colcount, nnz(L), flops = sum colcount^2) of P A P^T."""
    cp, ri = _csc(colptr, rowind)
    p = np.ascontiguousarray(perm, np.int32)
    parent = np.empty(n, np.int32)
    cc = np.empty(n, np.int32)
    nnz = C.c_int64()
    fl = C.c_int64()
    rc = load().orc_symbolic(n, _ptr(cp), _ptr(ri), _ptr(p), _ptr(parent), _ptr(cc), C.byref(nnz), C.byref(fl))
    if rc:
        raise OracleError(rc, "symbolic")
    return parent, cc, int(nnz.value), int(fl.value)


def pattern(n: int, colptr, rowind, perm, parent, colcount) -> Tuple[np.ndarray, np.ndarray]:
    """Column pattern (Lp int64[n+1], Li int32[nnz(L)]) of L."""
    cp, ri = _csc(colptr, rowind)
    p = np.ascontiguousarray(perm, np.int32)
    par = np.ascontiguousarray(parent, np.int32)
    cc = np.ascontiguousarray(colcount, np.int32)
    Lp = np.empty(n + 1, np.int64)
    Li = np.empty(int(cc.astype(np.int64).sum()), np.int32)
    rc = load().orc_pattern(n, _ptr(cp), _ptr(ri), _ptr(p), _ptr(par), _ptr(cc), _ptr(Lp), _ptr(Li))
    if rc:
        raise OracleError(rc, "pattern")
    return Lp, Li


def factor(n: int, colptr, rowind, values, perm, Lp, Li, ncols: Optional[int] = None) -> np.ndarray:
    """Values Lx of L (left-looking, FP64); only the first ncols columns if given."""
    cp, ri, v = _csc(colptr, rowind, values)
    p = np.ascontiguousarray(perm, np.int32)
    Lx = np.zeros(Li.size, np.float64)
    bad = C.c_int32(-1)
    nc = n if ncols is None else int(ncols)
    rc = load().orc_factor(n, _ptr(cp), _ptr(ri), _ptr(v), _ptr(p), _ptr(Lp), _ptr(Li), _ptr(Lx), nc, C.byref(bad))
    if rc:
        raise OracleError(rc, "factor", bad.value)
    return Lx


def solve(perm, Lp, Li, Lx, B: np.ndarray, part: int = 0) -> np.ndarray:
    """part 0: P^T L^-T L^-1 P B; 1: L^-1 P B; 2: P^T L^-T B.  B is n or n x k."""
    n = Lp.size - 1
    B2 = np.asfortranarray(B.reshape(n, -1), np.float64)
    X = np.empty_like(B2, order="F")
    p = np.ascontiguousarray(perm, np.int32)
    rc = load().orc_solve(n, _ptr(p), _ptr(Lp), _ptr(Li), _ptr(Lx), part, B2.shape[1], _ptr(B2), _ptr(X), n)
    if rc:
        raise OracleError(rc, "solve")
    return X.reshape(B.shape)


def apply(perm, Lp, Li, Lx, B: np.ndarray, part: int) -> np.ndarray:
    """part 1: P^T L B (B in pivot order); 2: L^T P B (result in pivot order).  B is n or n x k."""
    n = Lp.size - 1
    B2 = np.asfortranarray(B.reshape(n, -1), np.float64)
    X = np.empty_like(B2, order="F")
    p = np.ascontiguousarray(perm, np.int32)
    rc = load().orc_apply(n, _ptr(p), _ptr(Lp), _ptr(Li), _ptr(Lx), part, B2.shape[1], _ptr(B2), _ptr(X), n)
    if rc:
        raise OracleError(rc, "apply")
    return X.reshape(B.shape)


def symv(n: int, colptr, rowind, values, X: np.ndarray) -> np.ndarray:
    """A X with the full symmetric A stored by its lower CSC."""
    cp, ri, v = _csc(colptr, rowind, values)
    X2 = np.asfortranarray(X.reshape(n, -1), np.float64)
    Y = np.empty_like(X2, order="F")
    rc = load().orc_symv(n, _ptr(cp), _ptr(ri), _ptr(v), X2.shape[1], _ptr(X2), _ptr(Y), n)
    if rc:
        raise OracleError(rc, "symv")
    return Y.reshape(X.shape)


def residual(n: int, colptr, rowind, values, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Per-column relative residual ||A x - b||_2 / ||b||_2 (FP64)."""
    R = symv(n, colptr, rowind, values, X).reshape(n, -1) - B.reshape(n, -1)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B.reshape(n, -1), axis=0)


def grad(n: int, colptr, rowind, lam: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Gradient with respect to the stored lower entries given lambda and x."""
    cp, ri = _csc(colptr, rowind)
    l = np.ascontiguousarray(lam, np.float64)
    xx = np.ascontiguousarray(x, np.float64)
    g = np.empty(ri.size, np.float64)
    rc = load().orc_grad(n, _ptr(cp), _ptr(ri), _ptr(l), _ptr(xx), _ptr(g))
    if rc:
        raise OracleError(rc, "grad")
    return g


def check_nd(n: int, colptr, rowind, perm, tree: np.ndarray) -> int:
    """Number of violations of the nested dissection block structure (0 = valid)."""
    cp, ri = _csc(colptr, rowind)
    p = np.ascontiguousarray(perm, np.int32)
    t = np.ascontiguousarray(tree, np.int32).reshape(-1)
    r = load().orc_check_nd(n, _ptr(cp), _ptr(ri), _ptr(p), t.size // 6, _ptr(t))
    if r < 0:
        raise OracleError(int(r), "check_nd")
    return int(r)


@dataclasses.dataclass
class Factor:
    n: int
    perm: np.ndarray
    parent: np.ndarray
    colcount: np.ndarray
    nnzL: int
    flops: int
    Lp: np.ndarray
    Li: np.ndarray
    Lx: np.ndarray

    def solve(self, B: np.ndarray, part: int = 0) -> np.ndarray:
        return solve(self.perm, self.Lp, self.Li, self.Lx, B, part)

    def apply(self, B: np.ndarray, part: int) -> np.ndarray:
        return apply(self.perm, self.Lp, self.Li, self.Lx, B, part)

    def dense_L(self) -> np.ndarray:
        L = np.zeros((self.n, self.n))
        cols = np.repeat(np.arange(self.n), np.diff(self.Lp))
        L[self.Li, cols] = self.Lx
        return L


def theta_steps(m: dict, perm: np.ndarray, theta: float, dt: float, F: np.ndarray, u0: np.ndarray) -> np.ndarray:
    """Theta scheme in time (Section 5, eq:theta) for G = I (L2-orthonormal
    wavelets) and L = -K, K = the symmetric positive definite matrix m:
    (I + theta dt K) u_{i+1} = (I - (1 - theta) dt K) u_i + dt ((1 - theta) f_i + theta f_{i+1}).
    The left matrix is factored once (oracle Cholesky, ordering perm); the
    explicit part applies K itself.  F: n x (nsteps + 1); returns U: n x (nsteps + 1)
    with U[:, 0] = u0.  Plain NumPy around the C oracle's factor, solve and symv."""
    n = m["n"]
    colptr, rowind, kv = m["colptr"], m["rowind"], np.asarray(m["values"], np.float64)
    diag = np.asarray(colptr[:-1], np.int64)
    if not np.array_equal(np.asarray(rowind)[diag], np.arange(n)):
        raise ValueError("theta_steps: the first stored entry of every column must be its diagonal")
    av = theta * dt * kv
    av[diag] += 1.0
    fac = factorize(dict(m, values=av), perm)
    nsteps = F.shape[1] - 1
    U = np.empty((n, nsteps + 1))
    U[:, 0] = u0
    for i in range(nsteps):
        u = U[:, i]
        rhs = u - (1.0 - theta) * dt * symv(n, colptr, rowind, kv, u) + dt * ((1.0 - theta) * F[:, i] + theta * F[:, i + 1])
        U[:, i + 1] = fac.solve(rhs)
    return U


def factorize(m: dict, perm: np.ndarray) -> Factor:
    """Symbolic + pattern + numeric factor of one instance (dict from the workload generator)."""
    n = m["n"]
    parent, cc, nnzL, fl = symbolic(n, m["colptr"], m["rowind"], perm)
    Lp, Li = pattern(n, m["colptr"], m["rowind"], perm, parent, cc)
    Lx = factor(n, m["colptr"], m["rowind"], m["values"], perm, Lp, Li)
    return Factor(n, np.ascontiguousarray(perm, np.int32), parent, cc, nnzL, fl, Lp, Li, Lx)


# ---------------------------------------------------------------- LU (Section 5.1, eq:PCM2)

def lu(n: int, colptr, rowind, lval, uval, perm, Lp, Li, ncols: Optional[int] = None):
    """(Lx, Ux): P A P^T = L U without pivoting for a matrix with a symmetric
    pattern given by its stored lower entries and the values below/on
    (lval) and above (uval) the diagonal; Lx = L (unit diagonal stored),
    Ux = U^T, both in the Cholesky pattern (Lp, Li)."""
    cp, ri, lv = _csc(colptr, rowind, lval)
    uv = np.ascontiguousarray(uval, np.float64)
    p = np.ascontiguousarray(perm, np.int32)
    Lx = np.zeros(Li.size, np.float64)
    Ux = np.zeros(Li.size, np.float64)
    bad = C.c_int32(-1)
    nc = n if ncols is None else int(ncols)
    rc = load().orc_lu(n, _ptr(cp), _ptr(ri), _ptr(lv), _ptr(uv), _ptr(p), _ptr(Lp), _ptr(Li), _ptr(Lx), _ptr(Ux),
                       nc, C.byref(bad))
    if rc:
        raise OracleError(rc, "lu", bad.value)
    return Lx, Ux


def lu_solve(perm, Lp, Li, Lx, Ux, B: np.ndarray, part: int = 0) -> np.ndarray:
    """part 0: P^T U^-1 L^-1 P B; 1: L^-1 P B; 2: P^T U^-1 B.  B is n or n x k."""
    n = Lp.size - 1
    B2 = np.asfortranarray(B.reshape(n, -1), np.float64)
    X = np.empty_like(B2, order="F")
    p = np.ascontiguousarray(perm, np.int32)
    rc = load().orc_lu_solve(n, _ptr(p), _ptr(Lp), _ptr(Li), _ptr(Lx), _ptr(np.ascontiguousarray(Ux)), part,
                             B2.shape[1], _ptr(B2), _ptr(X), n)
    if rc:
        raise OracleError(rc, "lu_solve")
    return X.reshape(B.shape)


def gemv(n: int, colptr, rowind, lval, uval, X: np.ndarray) -> np.ndarray:
    """A X for the nonsymmetric A of lu()."""
    cp, ri, lv = _csc(colptr, rowind, lval)
    uv = np.ascontiguousarray(uval, np.float64)
    X2 = np.asfortranarray(X.reshape(n, -1), np.float64)
    Y = np.empty_like(X2, order="F")
    rc = load().orc_gemv(n, _ptr(cp), _ptr(ri), _ptr(lv), _ptr(uv), X2.shape[1], _ptr(X2), _ptr(Y), n)
    if rc:
        raise OracleError(rc, "gemv")
    return Y.reshape(X.shape)


def gemv_residual(n: int, colptr, rowind, lval, uval, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Per-column ||A x - b||_2 / ||b||_2 for the nonsymmetric A (FP64)."""
    R = gemv(n, colptr, rowind, lval, uval, X).reshape(n, -1) - B.reshape(n, -1)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B.reshape(n, -1), axis=0)


@dataclasses.dataclass
class LUFactor:
    n: int
    perm: np.ndarray
    Lp: np.ndarray
    Li: np.ndarray
    Lx: np.ndarray
    Ux: np.ndarray

    def solve(self, B: np.ndarray, part: int = 0) -> np.ndarray:
        return lu_solve(self.perm, self.Lp, self.Li, self.Lx, self.Ux, B, part)

    def dense(self):
        """(L, U) as dense matrices in pivot order."""
        L = np.zeros((self.n, self.n))
        cols = np.repeat(np.arange(self.n), np.diff(self.Lp))
        L[self.Li, cols] = self.Lx
        Ut = np.zeros((self.n, self.n))
        Ut[self.Li, cols] = self.Ux
        return L, Ut.T


def lu_factorize(m: dict, perm: np.ndarray) -> LUFactor:
    """Symbolic (Cholesky pattern of the symmetric pattern) + LU of one
    nonsymmetric instance: m holds colptr, rowind and the two value arrays
    "values" (lower and diagonal) and "upper" (above the diagonal)."""
    n = m["n"]
    parent, cc, _, _ = symbolic(n, m["colptr"], m["rowind"], perm)
    Lp, Li = pattern(n, m["colptr"], m["rowind"], perm, parent, cc)
    Lx, Ux = lu(n, m["colptr"], m["rowind"], m["values"], m["upper"], perm, Lp, Li)
    return LUFactor(n, np.ascontiguousarray(perm, np.int32), Lp, Li, Lx, Ux)


# ---------------------------------------------------------------- covariance-form sampling (Section 5.3)

def field_sample(cov: Factor, mass: Factor, abar: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Coefficients of Gaussian random field samples in the covariance form of
    Section 5.3 (eq:CholFastField): G^-1 (abar^G + L X), where L L^T is the
    Cholesky decomposition of the Galerkin covariance matrix C^G (here
    C^G = P_C^T L_C L_C^T P_C with its own ordering, so L = P_C^T L_C) and G
    is the mass matrix, solved with its own factor (its own ordering).  X: the
    standard normal vectors, n x k, indexed in the covariance factor's pivot
    order; abar: n or n x k.  Returns n x k."""
    n = cov.n
    X2 = X.reshape(n, -1)
    Y = cov.apply(X2, 1)                                   # P_C^T L_C X
    Y = Y + np.asarray(abar, np.float64).reshape(n, -1)
    return mass.solve(Y, 0)                                # G^-1 (abar + L X)
