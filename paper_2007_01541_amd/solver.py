"""Python binding of the wcs C ABI.

Argument marshalling only: every step of analyze/factor/solve runs inside
libwcs.so (host analysis in C++, numerics in gfx950 kernels).  PyTorch
provides the device memory (the caller-owned workspace and vectors) and the
stream.  There is no fallback: without the compiled library every call
raises.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import capi
from .capi import AnalyzeOpts, IRReport, SymbolicInfo, check, lib

FP64 = 0
FP32 = 1
LU64 = 2          # nonsymmetric A = P^T L U P (FP64 fronts)
SOLVE_FULL = 0
SOLVE_L = 1
SOLVE_LT = 2
APPLY_L = 1
APPLY_LT = 2


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dptr(t) -> int:
    return int(t.data_ptr())


class Symbolic:
    """Ordering + symbolic analysis of one pattern (host, deterministic)."""

    def __init__(self, n: int, colptr: np.ndarray, rowind: np.ndarray, coords: Optional[np.ndarray] = None,
                 leaf_size: int = 64, dense_degree_frac: float = 0.25, dense_degree_min: float = 1024.0,
                 user_perm: Optional[np.ndarray] = None, relax: bool = True):
        self._keep = []
        cp = np.ascontiguousarray(colptr, np.int64)
        ri = np.ascontiguousarray(rowind, np.int32)
        o = AnalyzeOpts()
        o.leaf_size = leaf_size
        o.dense_degree_frac = dense_degree_frac
        o.dense_degree_min = dense_degree_min
        o.relax = 1 if relax else 0
        if coords is not None:
            cc = np.ascontiguousarray(coords, np.float64)
            o.coords = cc.ctypes.data
            o.coord_dim = 1 if cc.ndim == 1 else cc.shape[1]
            self._keep.append(cc)
        if user_perm is not None:
            up = np.ascontiguousarray(user_perm, np.int32)
            o.user_perm = up.ctypes.data
            self._keep.append(up)
        h = C.c_void_p()
        check(lib().wcs_analyze(int(n), cp.ctypes.data, ri.ctypes.data, C.byref(o), C.byref(h)), "wcs_analyze")
        self._keep = []
        self.handle = h
        self.n = int(n)

    @classmethod
    def batch(cls, parts) -> "Symbolic":
        """Block-diagonal batch of independent analyses (wcs_symbolic_batch):
        instance b owns the unknowns seg_ptr[b]:seg_ptr[b+1]; its values follow
        those of instance b-1 in the batch's value array."""
        parts = list(parts)
        arr = (C.c_void_p * len(parts))(*[p.handle.value for p in parts])
        h = C.c_void_p()
        check(lib().wcs_symbolic_batch(len(parts), C.cast(arr, C.c_void_p), C.byref(h)), "wcs_symbolic_batch")
        self = cls.__new__(cls)
        self._keep = []
        self.handle = h
        self.n = int(sum(p.n for p in parts))
        return self

    @property
    def seg_ptr(self) -> np.ndarray:
        sp = np.empty(self.info["nseg"] + 1, np.int32)
        check(lib().wcs_symbolic_segments(self.handle, sp.ctypes.data), "wcs_symbolic_segments")
        return sp

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().wcs_symbolic_free(h)
            except Exception:
                pass
            self.handle = None

    @property
    def info(self) -> dict:
        inf = SymbolicInfo()
        check(lib().wcs_symbolic_info(self.handle, C.byref(inf)), "wcs_symbolic_info")
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def export(self) -> dict:
        inf = self.info
        n = self.n
        perm = np.empty(n, np.int32)
        parent = np.empty(n, np.int32)
        cc = np.empty(n, np.int32)
        sp = np.empty(inf["nsuper_fund"] + 1, np.int32)
        tree = np.empty(6 * inf["nsep_nodes"], np.int32)
        check(lib().wcs_symbolic_export(self.handle, perm.ctypes.data, parent.ctypes.data, cc.ctypes.data,
                                        sp.ctypes.data, tree.ctypes.data), "wcs_symbolic_export")
        rp = np.empty(inf["nsuper"] + 1, np.int32)
        fo = np.empty(inf["nsuper"], np.int32)
        check(lib().wcs_symbolic_fronts(self.handle, rp.ctypes.data, fo.ctypes.data), "wcs_symbolic_fronts")
        return {"perm": perm, "parent": parent, "colcount": cc, "super_ptr": sp, "sep_tree": tree.reshape(-1, 6),
                "relaxed_ptr": rp, "front_order": fo}

    def workspace_size(self, precision: int = FP64, max_nrhs: int = 1) -> int:
        b = C.c_size_t()
        check(lib().wcs_workspace_size(self.handle, precision, max_nrhs, C.byref(b)), "wcs_workspace_size")
        return int(b.value)


class Factor:
    """A device factor P A P^T = L L^T living in a torch-owned workspace."""

    def __init__(self, sym: Symbolic, precision: int = FP64, max_nrhs: int = 1, device=None, stream=None,
                 static_workspace: bool = False):
        """static_workspace=True: no workspace tensor; the factor lives in the
        library's static device array of the current device
        (wcs_factor_create_static: one such factor per device at a time)."""
        torch = _torch()
        self.sym = sym
        self.n = sym.n
        self.precision = precision
        self.max_nrhs = max_nrhs
        self.device = torch.device(device if device is not None else "cuda")
        h = C.c_void_p()
        if static_workspace:
            self.workspace = None
            check(lib().wcs_factor_create_static(sym.handle, precision, max_nrhs, _stream_ptr(stream), C.byref(h)),
                  "wcs_factor_create_static")
        else:
            nbytes = sym.workspace_size(precision, max_nrhs)
            # 256-byte aligned by the caching allocator
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            check(lib().wcs_factor_create(sym.handle, precision, max_nrhs, _dptr(self.workspace), nbytes,
                                          _stream_ptr(stream), C.byref(h)), "wcs_factor_create")
        self.handle = h
        self.values = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().wcs_factor_free(h)
            except Exception:
                pass
            self.handle = None

    def numeric(self, values, check_pivots: bool = True, stream=None) -> None:
        """Factor the matrix with device FP64 values (aligned with the pattern)."""
        torch = _torch()
        assert values.dtype == torch.float64 and values.is_cuda and values.is_contiguous()
        self.values = values
        if check_pivots:
            bad = C.c_int32(-1)
            rc = lib().wcs_factor_numeric(self.handle, _dptr(values), _stream_ptr(stream), C.byref(bad))
            check(rc, "wcs_factor_numeric", bad.value)
        else:
            check(lib().wcs_factor_numeric(self.handle, _dptr(values), _stream_ptr(stream), None),
                  "wcs_factor_numeric")

    def numeric_lu(self, lower, upper, check_pivots: bool = True, stream=None) -> None:
        """LU factorization (factor created with LU64) of the nonsymmetric matrix
        with device FP64 values on/below the diagonal (lower) and above it
        (upper), both aligned with the analysed lower pattern."""
        torch = _torch()
        for v in (lower, upper):
            assert v.dtype == torch.float64 and v.is_cuda and v.is_contiguous()
        self.values = (lower, upper)
        bad = C.c_int32(-1)
        rc = lib().wcs_factor_numeric_lu(self.handle, _dptr(lower), _dptr(upper), _stream_ptr(stream),
                                         C.byref(bad) if check_pivots else None)
        check(rc, "wcs_factor_numeric_lu", bad.value)

    def use_graphs(self, enable: bool = True) -> None:
        """Record the factorization and the sweeps into HIP graphs and replay them."""
        check(lib().wcs_factor_use_graphs(self.handle, 1 if enable else 0), "wcs_factor_use_graphs")

    def autotune(self, values, stream=None) -> dict:
        """Pick the trailing-update kernel per tree level by timing (leaves a valid factor):
        0 = 128x128 register-staged, 1 = 64x64, 2 = 128x128 streamed into LDS (four stages), 3 = the same
        with three stages."""
        self.values = values
        H = self.sym.info["nlevels"]
        tiles = np.zeros(max(H, 1), np.int32)
        ms = np.zeros(2, np.float64)
        check(lib().wcs_factor_autotune(self.handle, _dptr(values), _stream_ptr(stream), tiles.ctypes.data,
                                        ms.ctypes.data), "wcs_factor_autotune")
        return {"tiles": tiles[:H], "ms_default": float(ms[0]), "ms_tuned": float(ms[1])}

    def set_tiles(self, tiles) -> None:
        t = np.ascontiguousarray(tiles, np.int32)
        assert t.size == self.sym.info["nlevels"]
        check(lib().wcs_factor_set_tiles(self.handle, t.ctypes.data), "wcs_factor_set_tiles")

    def residuals(self) -> np.ndarray:
        """Relative residuals of the last refinement, shape (instances, nrhs)."""
        nseg = self.sym.info["nseg"]
        k = getattr(self, "_last_k", self.max_nrhs)
        out = np.empty(nseg * k, np.float64)
        check(lib().wcs_factor_residuals(self.handle, out.ctypes.data, out.size), "wcs_factor_residuals")
        return out.reshape(nseg, k)

    def profile(self, values, stream=None) -> dict:
        """One factorization with HIP events around every launch; per kernel class
        {launches, ms, flops, bytes} (algorithmic work)."""
        stats = (capi.KernelStat * len(capi.KERNEL_CLASSES))()
        self.values = values
        check(lib().wcs_factor_profile(self.handle, _dptr(values), _stream_ptr(stream), stats), "wcs_factor_profile")
        return {nm: {"launches": st.launches, "ms": st.ms, "flops": st.flops, "bytes": st.bytes}
                for nm, st in zip(capi.KERNEL_CLASSES, stats)}

    def profile_levels(self, values, stream=None) -> list:
        """One factorization timed per assembly-tree level: [{ms, flops}] from the leaves up."""
        nl = self.sym.info["nlevels"]
        stats = (capi.KernelStat * nl)()
        self.values = values
        check(lib().wcs_factor_profile_levels(self.handle, _dptr(values), _stream_ptr(stream), stats),
              "wcs_factor_profile_levels")
        return [{"ms": st.ms, "flops": st.flops} for st in stats]

    def pivot_check(self, stream=None) -> int:
        bad = C.c_int32(-1)
        rc = lib().wcs_factor_check(self.handle, _stream_ptr(stream), C.byref(bad))
        if rc not in (0, -4):
            check(rc, "wcs_factor_check")
        return bad.value

    def solve_(self, B, part: int = SOLVE_FULL, stream=None):
        """In-place solve on a device FP64 tensor B of shape (n,) or (n, k) (column-major view is made)."""
        torch = _torch()
        Bm = B if B.dim() == 2 else B.view(-1, 1)
        k = Bm.shape[1]
        # column-major n x k with ld = n == a contiguous (k, n) tensor transposed
        cm = Bm.t().contiguous()
        check(lib().wcs_solve(self.handle, part, k, _dptr(cm), self.n, _stream_ptr(stream)), "wcs_solve")
        Bm.copy_(cm.t())
        return B

    def solve(self, B, part: int = SOLVE_FULL, stream=None):
        return self.solve_(B.clone(), part, stream)

    def apply(self, B, part: int, stream=None):
        """Product with the factor: APPLY_L gives P^T L B (B in pivot order), APPLY_LT gives
        L^T P B (result in pivot order).  B: device FP64 tensor (n,) or (n, k); returns a new tensor."""
        Bm = B.clone() if B.dim() == 2 else B.clone().view(-1, 1)
        k = Bm.shape[1]
        cm = Bm.t().contiguous()
        check(lib().wcs_apply(self.handle, part, k, _dptr(cm), self.n, _stream_ptr(stream)), "wcs_apply")
        Bm.copy_(cm.t())
        return Bm if B.dim() == 2 else Bm.view(-1)

    def solve_refined(self, B, values=None, tol: float = 1e-10, max_iter: int = 10, stream=None):
        """X = A^-1 B by iterative refinement; returns (X, report dict).  If tol is
        not reached in max_iter corrections, raises WcsError (code -5) carrying
        .report and the last iterate as .result."""
        torch = _torch()
        vals = values if values is not None else self.values
        Bm = B if B.dim() == 2 else B.view(-1, 1)
        k = Bm.shape[1]
        bc = Bm.t().contiguous()
        xc = torch.empty_like(bc)
        rep = IRReport()
        self._last_k = k
        rc = lib().wcs_solve_refined(self.handle, _dptr(vals), k, _dptr(bc), _dptr(xc), self.n, tol, max_iter,
                                     C.byref(rep), _stream_ptr(stream))
        report = {"iterations": rep.iterations, "raw_residual": rep.raw_residual,
                  "final_residual": rep.final_residual}
        X = xc.t().contiguous()
        X = X if B.dim() == 2 else X.view(-1)
        if rc != 0:
            err = capi.WcsError(rc, "wcs_solve_refined", lib().wcs_last_error().decode(errors="replace"))
            err.report = report
            err.result = X if rc == -5 else None
            raise err
        return X, report

    def spmv(self, X, values=None, stream=None):
        torch = _torch()
        vals = values if values is not None else self.values
        Xm = X if X.dim() == 2 else X.view(-1, 1)
        xc = Xm.t().contiguous()
        yc = torch.empty_like(xc)
        check(lib().wcs_spmv(self.handle, _dptr(vals), Xm.shape[1], _dptr(xc), _dptr(yc), self.n,
                             _stream_ptr(stream)), "wcs_spmv")
        Y = yc.t().contiguous()
        return Y if X.dim() == 2 else Y.view(-1)

    def grad_pattern(self, lam, x, stream=None):
        torch = _torch()
        nnz = self.sym.info["nnz_lower"]
        g = torch.empty(nnz, dtype=torch.float64, device=lam.device)
        check(lib().wcs_grad_pattern(self.handle, _dptr(lam.contiguous()), _dptr(x.contiguous()), _dptr(g),
                                     _stream_ptr(stream)), "wcs_grad_pattern")
        return g

    def theta_matrix(self, K_values, theta: float, dt: float, stream=None):
        """Values of A = I + theta dt K on the stored lower pattern (device FP64)."""
        torch = _torch()
        A = torch.empty_like(K_values)
        check(lib().wcs_theta_matrix(self.handle, _dptr(K_values), theta, dt, _dptr(A), _stream_ptr(stream)),
              "wcs_theta_matrix")
        return A

    def theta_steps(self, A_values, theta: float, dt: float, F, u0, tol: float = 1e-10, stream=None):
        """nsteps = F.shape[1] - 1 theta-scheme steps over this factor of A = I + theta dt K
        (wcs_theta_steps); F: n x (nsteps + 1) device FP64, u0: n.  Returns (U, report) with
        U: n x (nsteps + 1), column 0 = u0."""
        torch = _torch()
        nsteps = F.shape[1] - 1
        fc = F.t().contiguous()                 # column-major n x (nsteps + 1)
        uc = torch.empty((nsteps + 1, self.n), dtype=torch.float64, device=F.device)
        uc[0] = u0
        rep = IRReport()
        rc = lib().wcs_theta_steps(self.handle, _dptr(A_values), theta, dt, nsteps, _dptr(fc), self.n, _dptr(uc),
                                   self.n, tol, C.byref(rep), _stream_ptr(stream))
        report = {"iterations": rep.iterations, "raw_residual": rep.raw_residual,
                  "final_residual": rep.final_residual}
        if rc != 0:
            err = capi.WcsError(rc, "wcs_theta_steps", lib().wcs_last_error().decode(errors="replace"))
            err.report = report
            raise err
        return uc.t().contiguous(), report

    def export_L(self, j0: int = 0, j1: Optional[int] = None):
        """Columns [j0, j1) of L in pivot order as host CSC (stored pattern, explicit zeros kept)."""
        return self._export("wcs_factor_export", j0, j1)

    def export_U(self, j0: int = 0, j1: Optional[int] = None):
        """LU factors: columns [j0, j1) of U^T (entry (i, j) = u(j, i)) in the format of export_L."""
        return self._export("wcs_factor_export_upper", j0, j1)

    def _export(self, call: str, j0: int, j1: Optional[int]):
        j1 = self.n if j1 is None else j1
        fn = getattr(lib(), call)
        Lp = np.empty(j1 - j0 + 1, np.int64)
        check(fn(self.handle, j0, j1, Lp.ctypes.data, None, None, _stream_ptr()), call)
        Li = np.empty(int(Lp[-1]), np.int32)
        Lx = np.empty(int(Lp[-1]), np.float64)
        check(fn(self.handle, j0, j1, Lp.ctypes.data, Li.ctypes.data, Lx.ctypes.data, _stream_ptr()), call)
        return Lp, Li, Lx


def field_sample(cov: Factor, mass: Factor, X, abar=None, stream=None):
    """Random field coefficients G^-1 (abar + L X) (Section 5.3, eq:CholFastField)
    from a Cholesky factor of the covariance matrix (cov) and one of the mass
    matrix (mass, its own ordering); X: device FP64 (n,) or (n, k) standard
    normal noise in cov's pivot order; abar: None, (n,) or (n, k).  Returns a
    new (n,) or (n, k) tensor in the original order."""
    torch = _torch()
    n = cov.n
    Xm = X if X.dim() == 2 else X.view(-1, 1)
    k = Xm.shape[1]
    xc = Xm.t().contiguous()                      # column-major n x k, ld = n
    out = torch.empty_like(xc)
    a = None
    lda = 0
    if abar is not None:
        am = abar if abar.dim() == 2 else abar.view(-1, 1)
        a = am.t().contiguous()
        lda = n if am.shape[1] > 1 else 0
    check(lib().wcs_field_sample(cov.handle, mass.handle, k, _dptr(a) if a is not None else None, lda, _dptr(xc), n,
                                 _dptr(out), n, _stream_ptr(stream)), "wcs_field_sample")
    res = out.t()
    return res.contiguous() if X.dim() == 2 else res.reshape(-1)


def _solve_op():
    torch = _torch()

    class SparseCholeskySolve(torch.autograd.Function):
        """y = A^-1 b with A given by its stored lower entries (values).

        Forward factors nothing: it uses a prepared Factor of A.  Backward reuses
        the same factor: lam = A^-1 gy, gb = lam, and the gradient with respect
        to the stored entries is -(lam_i y_j + lam_j y_i) off the diagonal and
        -lam_i y_i on it.  Only the factor and y are kept between the passes.
        """

        @staticmethod
        def forward(ctx, values, b, factor, refine, tol, max_iter):
            if refine:
                y, _ = factor.solve_refined(b.detach(), values.detach(), tol=tol, max_iter=max_iter)
            else:
                y = factor.solve(b.detach())
            ctx.factor = factor
            ctx.refine = refine
            ctx.tol = tol
            ctx.max_iter = max_iter
            ctx.save_for_backward(values, y)
            return y

        @staticmethod
        def backward(ctx, gy):
            values, y = ctx.saved_tensors
            f = ctx.factor
            if ctx.refine:
                lam, _ = f.solve_refined(gy.contiguous(), values, tol=ctx.tol, max_iter=ctx.max_iter)
            else:
                lam = f.solve(gy.contiguous())
            gvals = f.grad_pattern(lam, y) if ctx.needs_input_grad[0] else None
            gb = lam if ctx.needs_input_grad[1] else None
            return gvals, gb, None, None, None, None

    return SparseCholeskySolve


_OP = None


def cholesky_solve(values, b, factor: Factor, refine: bool = False, tol: float = 1e-10, max_iter: int = 10):
    """Differentiable x = A^-1 b (b a 1-D device FP64 tensor) through a prepared Factor."""
    global _OP
    if _OP is None:
        _OP = _solve_op()
    return _OP.apply(values, b, factor, refine, tol, max_iter)
