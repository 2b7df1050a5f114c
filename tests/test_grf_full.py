"""Gaussian random field form at full size (N = 2^18, a = 2, s = 3/4).

Sample x = P^T L^-T z (precision form: Cov(x) = A^-1), then y = A^-1 b with
b = x held fixed, loss 0.5 ||y - y*||^2, and its gradient with respect to
the stored entries of A and to b from the adjoint that reuses L.  The oracle
cannot factor this size in seconds, so the checks are its factorization of
the leading pivot columns, properties that hold at any size (residuals formed
by the oracle's product), the oracle's gradient formula evaluated on the same
lambda and y, and central finite differences on the GPU FP64 path at 32
sampled entries."""
import types

import numpy as np
import pytest

import oracle
import workloads
from tests.helpers import EPS32, EPS64, compare_columns, factor_tol, leading_columns_backward_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, FP64, SOLVE_LT, Factor, Symbolic, cholesky_solve  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def test_grf_sample_and_gradient_full_size():
    w = workloads.random_field()
    m = w.matrix()
    n = m["n"]
    print(f"grf workload {w.name} n={n} nnz={m['colptr'][-1]}", flush=True)
    sym = Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"])
    vals = dev(m["values"])
    f64 = Factor(sym, FP64)
    f64.numeric(vals)
    f32 = Factor(sym, FP32)
    f32.numeric(vals)

    # leading pivot columns of both factors against the oracle's left-looking
    # factorization of the same columns: FP64 entrywise, FP32 by the
    # componentwise backward error of those columns (kappa-free)
    perm = sym.export()["perm"]
    parent, cc, _, _ = oracle.symbolic(n, m["colptr"], m["rowind"], perm)
    Lp_o, Li_o = oracle.pattern(n, m["colptr"], m["rowind"], perm, parent, cc)
    k = int(np.searchsorted(np.cumsum(cc.astype(np.float64) ** 2), 1e10))
    Lx_o = oracle.factor(n, m["colptr"], m["rowind"], m["values"], perm, Lp_o, Li_o, ncols=k)
    orc = types.SimpleNamespace(Lp=Lp_o, Li=Li_o, Lx=Lx_o)
    Lp, Li, Lx = f64.export_L(0, k)
    worst, scale = compare_columns(Lp, Li, Lx, orc)
    print(f"leading {k} columns: FP64 max |L - L_oracle| / max |L| = {worst / scale:.3e}", flush=True)
    assert worst <= factor_tol(m, int(cc.max()), EPS64) * scale
    Lp, Li, Lx = f32.export_L(0, k)
    ratio = leading_columns_backward_error(m, perm, Lp, Li, Lx, EPS32)
    print(f"leading {k} columns: FP32 backward error / gamma bound = {ratio:.3e}", flush=True)
    assert ratio <= 1.0

    def symv(v):
        return oracle.symv(n, m["colptr"], m["rowind"], m["values"], np.asarray(v, np.float64))

    def rel_residual(v, rhs):
        v, rhs = np.asarray(v), np.asarray(rhs)
        return float(np.linalg.norm(symv(v) - rhs) / np.linalg.norm(rhs))

    # sample: x^T A x = z^T z for x = P^T L^-T z (exact identity with the exact factor)
    z = workloads.normal_rhs(n, 1, w.seed + 3)[:, 0]
    x = f64.solve(dev(z), part=SOLVE_LT)
    xh = x.cpu().numpy()
    q = float(xh @ symv(xh))
    zz = float(z @ z)
    print(f"x^T A x = {q:.15e}, z^T z = {zz:.15e}", flush=True)
    assert abs(q - zz) <= 1e-10 * zz
    x32 = f32.solve(dev(z), part=SOLVE_LT)
    rel32 = float(torch.linalg.norm(x32 - x) / torch.linalg.norm(x))
    print(f"FP32 sample relative difference {rel32:.3e}", flush=True)
    assert rel32 <= 1e-4

    # solve + adjoint through the FP32 factor with FP64 refinement
    ystar = dev(workloads.normal_rhs(n, 1, w.seed + 2)[:, 0])
    b = x.detach().clone().requires_grad_(True)
    v = vals.clone().requires_grad_(True)
    y = cholesky_solve(v, b, f32, refine=True, tol=1e-10)
    loss = 0.5 * ((y - ystar) ** 2).sum()
    loss.backward()
    gA = v.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()
    yh = y.detach().cpu().numpy()
    # y solves A y = b to 1e-10 (residual by the oracle's product)
    assert rel_residual(yh, b.detach().cpu().numpy()) <= 1e-10
    # gb = lambda solves A lambda = y - y* to 1e-10; gA is the oracle's formula on that lambda and y
    assert rel_residual(gb, yh - ystar.cpu().numpy()) <= 1e-10
    g_orc = oracle.grad(n, m["colptr"], m["rowind"], gb, yh)
    assert np.abs(gA - g_orc).max() <= 1e-14 * np.abs(g_orc).max()

    # central finite differences (h = 1e-6, FP64 factor) at 32 entries; the loss
    # difference is formed as sum (y+ - y-)(y+ + y- - 2 y*) / 2 to keep it accurate
    rng = np.random.Generator(np.random.PCG64(w.seed + 4))
    nnz = m["colptr"][-1]
    diag = m["colptr"][:-1]
    picks = np.concatenate([rng.choice(diag, 4, replace=False), rng.choice(nnz, 28, replace=False)])
    h = 1e-6
    bd = b.detach()
    gmax = np.abs(gA).max()
    worst = 0.0
    for t, e in enumerate(picks):
        ys = []
        for sgn in (1.0, -1.0):
            vp = vals.clone()
            vp[int(e)] += sgn * h
            f64.numeric(vp, check_pivots=False)
            ys.append(f64.solve(bd))
        fd = float(((ys[0] - ys[1]) * (ys[0] + ys[1] - 2 * ystar)).sum()) / 2 / (2 * h)
        err = abs(fd - gA[e])
        worst = max(worst, err / (1e-5 * abs(gA[e]) + 1e-7 * gmax))
        if t < 4 or err > 1e-5 * abs(gA[e]) + 1e-7 * gmax:
            print(f"entry {e}: fd {fd:.10e} adjoint {gA[e]:.10e} err {err:.3e}", flush=True)
    print(f"finite differences: worst error / tolerance = {worst:.3f}", flush=True)
    assert worst <= 1.0
