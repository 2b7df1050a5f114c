"""The persistent leaf-front launch and batches at the batching workload's sizes.

All leaf fronts of all instances of a batch are factored by one persistent
launch that pulls fronts from a device queue (largest first) and keeps each
front's pivot columns in LDS; the upper levels stay level-synchronous.
Checked here: the leaf kernel against the oracle and against the
level-synchronous kernels (within rounding: both are Cholesky factors of the
same matrix), a batch drawn from the batching workload at full instance size
(grid sides 2^5 and 2^6, N = 1,024 and 4,096) bitwise equal to every
instance's own factor and equal to the oracle's factor of the stacked matrix,
and refinement of a batch holding a 128 x 128 instance (N = 16,384) to 1e-10
per instance, with the residuals formed by the oracle's product.
"""
import numpy as np
import pytest

import oracle
from workloads import batch_instance, block_diagonal, normal_rhs
from tests.helpers import EPS32, EPS64, cholesky_backward_error, compare_columns
from tests.test_gpu_parity import dev, prepared

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, FP64, Factor, Symbolic  # noqa: E402


def leaf_fronts(sym):
    """Number of fronts with no child (the leaf fronts) from the exported tree."""
    ex = sym.export()
    rp = ex["relaxed_ptr"]
    ns = rp.size - 1
    snode = np.repeat(np.arange(ns), np.diff(rp))
    par = ex["parent"][rp[1:] - 1]
    sp = np.where(par >= 0, snode[np.maximum(par, 0)], -1)
    has_child = np.zeros(ns, bool)
    has_child[sp[sp >= 0]] = True
    return int((~has_child).sum())


@pytest.mark.parametrize("kind", ["small", "g6alg"])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_leaf_kernel_against_oracle_and_level_path(kind, prec, monkeypatch):
    m, sym, orc = prepared(kind)
    n = m["n"]
    print(f"{kind}: n={n} fronts={sym.info['nsuper']} leaf fronts {leaf_fronts(sym)}", flush=True)
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("WCS_LEAF_KERNEL", flag)      # read when the factor is created
        f = Factor(sym, prec, max_nrhs=4)
        vals = dev(m["values"])
        f.numeric(vals)
        out[flag] = f.export_L()
        if flag == "1":
            B = normal_rhs(n, 4, 71)
            if prec == FP64:
                X = f.solve(dev(B)).cpu().numpy()
                assert oracle.residual(n, m["colptr"], m["rowind"], m["values"], X, B).max() <= 1e-12
            else:
                X, rep = f.solve_refined(dev(B), vals, tol=1e-10)
                res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X.cpu().numpy(), B)
                assert res.max() <= 1e-10 and rep["iterations"] <= 3
    Lp, Li, Lx = out["1"]
    assert np.array_equal(Lp, out["0"][0]) and np.array_equal(Li, out["0"][1])
    worst, scale = compare_columns(Lp, Li, Lx, orc)
    if prec == FP64:
        assert worst <= 1e-12 * scale
        assert np.abs(Lx - out["0"][2]).max() <= 1e-12 * scale
    else:
        ratio = cholesky_backward_error(m, sym.export()["perm"], Lp, Li, Lx, EPS32)
        print(f"  FP32 backward error / gamma bound {ratio:.3e}; leaf vs level path "
              f"{np.abs(Lx - out['0'][2]).max() / scale:.3e}")
        assert ratio <= 1.0


_BATCH = {}


def config_batch():
    """The first instances of the batching workload with grid side 2^5 or 2^6
    (N = 1,024 or 4,096), at their own sizes and parameters."""
    if not _BATCH:
        ids = [i for i in range(24) if batch_instance(i).spec.grid_exp <= 6][:8]
        from workloads import make_matrix
        mats = [make_matrix(batch_instance(i).spec) for i in ids]
        syms = [Symbolic(x["n"], x["colptr"], x["rowind"], coords=x["coords"]) for x in mats]
        _BATCH.update(ids=ids, mats=mats, syms=syms)
    return _BATCH["ids"], _BATCH["mats"], _BATCH["syms"]


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_config_size_batch_equals_instances_and_oracle(prec):
    ids, mats, syms = config_batch()
    bs = Symbolic.batch(syms)
    big = block_diagonal(mats)
    print(f"batch instances {ids}: n={big['n']} sizes {[x['n'] for x in mats]} leaf fronts {leaf_fronts(bs)}",
          flush=True)
    fb = Factor(bs, prec)
    fb.numeric(dev(big["values"]))
    Lp, Li, Lx = fb.export_L()
    off = big["seg_ptr"]
    for b, (x, s) in enumerate(zip(mats, syms)):
        f = Factor(s, prec)
        f.numeric(dev(x["values"]))
        lp, li, lx = f.export_L()
        j0, j1 = off[b], off[b + 1]
        assert np.array_equal(Lx[Lp[j0]:Lp[j1]], lx), b          # bitwise the instance's own factor
        assert np.array_equal(Li[Lp[j0]:Lp[j1]] - j0, li)
    if prec == FP64:
        orc = oracle.factorize(big, bs.export()["perm"])
        worst, scale = compare_columns(Lp, Li, Lx, orc)
        assert worst <= 1e-11 * scale


def test_batch_with_128_grid_instance_refines_per_instance():
    ids, mats, syms = config_batch()
    j7 = next(i for i in range(24) if batch_instance(i).spec.grid_exp == 7)
    from workloads import make_matrix
    m7 = make_matrix(batch_instance(j7).spec)
    s7 = Symbolic(m7["n"], m7["colptr"], m7["rowind"], coords=m7["coords"])
    allm = mats[:3] + [m7]
    bs = Symbolic.batch(syms[:3] + [s7])
    big = block_diagonal(allm)
    n = big["n"]
    B = normal_rhs(n, 4, 72)
    f = Factor(bs, FP32, max_nrhs=4)
    vals = dev(big["values"])
    f.numeric(vals)
    X, rep = f.solve_refined(dev(B), vals, tol=1e-10)
    X = X.cpu().numpy()
    off = big["seg_ptr"]
    worst = 0.0
    for b, x in enumerate(allm):
        r = oracle.residual(x["n"], x["colptr"], x["rowind"], x["values"], X[off[b]:off[b + 1]], B[off[b]:off[b + 1]])
        worst = max(worst, float(r.max()))
    print(f"instances {[x['n'] for x in allm]}: {rep}, worst per-instance residual {worst:.3e}", flush=True)
    assert worst <= 1e-10 and rep["iterations"] <= 3
    assert np.allclose(f.residuals().max(), rep["final_residual"])
