"""Fused panel steps of large fronts against the panel kernel's schedule.

Fronts with at least WCS_STEP_MIN_COLS pivots (read when a factor is created)
are factored by k_diag_factor + k_step: each diagonal block one step ahead,
each panel's triangular solve fused with the update of the rest of its outer
block, panel rows parked in the front's upper triangle until the outer
block's last step moves them into place.  The arithmetic is the panel
kernel's (same diagonal-block factorization, same block forward substitution,
same update order), so the factor, and the solves with it, must be the same
bit for bit; the oracle parity of that factor is pinned by the other GPU
tests.  Outer blocks of 128 and 192 columns give many outer blocks (and a
ragged one) on the small parity cases; a diagonal-block threshold of 64
routes every FP32 front through the FP64 diagonal blocks.
"""
import numpy as np
import pytest

import oracle
from workloads import normal_rhs
from tests.helpers import EPS32, EPS64, cholesky_backward_error, compare_columns, factor_tol
from tests.test_gpu_parity import CASES, dev, prepared

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, FP64, Factor  # noqa: E402
from paper_2007_01541_amd.capi import WcsError  # noqa: E402

OFF = 10 ** 9   # threshold no front reaches: the panel kernel everywhere


def make(sym, prec, step_cols, monkeypatch, outer=None, diag=None, nrhs=1):
    monkeypatch.setenv("WCS_STEP_MIN_COLS", str(step_cols))
    if outer is None:
        monkeypatch.delenv("WCS_OUTER_BLOCK", raising=False)
    else:
        monkeypatch.setenv("WCS_OUTER_BLOCK", str(outer))
    if diag is None:
        monkeypatch.delenv("WCS_FP64_DIAG_COLS", raising=False)
    else:
        monkeypatch.setenv("WCS_FP64_DIAG_COLS", str(diag))
    return Factor(sym, prec, max_nrhs=nrhs)


@pytest.mark.parametrize("kind,leaf,coords", CASES)
@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("outer,diag", [(None, None), (128, 64), (192, None)])
def test_step_path_bitwise(kind, leaf, coords, prec, outer, diag, monkeypatch):
    m, sym, orc = prepared(kind, leaf, coords)
    p = np.diff(sym.export()["relaxed_ptr"])
    print(f"case {kind} prec={prec} outer={outer} diag={diag} n={m['n']} largest front {p.max()}", flush=True)
    assert p.max() > 128
    vals = dev(m["values"])
    B = normal_rhs(m["n"], 3, 71)
    out = []
    for cols in (OFF, 64):
        f = make(sym, prec, cols, monkeypatch, outer, diag, nrhs=3)
        f.numeric(vals)
        L = f.export_L()
        X = f.solve(dev(B)).cpu().numpy()
        out.append((L, X))
    (L0, X0), (L1, X1) = out
    for a, b in zip(L0, L1):
        assert np.array_equal(a, b)
    assert np.array_equal(X0, X1)
    eps = EPS64 if prec == FP64 else EPS32
    worst, scale = compare_columns(*L1, orc)
    assert worst <= factor_tol(m, int(orc.colcount.max()), eps) * scale


def test_step_path_refactor_and_backward_error(monkeypatch):
    """Refactorization over the same workspace (whose upper triangles still
    hold the previous run's parked panels) is bitwise reproducible, and the
    FP32 factor of the step path satisfies the kappa-free backward-error bound."""
    m, sym, orc = prepared("g6alg", 32, True)
    f = make(sym, FP32, 64, monkeypatch, outer=128, diag=64)
    vals = dev(m["values"])
    f.numeric(vals)
    a = f.export_L()
    f.numeric(dev(m["values"] * 3.0))
    f.numeric(vals)
    b = f.export_L()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    ratio = cholesky_backward_error(m, sym.export()["perm"], *b, EPS32)
    print(f"backward error / gamma bound = {ratio:.3e}")
    assert ratio <= 1.0


def test_step_path_refined_solve(monkeypatch):
    m, sym, orc = prepared("small")
    n = m["n"]
    B = normal_rhs(n, 8, 72)
    f = make(sym, FP32, 64, monkeypatch, outer=192, nrhs=8)
    vals = dev(m["values"])
    f.numeric(vals)
    X, rep = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X.cpu().numpy(), B)
    print(f"refined: {rep}, oracle residual {res.max():.3e}")
    assert res.max() <= 1e-10 and rep["iterations"] <= 3


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_step_path_reports_first_bad_pivot(prec, monkeypatch):
    """A non-positive pivot inside a stepped front (first or later diagonal
    block of an outer block) is reported with its pivot index, as by the
    panel kernel."""
    m, sym, _ = prepared("small")
    ex = sym.export()
    perm, rp = ex["perm"], ex["relaxed_ptr"]
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(perm.size)
    s = int(np.argmax(np.diff(rp)))
    # first block (k_diag_factor), second block (k_step), first and second
    # blocks of the second outer block of 128 columns
    for off in (0, 70, 130, 200):
        piv = int(rp[s]) + off
        col = int(perm[piv])
        v = m["values"].copy()
        v[m["colptr"][col]] = -1.0
        f = make(sym, prec, 64, monkeypatch, outer=128)
        with pytest.raises(WcsError) as e:
            f.numeric(dev(v))
        print(f"pivot {piv}: reported {e.value.bad_col}", flush=True)
        assert e.value.code == -4 and e.value.bad_col == piv


@pytest.mark.parametrize("kind,leaf,coords", CASES)
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_late_levels_bitwise(kind, leaf, coords, prec, monkeypatch):
    """Large fronts factored one level below their parent (WCS_LATE_MIN_PIVOTS)
    share other launches but keep every front's arithmetic and the order of
    the extend-add rounds: the factor and the solves are the same bit for bit."""
    m, sym, orc = prepared(kind, leaf, coords)
    vals = dev(m["values"])
    B = normal_rhs(m["n"], 3, 73)
    out = []
    for late in ("0", "64", "200", "1024"):
        monkeypatch.setenv("WCS_LATE_MIN_PIVOTS", late)
        f = Factor(sym, prec, max_nrhs=3)
        f.numeric(vals)
        out.append((f.export_L(), f.solve(dev(B)).cpu().numpy()))
    print(f"case {kind} prec={prec} n={m['n']}", flush=True)
    for L, X in out[1:]:
        for a, b in zip(out[0][0], L):
            assert np.array_equal(a, b)
        assert np.array_equal(out[0][1], X)
