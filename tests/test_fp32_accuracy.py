"""Accuracy of the FP32 factor itself, independent of the condition number.

The FP32 path factors every front in FP32 on the matrix cores, except that
fronts with many pivots factor their 64 x 64 diagonal blocks in FP64 and round
them to FP32 (the FP64 diagonal-block factorization of the root separators).
These tests pin

  * the componentwise backward error of the exported FP32 factor,
    |L L^T - P A P^T| <= gamma_{c+2}(eps32) |L||L^T| (Section 4 defines
    the factor by P A P^T = L L^T; the bound is the textbook one for
    Cholesky in any summation order, taken without a safety factor), for the default routing and with every
    front of 64 or more pivots routed through the FP64 diagonal blocks;
  * a front with more than 1024 pivots (not a multiple of 64) that takes the
    FP64 diagonal-block route at the default threshold, against the oracle;
  * the raw FP32 solve: its residual under c kappa eps32, and refinement to
    1e-10 in at most three corrections.
"""
import numpy as np
import pytest

import oracle
from workloads import tiny, normal_rhs
from tests.helpers import EPS32, cholesky_backward_error, compare_columns, factor_tol, gershgorin_kappa
from tests.test_gpu_parity import CASES, dev, prepared

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, Factor, Symbolic  # noqa: E402


def fp64diag_launches(f, vals):
    return f.profile(vals)["panel_fp64diag"]["launches"]


@pytest.mark.parametrize("kind,leaf,coords", CASES)
@pytest.mark.parametrize("diag_cols", ["1024", "64"])
def test_fp32_factor_backward_error(kind, leaf, coords, diag_cols, monkeypatch):
    """kappa-free check of the FP32 factor on every parity case, with the
    default FP64 diagonal-block threshold and with it lowered to 64 pivots
    (read when the factor is created), so every front of >= 64 pivots factors
    its diagonal blocks in FP64."""
    monkeypatch.setenv("WCS_FP64_DIAG_COLS", diag_cols)
    m, sym, orc = prepared(kind, leaf, coords)
    print(f"case {kind} diag_cols={diag_cols} n={m['n']}", flush=True)
    f = Factor(sym, FP32)
    vals = dev(m["values"])
    f.numeric(vals)
    if diag_cols == "64":
        assert fp64diag_launches(f, vals) > 0
        f.numeric(vals)
    Lp, Li, Lx = f.export_L()
    perm = sym.export()["perm"]
    ratio = cholesky_backward_error(m, perm, Lp, Li, Lx, EPS32)
    print(f"  backward error / gamma bound = {ratio:.3e}")
    assert ratio <= 1.0
    worst, scale = compare_columns(Lp, Li, Lx, orc)
    assert worst <= factor_tol(m, int(orc.colcount.max()), EPS32) * scale


@pytest.mark.parametrize("kind", ["small", "g6alg"])
def test_fp64_diag_blocks_refined_solve(kind, monkeypatch):
    """Every front of >= 64 pivots on the FP64 diagonal-block panel: the
    refined solve reaches 1e-10 against the oracle's residual in at most three
    corrections, and its solution matches the oracle's."""
    monkeypatch.setenv("WCS_FP64_DIAG_COLS", "64")
    m, sym, orc = prepared(kind)
    n = m["n"]
    B = normal_rhs(n, 8, 61)
    f = Factor(sym, FP32, max_nrhs=8)
    vals = dev(m["values"])
    f.numeric(vals)
    X, rep = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    X = X.cpu().numpy()
    res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X, B)
    print(f"{kind}: {rep}, oracle residual {res.max():.3e}")
    assert res.max() <= 1e-10 and rep["iterations"] <= 3
    Xo = orc.solve(B)
    assert np.abs(X - Xo).max() <= 1e-10 * gershgorin_kappa(m) * np.abs(Xo).max()


_BIG = {}


def big_front():
    """N = 4096 with the vertices of degree >= 250 peeled into the root
    separator: the root front has 1276 pivots (19 full 64-column panels and a
    ragged one of 60), above the default FP64 diagonal-block threshold."""
    if not _BIG:
        m = tiny(6, 1.5, seed=42).matrix()
        sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"], dense_degree_frac=0.0,
                       dense_degree_min=250)
        orc = oracle.factorize(m, sym.export()["perm"])
        _BIG.update(m=m, sym=sym, orc=orc)
    return _BIG["m"], _BIG["sym"], _BIG["orc"]


def test_big_front_fp64_diag_default_threshold(monkeypatch):
    monkeypatch.delenv("WCS_FP64_DIAG_COLS", raising=False)
    m, sym, orc = big_front()
    p = np.diff(sym.export()["relaxed_ptr"])
    assert p.max() >= 1024 and p.max() % 64 != 0
    print(f"big front: n={m['n']} largest front {p.max()} pivots", flush=True)
    f = Factor(sym, FP32, max_nrhs=4)
    vals = dev(m["values"])
    assert fp64diag_launches(f, vals) > 0
    f.numeric(vals)
    Lp, Li, Lx = f.export_L()
    ratio = cholesky_backward_error(m, sym.export()["perm"], Lp, Li, Lx, EPS32)
    worst, scale = compare_columns(Lp, Li, Lx, orc)
    print(f"  backward error / gamma bound {ratio:.3e}; max |L - L_oracle| / max |L| = {worst / scale:.3e}")
    assert ratio <= 1.0
    assert worst <= factor_tol(m, int(orc.colcount.max()), EPS32) * scale
    B = normal_rhs(m["n"], 4, 62)
    X, rep = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    res = oracle.residual(m["n"], m["colptr"], m["rowind"], m["values"], X.cpu().numpy(), B)
    assert res.max() <= 1e-10 and rep["iterations"] <= 3


@pytest.mark.parametrize("kind,leaf,coords", CASES)
def test_raw_fp32_residual_bound(kind, leaf, coords):
    """One FP32 solve without refinement: relative residual (oracle symv, FP64)
    below c kappa eps32 with c the longest column of L and kappa the
    Gershgorin bound of the condition number; the value is printed (the raw
    FP32 error the report states)."""
    m, sym, orc = prepared(kind, leaf, coords)
    n = m["n"]
    B = normal_rhs(n, 4, 63)
    f = Factor(sym, FP32, max_nrhs=4)
    f.numeric(dev(m["values"]))
    X = f.solve(dev(B)).cpu().numpy()
    res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X, B).max()
    bound = int(orc.colcount.max()) * gershgorin_kappa(m) * EPS32
    Xo = orc.solve(B)
    err = np.abs(X - Xo).max() / np.abs(Xo).max()
    print(f"{kind}: raw FP32 residual {res:.3e} (bound {bound:.3e}), error vs FP64 oracle {err:.3e}")
    assert res <= bound
