"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Sizes here run through several tiles, ragged tails and multi-level trees
while the oracle finishes in seconds."""
import numpy as np
import pytest

import oracle
from workloads import small_fp64, tiny, WaveletSpec, make_matrix, normal_rhs
from tests.helpers import EPS32, EPS64, compare_columns, factor_tol, gershgorin_kappa

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import (APPLY_L, APPLY_LT, FP32, FP64, SOLVE_FULL, SOLVE_L, SOLVE_LT, Factor,  # noqa: E402
                                  Symbolic, cholesky_solve)
from paper_2007_01541_amd.capi import WcsError  # noqa: E402


def instance(kind):
    if kind == "small":
        return small_fp64().matrix()
    if kind == "g5a13":
        return tiny(5, 1.3, seed=21).matrix()
    if kind == "g4a2":
        return tiny(4, 2.0, seed=22).matrix()
    if kind == "g6alg":
        return make_matrix(WaveletSpec(6, 2.0, 0.75, "alg", 0.3, 1.75, 23))
    raise KeyError(kind)


_CACHE = {}


def prepared(kind, leaf=64, coords=True):
    key = (kind, leaf, coords)
    if key not in _CACHE:
        m = instance(kind)
        sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"] if coords else None, leaf_size=leaf,
                       dense_degree_min=64 if m["n"] < 4096 else 1024)
        perm = sym.export()["perm"]
        orc = oracle.factorize(m, perm)
        _CACHE[key] = (m, sym, orc)
    return _CACHE[key]


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


CASES = [("small", 64, True), ("g5a13", 16, True), ("g4a2", 8, False), ("g6alg", 32, True)]


@pytest.mark.parametrize("kind,leaf,coords", CASES)
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_factor_matches_oracle(kind, leaf, coords, prec):
    m, sym, orc = prepared(kind, leaf, coords)
    print(f"case {kind} leaf={leaf} prec={prec} n={m['n']} fronts={sym.info['nsuper']}", flush=True)
    f = Factor(sym, prec)
    f.numeric(dev(m["values"]))
    Lp, Li, Lx = f.export_L()
    worst, scale = compare_columns(Lp, Li, Lx, orc)
    tol = factor_tol(m, int(orc.colcount.max()), EPS64 if prec == FP64 else EPS32)
    assert worst <= tol * scale, (worst / scale, tol)


@pytest.mark.parametrize("kind,leaf,coords", CASES)
@pytest.mark.parametrize("k", [1, 3, 9, 64, 70])
def test_fp64_solve(kind, leaf, coords, k):
    m, sym, orc = prepared(kind, leaf, coords)
    n = m["n"]
    B = normal_rhs(n, k, 77)
    f = Factor(sym, FP64, max_nrhs=k)
    f.numeric(dev(m["values"]))
    X = f.solve(dev(B)).cpu().numpy()
    res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X, B)
    assert res.max() <= 1e-12
    Xo = orc.solve(B)
    tol = factor_tol(m, int(orc.colcount.max()), EPS64)
    assert np.abs(X - Xo).max() <= tol * np.abs(Xo).max()


@pytest.mark.parametrize("kind,leaf,coords", CASES)
@pytest.mark.parametrize("k", [5, 9, 16])
def test_solve_sixteen_column_kernels(kind, leaf, coords, k, monkeypatch):
    """5..16 right-hand sides through the 16-column sweep kernels (routed
    there by WCS_SOLVE_KT16_MAX, read by every solve; by default they take the
    64-column ones): oracle residual and agreement with the default route."""
    m, sym, orc = prepared(kind, leaf, coords)
    n = m["n"]
    B = normal_rhs(n, k, 79)
    f = Factor(sym, FP64, max_nrhs=k)
    f.numeric(dev(m["values"]))
    X64 = f.solve(dev(B)).cpu().numpy()
    monkeypatch.setenv("WCS_SOLVE_KT16_MAX", "16")
    X16 = f.solve(dev(B)).cpu().numpy()
    res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X16, B)
    assert res.max() <= 1e-12
    tol = factor_tol(m, int(orc.colcount.max()), EPS64)
    assert np.abs(X16 - X64).max() <= tol * np.abs(X64).max()


@pytest.mark.parametrize("part", [SOLVE_L, SOLVE_LT])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_half_solves(part, prec):
    m, sym, orc = prepared("small")
    n = m["n"]
    B = normal_rhs(n, 2, 5)
    f = Factor(sym, prec, max_nrhs=2)
    f.numeric(dev(m["values"]))
    X = f.solve(dev(B), part).cpu().numpy()
    Xo = orc.solve(B, part)
    tol = factor_tol(m, int(orc.colcount.max()), EPS64 if prec == FP64 else EPS32)
    assert np.abs(X - Xo).max() <= tol * np.abs(Xo).max()


@pytest.mark.parametrize("kind,leaf,coords", CASES)
@pytest.mark.parametrize("k", [1, 8, 64])
def test_fp32_refined_reaches_1e10(kind, leaf, coords, k):
    m, sym, orc = prepared(kind, leaf, coords)
    n = m["n"]
    B = normal_rhs(n, k, 9)
    f = Factor(sym, FP32, max_nrhs=k)
    vals = dev(m["values"])
    f.numeric(vals)
    X, rep = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    X = X.cpu().numpy()
    res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X, B)
    print(f"{kind} k={k}: iterations={rep['iterations']} raw={rep['raw_residual']:.3e} final={res.max():.3e}")
    assert res.max() <= 1e-10
    assert rep["final_residual"] <= 1e-10
    assert rep["raw_residual"] > rep["final_residual"] or rep["iterations"] == 0
    assert rep["iterations"] <= 3
    Xo = orc.solve(B)
    assert np.abs(X - Xo).max() <= 1e-10 * gershgorin_kappa(m) * np.abs(Xo).max()


@pytest.mark.parametrize("kind", ["small", "g6alg"])
@pytest.mark.parametrize("k", [4, 8, 32, 64])
def test_updated_residual_tracks_true_residual(kind, k):
    """With an FP32 factor and 4, 8, 16, 32 or 64 right-hand sides the residual
    is updated from the FP32 corrections (R -= A D) instead of being recomputed
    from X (k = 4 in the four-column form of the SpMV); the reported
    per-column residuals must stay the true ones ||b - A x|| / ||b|| (oracle,
    FP64) up to the FP64 rounding of x, through several corrections
    (tolerance far below what one correction reaches)."""
    m, sym, _ = prepared(kind)
    n = m["n"]
    B = normal_rhs(n, k, 31) * np.logspace(-3, 3, k)     # columns of very different scales
    f = Factor(sym, FP32, max_nrhs=k)
    vals = dev(m["values"])
    f.numeric(vals)
    with pytest.raises(WcsError) as e:      # tolerance 0: every correction is taken
        f.solve_refined(dev(B), vals, tol=0.0, max_iter=3)
    X, rep = e.value.result, e.value.report
    true = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X.cpu().numpy(), B)
    upd = f.residuals()[0]
    kap = gershgorin_kappa(m)
    print(f"{kind} k={k}: iterations {rep['iterations']}, reported {upd.max():.3e}, true {true.max():.3e}, "
          f"largest gap {np.abs(upd - true).max():.3e}, kappa bound {kap:.1f}")
    assert rep["iterations"] == 3
    assert np.all(np.abs(upd - true) <= 8 * rep["iterations"] * EPS64 * kap)
    assert true.max() <= 1e-12


def test_fp64_refined_no_iterations_needed():
    m, sym, _ = prepared("small")
    B = normal_rhs(m["n"], 1, 3)
    f = Factor(sym, FP64)
    vals = dev(m["values"])
    f.numeric(vals)
    X, rep = f.solve_refined(dev(B), vals, tol=1e-12, max_iter=0)
    assert rep["iterations"] == 0 and rep["final_residual"] <= 1e-12


def test_refinement_not_converged_reports():
    m, sym, _ = prepared("small")
    B = normal_rhs(m["n"], 1, 3)
    f = Factor(sym, FP32)
    vals = dev(m["values"])
    f.numeric(vals)
    with pytest.raises(WcsError) as e:
        f.solve_refined(dev(B), vals, tol=1e-30, max_iter=0)
    assert e.value.code == -5 and e.value.report["iterations"] == 0


@pytest.mark.parametrize("k", [1, 3, 4, 8, 9, 16, 32, 64, 70])
def test_spmv_matches_oracle(k):
    m, sym, _ = prepared("small")
    X = normal_rhs(m["n"], k, 4)
    f = Factor(sym, FP64, max_nrhs=k)
    Y = f.spmv(dev(X), dev(m["values"])).cpu().numpy().reshape(m["n"], k)
    Yo = oracle.symv(m["n"], m["colptr"], m["rowind"], m["values"], X).reshape(m["n"], k)
    assert np.abs(Y - Yo).max() <= 1e-13 * np.abs(Yo).max()


_MEDIUM = {}


def medium():
    """N = 65536: the coarsest wavelets couple to every unknown, so rows of up to
    65536 entries are split into several SpMV work items (chunks of 4096)."""
    if not _MEDIUM:
        from workloads import medium_fp64
        m = medium_fp64().matrix()
        _MEDIUM["m"] = m
        _MEDIUM["sym"] = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"])
    return _MEDIUM["m"], _MEDIUM["sym"]


@pytest.mark.parametrize("k", [1, 8, 64])
def test_spmv_long_rows_match_oracle(k):
    m, sym = medium()
    n = m["n"]
    deg = np.diff(m["colptr"]) + np.bincount(m["rowind"], minlength=n) - 1
    print(f"medium n={n}: longest row {deg.max()} entries, {(deg > 4096).sum()} rows over 4096", flush=True)
    assert deg.max() > 4 * 4096
    X = normal_rhs(n, k, 12)
    f = Factor(sym, FP64, max_nrhs=k)
    Y = f.spmv(dev(X), dev(m["values"])).cpu().numpy().reshape(n, k)
    Yo = oracle.symv(n, m["colptr"], m["rowind"], m["values"], X).reshape(n, k)
    assert np.abs(Y - Yo).max() <= 1e-13 * np.abs(Yo).max()


@pytest.mark.parametrize("k", [4, 64])
def test_fp32_refined_long_rows(k):
    """The FP32-row residual forms (first residual and updates; k = 4 in the
    four-column form) over split rows."""
    m, sym = medium()
    n = m["n"]
    B = normal_rhs(n, k, 13)
    f = Factor(sym, FP32, max_nrhs=k)
    vals = dev(m["values"])
    f.numeric(vals)
    X, rep = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X.cpu().numpy(), B)
    print(f"medium k={k}: {rep}, true residual {res.max():.3e}", flush=True)
    assert res.max() <= 1e-10 and abs(res.max() - rep["final_residual"]) <= 1e-12


@pytest.mark.parametrize("kind", ["small", "medium"])
def test_refined_independent_of_expansion_grid(kind, monkeypatch):
    """The matrix values for the residual are expanded on a side stream with a
    bounded grid (environment WCS_EXPAND_BLOCKS, read at each call): one
    workgroup (the eight-deep loop runs from 1,793 entries on), the default and
    a grid larger than the work must give bitwise the same refined solution
    and report, and that solution reaches 1e-10 against the oracle."""
    if kind == "medium":
        m, sym = medium()
    else:
        m, sym, _ = prepared(kind)
    n, k = m["n"], 8
    nnz_full = 2 * len(m["rowind"]) - n
    B = normal_rhs(n, k, 57)
    f = Factor(sym, FP32, max_nrhs=k)
    vals = dev(m["values"])
    f.numeric(vals)
    out = []
    for blocks in ("1", "256", "65536"):
        monkeypatch.setenv("WCS_EXPAND_BLOCKS", blocks)
        print(f"case {kind} n={n} nnz={nnz_full} expansion blocks {blocks}", flush=True)
        X, rep = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
        out.append((X.cpu().numpy(), rep))
    for X, rep in out[1:]:
        assert np.array_equal(X, out[0][0]) and rep == out[0][1]
    res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], out[0][0], B)
    assert res.max() <= 1e-10


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("k", [1, 3, 64, 70])
def test_factor_products_match_oracle(prec, k):
    """P^T L B and L^T P B against the oracle's products with the same (exported)
    L, entrywise within the rounding bound of a sum of at most n terms, and
    their composition against the oracle's A B."""
    m, sym, _ = prepared("small")
    n = m["n"]
    print(f"factor products prec={prec} k={k} n={n}", flush=True)
    f = Factor(sym, prec, max_nrhs=k)
    f.numeric(dev(m["values"]))
    Lp, Li, Lx = f.export_L()
    perm = sym.export()["perm"]
    eps = EPS64 if prec == FP64 else EPS32
    B = normal_rhs(n, k, 21)
    for part in (APPLY_L, APPLY_LT):
        X = f.apply(dev(B), part).cpu().numpy()
        ref = oracle.apply(perm, Lp, Li, Lx, B, part)
        bound = (n + 2) * eps * oracle.apply(perm, Lp, Li, np.abs(Lx), np.abs(B), part)
        assert np.all(np.abs(X - ref) <= bound), part
    X = f.apply(f.apply(dev(B), APPLY_LT), APPLY_L).cpu().numpy()
    AB = oracle.symv(n, m["colptr"], m["rowind"], m["values"], B)
    tol = 1e-12 if prec == FP64 else 1e-4
    assert np.abs(X - AB).max() <= tol * np.abs(AB).max()
    if prec == FP64:
        # the forward solve undone by the product: P^T L (L^-1 P B) = B
        Y = f.apply(f.solve(dev(B), SOLVE_L), APPLY_L).cpu().numpy()
        assert np.abs(Y - B).max() <= 1e-11 * np.abs(B).max()


def test_factor_products_reject_bad_arguments():
    m, sym, _ = prepared("small")
    f = Factor(sym, FP64, max_nrhs=2)
    B = dev(normal_rhs(m["n"], 2, 1))
    with pytest.raises(Exception):
        f.apply(B, APPLY_L)          # no numeric factorization yet
    f.numeric(dev(m["values"]))
    with pytest.raises(Exception):
        f.apply(B, 0)                # not a product part
    with pytest.raises(Exception):
        f.apply(dev(normal_rhs(m["n"], 3, 1)), APPLY_L)   # more columns than max_nrhs


@pytest.mark.parametrize("kind", ["small", "g5a13"])
def test_gradient_matches_oracle(kind):
    m, sym, orc = prepared(kind, *{"small": (64, True), "g5a13": (16, True)}[kind])
    n = m["n"]
    g = np.random.default_rng(3)
    b = g.standard_normal(n)
    ystar = g.standard_normal(n)
    f = Factor(sym, FP64)
    vals = dev(m["values"]).requires_grad_(True)
    f.numeric(vals.detach())
    bt = dev(b).requires_grad_(True)
    y = cholesky_solve(vals, bt, f)
    loss = 0.5 * ((y - dev(ystar)) ** 2).sum()
    loss.backward()
    x = orc.solve(b)
    lam = orc.solve(x - ystar)
    gA = oracle.grad(n, m["colptr"], m["rowind"], lam, x)
    assert np.abs(vals.grad.cpu().numpy() - gA).max() <= 1e-10 * np.abs(gA).max()
    assert np.abs(bt.grad.cpu().numpy() - lam).max() <= 1e-10 * np.abs(lam).max()


def test_not_spd_reports_first_pivot():
    m, sym, _ = prepared("g5a13", 16, True)
    perm = sym.export()["perm"]
    iperm = np.empty_like(perm); iperm[perm] = np.arange(perm.size)
    col = int(perm[perm.size // 3])
    v = m["values"].copy()
    v[m["colptr"][col]] = -1.0
    f = Factor(sym, FP64)
    with pytest.raises(WcsError) as e:
        f.numeric(dev(v))
    assert e.value.code == -4 and e.value.bad_col == iperm[col]
    v[m["colptr"][col]] = np.nan
    with pytest.raises(WcsError) as e:
        f.numeric(dev(v))
    assert e.value.code == -4 and e.value.bad_col <= iperm[col]


def test_refactor_and_determinism():
    m, sym, _ = prepared("small")
    f = Factor(sym, FP64)
    f.numeric(dev(m["values"]))
    a = f.export_L()[2].copy()
    f.numeric(dev(m["values"] * 2.0))
    b = f.export_L()[2].copy()
    f.numeric(dev(m["values"]))
    c = f.export_L()[2]
    assert np.array_equal(a, c)                      # bitwise reproducible
    # L(2A) = sqrt(2) L(A): exact up to rounding, measured against max |L|
    assert np.abs(b - a * np.sqrt(2.0)).max() <= 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("kind,leaf,coords", CASES)
@pytest.mark.parametrize("k", [1, 9, 64, 70])
@pytest.mark.parametrize("rows", ["100000", "64"])
def test_solve_fused_fronts(kind, leaf, coords, k, rows, monkeypatch):
    """Fronts of at most `rows` rows solved one workgroup per front for the whole
    sweep (all of them, or the small ones beside super-block fronts; the plan
    reads the routing threshold when the factor is created; by default every
    front takes the super-block path): same solution as the oracle."""
    monkeypatch.setenv("WCS_SOLVE_STEP_ROWS", rows)
    m, sym, orc = prepared(kind, leaf, coords)
    n = m["n"]
    B = normal_rhs(n, k, 78)
    for prec, eps in ((FP64, EPS64), (FP32, EPS32)):
        f = Factor(sym, prec, max_nrhs=k)
        f.numeric(dev(m["values"]))
        X = f.solve(dev(B)).cpu().numpy()
        Xo = orc.solve(B)
        tol = factor_tol(m, int(orc.colcount.max()), eps)
        print(f"case {kind} k={k} prec={prec}", flush=True)
        assert np.abs(X - Xo).max() <= tol * np.abs(Xo).max()


@pytest.mark.parametrize("kind", ["small", "g6alg"])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_update_variants_bitwise(kind, prec):
    """Every trailing-update kernel (128 x 128 register-staged, 64 x 64,
    128 x 128 streamed with four or three chunks in flight or two chunks of
    twice the depth) sums the same
    products in the same order: the factor is bitwise the same on fronts with
    many tiles and ragged edges."""
    m, sym, orc = prepared(kind)
    vals = dev(m["values"])
    out = []
    for v in range(5):
        f = Factor(sym, prec)
        f.set_tiles(np.full(sym.info["nlevels"], v, np.int32))
        f.numeric(vals)
        out.append(f.export_L()[2])
    for v in range(1, 5):
        assert np.array_equal(out[v], out[0]), v
    Lp, Li, _ = f.export_L()
    worst, scale = compare_columns(Lp, Li, out[3], orc)
    assert worst <= factor_tol(m, int(orc.colcount.max()), EPS64 if prec == FP64 else EPS32) * scale
