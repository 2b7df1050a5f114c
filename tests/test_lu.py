"""GPU LU of nonsymmetric matrices on the Cholesky plan against the oracle.

Section 5.1 (eq:PCM2): the PCM system matrix is not symmetric and Section 6.1
factors it by LU on the nested dissection ordering of its (symmetric)
pattern.  The GPU factors P A P^T = L U without pivoting in two sets of
fronts (L, and U^T), with the same MFMA trailing updates as the Cholesky
path; the oracle is the left-looking LU of oracle.c.  Inputs are strictly
diagonally dominant by rows and columns, so the factorization exists and is
stable without pivoting.
"""
import numpy as np
import pytest

import oracle
from workloads import WaveletSpec, make_nonsymmetric, normal_rhs
from tests.helpers import EPS64, compare_columns, gamma

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP64, LU64, SOLVE_FULL, SOLVE_L, SOLVE_LT, Factor, Symbolic  # noqa: E402
from paper_2007_01541_amd.capi import WcsError  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


SPECS = {
    # (grid exponent, a, kind, leaf size, peel threshold)
    "g5": (WaveletSpec(5, 1.5, 0.5, "exp", 0.3, 1.5, 81), 16, 64),
    "g6": (WaveletSpec(6, 2.0, 0.75, "alg", 0.3, 1.75, 82), 32, 1024),
    "g6peel": (WaveletSpec(6, 1.5, 0.5, "exp", 0.3, 1.5, 83), 64, 250),   # root front of > 1024 pivots
}
_CACHE = {}


def prepared(kind):
    if kind not in _CACHE:
        spec, leaf, peel = SPECS[kind]
        m = make_nonsymmetric(spec, 0.5, 9)
        sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"], leaf_size=leaf,
                       dense_degree_frac=0.0 if kind == "g6peel" else 0.25, dense_degree_min=peel)
        orc = oracle.lu_factorize(m, sym.export()["perm"])
        _CACHE[kind] = (m, sym, orc)
    return _CACHE[kind]


def dense_permuted_nonsym(m, perm):
    n = m["n"]
    A = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    A[m["rowind"], cols] = m["values"]
    off = m["rowind"] != cols
    A[cols[off], m["rowind"][off]] = m["upper"][off]
    return A[np.ix_(perm, perm)]


def dense_from_export(Lp, Li, Lx, n):
    M = np.zeros((n, n))
    M[Li, np.repeat(np.arange(n), np.diff(Lp))] = Lx
    return M


@pytest.mark.parametrize("kind", list(SPECS))
def test_lu_factors_match_oracle(kind):
    m, sym, orc = prepared(kind)
    n = m["n"]
    p = np.diff(sym.export()["relaxed_ptr"])
    print(f"LU case {kind}: n={n} fronts={sym.info['nsuper']} largest front {p.max()} pivots", flush=True)
    f = Factor(sym, LU64)
    f.numeric_lu(dev(m["values"]), dev(m["upper"]))
    Lp, Li, Lx = f.export_L()
    Up, Ui, Ux = f.export_U()
    assert np.array_equal(Lp, Up) and np.array_equal(Li, Ui)
    # entrywise against the oracle's factors
    wl, sl = compare_columns(Lp, Li, Lx, orc)
    wu, su = compare_columns(Up, Ui, Ux, oracle.Factor(n, orc.perm, None, None, 0, 0, orc.Lp, orc.Li, orc.Ux))
    print(f"  max |L - L_oracle| / max|L| = {wl / sl:.3e}, max |U - U_oracle| / max|U| = {wu / su:.3e}")
    assert wl <= 1e-11 * sl and wu <= 1e-11 * su
    # kappa-free: |L U - P A P^T| <= gamma_c |L||U| entrywise (textbook LU backward error)
    L = dense_from_export(Lp, Li, Lx, n)
    U = dense_from_export(Up, Ui, Ux, n).T
    C = dense_permuted_nonsym(m, sym.export()["perm"])
    c = int(np.diff(Lp).max())
    ratio = np.max(np.abs(L @ U - C) / (gamma(c, EPS64) * (np.abs(L) @ np.abs(U)) + 1e-300))
    print(f"  backward error / gamma bound = {ratio:.3e}")
    assert ratio <= 1.0
    assert np.all(np.diag(L) == 1.0)


@pytest.mark.parametrize("kind", list(SPECS))
@pytest.mark.parametrize("k", [1, 3, 64, 70])
def test_lu_solve_matches_oracle(kind, k):
    m, sym, orc = prepared(kind)
    n = m["n"]
    B = normal_rhs(n, k, 91)
    f = Factor(sym, LU64, max_nrhs=k)
    f.numeric_lu(dev(m["values"]), dev(m["upper"]))
    X = f.solve(dev(B)).cpu().numpy()
    res = oracle.gemv_residual(n, m["colptr"], m["rowind"], m["values"], m["upper"], X, B)
    Xo = orc.solve(B)
    print(f"{kind} k={k}: residual {res.max():.3e}, max |X - X_oracle| / max|X| = "
          f"{np.abs(X - Xo).max() / np.abs(Xo).max():.3e}", flush=True)
    assert res.max() <= 1e-12
    assert np.abs(X - Xo).max() <= 1e-11 * np.abs(Xo).max()


@pytest.mark.parametrize("part", [SOLVE_L, SOLVE_LT])
def test_lu_half_solves(part):
    m, sym, orc = prepared("g6")
    n = m["n"]
    B = normal_rhs(n, 4, 92)
    f = Factor(sym, LU64, max_nrhs=4)
    f.numeric_lu(dev(m["values"]), dev(m["upper"]))
    X = f.solve(dev(B), part).cpu().numpy()
    Xo = orc.solve(B, part)
    assert np.abs(X - Xo).max() <= 1e-11 * np.abs(Xo).max()


def test_lu_refactor_bitwise_and_singular_pivot():
    m, sym, _ = prepared("g5")
    f = Factor(sym, LU64)
    lo, up = dev(m["values"]), dev(m["upper"])
    f.numeric_lu(lo, up)
    a = f.export_L()[2].copy(), f.export_U()[2].copy()
    f.numeric_lu(lo, up)
    b = f.export_L()[2], f.export_U()[2]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    perm = sym.export()["perm"]
    v = m["values"].copy()
    v[m["colptr"][perm[0]]] = 0.0          # the first pivot is a_{perm[0], perm[0]} itself
    with pytest.raises(WcsError) as e:
        f.numeric_lu(dev(v), up)
    assert e.value.code == -7 and e.value.bad_col == 0


def test_lu_rejects_cholesky_only_calls():
    m, sym, _ = prepared("g5")
    f = Factor(sym, LU64, max_nrhs=2)
    with pytest.raises(WcsError):
        f.numeric(dev(m["values"]))
    f.numeric_lu(dev(m["values"]), dev(m["upper"]))
    B = dev(normal_rhs(m["n"], 2, 1))
    with pytest.raises(WcsError):
        f.solve_refined(B, dev(m["values"]))
    chol = Factor(sym, FP64)
    with pytest.raises(WcsError):
        chol.numeric_lu(dev(m["values"]), dev(m["upper"]))
