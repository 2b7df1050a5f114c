"""Shared helpers of the parity tests (tolerances derived from the arithmetic)."""
import numpy as np

EPS64 = np.finfo(np.float64).eps
EPS32 = float(np.finfo(np.float32).eps)


def gershgorin_kappa(m):
    """Upper bound of the 2-norm condition number from Gershgorin discs:
    lambda in [min(a_ii - r_i), max(a_ii + r_i)], r_i = sum_{k != i} |a_ik|."""
    n = m["n"]
    cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    rows = m["rowind"]
    v = m["values"]
    off = rows != cols
    r = np.bincount(rows[off], np.abs(v[off]), n) + np.bincount(cols[off], np.abs(v[off]), n)
    d = v[m["colptr"][:-1]]
    lo, hi = np.min(d - r), np.max(d + r)
    assert lo > 0
    return hi / lo


def factor_tol(m, colcount_max, eps):
    """Forward-error scale of a computed Cholesky factor: kappa * c * eps, with a
    safety factor 10 (relative to max |L|)."""
    return 10.0 * gershgorin_kappa(m) * colcount_max * eps


def compare_columns(Lp, Li, Lx, orc, j0=0):
    """Max |L_gpu - L_oracle| over columns [j0, j0 + len(Lp) - 1) in pivot order.
    The GPU pattern may hold extra (amalgamation) rows: those must be exactly 0
    and every oracle row must be present.  Returns (max abs diff, max |L|)."""
    worst = 0.0
    scale = 0.0
    for t in range(Lp.size - 1):
        j = j0 + t
        gr = Li[Lp[t]:Lp[t + 1]]
        gv = Lx[Lp[t]:Lp[t + 1]]
        orow = orc.Li[orc.Lp[j]:orc.Lp[j + 1]]
        oval = orc.Lx[orc.Lp[j]:orc.Lp[j + 1]]
        pos = np.searchsorted(gr, orow)
        assert np.all(pos < gr.size) and np.array_equal(gr[pos], orow), f"column {j}: oracle rows missing"
        extra = np.ones(gr.size, bool)
        extra[pos] = False
        assert np.all(gv[extra] == 0.0), f"column {j}: nonzero outside the pattern"
        worst = max(worst, float(np.max(np.abs(gv[pos] - oval))))
        scale = max(scale, float(np.max(np.abs(oval))))
    return worst, scale


def dense_lower_export(Lp, Li, Lx, n):
    """Dense n x n lower-triangular L from a column export (pivot order)."""
    L = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(Lp))
    L[Li, cols] = Lx
    return L


def dense_permuted(m, perm):
    """P A P^T as a dense matrix (full symmetric A from its stored lower CSC)."""
    n = m["n"]
    A = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    A[m["rowind"], cols] = m["values"]
    A = A + np.tril(A, -1).T
    return A[np.ix_(perm, perm)]


def gamma(k, eps):
    """gamma_k = k u / (1 - k u) with the unit roundoff u = eps / 2."""
    u = eps / 2.0
    return k * u / (1.0 - k * u)


def cholesky_backward_error(m, perm, Lp, Li, Lx, eps):
    """Largest ratio |L L^T - P A P^T|_ij / (gamma_{c+2} |L||L^T|)_ij over the
    entries where the bound is nonzero, for a factor computed in a precision of
    machine epsilon eps.  The textbook componentwise backward error of Cholesky
    (Higham, Accuracy and Stability of Numerical Algorithms, Thm 10.3) bounds
    |L L^T - C| by gamma_{c+1} |L||L^T| for c = the longest column; one more u
    covers rounding the FP64 input to the working precision.
    the bound with a safety factor of 10; it does not depend on the condition
    number.  Entries where the bound is zero must match exactly."""
    n = m["n"]
    L = dense_lower_export(Lp, Li, Lx, n)
    C = dense_permuted(m, perm)
    E = np.abs(L @ L.T - C)
    c = int(np.diff(Lp).max())
    B = gamma(c + 2, eps) * (np.abs(L) @ np.abs(L).T)
    pos = B > 0
    assert np.all(E[~pos] == 0.0)
    return float(np.max(E[pos] / B[pos]))


def leading_columns_backward_error(m, perm, Lp, Li, Lx, eps):
    """cholesky_backward_error restricted to the columns [0, k) of L (pivot
    order) given by a column export of those columns: every entry (i, j) of
    L L^T with j < k sums products of columns t <= j only, so it is fixed by
    them, and the check runs at any size (sparse, the rows of all n pivots)."""
    import scipy.sparse as sp
    n = m["n"]
    k = Lp.size - 1
    cols = np.repeat(np.arange(k), np.diff(Lp))
    L = sp.csr_matrix((Lx, (Li, cols)), shape=(n, k))
    Lt = L[:k].T.tocsc()
    M = (L @ Lt).tocoo()                         # (L L^T)(:, 0:k), all rows
    Ab = (abs(L) @ abs(Lt)).tocsr()
    iperm = np.empty(n, np.int64)
    iperm[np.asarray(perm)] = np.arange(n)
    acols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    pi, pj = iperm[m["rowind"]], iperm[acols]
    hi, lo = np.maximum(pi, pj), np.minimum(pi, pj)
    keep = lo < k
    C = sp.csr_matrix((np.asarray(m["values"])[keep], (hi[keep], lo[keep])), shape=(n, k))
    mask = M.row >= M.col                         # lower triangle (the symmetric part is the same)
    E = sp.csr_matrix((M.data[mask], (M.row[mask], M.col[mask])), shape=(n, k)) - C
    E = E.tocoo()
    c = int(np.diff(Lp).max())
    bound = np.asarray(Ab[E.row, E.col]).ravel() * gamma(c + 2, eps)
    err = np.abs(E.data)
    assert np.all(err[bound == 0] == 0.0)
    pos = bound > 0
    return float(np.max(err[pos] / bound[pos])) if pos.any() else 0.0
