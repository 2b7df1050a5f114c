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
