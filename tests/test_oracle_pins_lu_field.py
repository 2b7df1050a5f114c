"""Pins of the oracle's LU (Section 5.1, eq:PCM2) and covariance-form field
sampling (Section 5.3, eq:CholFastField) against independent routes: a
library dense LU with partial pivoting (which exchanges no rows on these
column-dominant matrices), the Cholesky oracle on symmetric input, dense
solves and products, and the covariance identity of the samples."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from workloads import WaveletSpec, make_matrix, make_nonsymmetric, mass_spec


def perms(n, seed):
    if seed == 0:
        return np.arange(n, dtype=np.int32)
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


def dense_nonsym(m):
    """Dense A from the stored lower pattern with values (lower) and upper."""
    n = m["n"]
    A = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    A[m["rowind"], cols] = m["values"]
    off = m["rowind"] != cols
    A[cols[off], m["rowind"][off]] = m["upper"][off]
    return A


def dense_sym(m):
    n = m["n"]
    A = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    A[m["rowind"], cols] = m["values"]
    return A + np.tril(A, -1).T


def nonsym(G=3, a=1.5, seed=11, eta=0.5):
    return make_nonsymmetric(WaveletSpec(G, a, 0.5, "exp", 0.3, 1.5, seed), eta, 5)


@pytest.mark.parametrize("pseed", [0, 3, 4])
def test_lu_matches_library_dense_lu(pseed):
    """scipy's LU with partial pivoting on C = P A P^T: on a matrix strictly
    dominant by columns it exchanges no rows, so its L and U are the unique
    no-pivot factors the oracle must produce."""
    m = nonsym()
    n = m["n"]
    perm = perms(n, pseed)
    f = oracle.lu_factorize(m, perm)
    C = dense_nonsym(m)[np.ix_(perm, perm)]
    P, Lr, Ur = scipy.linalg.lu(C)
    assert np.array_equal(P, np.eye(n))
    L, U = f.dense()
    assert np.max(np.abs(L - Lr)) <= 1e-13 * np.max(np.abs(Lr))
    assert np.max(np.abs(U - Ur)) <= 1e-13 * np.max(np.abs(Ur))


def test_lu_of_symmetric_matrix_is_scaled_cholesky():
    """For symmetric positive definite input, L U = P A P^T = R R^T gives
    L = R D^-1 and U = D R^T with D = diag(R) (the Cholesky oracle's factor)."""
    m = make_matrix(WaveletSpec(4, 1.5, 0.5, "exp", 0.3, 1.5, 13))
    m["upper"] = m["values"].copy()
    n = m["n"]
    perm = perms(n, 5)
    f = oracle.lu_factorize(m, perm)
    ch = oracle.factorize(m, perm)
    R = ch.dense_L()
    d = np.diag(R)
    L, U = f.dense()
    assert np.max(np.abs(L - R / d[None, :])) <= 1e-13
    assert np.max(np.abs(U - d[:, None] * R.T)) <= 1e-13 * np.max(np.abs(U))


def test_lu_backward_error_and_pattern():
    """|L U - C| within gamma_c |L||U| entrywise (textbook LU backward error,
    any summation order), and the symbolic pattern is the numerical one for
    both factors (no cancellation for random values)."""
    m = nonsym(G=4, a=1.5, seed=17)
    n = m["n"]
    perm = perms(n, 6)
    f = oracle.lu_factorize(m, perm)
    L, U = f.dense()
    C = dense_nonsym(m)[np.ix_(perm, perm)]
    c = int(np.diff(f.Lp).max())
    u = np.finfo(float).eps / 2
    gam = c * u / (1 - c * u)
    assert np.all(np.abs(L @ U - C) <= gam * (np.abs(L) @ np.abs(U)) + 1e-300)
    assert np.count_nonzero(f.Lx) == f.Lx.size and np.count_nonzero(f.Ux) == f.Ux.size
    assert np.all(np.diag(L) == 1.0)


@pytest.mark.parametrize("part", [0, 1, 2])
def test_lu_solve_against_dense(part):
    m = nonsym(G=3, a=1.2, seed=19)
    n = m["n"]
    perm = perms(n, 7)
    f = oracle.lu_factorize(m, perm)
    A = dense_nonsym(m)
    C = A[np.ix_(perm, perm)]
    _, L, U = scipy.linalg.lu(C)
    B = np.random.default_rng(8).standard_normal((n, 3))
    X = f.solve(B, part)
    if part == 0:
        ref = np.linalg.solve(A, B)
    elif part == 1:
        ref = scipy.linalg.solve_triangular(L, B[perm], lower=True, unit_diagonal=True)
    else:
        ref = np.empty_like(B)
        ref[perm] = scipy.linalg.solve_triangular(U, B, lower=False)
    assert np.max(np.abs(X - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_gemv_and_residual_against_dense():
    m = nonsym(G=4, a=1.5, seed=23)
    n = m["n"]
    A = dense_nonsym(m)
    X = np.random.default_rng(9).standard_normal((n, 2))
    assert np.max(np.abs(oracle.gemv(n, m["colptr"], m["rowind"], m["values"], m["upper"], X) - A @ X)) <= 1e-13 * np.abs(A @ X).max()
    f = oracle.lu_factorize(m, perms(n, 2))
    B = np.random.default_rng(10).standard_normal((n, 4))
    res = oracle.gemv_residual(n, m["colptr"], m["rowind"], m["values"], m["upper"], f.solve(B), B)
    assert res.max() <= 1e-13


def test_lu_leading_columns():
    m = nonsym(G=4, a=1.5, seed=29)
    n = m["n"]
    perm = perms(n, 4)
    f = oracle.lu_factorize(m, perm)
    k = n // 3
    Lx, Ux = oracle.lu(n, m["colptr"], m["rowind"], m["values"], m["upper"], perm, f.Lp, f.Li, ncols=k)
    e = f.Lp[k]
    assert np.array_equal(Lx[:e], f.Lx[:e])
    # U^T columns < k hold u(j, i) for rows i < k only once column i is done
    rows = f.Li[:e]
    done = rows < k
    assert np.array_equal(Ux[:e][done], f.Ux[:e][done])


def test_lu_singular_pivot_reported():
    """A zero pivot stops the factorization with its column: in the natural
    order the first pivot is a_00 itself."""
    m = nonsym(G=3, a=1.5, seed=31)
    m["values"][m["colptr"][0]] = 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.lu_factorize(m, perms(m["n"], 0))
    assert e.value.code == -5 and e.value.bad_col == 0


def field_case(G=3, seed=41):
    cov = make_matrix(WaveletSpec(G, 1.5, 0.5, "exp", 0.25, 1.5, seed))
    mass = make_matrix(mass_spec(G, seed + 1))
    return cov, mass


def test_field_sample_covariance_identity():
    """With X the identity (all n unit noise vectors) and no mean, the samples
    S = G^-1 L satisfy S S^T = G^-1 C^G G^-1, the covariance of the
    coefficients (Section 5.3), whatever the two orderings; checked against
    dense inverses."""
    cov, mass = field_case()
    n = cov["n"]
    fc = oracle.factorize(cov, perms(n, 3))
    fg = oracle.factorize(mass, perms(n, 4))
    S = oracle.field_sample(fc, fg, np.zeros(n), np.eye(n))
    Ginv = np.linalg.inv(dense_sym(mass))
    ref = Ginv @ dense_sym(cov) @ Ginv
    assert np.max(np.abs(S @ S.T - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_field_sample_mean_and_noise_terms():
    """Linearity: zero noise gives G^-1 abar; the noise part is G^-1 P^T L X with
    the Cholesky factor of C^G (dense library Cholesky of the permuted C^G)."""
    cov, mass = field_case(G=3, seed=43)
    n = cov["n"]
    pc = perms(n, 5)
    fc = oracle.factorize(cov, pc)
    fg = oracle.factorize(mass, perms(n, 6))
    G = dense_sym(mass)
    abar = np.random.default_rng(1).standard_normal(n)
    X = np.random.default_rng(2).standard_normal((n, 3))
    s0 = oracle.field_sample(fc, fg, abar, np.zeros((n, 1)))
    assert np.max(np.abs(s0[:, 0] - np.linalg.solve(G, abar))) <= 1e-12 * np.abs(s0).max()
    Lc = np.linalg.cholesky(dense_sym(cov)[np.ix_(pc, pc)])
    Y = np.empty((n, 3))
    Y[pc] = Lc @ X
    s = oracle.field_sample(fc, fg, abar, X)
    ref = np.linalg.solve(G, abar[:, None] + Y)
    assert np.max(np.abs(s - ref)) <= 1e-12 * np.abs(ref).max()


def test_mass_pattern_is_sub_pattern_of_system():
    """Section 6.3: the mass matrix's pattern is contained in the system
    matrix's, yet it is much sparser (own ordering, less fill)."""
    cov, mass = field_case(G=5, seed=45)
    n = cov["n"]
    def pairs(m):
        cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
        return set(zip(m["rowind"].tolist(), cols.tolist()))
    pm, pc = pairs(mass), pairs(cov)
    assert pm <= pc and len(pm) < len(pc) / 3
