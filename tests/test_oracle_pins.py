"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: each compares it with an
independent route to the same answer (a library dense Cholesky, a brute-force
reading of Lemma 4.1, closed forms, exact invariants, finite differences).
"""
import numpy as np
import pytest

import oracle
from workloads import tiny, small_fp64, WaveletSpec, make_matrix, full_nnz


def dense_from_lower(m):
    n = m["n"]
    A = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    A[m["rowind"], cols] = m["values"]
    A = A + np.tril(A, -1).T
    return A


def random_sparse_spd(n, deg, seed):
    """A random sparse SPD matrix (diagonally dominant) as a lower CSC dict."""
    g = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        nb = g.choice(n, size=min(n - 1, deg), replace=False)
        for j in nb:
            if j != i:
                rows.append(max(i, j)); cols.append(min(i, j))
    pairs = sorted(set(zip(cols, rows)))
    A = np.zeros((n, n))
    for c, r in pairs:
        v = g.uniform(-1, 1)
        A[r, c] = A[c, r] = v
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(1) + 1.0
    return lower_csc(A)


def lower_csc(A):
    n = A.shape[0]
    colptr = [0]
    rowind, vals = [], []
    for j in range(n):
        r = np.nonzero(A[j:, j])[0] + j
        if r.size == 0 or r[0] != j:
            r = np.concatenate([[j], r])
        rowind.extend(r.tolist()); vals.extend(A[r, j].tolist())
        colptr.append(len(rowind))
    return {"n": n, "colptr": np.array(colptr, np.int64), "rowind": np.array(rowind, np.int32),
            "values": np.array(vals)}


def sparse_haar(G=3, a=1.2, seed=11):
    return make_matrix(WaveletSpec(G, a, 0.5, "exp", 0.3, 1.5, seed))


def lemma41_pattern(A_pattern, perm):
    """Brute force of Lemma 4.1: l_ij != 0 (i > j, pivot order) iff there is a
    path i = v1, ..., v_{k+1} = j in the graph of A whose interior vertices are
    all numbered below min(pi(i), pi(j)).  Returns a dense boolean lower
    pattern in pivot order."""
    n = A_pattern.shape[0]
    pi = np.empty(n, int)
    pi[perm] = np.arange(n)
    nbrs = [np.nonzero(A_pattern[v])[0] for v in range(n)]
    P = np.zeros((n, n), bool)
    for jv in range(n):
        j = pi[jv]
        # BFS from jv through vertices numbered below j; every vertex reached
        # with number above j is a row i with l_ij != 0
        seen = {jv}
        stack = [jv]
        while stack:
            u = stack.pop()
            for w in nbrs[u]:
                if w in seen or w == u:
                    continue
                seen.add(w)
                if pi[w] < j:
                    stack.append(w)
                elif pi[w] > j:
                    P[pi[w], j] = True
        P[j, j] = True
    return P


PERM_SEEDS = [0, 1, 2]


def perms(n, seed):
    if seed == 0:
        return np.arange(n, dtype=np.int32)
    if seed == 1:
        return np.arange(n - 1, -1, -1, dtype=np.int32)
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


@pytest.mark.parametrize("seed", PERM_SEEDS)
@pytest.mark.parametrize("make", ["haar", "rand"])
def test_symbolic_matches_lemma41(make, seed):
    m = sparse_haar() if make == "haar" else random_sparse_spd(120, 3, 5)
    n = m["n"]
    A = dense_from_lower(m)
    perm = perms(n, seed)
    parent, cc, nnzL, flops = oracle.symbolic(n, m["colptr"], m["rowind"], perm)
    Lp, Li = oracle.pattern(n, m["colptr"], m["rowind"], perm, parent, cc)
    P = lemma41_pattern(A != 0, perm)
    got = np.zeros((n, n), bool)
    got[Li, np.repeat(np.arange(n), np.diff(Lp))] = True
    assert np.array_equal(got, P)
    assert nnzL == int(P.sum())
    assert np.array_equal(cc, P.sum(0))
    assert flops == int((P.sum(0).astype(np.int64) ** 2).sum())
    # etree: parent[j] = min{i > j : l_ij != 0}
    for j in range(n):
        below = np.nonzero(P[j + 1:, j])[0]
        assert parent[j] == (below[0] + j + 1 if below.size else -1)


def test_dense_closed_forms():
    """N = 16 (grid 4x4): every pair is kept for a >= 1.2, so L is dense:
    nnz(L) = N(N+1)/2 = 136 and sum c_j^2 = N(N+1)(2N+1)/6 = 1496 for any P."""
    m = tiny(2, a=1.2).matrix()
    assert full_nnz(m) == 16 * 16
    for seed in PERM_SEEDS:
        perm = perms(16, seed)
        _, cc, nnzL, flops = oracle.symbolic(16, m["colptr"], m["rowind"], perm)
        assert nnzL == 136
        assert flops == 1496
        assert sorted(cc.tolist()) == list(range(1, 17))


@pytest.mark.parametrize("seed", PERM_SEEDS)
@pytest.mark.parametrize("make", ["haar", "rand", "haar16"])
def test_numeric_matches_dense_cholesky(make, seed):
    m = {"haar": sparse_haar, "rand": lambda: random_sparse_spd(150, 4, 9),
         "haar16": lambda: tiny(4, 1.5).matrix()}[make]()
    n = m["n"]
    perm = perms(n, seed)
    f = oracle.factorize(m, perm)
    A = dense_from_lower(m)
    C = A[np.ix_(perm, perm)]
    Lref = np.linalg.cholesky(C)
    L = f.dense_L()
    assert np.max(np.abs(L - Lref)) <= 1e-13 * np.max(np.abs(Lref))
    # upper triangle untouched, diagonal positive
    assert np.all(np.diag(L) > 0)


def test_backward_error_bound_and_nnz_prediction():
    """|L L^T - P A P^T| <= 10 gamma_{c+1} |L||L^T| entrywise on pattern(L)
    (textbook Cholesky backward error), and the predicted pattern is the
    numerical one (no cancellation for random values)."""
    m = tiny(5, 1.5).matrix()
    n = m["n"]
    # an ND-like ordering is not needed for the bound; a random one exercises fill
    perm = perms(n, 2)[:]
    f = oracle.factorize(m, perm)
    L = f.dense_L()
    A = dense_from_lower(m)
    C = A[np.ix_(perm, perm)]
    E = np.abs(L @ L.T - C)
    c = int(f.colcount.max())
    u = np.finfo(float).eps / 2
    gamma = (c + 1) * u / (1 - (c + 1) * u)
    B = 10 * gamma * (np.abs(L) @ np.abs(L).T)
    assert np.all(E <= B + 1e-300)
    assert int(np.count_nonzero(f.Lx)) == f.nnzL


@pytest.mark.parametrize("part", [0, 1, 2])
def test_solves_against_dense(part):
    m = sparse_haar(G=3, a=1.5)
    n = m["n"]
    perm = perms(n, 2)
    f = oracle.factorize(m, perm)
    L = f.dense_L()
    A = dense_from_lower(m)
    B = np.random.default_rng(3).standard_normal((n, 3))
    X = f.solve(B, part)
    if part == 0:
        ref = np.linalg.solve(A, B)
    elif part == 1:
        ref = np.linalg.solve(L, B[perm])
    else:
        Z = np.linalg.solve(L.T, B)
        ref = np.empty_like(Z)
        ref[perm] = Z
    assert np.allclose(X, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_residual_haar1024():
    """Exactness claim (Section 1): the solve reproduces A x = b to roundoff."""
    w = tiny(5, 1.5)
    m = w.matrix()
    n = m["n"]
    b = w.rhs()
    perm = perms(n, 2)
    f = oracle.factorize(m, perm)
    x = f.solve(b)
    r = oracle.residual(n, m["colptr"], m["rowind"], m["values"], x, b)
    assert r.max() <= 1e-12


def test_gradient_against_finite_differences():
    """loss = 0.5 ||A^-1 b - y*||^2 over the stored lower entries of A; the
    oracle's pattern gradient -(lam_i x_j + lam_j x_i) must match central
    differences of a dense library solve."""
    m = sparse_haar(G=3, a=1.3, seed=5)
    n = m["n"]
    g = np.random.default_rng(1)
    b = g.standard_normal(n)
    ystar = g.standard_normal(n)
    perm = perms(n, 2)
    f = oracle.factorize(m, perm)
    x = f.solve(b)
    lam = f.solve(x - ystar)
    gA = oracle.grad(n, m["colptr"], m["rowind"], lam, x)

    def loss(vals):
        A = dense_from_lower({**m, "values": vals})
        y = np.linalg.solve(A, b)
        return 0.5 * np.sum((y - ystar) ** 2)

    h = 1e-6
    idx = np.random.default_rng(2).choice(m["values"].size, 25, replace=False)
    for e in idx:
        vp = m["values"].copy(); vp[e] += h
        vm = m["values"].copy(); vm[e] -= h
        fd = (loss(vp) - loss(vm)) / (2 * h)
        assert abs(fd - gA[e]) <= 1e-6 * abs(gA[e]) + 1e-8 * np.abs(gA).max()


def test_gradient_against_torch_autograd():
    torch = pytest.importorskip("torch")
    m = random_sparse_spd(40, 3, 21)
    n = m["n"]
    g = np.random.default_rng(4)
    b = g.standard_normal(n)
    ystar = g.standard_normal(n)
    f = oracle.factorize(m, perms(n, 1))
    x = f.solve(b)
    lam = f.solve(x - ystar)
    gA = oracle.grad(n, m["colptr"], m["rowind"], lam, x)
    cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    v = torch.tensor(m["values"], dtype=torch.float64, requires_grad=True)
    A = torch.zeros(n, n, dtype=torch.float64)
    A = A.index_put((torch.tensor(m["rowind"], dtype=torch.long), torch.tensor(cols)), v)
    A = A + torch.tril(A, -1).T
    y = torch.linalg.solve(A, torch.tensor(b))
    loss = 0.5 * ((y - torch.tensor(ystar)) ** 2).sum()
    loss.backward()
    assert np.allclose(v.grad.numpy(), gA, rtol=1e-9, atol=1e-12)


def test_not_spd_reports_column():
    m = random_sparse_spd(30, 3, 2)
    perm = np.arange(30, dtype=np.int32)
    vals = m["values"].copy()
    # negate the diagonal of original column 7: pivot 7 fails first
    vals[m["colptr"][7]] = -abs(vals[m["colptr"][7]])
    parent, cc, _, _ = oracle.symbolic(30, m["colptr"], m["rowind"], perm)
    Lp, Li = oracle.pattern(30, m["colptr"], m["rowind"], perm, parent, cc)
    with pytest.raises(oracle.OracleError) as e:
        oracle.factor(30, m["colptr"], m["rowind"], vals, perm, Lp, Li)
    assert e.value.code == -4 and e.value.bad_col == 7


def test_partial_factor_columns_are_exact():
    m = sparse_haar(G=3, a=1.5)
    n = m["n"]
    perm = perms(n, 2)
    f = oracle.factorize(m, perm)
    Lx_part = oracle.factor(n, m["colptr"], m["rowind"], m["values"], perm, f.Lp, f.Li, ncols=20)
    k = f.Lp[20]
    assert np.array_equal(Lx_part[:k], f.Lx[:k])


def _path_graph_nd(n):
    """Path 0-1-...-(n-1) with a hand-made nested dissection (middle vertex separators)."""
    A = np.eye(n) * 4
    for i in range(n - 1):
        A[i, i + 1] = A[i + 1, i] = -1
    m = lower_csc(A)
    perm, tree = [], []

    def rec(verts):
        idx = len(tree)
        tree.append(None)
        lo = len(perm)
        if len(verts) <= 2:
            perm.extend(verts)
            tree[idx] = [lo, -1, lo, len(perm), -1, -1]
            return idx
        mid_v = verts[len(verts) // 2]
        left, right = verts[:len(verts) // 2], verts[len(verts) // 2 + 1:]
        c1 = rec(left)
        mid = len(perm)
        c2 = rec(right)
        sep = len(perm)
        perm.append(mid_v)
        tree[idx] = [lo, mid, sep, len(perm), c1, c2]
        return idx

    rec(list(range(n)))
    return m, np.array(perm, np.int32), np.array(tree, np.int32)


def test_check_nd_accepts_valid_and_rejects_invalid():
    m, perm, tree = _path_graph_nd(31)
    assert oracle.check_nd(31, m["colptr"], m["rowind"], perm, tree) == 0
    # swap the root separator vertex with a vertex of V1: edges now cross V1-V2
    bad = perm.copy()
    root = tree[0]
    bad[root[2]], bad[root[0] + 3] = bad[root[0] + 3], bad[root[2]]
    assert oracle.check_nd(31, m["colptr"], m["rowind"], bad, tree) > 0
    assert oracle.check_perm(perm)
    assert not oracle.check_perm(np.zeros(31, np.int32))


def test_nd_ordering_reduces_fill_on_path():
    m, perm, _ = _path_graph_nd(31)
    # a path has no fill in natural order; ND gives at most log-many extra entries
    _, _, nnz_nat, _ = oracle.symbolic(31, m["colptr"], m["rowind"], np.arange(31, dtype=np.int32))
    _, _, nnz_nd, _ = oracle.symbolic(31, m["colptr"], m["rowind"], perm)
    assert nnz_nat == 31 + 30
    assert nnz_nat <= nnz_nd <= nnz_nat + 31 * 5


def test_permutation_preserves_nnz(small_matrix):
    """Fig. 1: the reordering does not change nnz(A) (both triangles)."""
    m = small_matrix
    n = m["n"]
    perm = perms(n, 2)
    iperm = np.empty(n, np.int64); iperm[perm] = np.arange(n)
    cols = np.repeat(np.arange(n), np.diff(m["colptr"]))
    r, c = iperm[m["rowind"]], iperm[cols]
    assert np.unique(np.stack([np.maximum(r, c), np.minimum(r, c)]), axis=1).shape[1] == m["rowind"].size
    assert full_nnz(m) == 1254448


def test_factor_products_compose_to_A():
    """P^T L (L^T P b) = A b: the two factor products of the oracle against its
    symmetric product with the stored matrix (a different code path), and
    P^T L (L^-1 P b) = b against its forward solve."""
    w = tiny(4, 1.5)
    m = w.matrix()
    n = m["n"]
    perm = perms(n, 2)
    f = oracle.factorize(m, perm)
    B = np.random.default_rng(7).standard_normal((n, 3))
    AB = oracle.symv(n, m["colptr"], m["rowind"], m["values"], B)
    X = f.apply(f.apply(B, 2), 1)
    assert np.abs(X - AB).max() <= 1e-12 * np.abs(AB).max()
    Y = f.apply(f.solve(B, 1), 1)
    assert np.abs(Y - B).max() <= 1e-12 * np.abs(B).max()


@pytest.mark.parametrize("part", [1, 2])
def test_factor_products_against_dense(part):
    m = sparse_haar(G=3, a=1.5)
    n = m["n"]
    perm = perms(n, 2)
    f = oracle.factorize(m, perm)
    L = f.dense_L()
    B = np.random.default_rng(4).standard_normal((n, 2))
    X = f.apply(B, part)
    if part == 1:
        ref = np.empty_like(B)
        ref[perm] = L @ B
    else:
        ref = L.T @ B[perm]
    assert np.abs(X - ref).max() <= 1e-13 * np.abs(ref).max()


# ---- theta scheme (Section 5, eq:theta with G = I, L = -K)

def _theta_case(G=3, scale=None):
    m = tiny(G, 1.5).matrix()
    if scale is not None:        # rescale K so that its largest eigenvalue is `scale`
        lmax = np.linalg.eigvalsh(dense_from_lower(m)).max()
        m = dict(m, values=m["values"] * (scale / lmax))
    return m, perms(m["n"], 2)


@pytest.mark.parametrize("theta", [0.5, 0.75, 1.0])
def test_theta_eigenmode_amplification(theta):
    """An eigenvector v of K (K v = lambda v) without forcing decays by the
    closed-form factor rho = (1 - (1 - theta) dt lambda) / (1 + theta dt lambda)
    per step (eigenpairs from a library dense eigensolver)."""
    m, perm = _theta_case()
    n = m["n"]
    lam, V = np.linalg.eigh(dense_from_lower(m))
    dt, nsteps = 0.02, 12
    F = np.zeros((n, nsteps + 1))
    for q in (0, n // 2, n - 1):
        U = oracle.theta_steps(m, perm, theta, dt, F, V[:, q])
        rho = (1 - (1 - theta) * dt * lam[q]) / (1 + theta * dt * lam[q])
        ref = V[:, q][:, None] * rho ** np.arange(nsteps + 1)[None, :]
        assert np.abs(U - ref).max() <= 1e-12, (theta, q)


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_theta_steady_state_is_fixed_point(theta):
    """With constant forcing f the stationary solution u = K^-1 f (library dense
    solve) is reproduced by every step."""
    m, perm = _theta_case()
    n = m["n"]
    f = np.random.default_rng(3).standard_normal(n)
    u = np.linalg.solve(dense_from_lower(m), f)
    U = oracle.theta_steps(m, perm, theta, 0.05, np.repeat(f[:, None], 9, axis=1), u)
    assert np.abs(U - u[:, None]).max() <= 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("theta", [0.5, 0.75])
def test_theta_forcing_weights(theta):
    """From u_0 = 0 a unit impulse of f at t_0 gives u_1 = (1 - theta) dt A^-1 g and
    one at t_1 gives theta dt A^-1 g, A = I + theta dt K (library dense solve):
    the trapezoid-type weights of the forcing."""
    m, perm = _theta_case()
    n = m["n"]
    dt = 0.1
    g = np.random.default_rng(5).standard_normal(n)
    Ainv_g = np.linalg.solve(np.eye(n) + theta * dt * dense_from_lower(m), g)
    for i, wgt in ((0, 1 - theta), (1, theta)):
        F = np.zeros((n, 2))
        F[:, i] = g
        U = oracle.theta_steps(m, perm, theta, dt, F, np.zeros(n))
        assert np.abs(U[:, 1] - wgt * dt * Ainv_g).max() <= 1e-13 * np.abs(Ainv_g).max()


def test_crank_nicolson_is_second_order():
    """theta = 1/2 converges at second order to the exact flow exp(-t K) u_0
    (library matrix exponential): halving dt divides the error at T = 1 by 4
    (K scaled so that dt lambda <= 1/4, the asymptotic regime); theta = 1 is
    first order (ratio 2)."""
    from scipy.linalg import expm
    m, perm = _theta_case(scale=5.0)
    n = m["n"]
    u0 = np.random.default_rng(9).standard_normal(n)
    exact = expm(-dense_from_lower(m)) @ u0
    for theta, order in ((0.5, 4.0), (1.0, 2.0)):
        err = []
        for nsteps in (20, 40, 80):
            U = oracle.theta_steps(m, perm, theta, 1.0 / nsteps, np.zeros((n, nsteps + 1)), u0)
            err.append(np.abs(U[:, -1] - exact).max())
        r1, r2 = err[0] / err[1], err[1] / err[2]
        assert abs(r1 - order) <= 0.1 * order and abs(r2 - order) <= 0.1 * order, (theta, err)
