"""The residual product by groups of rows with one column pattern, against
the oracle's symmetric product: patterns shared by six rows (groups of four
and two), rows with patterns of their own, and rows longer than one work
item's chunk (4,096 entries) in split groups."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import normal_rhs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP64, Factor, Symbolic  # noqa: E402


def lower_csc(A):
    """Lower triangle (diagonal included) of a symmetric scipy matrix as CSC arrays."""
    L = sp.tril(A, format="csc")
    L.sort_indices()
    return L.indptr.astype(np.int64), L.indices.astype(np.int32), L.data.astype(np.float64)


def block_matrix(nblk, bs, dense_blocks, seed):
    """kron(P, ones(bs, bs)) for a random symmetric block pattern P (the rows
    of a block share one pattern), with `dense_blocks` blocks coupled to every
    block; symmetric random values."""
    rng = np.random.default_rng(seed)
    P = sp.random(nblk, nblk, density=4.0 / nblk, random_state=rng, format="csr")
    P = ((P + P.T) != 0).astype(np.float64) + sp.identity(nblk)
    P = P.tolil()
    for d in range(dense_blocks):
        P[d, :] = 1.0
        P[:, d] = 1.0
    P = sp.csr_matrix(P)
    pat = sp.kron(P, np.ones((bs, bs)), format="csr")
    pat.data[:] = 1.0
    V = sp.triu(pat, format="coo")
    vals = rng.standard_normal(V.nnz)
    U = sp.coo_matrix((vals, (V.row, V.col)), shape=pat.shape)
    return (U + sp.triu(U, k=1).T).tocsr()


def random_matrix(n, seed):
    rng = np.random.default_rng(seed)
    R = sp.random(n, n, density=6.0 / n, random_state=rng, format="csr")
    return (R + R.T + sp.diags(rng.standard_normal(n) + 10.0)).tocsr()


def check(A, ks, seed):
    n = A.shape[0]
    colptr, rowind, values = lower_csc(A)
    sym = Symbolic(n, colptr, rowind)
    f = Factor(sym, FP64, max_nrhs=max(ks))
    for k in ks:
        X = normal_rhs(n, k, seed + k)
        Y = f.spmv(torch.as_tensor(X, device="cuda:0"), torch.as_tensor(values, device="cuda:0")).cpu().numpy()
        Yo = oracle.symv(n, colptr, rowind, values, X)
        err = np.abs(Y.reshape(n, k) - Yo.reshape(n, k)).max()
        print(f"n={n} k={k}: max |Y - Yo| = {err:.3e} (max |Yo| {np.abs(Yo).max():.3e})", flush=True)
        assert err <= 1e-13 * np.abs(Yo).max()


@pytest.mark.parametrize("bs", [3, 6])
def test_shared_patterns_and_split_groups(bs):
    # 1,100 blocks of bs rows; two blocks touch every block, so their rows
    # (6,600 entries when bs = 6) are split into chunks
    A = block_matrix(1100, bs, 2, 31 + bs)
    lens = np.diff(A.indptr)
    print(f"bs={bs}: n={A.shape[0]}, longest row {lens.max()}, rows over 4096: {(lens > 4096).sum()}", flush=True)
    check(A, (4, 8, 64), 40)


def test_rows_with_patterns_of_their_own():
    check(random_matrix(3000, 41), (4, 16, 64), 50)
