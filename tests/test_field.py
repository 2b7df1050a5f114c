"""Covariance-form random field samples G^-1 (abar + L X) on the GPU (Section
5.3, eq:CholFastField) against the oracle: the covariance matrix C^G and
the mass matrix G are analysed and factored separately (each its own nested
dissection ordering, Section 6.3), the sample is one product with the
covariance factor and one solve with the mass factor."""
import numpy as np
import pytest

import oracle
from workloads import WaveletSpec, make_matrix, mass_spec, normal_rhs, covariance_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, FP64, Factor, Symbolic, field_sample  # noqa: E402
from paper_2007_01541_amd.capi import WcsError  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


_CACHE = {}


def case(G):
    if G not in _CACHE:
        cov = make_matrix(WaveletSpec(G, 2.0, 0.5, "exp", 0.25, 1.5, 7100 + G))
        mass = make_matrix(mass_spec(G, 7200 + G))
        sc = Symbolic(cov["n"], cov["colptr"], cov["rowind"], coords=cov["coords"], leaf_size=32, dense_degree_min=256)
        sg = Symbolic(mass["n"], mass["colptr"], mass["rowind"], coords=mass["coords"], leaf_size=32,
                      dense_degree_min=256)
        oc = oracle.factorize(cov, sc.export()["perm"])
        og = oracle.factorize(mass, sg.export()["perm"])
        _CACHE[G] = (cov, mass, sc, sg, oc, og)
    return _CACHE[G]


@pytest.mark.parametrize("G", [5, 6])
@pytest.mark.parametrize("k", [1, 4, 64])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_field_sample_matches_oracle(G, k, prec):
    cov, mass, sc, sg, oc, og = case(G)
    n = cov["n"]
    assert not np.array_equal(sc.export()["perm"], sg.export()["perm"])     # two orderings
    print(f"field n={n} k={k} prec={prec}: nnz(L_C)={sc.info['nnz_l']} nnz(L_G)={sg.info['nnz_l']}", flush=True)
    X = normal_rhs(n, k, 31 + k)
    abar = np.sin(np.arange(n) * 0.01)
    fc = Factor(sc, prec, max_nrhs=k)
    fc.numeric(dev(cov["values"]))
    fg = Factor(sg, prec, max_nrhs=k)
    fg.numeric(dev(mass["values"]))
    S = field_sample(fc, fg, dev(X), dev(abar)).cpu().numpy().reshape(n, k)
    ref = oracle.field_sample(oc, og, abar, X).reshape(n, k)
    err = np.abs(S - ref).max() / np.abs(ref).max()
    print(f"  max |sample - oracle| / max|oracle| = {err:.3e}")
    assert err <= (1e-12 if prec == FP64 else 1e-4)
    # a per-sample mean (lda = n) gives the same as the shared one
    S2 = field_sample(fc, fg, dev(X), dev(np.repeat(abar[:, None], k, axis=1))).cpu().numpy().reshape(n, k)
    assert np.array_equal(S, S2)


def test_field_sample_covariance_identity():
    """Unit noise vectors as the samples (X = I, no mean): S S^T equals the
    coefficient covariance G^-1 C^G G^-1 (dense inverses)."""
    cov, mass, sc, sg, _, _ = case(4)
    n = cov["n"]
    fc = Factor(sc, FP64, max_nrhs=n)
    fc.numeric(dev(cov["values"]))
    fg = Factor(sg, FP64, max_nrhs=n)
    fg.numeric(dev(mass["values"]))
    S = field_sample(fc, fg, dev(np.eye(n))).cpu().numpy()

    def dense(m):
        A = np.zeros((n, n))
        A[m["rowind"], np.repeat(np.arange(n), np.diff(m["colptr"]))] = m["values"]
        return A + np.tril(A, -1).T
    Gi = np.linalg.inv(dense(mass))
    ref = Gi @ dense(cov) @ Gi
    assert np.abs(S @ S.T - ref).max() <= 1e-12 * np.abs(ref).max()


def test_field_sample_bad_arguments():
    cov, mass, sc, sg, _, _ = case(5)
    fc = Factor(sc, FP64, max_nrhs=2)
    fg = Factor(sg, FP64, max_nrhs=2)
    X = dev(normal_rhs(cov["n"], 2, 1))
    with pytest.raises(WcsError):
        field_sample(fc, fg, X)                       # no numeric factorization yet
    fc.numeric(dev(cov["values"]))
    fg.numeric(dev(mass["values"]))
    with pytest.raises(WcsError):
        field_sample(fc, fg, dev(normal_rhs(cov["n"], 3, 1)))     # more samples than max_nrhs
    small = case(4)
    fs = Factor(small[3], FP64)
    fs.numeric(dev(small[1]["values"]))
    with pytest.raises(WcsError):
        field_sample(fc, fs, X[:, :1])                # different n
