"""Matrix values of the refinement's residual.

wcs_solve_refined forms the residual with the values it is given, in the
CSR order of the factor's pattern: the same values give the same result bit
for bit whatever ran in between (wcs_spmv with other values), and values of a
nearby matrix with the same pattern are refined against with the factor of
the first one (its residual is the nearby matrix's)."""
import numpy as np
import pytest

import oracle
from workloads import normal_rhs
from tests.test_gpu_parity import dev, prepared

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, FP64, Factor  # noqa: E402


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_residual_values_follow_the_call(prec):
    m, sym, orc = prepared("small", 64, True)
    n, k = m["n"], 8
    cp, ri, va = m["colptr"], m["rowind"], m["values"]
    print(f"case small prec={prec} n={n} k={k}", flush=True)
    B = normal_rhs(n, k, 31)
    vals = dev(va)
    f = Factor(sym, prec, max_nrhs=k)
    f.numeric(vals)
    X0, _ = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    X0 = X0.cpu().numpy()
    assert oracle.residual(n, cp, ri, va, X0, B).max() <= 1e-10
    # other values through wcs_spmv in between: the same refinement again gives
    # the same result, bit for bit
    f.spmv(dev(normal_rhs(n, k, 32)), dev(2.0 * va))
    X1, _ = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    assert np.array_equal(X1.cpu().numpy(), X0)
    # refinement against a nearby matrix of the same pattern (diagonal raised
    # by 0.1%) with the factor of the first: its residual is the nearby matrix's
    col = np.repeat(np.arange(n), np.diff(cp))
    near = va.copy()
    near[ri == col] *= 1.001
    X2, rep = f.solve_refined(dev(B), dev(near), tol=1e-10, max_iter=30)
    X2 = X2.cpu().numpy()
    print(f"nearby matrix: iterations={rep['iterations']} final={rep['final_residual']:.3e}", flush=True)
    assert rep["iterations"] >= 1
    assert oracle.residual(n, cp, ri, near, X2, B).max() <= 1e-10
    assert oracle.residual(n, cp, ri, va, X2, B).max() > 1e-6
    # and the factorization's values once more
    X3, _ = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    assert np.array_equal(X3.cpu().numpy(), X0)
