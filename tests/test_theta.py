"""Theta-scheme time stepping over one factor (Section 5, eq:theta, G = I, L = -K).

wcs_theta_matrix builds A = I + theta dt K from K's values on the device and
wcs_theta_steps runs the steps over the factor of A, forming the explicit
part from A itself.  Parity: every step of the whole trajectory (150
Crank-Nicolson steps over [0, 3] with the moving heat-spot forcing) against
the oracle, which applies K directly and factors A on the CPU.  At the
time-stepping workload's size (N = 262144), where the oracle is too slow,
properties that hold at any size: the stationary solution is a fixed point,
and sampled steps satisfy their equation with K (FP64 products) to 1e-10."""
import numpy as np
import pytest

import oracle
import workloads
from workloads import NSTEPS, T_END, THETA, heat_spot_forcing, small_fp64, tiny

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, FP64, Factor, Symbolic  # noqa: E402
from paper_2007_01541_amd.capi import WcsError  # noqa: E402

DT = T_END / NSTEPS


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def case(kind):
    w = small_fp64() if kind == "small" else tiny(5, 1.5)
    m = w.matrix()
    F = heat_spot_forcing(w.spec, np.linspace(0.0, T_END, NSTEPS + 1))
    return m, F


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("kind", ["tiny5", "small"])
def test_theta_steps_match_oracle(kind, prec):
    m, F = case(kind)
    n = m["n"]
    sym = Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"])
    print(f"theta scheme {kind} n={n} prec={prec}: {NSTEPS} steps", flush=True)
    kv = dev(m["values"])
    f = Factor(sym, prec)
    A = f.theta_matrix(kv, THETA, DT)
    # the matrix of the steps: theta dt K on every stored entry, plus 1 on the diagonal
    ref = THETA * DT * m["values"]
    ref[m["colptr"][:-1]] += 1.0
    np.testing.assert_allclose(A.cpu().numpy(), ref, rtol=2e-16, atol=0)
    f.numeric(A)
    u0 = np.zeros(n)
    U, rep = f.theta_steps(A, THETA, DT, dev(F), dev(u0), tol=1e-10)
    U = U.cpu().numpy()
    Uo = oracle.theta_steps(m, sym.export()["perm"], THETA, DT, F, u0)
    err = np.abs(U - Uo).max() / np.abs(Uo).max()
    print(f"  max |U - U_oracle| / max |U_oracle| = {err:.3e}, report {rep}", flush=True)
    assert U.shape == (n, NSTEPS + 1) and np.array_equal(U[:, 0], u0)
    assert err <= (1e-11 if prec == FP64 else 1e-9)
    if prec == FP32:
        assert 1 <= rep["iterations"] <= 3 and rep["final_residual"] <= 1e-10
    else:
        assert rep["iterations"] == 0 and rep["final_residual"] == -1


def test_theta_rejects_bad_arguments():
    m, F = case("tiny5")
    n = m["n"]
    sym = Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"])
    f = Factor(sym, FP64)
    kv = dev(m["values"])
    for theta, dt in ((0.0, DT), (1.5, DT), (0.5, 0.0), (0.5, -1.0)):
        with pytest.raises(WcsError) as e:
            f.theta_matrix(kv, theta, dt)
        assert e.value.code == -1
    A = f.theta_matrix(kv, THETA, DT)
    with pytest.raises(WcsError) as e:                  # no numeric factorization yet
        f.theta_steps(A, THETA, DT, dev(F), dev(np.zeros(n)))
    assert e.value.code == -6
    f.numeric(A)
    with pytest.raises(WcsError) as e:                  # nsteps = 0
        f.theta_steps(A, THETA, DT, dev(F[:, :1]), dev(np.zeros(n)))
    assert e.value.code == -1


def test_theta_full_size_properties():
    w = workloads.theta_scheme()
    m = w.matrix()
    n = m["n"]
    print(f"theta workload {w.name} n={n} nnz={m['colptr'][-1]}", flush=True)
    sym = Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"])
    kv = dev(m["values"])
    fk = Factor(sym, FP64)                       # factor of K: the stationary solution
    fk.numeric(kv)
    fa = Factor(sym, FP64)
    A = fa.theta_matrix(kv, THETA, DT)
    fa.numeric(A)
    nst = 20
    f0 = heat_spot_forcing(w.spec, np.array([0.25]))[:, 0]
    ustar = fk.solve(dev(f0))
    U, _ = fa.theta_steps(A, THETA, DT, dev(np.repeat(f0[:, None], nst + 1, axis=1)), ustar)
    drift = float((U - ustar[:, None]).abs().max() / ustar.abs().max())
    print(f"  stationary solution over {nst} steps: max drift {drift:.3e}", flush=True)
    assert drift <= 1e-10
    # the full trajectory in FP64 and with the FP32 factor + refinement; sampled steps against eq:theta with K
    F = heat_spot_forcing(w.spec, np.linspace(0.0, T_END, NSTEPS + 1))
    Fd = dev(F)
    f32 = Factor(sym, FP32)
    f32.numeric(A)
    U64, _ = fa.theta_steps(A, THETA, DT, Fd, dev(np.zeros(n)))
    U32, rep = f32.theta_steps(A, THETA, DT, Fd, dev(np.zeros(n)), tol=1e-10)
    print(f"  FP32 + refinement report {rep}", flush=True)
    def K(v):        # the oracle's product with K
        return oracle.symv(n, m["colptr"], m["rowind"], m["values"], v)

    for U in (U64, U32):
        Uh = U.cpu().numpy()
        for i in (0, 1, 37, 74, NSTEPS - 1):
            lhs = Uh[:, i + 1] + THETA * DT * K(Uh[:, i + 1])
            rhs = Uh[:, i] - (1 - THETA) * DT * K(Uh[:, i]) + DT * ((1 - THETA) * F[:, i] + THETA * F[:, i + 1])
            rel = float(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))
            assert rel <= 1e-10, (i, rel)
    diff = float((U32 - U64).abs().max() / U64.abs().max())
    print(f"  FP32 + refinement vs FP64 trajectory: {diff:.3e}", flush=True)
    assert diff <= 1e-8
