"""The allocation-free factor (wcs_factor_create_static) against the regular one.

A factor created in the library's static device array must give the same
factor, solves and refined solves as one created in a caller workspace, on
two systems in a row (the second smaller, so stale contents of the array
from the first would show), and both must meet the oracle's residual bar.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from workloads import normal_rhs, tiny

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, FP64, Factor, Symbolic, capi  # noqa: E402
from paper_2007_01541_amd.capi import WcsError  # noqa: E402

STATIC_BYTES = 64 << 20


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def system(G, seed):
    m = tiny(G, 1.5, seed=seed).matrix()
    sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"], leaf_size=16, dense_degree_min=64)
    return m, sym


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_static_factor_matches_workspace_factor(prec):
    k = 8
    for G, seed in ((5, 71), (4, 72)):           # N = 1024, then N = 256
        m, sym = system(G, seed)
        n = m["n"]
        assert sym.workspace_size(prec, k) <= STATIC_BYTES
        print(f"static workspace: n={n} prec={prec} k={k} needs {sym.workspace_size(prec, k)} bytes", flush=True)
        vals = dev(m["values"])
        B = normal_rhs(n, k, seed + 1)
        ref = Factor(sym, prec, max_nrhs=k)
        ref.numeric(vals)
        fs = Factor(sym, prec, max_nrhs=k, static_workspace=True)
        assert fs.workspace is None
        fs.numeric(vals)
        torch.cuda.synchronize()
        assert all(np.array_equal(a, b) for a, b in zip(fs.export_L(), ref.export_L()))
        X = fs.solve(dev(B)).cpu().numpy()
        assert np.array_equal(X, ref.solve(dev(B)).cpu().numpy())
        Xr, rep = fs.solve_refined(dev(B), vals, tol=1e-10)
        Xr2, rep2 = ref.solve_refined(dev(B), vals, tol=1e-10)
        assert np.array_equal(Xr.cpu().numpy(), Xr2.cpu().numpy()) and rep == rep2
        res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], Xr.cpu().numpy(), B)
        res_direct = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X, B)
        print(f"  n={n}: refined residual {res.max():.3e}, direct {res_direct.max():.3e}", flush=True)
        assert res.max() <= 1e-10
        if prec == FP64:
            assert res_direct.max() <= 1e-12
        del fs, ref


def test_static_factor_one_per_device_and_size_limit():
    m, sym = system(4, 73)
    a = Factor(sym, FP64, static_workspace=True)
    with pytest.raises(WcsError) as e:
        Factor(sym, FP64, static_workspace=True)      # the array is held by `a`
    assert e.value.code == -6
    del a
    b = Factor(sym, FP64, static_workspace=True)      # released by the free
    b.numeric(dev(m["values"]))
    del b
    big = tiny(6, 1.5, seed=74).matrix()              # N = 4096: above the static size
    sb = Symbolic(big["n"], big["colptr"], big["rowind"], coords=big["coords"])
    assert sb.workspace_size(FP64, 1) > STATIC_BYTES
    h = C.c_void_p()
    rc = capi.lib().wcs_factor_create_static(sb.handle, FP64, 1, None, C.byref(h))
    assert rc == -2 and not h.value
    assert "static workspace too small" in capi.lib().wcs_last_error().decode()
