"""Batches of independent uneven instances (block-diagonal union of analyses).

Host part: the combined analysis must be the analysis of diag(A_0, A_1, ...)
with each block in its own order — checked against the oracle's own symbolic
factorization of the stacked matrix.  GPU part: the batch factor equals every
instance's own factor, matches the oracle, and refinement reaches 1e-10 per
instance and column."""
import numpy as np
import pytest

import oracle
from workloads import batch_instance, block_diagonal, normal_rhs

torch = pytest.importorskip("torch")

from paper_2007_01541_amd import FP32, FP64, Factor, Symbolic  # noqa: E402

# a small uneven batch: tiny grids (2^3, 2^4, 2^5) with the batch's parameter draws
SMALL_IDS = [0, 1, 2, 3, 4, 5]


def small_instances(ids=SMALL_IDS):
    out = []
    for i in ids:
        w = batch_instance(i)
        spec = w.spec
        # shrink the grid so the oracle runs in seconds: J in {3, 4, 5}
        from workloads import WaveletSpec, make_matrix
        small = WaveletSpec(spec.grid_exp - 2, spec.a, spec.s, spec.kind, spec.ell, spec.decay, spec.seed)
        out.append(make_matrix(small))
    return out


def analyses(mats, leaf=16):
    return [Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"], leaf_size=leaf,
                     dense_degree_min=64 if m["n"] < 4096 else 1024) for m in mats]


def test_batch_symbolic_is_block_diagonal_analysis():
    mats = small_instances()
    syms = analyses(mats)
    bs = Symbolic.batch(syms)
    big = block_diagonal(mats)
    info = bs.info
    assert info["nseg"] == len(mats)
    assert np.array_equal(bs.seg_ptr, big["seg_ptr"])
    assert info["n"] == big["n"] and info["nnz_lower"] == big["colptr"][-1]
    parts = [s.export() for s in syms]
    ex = bs.export()
    off = big["seg_ptr"]
    # the permutation is each instance's own, shifted into its block
    assert np.array_equal(ex["perm"], np.concatenate([p["perm"] + off[b] for b, p in enumerate(parts)]))
    # independent check: the oracle's symbolic factorization of the stacked matrix under that permutation
    parent, cc, nnzL, fl = oracle.symbolic(big["n"], big["colptr"], big["rowind"], ex["perm"])
    assert np.array_equal(ex["parent"], parent)
    assert np.array_equal(ex["colcount"], cc)
    assert info["nnz_l"] == nnzL and info["flops"] == fl
    assert info["nnz_l"] == sum(s.info["nnz_l"] for s in syms)
    assert info["nsuper"] == sum(s.info["nsuper"] for s in syms)
    assert info["nlevels"] == max(s.info["nlevels"] for s in syms)
    # separator trees: one per instance, node and position indices shifted
    toff = 0
    rows = []
    for b, p in enumerate(parts):
        t = p["sep_tree"].copy()
        for c in range(4):
            t[:, c] = np.where(t[:, c] < 0, -1, t[:, c] + off[b])
        for c in (4, 5):
            t[:, c] = np.where(t[:, c] < 0, -1, t[:, c] + toff)
        rows.append(t)
        toff += p["sep_tree"].shape[0]
    assert np.array_equal(ex["sep_tree"], np.concatenate(rows))


def test_batch_of_one_equals_single():
    mats = small_instances([2])
    s = analyses(mats)[0]
    b = Symbolic.batch([s])
    for k, v in s.export().items():
        assert np.array_equal(v, b.export()[k]), k
    si, bi = s.info, b.info
    assert si == bi


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_batch_factor_equals_instances(prec):
    mats = small_instances()
    syms = analyses(mats)
    bs = Symbolic.batch(syms)
    big = block_diagonal(mats)
    print(f"batch of {len(mats)} n={big['n']} prec={prec}", flush=True)
    fb = Factor(bs, prec)
    fb.numeric(dev(big["values"]))
    Lp, Li, Lx = fb.export_L()
    off = big["seg_ptr"]
    for b, (m, s) in enumerate(zip(mats, syms)):
        f = Factor(s, prec)
        f.numeric(dev(m["values"]))
        lp, li, lx = f.export_L()
        j0, j1 = off[b], off[b + 1]
        # same kernels on the same fronts: the batch factor is bitwise the instance's factor
        assert np.array_equal(Lp[j0:j1 + 1] - Lp[j0], lp)
        assert np.array_equal(Li[Lp[j0]:Lp[j1]] - j0, li)
        assert np.array_equal(Lx[Lp[j0]:Lp[j1]], lx)
    if prec == FP64:
        # and it is the Cholesky factor of the stacked matrix (oracle, same permutation)
        orc = oracle.factorize(big, bs.export()["perm"])
        from tests.helpers import compare_columns
        worst, scale = compare_columns(Lp, Li, Lx, orc)
        assert worst <= 1e-11 * scale, (worst, scale)


@pytest.mark.gpu
def test_batch_refinement_per_instance():
    mats = small_instances()
    syms = analyses(mats)
    bs = Symbolic.batch(syms)
    big = block_diagonal(mats)
    k = 4
    # per-instance right-hand sides with very different scales, stacked
    Bs = [normal_rhs(m["n"], k, 4100 + b) * 10.0 ** (3 * (b % 3) - 3) for b, m in enumerate(mats)]
    B = np.vstack(Bs)
    f = Factor(bs, FP32, max_nrhs=k)
    vals = dev(big["values"])
    f.numeric(vals)
    X, rep = f.solve_refined(dev(B), vals, tol=1e-10, max_iter=10)
    rel = f.residuals()
    print(f"report {rep} per-instance max {rel.max(axis=1)}", flush=True)
    assert rel.shape == (len(mats), k)
    assert np.all(rel <= 1e-10)
    assert rep["final_residual"] == rel.max()
    # every instance's block solves its own system (oracle residual, FP64)
    Xh = X.cpu().numpy()
    off = big["seg_ptr"]
    for b, m in enumerate(mats):
        xb = Xh[off[b]:off[b + 1]]
        r = oracle.symv(m["n"], m["colptr"], m["rowind"], m["values"], xb) - Bs[b]
        assert np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(Bs[b], axis=0)) <= 1e-10


@pytest.mark.gpu
def test_graph_replay_matches_eager():
    """Recorded factorization and sweeps, replayed several times with other work
    in between and with changing values, give bitwise the eager results."""
    mats = small_instances()
    bs = Symbolic.batch(analyses(mats))
    big = block_diagonal(mats)
    k = 4
    B = dev(np.vstack([normal_rhs(m["n"], k, 4200 + b) for b, m in enumerate(mats)]))
    vals = [dev(big["values"]), dev(big["values"] * 1.25)]
    eager = Factor(bs, FP32, max_nrhs=k)
    ref = []
    for v in vals:
        eager.numeric(v)
        ref.append((eager.export_L()[2], eager.solve(B).cpu().numpy()))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = Factor(bs, FP32, max_nrhs=k)
        g.use_graphs(True)
        for rep in range(5):
            which = (rep // 2) % 2          # same pointer twice (replay), then a new one (record again)
            print(f"replay {rep} values {which}", flush=True)
            junk = torch.randn(1 << 20, device="cuda").sum()    # unrelated eager work between replays
            g.numeric(vals[which])
            X = g.solve(B)
            s.synchronize()
            assert np.array_equal(g.export_L()[2], ref[which][0])
            assert np.array_equal(X.cpu().numpy(), ref[which][1])
            del junk


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_autotune_keeps_factor_exact(prec):
    """Every update kernel variant sums the same products in the same order,
    so the factor is bitwise the same whichever the autotuner picks."""
    mats = small_instances()
    bs = Symbolic.batch(analyses(mats))
    big = block_diagonal(mats)
    vals = dev(big["values"])
    f = Factor(bs, prec)
    f.numeric(vals)
    L0 = f.export_L()[2]
    res = f.autotune(vals)
    print(f"autotune {res}", flush=True)
    assert set(res["tiles"].tolist()) <= {0, 1, 2, 3, 4}
    assert res["ms_tuned"] <= res["ms_default"] + 1e-9
    assert np.array_equal(f.export_L()[2], L0)
    for v in (0, 1, 2, 3, 4):
        f.set_tiles(np.full(bs.info["nlevels"], v, np.int32))
        f.numeric(vals)
        assert np.array_equal(f.export_L()[2], L0), v
