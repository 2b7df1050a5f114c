#!/usr/bin/env python3
"""Benchmark of the sparse Cholesky hot path on one MI355X.

Workload (default): the 512 x 512 Haar grid, N = 2^18, a = 2, s = 0.75,
algebraic decay, 64 right-hand sides.  One step is the whole path on inputs
already resident in HBM: value load into the fronts, numeric factorization,
and the solve of all 64 right-hand sides to relative residual 1e-10 — in
FP32 on the matrix cores with FP64 iterative refinement (the measured path),
and the same step with the plain FP64 factor for comparison.  The ordering
and symbolic analysis (host, once per pattern) are outside the timed region.

Prints one JSON line (metric, value = factor TFLOP/s of the FP32+IR path from
the symbolic flop count sum(colcount^2), ...), with a roofline object for the
dominant kernel (per-launch HIP events on the launch stream) and the CPU
oracle timed on a bounded sample of the same factorization.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma_tflops": 157.3, "fp64_mfma_tflops": 78.6, "hbm_gbs": 8000.0}
METRIC = "factor TFLOP/s + % MFMA peak, N=2^18: FP32+IR vs FP64 at resid 1e-10"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "update_fp32_headline_hbm_traffic.txt")
# the update kernels' source: their own file and the definitions it includes
KERNEL_SRC = [os.path.join(ROOT, "paper_2007_01541_amd", "csrc", f) for f in ("common.h", "update.h")]


def update_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the FP32 update kernel class from the committed
    counter summary, or None when the update kernels' source changed since."""
    try:
        fields = dict(l.split(": ", 1) for l in open(TRAFFIC_FILE).read().splitlines() if ": " in l)
        src = update_source_sha256()
    except OSError:
        return None
    if fields.get("update_source_sha256", "").strip() != src:
        return None
    return float(fields["traffic_bytes_per_launch"])


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def sample_flops(Lp, Li, ncols: int) -> float:
    """Exact flops the left-looking oracle performs for its first ncols columns
    (sqrt and divisions of those columns, 2 per multiply-add of every update
    they receive), in the same counting as sum(colcount^2)."""
    import numpy as np
    total = float(Lp[ncols] - Lp[0])              # one sqrt or division per entry of the sample columns
    for k in range(ncols):
        rows = Li[Lp[k] + 1:Lp[k + 1]]
        c = rows.size
        t = np.searchsorted(rows, ncols)          # off-diagonal rows that are sample columns
        # an update into column rows[i] touches the c - i rows at or below it
        total += 2.0 * float(np.sum(c - np.arange(t)))
    return total


def cpu_baseline(m, perm, target_seconds: float, analysis=None, X=None, B=None) -> dict:
    """The oracle on the host: its symbolic analysis of the same ordering
    (compared with the library's, `analysis` = (export dict, info dict)), the
    true residual of the GPU solution X of A X = B formed with the oracle's
    product on four of its columns, and the timed sample of its numeric
    factorization."""
    import numpy as np
    import oracle
    n = m["n"]
    t0 = time.perf_counter()
    parent, cc, nnzL, flops = oracle.symbolic(n, m["colptr"], m["rowind"], perm)
    Lp, Li = oracle.pattern(n, m["colptr"], m["rowind"], perm, parent, cc)
    log(f"oracle symbolic+pattern {time.perf_counter() - t0:.1f}s")
    checks = {}
    if analysis is not None:
        ex, inf = analysis
        same = (np.array_equal(ex["parent"], parent) and np.array_equal(ex["colcount"], cc)
                and inf["nnz_l"] == nnzL and inf["flops"] == flops)
        log(f"analysis vs oracle symbolic: {'bit-exact' if same else 'MISMATCH'}")
        assert same, "symbolic analysis differs from the oracle"
        checks["symbolic_bit_exact"] = True
    if X is not None:
        cols = np.linspace(0, X.shape[1] - 1, min(4, X.shape[1])).astype(int)
        res = oracle.residual(n, m["colptr"], m["rowind"], m["values"], X[:, cols], B[:, cols])
        checks["oracle_true_residual"] = float(res.max())
        log(f"oracle residual of the FP32+IR solution (columns {cols.tolist()}): {res.max():.3e}")
    # first a short calibration, then a sample sized for the target time from
    # the flops the oracle actually performs on a leading block of columns
    cum = np.cumsum(cc.astype(np.float64) ** 2)
    k_cal = min(int(np.searchsorted(cum, 2e9)) + 1, n)
    t0 = time.perf_counter()
    oracle.factor(n, m["colptr"], m["rowind"], m["values"], perm, Lp, Li, ncols=k_cal)
    t_cal = time.perf_counter() - t0
    k, t = k_cal, t_cal
    for _ in range(3):                            # re-size from the last measured rate until the sample is long enough
        if t >= 0.6 * target_seconds or k == n:
            break
        want = sample_flops(Lp, Li, k) / max(t, 1e-3) * target_seconds
        lo, hi = k, n
        while lo < hi:                            # smallest k whose sample reaches the target flops
            mid = (lo + hi) // 2
            if sample_flops(Lp, Li, mid) >= want:
                hi = mid
            else:
                lo = mid + 1
        k = lo
        t0 = time.perf_counter()
        oracle.factor(n, m["colptr"], m["rowind"], m["values"], perm, Lp, Li, ncols=k)
        t = time.perf_counter() - t0
    fl = sample_flops(Lp, Li, k)
    log(f"oracle sample: {k} leading pivot columns, {fl / 1e9:.1f} GFLOP in {t:.1f}s")
    return dict({"value": fl / t / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
                 "sample": f"left-looking FP64 factorization of the first {k} of {n} pivot columns "
                           f"(nested dissection order) of the same matrix: {fl:.4g} flops in {t:.2f} s, "
                           f"single thread"}, **checks)


def bench_batch(args) -> int:
    """Many uneven instances factored and solved together: grid side 2^J with J
    uniform in {5,6,7}, 4 right-hand sides each, FP32 factor + FP64 refinement
    per instance to the tolerance, update tiles from the autotuner, factor and
    sweeps replayed from HIP graphs.  Also times the same instances factored
    one after another (eager, one handle each) for comparison."""
    import numpy as np
    import workloads
    t0 = time.perf_counter()
    mats = workloads.batch_matrices(args.instances, workers=8)     # forked workers: before any GPU work
    log(f"generated {len(mats)} instances in {time.perf_counter() - t0:.1f}s")
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2007_01541_amd import FP32, Factor, Symbolic
    t0 = time.perf_counter()
    with ThreadPoolExecutor(8) as ex:
        syms = list(ex.map(lambda m: Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"]), mats))
    t_an = time.perf_counter() - t0
    t0 = time.perf_counter()
    bs = Symbolic.batch(syms)
    info = bs.info
    t_comb = time.perf_counter() - t0
    log(f"analyze {t_an:.1f}s (8 threads), combine {t_comb:.1f}s: n={info['n']} nnz(L)={info['nnz_l']} "
        f"flops={info['flops']:.4e} fronts={info['nsuper']} levels={info['nlevels']}")
    ws = workloads.batch(args.instances)
    k = 4
    B = np.vstack([workloads.normal_rhs(m["n"], k, w.seed + 1) for m, w in zip(mats, ws)])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    vals = torch.as_tensor(np.concatenate([m["values"] for m in mats]), device=dev)
    Bd = torch.as_tensor(B, device=dev)
    F = float(info["flops"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        f = Factor(bs, FP32, max_nrhs=k)
        log(f"workspace {f.workspace.numel() / 2**30:.1f} GiB")
        f.numeric(vals)
        tune = f.autotune(vals)
        log(f"autotune: tiles per level {tune['tiles'].tolist()}, level sum {tune['ms_default']:.2f} ms with "
            f"128x128 -> {tune['ms_tuned']:.2f} ms")
        f.use_graphs(True)
        reps = []

        def step():
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            f.numeric(vals, check_pivots=False)
            e1.record(stream)
            X, rep = f.solve_refined(Bd, vals, tol=args.tol, max_iter=10)
            reps.append(rep)
            return e0, e1
        for _ in range(args.warmup):
            step()
        stream.synchronize()
        reps.clear()
        t0 = time.perf_counter()
        evs = [step() for _ in range(args.steps)]
        stream.synchronize()
        t_step = (time.perf_counter() - t0) / args.steps
        fact_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        assert f.pivot_check() == -1
        rel = f.residuals()
        log(f"{args.steps} steps: {t_step * 1e3:.1f} ms/step, factor {fact_ms:.2f} ms ({F / fact_ms / 1e9:.1f} "
            f"TFLOP/s), refinement {reps[-1]}, worst instance residual {rel.max():.3e}")
        del f
        torch.cuda.empty_cache()
        # the same instances one after another, each with its own handle (eager launches)
        one = []
        for s_, m in zip(syms, mats):
            fi = Factor(s_, FP32, max_nrhs=k)
            one.append((fi, torch.as_tensor(m["values"], device=dev)))
        for fi, v in one:
            fi.numeric(v, check_pivots=False)
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for fi, v in one:
            fi.numeric(v, check_pivots=False)
        e1.record(stream)
        stream.synchronize()
        seq_ms = e0.elapsed_time(e1)
        log(f"one instance at a time: factor {seq_ms:.2f} ms")
    out = {
        "metric": "batched factor TFLOP/s, 256 uneven instances (FP32 + FP64 refinement per instance to 1e-10)",
        "value": F / fact_ms / 1e9, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch{args.instances}_J5-7_nrhs4", "instances": args.instances, "n": info["n"],
                   "nnz_lower": info["nnz_lower"], "nnz_l": info["nnz_l"], "flops": info["flops"],
                   "fronts": info["nsuper"], "levels": info["nlevels"]},
        "factor_ms": fact_ms, "sequential_factor_ms": seq_ms, "batching_speedup": seq_ms / fact_ms,
        "autotune": {"tiles": tune["tiles"].tolist(), "ms_128": tune["ms_default"], "ms_tuned": tune["ms_tuned"]},
        "ir": reps[-1], "worst_instance_residual": float(rel.max()),
        "host": {"analyze_s": round(t_an, 2), "combine_s": round(t_comb, 2)},
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_theta(args) -> int:
    """Time stepping over one factor (Section 6, parabolic problem): A = I +
    theta dt K with theta = 1/2 (Crank-Nicolson), 150 steps over [0, 3] of the
    moving heat-spot forcing, one trajectory, N = 262144, s = 3/8.  A step of
    this line is one whole trajectory (150 SpMVs + 150 solves) with A factored
    beforehand (its factorization is reported beside).  The FP64 factor (as in
    the paper) gives the value; the FP32 factor with every step refined to the
    tolerance is reported beside it."""
    import numpy as np
    import torch
    import workloads
    from workloads import NSTEPS, T_END, THETA
    from paper_2007_01541_amd import FP32, FP64, Factor, Symbolic
    w = workloads.theta_scheme()
    t0 = time.perf_counter()
    m = w.matrix()
    n = m["n"]
    F = workloads.heat_spot_forcing(w.spec, np.linspace(0.0, T_END, NSTEPS + 1))
    log(f"{w.name}: generated in {time.perf_counter() - t0:.1f}s, nnz_lower={m['colptr'][-1]}")
    t0 = time.perf_counter()
    sym = Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"])
    t_an = time.perf_counter() - t0
    info = sym.info
    dt = T_END / NSTEPS
    if args.graphs:     # recording needs a created stream
        torch.cuda.set_stream(torch.cuda.Stream())
    kv = torch.as_tensor(m["values"], device="cuda")
    Fd = torch.as_tensor(F, device="cuda")
    u0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    res = {}
    for prec, nm in ((FP64, "fp64"), (FP32, "fp32_ir")):
        f = Factor(sym, prec)
        A = f.theta_matrix(kv, THETA, dt)
        f.numeric(A)
        if args.graphs:
            f.use_graphs(True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        f.numeric(A, check_pivots=False)
        e1.record()
        torch.cuda.synchronize()
        fact_ms = e0.elapsed_time(e1)
        for _ in range(args.warmup):
            f.theta_steps(A, THETA, dt, Fd, u0, tol=args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            U, rep_ = f.theta_steps(A, THETA, dt, Fd, u0, tol=args.tol)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        res[nm] = {"trajectory_ms": t * 1e3, "ms_per_time_step": t * 1e3 / NSTEPS, "factor_ms": fact_ms,
                   "report": rep_, "u_final_norm": float(torch.linalg.norm(U[:, -1]))}
        log(f"  {nm}: factor {fact_ms:.2f} ms, {NSTEPS} steps in {t * 1e3:.1f} ms "
            f"({t * 1e3 / NSTEPS:.3f} ms per step), report {rep_}")
        del f, A
        torch.cuda.empty_cache()
    out = {
        "metric": "theta-scheme time steps/s (150 Crank-Nicolson steps over one FP64 factor, one trajectory)",
        "value": NSTEPS / (res["fp64"]["trajectory_ms"] / 1e3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["fp64"]["trajectory_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n": n, "nnz_lower": int(m["colptr"][-1]), "nnz_l": int(info["nnz_l"]),
                   "theta": THETA, "t_end": T_END, "time_steps": NSTEPS, "analyze_s": round(t_an, 2)},
        "fp64": res["fp64"], "fp32_ir": res["fp32_ir"], "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def lu_flops(colcount) -> float:
    """Flops of LU without pivoting on the Cholesky pattern: column j (count
    c_j, diagonal included) takes c_j - 1 divisions and a rank-one update of
    the (c_j - 1)^2 entries below and right of its pivot (2 flops each)."""
    import numpy as np
    c = np.asarray(colcount, np.float64)
    return float(np.sum((c - 1.0) * (2.0 * c - 1.0)))


def lu_sample_flops(Lp, Li, ncols: int) -> float:
    """Flops of the oracle's left-looking LU over its first ncols columns:
    pivot t < ncols contributes its c_t - 1 divisions and, for every row j of
    its column with j < ncols (a column of U it updates), 2 (c_t - 1) flops."""
    import numpy as np
    total = 0.0
    for t in range(ncols):
        rows = Li[Lp[t] + 1:Lp[t + 1]]
        c1 = rows.size
        total += c1 + 2.0 * c1 * int(np.searchsorted(rows, ncols))
    return total


def bench_lu(args) -> int:
    """LU of the nonsymmetric PCM stand-in (Section 5.1, eq:PCM2) on the
    nested dissection ordering of its symmetric pattern, FP64: value load and
    factorization timed with HIP events, then the solve of the right-hand
    sides; the oracle's left-looking LU timed on the leading pivot columns."""
    import numpy as np
    import torch
    import oracle
    import workloads
    from paper_2007_01541_amd import LU64, Factor, Symbolic
    w = workloads.pcm_lu(args.grid, 8)
    t0 = time.perf_counter()
    m = w.matrix()
    n = m["n"]
    B = w.rhs()
    log(f"{w.name}: generated in {time.perf_counter() - t0:.1f}s, nnz_lower={m['colptr'][-1]}")
    t0 = time.perf_counter()
    sym = Symbolic(n, m["colptr"], m["rowind"], coords=m["coords"])
    t_an = time.perf_counter() - t0
    ex = sym.export()
    F = lu_flops(ex["colcount"])
    log(f"analyze {t_an:.1f}s: nnz(L) = nnz(U) = {sym.info['nnz_l']}, LU flops {F:.4e}")
    lo = torch.as_tensor(m["values"], device="cuda")
    up = torch.as_tensor(m["upper"], device="cuda")
    Bd = torch.as_tensor(B, device="cuda")
    f = Factor(sym, LU64, max_nrhs=w.nrhs)
    log(f"LU workspace {f.workspace.numel() / 2**30:.1f} GiB")
    for _ in range(args.warmup):
        f.numeric_lu(lo, up)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    fact, sol = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        f.numeric_lu(lo, up, check_pivots=False)
        e1.record(stream)
        X = f.solve(Bd)
        e2.record(stream)
        torch.cuda.synchronize()
        fact.append(e0.elapsed_time(e1))
        sol.append(e1.elapsed_time(e2))
    t_step = (time.perf_counter() - t0) / args.steps
    f.numeric_lu(lo, up)          # pivot check
    fact_ms, sol_ms = float(np.median(fact)), float(np.median(sol))
    log(f"  LU factor {fact_ms:.2f} ms ({F / fact_ms / 1e9:.1f} TFLOP/s), solve of {w.nrhs} RHS {sol_ms:.2f} ms")
    cpu = None
    Xh = X.cpu().numpy()
    res = float(oracle.gemv_residual(n, m["colptr"], m["rowind"], m["values"], m["upper"], Xh, B).max())
    log(f"  residual of the LU solution (oracle product): {res:.3e}")
    if not args.no_cpu_baseline:
        parent, cc, _, _ = oracle.symbolic(n, m["colptr"], m["rowind"], ex["perm"])
        assert np.array_equal(parent, ex["parent"]) and np.array_equal(cc, ex["colcount"])
        Lp, Li = oracle.pattern(n, m["colptr"], m["rowind"], ex["perm"], parent, cc)
        cum = np.cumsum((cc.astype(np.float64) - 1) * (2 * cc.astype(np.float64) - 1))
        k = min(int(np.searchsorted(cum, 3e9 * args.cpu_seconds / 20.0)) + 1, n)
        t0 = time.perf_counter()
        oracle.lu(n, m["colptr"], m["rowind"], m["values"], m["upper"], ex["perm"], Lp, Li, ncols=k)
        t = time.perf_counter() - t0
        fl = lu_sample_flops(Lp, Li, k)
        cpu = {"value": fl / t / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"left-looking FP64 LU of the first {k} of {n} pivot columns of the same matrix: "
                         f"{fl:.4g} flops in {t:.2f} s, single thread"}
        log(f"  oracle LU sample: {cpu['sample']}")
    out = {
        "metric": "LU factor TFLOP/s (FP64, nonsymmetric PCM stand-in on the nested dissection ordering)",
        "value": F / fact_ms / 1e9, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n": n, "nnz_lower": int(m["colptr"][-1]), "nnz_l": int(sym.info["nnz_l"]),
                   "lu_flops": F, "nrhs": w.nrhs, "analyze_s": round(t_an, 2)},
        "pct_fp64_mfma_peak": 100 * F / fact_ms / 1e9 / PEAK["fp64_mfma_tflops"],
        "factor_ms": fact_ms, "solve_ms": sol_ms, "residual": res, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_field(args) -> int:
    """Random field samples in covariance form (Section 5.3,
    eq:CholFastField): the covariance matrix and the mass matrix analysed
    and factored separately, then batches of samples G^-1 (abar + L X); the
    factors are set up once, the samples are the timed work (the paper times
    one sample, averaged over 1000)."""
    import numpy as np
    import torch
    import workloads
    from paper_2007_01541_amd import FP32, FP64, Factor, Symbolic, field_sample
    w = workloads.covariance_field(args.grid + 1 if args.grid else 9)
    t0 = time.perf_counter()
    mc, mg = w.cov_matrix(), w.mass_matrix()
    n = w.n
    log(f"{w.name}: generated in {time.perf_counter() - t0:.1f}s; nnz_lower C {mc['colptr'][-1]}, G {mg['colptr'][-1]}")
    t0 = time.perf_counter()
    sc = Symbolic(n, mc["colptr"], mc["rowind"], coords=mc["coords"])
    sg = Symbolic(n, mg["colptr"], mg["rowind"], coords=mg["coords"])
    t_an = time.perf_counter() - t0
    log(f"analyze {t_an:.1f}s: nnz(L_C) {sc.info['nnz_l']}, nnz(L_G) {sg.info['nnz_l']}")
    vc = torch.as_tensor(mc["values"], device="cuda")
    vg = torch.as_tensor(mg["values"], device="cuda")
    abar = torch.as_tensor(w.mean(), device="cuda")
    res = {}
    for prec, nm in ((FP64, "fp64"), (FP32, "fp32")):
        fc = Factor(sc, prec, max_nrhs=64)
        fg = Factor(sg, prec, max_nrhs=64)
        fc.numeric(vc)
        fg.numeric(vg)
        per = {}
        for k in (1, 64):
            X = torch.as_tensor(w.noise(k), device="cuda")
            for _ in range(max(1, args.warmup)):
                field_sample(fc, fg, X, abar)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = max(3, args.steps)
            e0.record()
            for _ in range(reps):
                S = field_sample(fc, fg, X, abar)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            per[f"k{k}"] = {"ms_per_call": ms, "samples_per_s": k / ms * 1e3,
                            "ms_per_sample": ms / k}
            log(f"  {nm}: {k} sample(s) per call: {ms:.3f} ms ({k / ms * 1e3:.0f} samples/s)")
        res[nm] = per
        del fc, fg
        torch.cuda.empty_cache()
    out = {
        "metric": "random field samples/s (covariance form G^-1 (abar + L X), FP64, one sample per call)",
        "value": res["fp64"]["k1"]["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": max(3, args.steps),
        "warmup": args.warmup, "ms_per_step": res["fp64"]["k1"]["ms_per_call"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n": n, "nnz_lower_cov": int(mc["colptr"][-1]),
                   "nnz_lower_mass": int(mg["colptr"][-1]), "nnz_l_cov": int(sc.info["nnz_l"]),
                   "nnz_l_mass": int(sg.info["nnz_l"]), "analyze_s": round(t_an, 2)},
        "fp64": res["fp64"], "fp32": res["fp32"], "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "medium", "small", "batch", "theta", "lu", "field"])
    ap.add_argument("--grid", type=int, default=8,
                    help="lu workload: grid exponent (2^grid squared cells, N = 4^grid); field: grid + 1")
    ap.add_argument("--instances", type=int, default=256, help="batch workload: number of instances")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default update kernel on every level instead of timing the variants first")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--graphs", action="store_true",
                    help="replay the factorization and the triangular sweeps from HIP graphs")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 1 GiB FP32 tensor three times (a kernel of known traffic for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (sharding the "
              "elimination tree across GPUs is a design note, not code).", file=sys.stderr)
        return 2

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "theta":
        return bench_theta(args)
    if args.workload == "lu":
        return bench_lu(args)
    if args.workload == "field":
        return bench_field(args)

    import numpy as np
    import torch
    import workloads
    from paper_2007_01541_amd import FP32, FP64, Factor, Symbolic

    w = {"headline": workloads.headline, "medium": workloads.medium_fp64, "small": workloads.small_fp64}[args.workload]()
    nrhs = 64 if args.workload == "headline" else w.nrhs
    t0 = time.perf_counter()
    m = w.matrix()
    B = workloads.normal_rhs(w.n, nrhs, w.seed + 1)
    log(f"generated {w.name}: n={m['n']} nnz_lower={m['colptr'][-1]} in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    sym = Symbolic(m["n"], m["colptr"], m["rowind"], coords=m["coords"])
    info = sym.info
    t_analyze = time.perf_counter() - t0
    log(f"analyze {t_analyze:.1f}s: nnz(L)={info['nnz_l']} flops={info['flops']:.4e} fronts={info['nsuper']} "
        f"max front={info['max_front']}")
    F = float(info["flops"])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 copies of 1 GiB done")
    vals = torch.as_tensor(m["values"], device=dev)
    Bd = torch.as_tensor(B, device=dev)
    if args.graphs:     # recording needs a created stream
        torch.cuda.set_stream(torch.cuda.Stream())
    stream = torch.cuda.current_stream()

    tuned = {}

    def run_path(prec, refine):
        f = Factor(sym, prec, max_nrhs=nrhs, device=dev)
        log(f"{'FP32' if prec == FP32 else 'FP64'} workspace {f.workspace.numel() / 2**30:.1f} GiB")
        reports = []
        if not args.no_autotune:
            # setup, like the analysis: time the update kernel variants per tree level
            tune = f.autotune(vals)
            torch.cuda.synchronize()
            tuned[prec] = tune["tiles"].tolist()
            log(f"  autotune: variants per level {tuned[prec]}, levels {tune['ms_default']:.2f} ms with the "
                f"default, {tune['ms_tuned']:.2f} ms tuned")
        if args.graphs:
            f.use_graphs(True)

        def step():
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            f.numeric(vals, check_pivots=False)
            e1.record(stream)
            if refine:
                X, rep = f.solve_refined(Bd, vals, tol=args.tol, max_iter=10)
            else:
                X, rep = f.solve_refined(Bd, vals, tol=args.tol, max_iter=0)
            reports.append(rep)
            return e0, e1, X

        for i in range(args.warmup):
            step()
            torch.cuda.synchronize()
            log(f"  warmup {i} done: {reports[-1]}")
        reports.clear()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs = []
        for i in range(args.steps):
            e0, e1, X = step()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t0
        fact_ms = [a.elapsed_time(b) for a, b in evs]
        bad = f.pivot_check()
        assert bad == -1, f"pivot {bad} failed"
        log(f"  {args.steps} steps: {t_total * 1e3 / args.steps:.1f} ms/step, factor {np.mean(fact_ms):.2f} ms; "
            f"last report {reports[-1]}")
        return f, t_total / args.steps, float(np.mean(fact_ms)), reports[-1], X

    f32, step32, fact32, rep32, X32 = run_path(FP32, True)
    # outside the timed steps: the true residual max_c ||b - A x|| / ||b|| of the last
    # refined solution (the refinement tracks an updated residual, see wcs_solve_refined)
    res_true = torch.linalg.norm(f32.spmv(X32, vals) - Bd, dim=0) / torch.linalg.norm(Bd, dim=0)
    rep32 = dict(rep32, true_residual=float(res_true.max()))
    log(f"  true residual of the last FP32+IR solution: {rep32['true_residual']:.3e}")
    assert rep32["true_residual"] <= args.tol, rep32
    X32_host = X32.cpu().numpy()
    prof = f32.profile(vals)
    torch.cuda.synchronize()
    for st_ in prof.values():      # algorithmic HBM bytes of the bandwidth-bound classes per second
        st_["gbps"] = st_["bytes"] / st_["ms"] / 1e6 if st_["ms"] > 0 else 0.0
    for nm, st in prof.items():
        log(f"  kernel class {nm}: {st['launches']} launches, {st['ms']:.2f} ms, "
            f"{st['flops'] / 1e9:.1f} GFLOP, {st['bytes'] / 1e9:.2f} GB")
    # products with the factor (P^T L B and L^T P B, 64 RHS): 2 nnz(L) k flops each
    from paper_2007_01541_amd import APPLY_L, APPLY_LT
    products = {}
    for nm_, part in (("L", APPLY_L), ("LT", APPLY_LT)):
        f32.apply(Bd, part)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            f32.apply(Bd, part)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        products[nm_] = {"ms": ms, "tflops": 2 * info["nnz_l"] * nrhs / ms / 1e9}
    log(f"  products with the factor ({nrhs} RHS, FP32): " +
        ", ".join(f"{k_} {v['ms']:.2f} ms ({v['tflops']:.1f} TFLOP/s)" for k_, v in products.items()))

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # one FP32 solve of all right-hand sides: flops 2 (2 nnz(L) - n) k; the factor is read once per sweep
    sol_ms = timed(lambda: f32.solve(Bd))
    solve = {"ms": sol_ms, "tflops": 2 * (2 * info["nnz_l"] - w.n) * nrhs / sol_ms / 1e9,
             "factor_gbps": 2 * info["nnz_l"] * 4 / sol_ms / 1e6}
    log(f"  one FP32 solve ({nrhs} RHS): {sol_ms:.2f} ms, {solve['tflops']:.1f} TFLOP/s, "
        f"{solve['factor_gbps']:.0f} GB/s of factor reads")
    # Gaussian random field form on the same operator: sample x = P^T L^-T z, y = A^-1 x (refined),
    # adjoint lambda = A^-1 (y - y*) (refined, same factor), gradient on the stored pattern
    from paper_2007_01541_amd import SOLVE_LT
    zs = torch.as_tensor(workloads.normal_rhs(w.n, 1, w.seed + 3)[:, 0], device=dev)
    ystar = torch.as_tensor(workloads.normal_rhs(w.n, 1, w.seed + 2)[:, 0], device=dev)

    def grf_step():
        x = f32.solve(zs, part=SOLVE_LT)
        y, _ = f32.solve_refined(x, vals, tol=args.tol)
        lam, _ = f32.solve_refined(y - ystar, vals, tol=args.tol)
        return f32.grad_pattern(lam, y)
    grf = {"ms": timed(grf_step)}
    log(f"  random-field sample + refined solve + refined adjoint + pattern gradient (1 RHS): {grf['ms']:.2f} ms")
    levels = f32.profile_levels(vals)
    torch.cuda.synchronize()
    top = levels[-3:]
    root_ms = sum(l["ms"] for l in top)
    root_flops = sum(l["flops"] for l in top)
    root = {"levels": len(top), "schedule": "height in the assembly tree; fronts of >= 1024 pivots one level below "
                                            "their parent", "ms": root_ms, "tflops": root_flops / root_ms / 1e9,
            "pct_fp32_mfma_peak": 100 * root_flops / root_ms / 1e9 / PEAK["fp32_mfma_tflops"],
            "per_level": [{"ms": round(l["ms"], 3), "tflops": round(l["flops"] / max(l["ms"], 1e-9) / 1e9, 2)}
                          for l in levels]}
    log(f"  root-level fronts (top 3 schedule levels): {root_ms:.2f} ms, {root['tflops']:.1f} TFLOP/s "
        f"({root['pct_fp32_mfma_peak']:.1f}% of FP32 MFMA peak)")
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    del f32
    torch.cuda.empty_cache()
    fp64 = None
    if not args.no_fp64:
        f64, step64, fact64, rep64, _ = run_path(FP64, False)
        fp64 = {"ms_per_step": step64 * 1e3, "factor_ms": fact64, "factor_tflops": F / fact64 / 1e9,
                "pct_fp64_mfma_peak": 100 * F / fact64 / 1e9 / PEAK["fp64_mfma_tflops"],
                "final_residual": rep64["final_residual"]}
        del f64
        torch.cuda.empty_cache()

    if d["flops"] > 0:
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp32_mfma_tflops"], "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp32_mfma_tflops"],
                "traffic": measured_traffic() if dom == "update" else None, "kernel": dom,
                "launches": d["launches"], "avg_launch_us": d["ms"] * 1e3 / max(1, d["launches"])}
    else:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                "frac": achieved / PEAK["hbm_gbs"], "traffic": None, "kernel": dom,
                "launches": d["launches"], "avg_launch_us": d["ms"] * 1e3 / max(1, d["launches"])}

    cpu = None
    if not args.no_cpu_baseline:
        ex = sym.export()
        cpu = cpu_baseline(m, ex["perm"], args.cpu_seconds, analysis=(ex, info), X=X32_host, B=B)
        if "oracle_true_residual" in cpu:
            rep32["oracle_true_residual"] = cpu["oracle_true_residual"]
            assert cpu["oracle_true_residual"] <= args.tol

    value = F / fact32 / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": int(m["n"]), "nnz_lower": int(m["colptr"][-1]), "nrhs": nrhs,
                   "nnz_l": int(info["nnz_l"]), "flops": int(info["flops"]), "fronts": int(info["nsuper"]),
                   "max_front": int(info["max_front"]), "analyze_s": round(t_analyze, 2)},
        "pct_fp32_mfma_peak": 100 * value / PEAK["fp32_mfma_tflops"],
        "root_fronts": root,
        "factor_products": products,
        "solve": solve,
        "grf_gradient_step": grf,
        "factor_ms": fact32,
        "ir": rep32,
        "fp64": fp64,
        "speedup_e2e_vs_fp64": (fp64["ms_per_step"] / (step32 * 1e3)) if fp64 else None,
        "kernels": prof,
        "update_variants": {("fp32" if k == FP32 else "fp64"): v for k, v in tuned.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
