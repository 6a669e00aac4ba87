#!/usr/bin/env python3
"""Benchmark of the inversion-based triangular solve on one MI355X.

One step = one pass of the hot path over the workload: invert the n0 x n0
diagonal blocks of L (Alg. Diagonal-Inverter / Alg. RecTriInv) and run the
blocked sweep (Alg. It-Inv-TRSM) for all k right-hand sides, in binary64.
Default workload: n = k = 16384, L with diagonal U[1,2] and strict lower
U[-1,1]/n, B ~ N(0,1), seed 0.  The metric credits n^2 k flops per step.

Prints ONE JSON line.  Also reported in that line:
  roofline      -- the matrix-core GEMM kernel (every product launch of a step),
                   timed live with hipEvents on the solve stream;
  cpu_baseline  -- the CPU oracle (plain forward substitution) on a column
                   sample of the same workload;
  mixed         -- refined bfloat16 / half solves of the same system,
                   compared with the binary64 solve;
  check         -- backward error of the benchmarked X (binary64 residual).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MIXED_TOL = 1e-12   # relative error target of the mixed-precision comparison
METRIC = ("TRSM TFLOP/s (n²k) at n=k=16384; served p50/p99 latency; "
          "mixed vs plain FP64")
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}   # TFLOP/s, dense
KERNEL_SRC = os.path.join(ROOT, "paper_1612_01855_amd", "csrc", "gemm.hpp")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profiles(workload: str, n0: int, large_tiles: bool):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source with the same block size and tile
    policy; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_gemm_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if (d.get("kernel_sha") != kernel_hash() or int(d.get("n0", -1)) != int(n0)
                or bool(d.get("large_tiles", False)) != bool(large_tiles)):
            return None
        return float(d["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(L, B, seconds_hint: float = 15.0):
    """Time the oracle on the first columns of the same B (column sample)."""
    import oracle
    threads = oracle.max_threads()
    k_s = min(B.shape[1], 128 * threads)
    n = L.shape[0]
    t0 = time.perf_counter()
    oracle.trsm(L, B[:, :k_s])
    dt = time.perf_counter() - t0
    return {"value": n * n * k_s / dt / 1e12, "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"n={n}, first k={k_s} of the {B.shape[1]} columns of the same L and B "
                      f"(columns are independent), binary64 forward substitution"}


def serving_bench(args, torch, T, gen, dev, chol=False):
    """Continuous-batching serving: resident factors with cached inverted
    blocks, Poisson arrivals of binary64 solves (binary32 sweeps, binary64
    residuals, refined until each request's own stopping test holds).
    Reports saturation throughput and p50/p99 latency at fixed arrival rates.
    chol: the factors are registered as Cholesky factors and every request
    solves A X = B with A = L L^T."""
    import numpy as np
    nf = args.serve_factors
    sizes = gen.serving_factor_sizes(nf, args.seed + 11)
    n0 = args.serve_n0
    tune = None
    if n0 == 0:
        # the block size from the batch autotuner: one system per factor, k
        # drawn from the requests' width distribution, binary32 sweeps (the
        # server's); timed as graph replays of the batched sweep
        ks = gen.log_uniform_int(gen.rng(args.seed + 13), 1, 512, size=nf)
        t0 = time.perf_counter()
        r = T.trsm_batch_autotune([int(v) for v in sizes], [int(v) for v in ks], T.F32, 3)
        n0 = int(r.n0)
        tune = {"n0": n0, "ms": round(r.ms, 3), "full_inversion_n0": int(r.default_n0),
                "full_inversion_ms": round(r.default_ms, 3), "candidates": int(r.candidates),
                "seconds": round(time.perf_counter() - t0, 1)}
        log(f"serving: batch autotune n0={n0} ({r.ms:.2f} ms per batched sweep; full inversion "
            f"{r.default_ms:.2f} ms), {r.candidates} candidates in {tune['seconds']} s")
        torch.cuda.empty_cache()
    resident = 0
    for n in sizes:
        n0f = min(n0, 512 if chol else n0, 1 << (int(n) - 1).bit_length())
        m = -(-int(n) // n0f)
        per = 12 * int(n) * (int(n) + 4) + 12 * m * n0f * n0f + 4096
        resident += per + (12 * int(n) * (int(n) + 4) + 4 * m * n0f * n0f if chol else 0)
    budget = resident + (6 << 30)
    srv = T.trsm_server_create(budget, 512, n0)
    try:
        t0 = time.perf_counter()
        lids = []
        for i, n in enumerate(sizes):
            n = int(n)
            g = torch.Generator(device=dev).manual_seed(args.seed * 7919 + i)
            L = torch.rand((n, n), generator=g, device=dev, dtype=torch.float64)
            L.mul_(2.0).sub_(1.0).mul_(1.0 / n)
            L = torch.tril(L, -1)
            L.diagonal().copy_(torch.rand(n, generator=g, device=dev, dtype=torch.float64) + 1.0)
            torch.cuda.synchronize()
            reg = T.trsm_server_register_chol if chol else T.trsm_server_register_L
            lids.append(reg(srv, L.data_ptr(), n, n))
            del L
        log(f"serving: registered {nf} factors (n in [{int(sizes.min())}, {int(sizes.max())}]) "
            f"in {time.perf_counter() - t0:.1f} s; resident {resident / 2**30:.2f} GiB")

        def make_requests(stream):
            bufs = []
            g = torch.Generator(device=dev).manual_seed(args.seed * 104729 + len(stream))
            for r in stream:
                n = int(sizes[r.factor])
                B = torch.randn((n, r.k), generator=g, device=dev, dtype=torch.float64)
                bufs.append((r, n, B, torch.empty_like(B)))
            torch.cuda.synchronize()
            return bufs

        def drive(bufs, timed_arrivals):
            outstanding = {}
            iters = []
            i = 0
            t_start = time.perf_counter()
            flops = 0.0
            while i < len(bufs) or outstanding:
                now = time.perf_counter() - t_start
                while i < len(bufs) and (not timed_arrivals or bufs[i][0].t_arrival <= now):
                    r, n, B, X = bufs[i]
                    t = T.trsm_serve_submit(srv, lids[r.factor], B.data_ptr(), r.k, r.k,
                                            X.data_ptr(), r.k)
                    outstanding[t] = (n, r.k)
                    i += 1
                for t in list(outstanding):
                    st, status, info = T.trsm_serve_poll(srv, t)
                    if st == T.REQ_DONE:
                        n, k = outstanding.pop(t)
                        if status != T.OK:
                            raise RuntimeError(f"serving request: {T.status_string(status)}")
                        iters.append(info.iterations)
                        flops += (2.0 if chol else 1.0) * float(n) * n * k
                    elif st == T.REQ_ERROR:
                        raise RuntimeError(f"serving request failed: {T.status_string(status)}")
                if i < len(bufs) and timed_arrivals:
                    wait = bufs[i][0].t_arrival - (time.perf_counter() - t_start)
                    if wait > 0:
                        time.sleep(min(wait, 2e-4))
                elif outstanding:
                    time.sleep(5e-5)
            return time.perf_counter() - t_start, iters, flops

        # saturation: everything submitted at once
        sat = gen.request_stream(min(1000, args.serve_requests), 1.0, nf, args.seed + 21)
        bufs = make_requests(sat)
        drive(bufs[:50], False)                       # warm the kernels
        T.trsm_server_reset_stats(srv)
        wall, iters, flops = drive(bufs, False)
        sat_rps = len(bufs) / wall
        st = T.trsm_server_stats(srv)
        log(f"serving: saturation {sat_rps:.0f} requests/s, {flops / wall / 1e12:.2f} TFLOP/s, "
            f"{st.batches} batches, {st.passes} passes, mean corrections {np.mean(iters):.2f}")
        del bufs
        # Poisson streams at fixed fractions of the saturation rate
        sweep = []
        headline = None
        for load in sorted(set([0.25, args.serve_load, 0.75])):
            rate = load * sat_rps
            stream = gen.request_stream(args.serve_requests, rate, nf, args.seed + 31)
            bufs = make_requests(stream)
            T.trsm_server_reset_stats(srv)
            wall, iters, flops = drive(bufs, True)
            st = T.trsm_server_stats(srv)   # latency: submit -> completion, server side
            log(f"serving: {st.completed} requests at {rate:.0f}/s (load {load}): "
                f"p50 {st.p50_us:.0f} us, p99 {st.p99_us:.0f} us, "
                f"{flops / wall / 1e12:.2f} TFLOP/s, {st.batches} batches, {st.passes} passes, "
                f"max in flight {st.max_in_flight}")
            rec = {"load_fraction": load, "rate_hz": round(rate, 1), "requests": int(st.completed),
                   "p50_us": round(st.p50_us, 1), "p99_us": round(st.p99_us, 1),
                   "mean_us": round(st.mean_us, 1),
                   "tflops_n2k": round(flops / wall / 1e12, 4), "batches": int(st.batches),
                   "passes": int(st.passes), "mean_corrections": round(float(np.mean(iters)), 3),
                   "max_in_flight": int(st.max_in_flight)}
            sweep.append(rec)
            if load == args.serve_load:
                headline = rec
            del bufs
        out = {"factors": nf, "n_range": [int(sizes.min()), int(sizes.max())],
               "k_range": [1, 512], "saturation_rps": round(sat_rps, 1),
               "hbm_budget_gib": round(budget / 2**30, 2), "n0_max": n0,
               "n0_source": "batch autotune" if tune else "fixed", "batch_autotune": tune,
               "precision": "binary64 in/out; binary32 sweeps, binary64 residuals, refined per "
                            "request to ||B-LX||_F <= sqrt(n) 2^-53 ||L||_F ||X||_F",
               "problem": "A X = B, A = L L^T (flops 2 n^2 k)" if chol else "L X = B"}
        out.update(headline)
        out["rate_sweep"] = sweep
        return out
    finally:
        T.trsm_server_destroy(srv)


def time_solves(T, torch, dev, L64, B64, precision, n0, flags, reps, invert_each=True):
    """Median milliseconds of (invert + solve) over `reps` runs, plus the plan."""
    import numpy as np
    n, k = B64.shape
    dt = torch.float32 if precision == "f32" else torch.float64
    Ld = L64.to(dt)
    Bd = B64.to(dt)
    Xd = torch.empty_like(Bd)
    s = T.Solver.create(n, k, precision, n0, flags, device=dev)
    rec = bool(flags & T.FLAG_RECURSIVE)
    if not rec:
        s.invert(Ld)
    s.solve(Ld, Bd, Xd)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if not rec and invert_each:
            s.invert(Ld)
        s.solve(Ld, Bd, Xd)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    info = s.info
    s.close()
    del Ld, Bd
    return float(np.median(times)), info, Xd


def cholesky_bench(args, torch, T, gen, dev, emit):
    """Blocked Cholesky A = L L^T (binary64) with the inverted-block panel
    solve: median of 3 timed factorizations after a warm one, flops n^3 / 3,
    and the backward error ||A - L L^T|| / ||A|| on 64 sampled rows."""
    sizes = (args.chol_n,) if args.chol_n else (4096, 8192, 16384)
    blocks = (args.chol_nb,) if args.chol_nb is not None else (0, 128, 256, 512, 1024)
    for n in sizes:
        A0 = gen.spd_on(torch, dev, n, args.seed)
        for nb in blocks:
            if nb > n // 4:
                continue
            c = T.Cholesky(n, nb, device=dev)
            A = torch.empty_like(A0)
            times = []
            for it in range(4):
                A.copy_(A0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                c.factor(A)
                e1.record()
                torch.cuda.synchronize()
                if it:
                    times.append(e0.elapsed_time(e1))
            st, idx = c.check()
            gcpu = torch.Generator().manual_seed(args.seed)
            rows = torch.randint(0, n, (64,), generator=gcpu).to(dev)
            L = torch.tril(A)
            R = A0[rows] - L[rows] @ L.t()
            be = float(torch.linalg.norm(R).item() / torch.linalg.norm(A0[rows]).item())
            ms = sorted(times)[1]
            tf = float(n) ** 3 / 3.0 / (ms * 1e-3) / 1e12
            emit({"suite": "cholesky", "n": n, "nb": int(c.nb), "auto": nb == 0,
                  "ms": round(ms, 3), "tflops_n3_3": round(tf, 2),
                  "frac_peak": round(tf / PEAK["f64"], 4), "status": T.status_string(st),
                  "sampled_backward_error": be})
            log(f"suite cholesky n={n} nb={c.nb}: {ms:.2f} ms {tf:.2f} TF backward {be:.2e}")
            del c, A, L, R
        del A0
        torch.cuda.empty_cache()


def lu_bench(args, torch, T, gen, dev, emit):
    """Blocked LU without row exchanges (binary64) on strictly column
    diagonally dominant matrices: median of 3 timed factorizations after a warm
    one, flops 2 n^3 / 3, backward error ||A - L U|| / ||A|| on 64 sampled
    rows."""
    sizes = (args.chol_n,) if args.chol_n else (4096, 8192, 16384)
    blocks = (args.chol_nb,) if args.chol_nb is not None else (0, 128, 256, 512)
    for n in sizes:
        A0 = gen.diag_dominant_on(torch, dev, n, args.seed)
        for nb in blocks:
            if nb > n // 4:
                continue
            f = T.LU(n, nb, device=dev)
            A = torch.empty_like(A0)
            times = []
            for it in range(4):
                A.copy_(A0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                f.factor(A)
                e1.record()
                torch.cuda.synchronize()
                if it:
                    times.append(e0.elapsed_time(e1))
            st, idx = f.check()
            gcpu = torch.Generator().manual_seed(args.seed)
            rows = torch.randint(0, n, (64,), generator=gcpu).to(dev)
            Ar = A.index_select(0, rows)
            cols = torch.arange(n, device=dev)
            Lr = torch.where(cols[None, :] < rows[:, None], Ar, torch.zeros_like(Ar))
            Lr.scatter_(1, rows[:, None], 1.0)           # rows of L: unit diagonal
            R = A0.index_select(0, rows) - Lr @ torch.triu(A)
            be = float(torch.linalg.norm(R).item() / torch.linalg.norm(A0.index_select(0, rows)).item())
            ms = sorted(times)[1]
            tf = 2.0 * float(n) ** 3 / 3.0 / (ms * 1e-3) / 1e12
            emit({"suite": "lu_nopiv", "n": n, "nb": int(f.nb), "auto": nb == 0,
                  "ms": round(ms, 3), "tflops_2n3_3": round(tf, 2),
                  "frac_peak": round(tf / PEAK["f64"], 4), "status": T.status_string(st),
                  "sampled_backward_error": be})
            log(f"suite lu n={n} nb={f.nb}: {ms:.2f} ms {tf:.2f} TF backward {be:.2e}")
            del f, A, Ar, Lr, R
        del A0
        torch.cuda.empty_cache()


def lu_piv_bench(args, torch, T, gen, dev, emit):
    """Blocked LU with partial pivoting (binary64) on Gaussian random matrices
    (no diagonal dominance: exchanges happen at nearly every step): median of
    3 timed factorizations after a warm one, flops 2 n^3 / 3, backward error
    ||P A - L U|| / ||P A|| on 64 sampled rows of P A."""
    sizes = (args.chol_n,) if args.chol_n else (4096, 8192, 16384)
    blocks = (args.chol_nb,) if args.chol_nb is not None else (0, 256, 512)
    for n in sizes:
        g = torch.Generator(device=dev).manual_seed(args.seed + n)
        A0 = torch.randn((n, n), generator=g, device=dev, dtype=torch.float64)
        for nb in blocks:
            f = T.LUPiv(n, nb, device=dev)
            if nb and f.nb != nb:
                continue
            A = torch.empty_like(A0)
            times = []
            for it in range(4):
                A.copy_(A0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                f.factor(A)
                e1.record()
                torch.cuda.synchronize()
                if it:
                    times.append(e0.elapsed_time(e1))
            st, idx = f.check()
            # rows of P A: apply the exchanges to a copy of A0
            PA = A0.clone()
            f.apply(PA)
            gcpu = torch.Generator().manual_seed(args.seed)
            rows = torch.randint(0, n, (64,), generator=gcpu).to(dev)
            Ar = A.index_select(0, rows)
            cols = torch.arange(n, device=dev)
            Lr = torch.where(cols[None, :] < rows[:, None], Ar, torch.zeros_like(Ar))
            Lr.scatter_(1, rows[:, None], 1.0)
            R = PA.index_select(0, rows) - Lr @ torch.triu(A)
            be = float(torch.linalg.norm(R).item() / torch.linalg.norm(PA.index_select(0, rows)).item())
            ms = sorted(times)[1]
            tf = 2.0 * float(n) ** 3 / 3.0 / (ms * 1e-3) / 1e12
            emit({"suite": "lu_piv", "n": n, "nb": int(f.nb), "auto": nb == 0,
                  "ms": round(ms, 3), "tflops_2n3_3": round(tf, 2),
                  "frac_peak": round(tf / PEAK["f64"], 4), "status": T.status_string(st),
                  "sampled_backward_error": be})
            log(f"suite lu_piv n={n} nb={f.nb}: {ms:.2f} ms {tf:.2f} TF backward {be:.2e}")
            del f, A, Ar, Lr, R, PA
        del A0
        torch.cuda.empty_cache()


def run_suite(args, torch, T, gen, dev):
    """The workload sweeps: n0 sweep and the recursive baseline at n = k = 8192
    (binary64 and binary32), the n/k sweep at n = 16384, and the hard factor in
    mixed precision.  One JSON line per measurement."""
    out = []

    def emit(rec):
        print(json.dumps(rec), flush=True)
        out.append(rec)

    # n0 sweep at n = k = 8192 (easy L), plus the recursive baseline
    n = k = 8192
    L, B = gen.easy_system(n, k, args.seed)
    L64 = torch.from_numpy(L).to(dev)
    B64 = torch.from_numpy(B).to(dev)
    del L, B
    for prec in ("f64", "f32"):
        peak = PEAK[prec]
        for n0 in (64, 128, 256, 512, 1024, 8192, 0):
            ms, info, _ = time_solves(T, torch, dev, L64, B64, prec, n0, 0, 3)
            tf = float(n) * n * k / (ms * 1e-3) / 1e12
            emit({"suite": "n0_sweep", "n": n, "k": k, "precision": prec,
                  "n0": int(info.n0), "auto": n0 == 0, "ms": round(ms, 3),
                  "tflops_n2k": round(tf, 2), "frac_peak": round(tf / peak, 4),
                  "inversion_flops_share": round(info.inv_flops / info.solve_flops, 5)})
            log(f"suite n0 {prec} n0={info.n0}: {ms:.2f} ms {tf:.2f} TF")
        ms, info, _ = time_solves(T, torch, dev, L64, B64, prec, 0, T.FLAG_RECURSIVE, 2)
        tf = float(n) * n * k / (ms * 1e-3) / 1e12
        emit({"suite": "recursive_baseline", "n": n, "k": k, "precision": prec,
              "leaf": 64, "ms": round(ms, 3), "tflops_n2k": round(tf, 2),
              "frac_peak": round(tf / peak, 4)})
        log(f"suite recursive {prec}: {ms:.2f} ms {tf:.2f} TF")
    del L64, B64
    torch.cuda.empty_cache()

    # n/k sweep at n = 16384, L the Cholesky factor of G G^T / 2n + I
    n = 16384
    L64 = gen.chol_lower_on(torch, dev, n, args.seed)
    for k in (128, 2048, 32768):
        B64 = torch.from_numpy(gen.rhs(n, k, args.seed)).to(dev)
        for prec, n0 in [(p_, n0_) for p_ in ("f64", "f32")
                         for n0_ in ((0, 256, 512) if k == 128 else (0,))]:
            es = 4 if prec == "f32" else 8
            ms, info, _ = time_solves(T, torch, dev, L64, B64, prec, n0, 0, 3)
            tf = float(n) * n * k / (ms * 1e-3) / 1e12
            alg_bytes = es * (n * (n + 1) / 2 + 2 * n * k)
            emit({"suite": "nk_sweep", "n": n, "k": k, "precision": prec, "n0": int(info.n0),
                  "auto": n0 == 0,
                  "n0_paper_rule": int(info.n0_paper_rule), "ms": round(ms, 3),
                  "tflops_n2k": round(tf, 2), "frac_peak": round(tf / PEAK[prec], 4),
                  "algorithmic_GBps": round(alg_bytes / (ms * 1e-3) / 1e9, 1)})
            log(f"suite nk {prec} k={k} n0={info.n0}: {ms:.2f} ms {tf:.2f} TF "
                f"{alg_bytes / (ms * 1e-3) / 1e9:.0f} GB/s")
        del B64
        torch.cuda.empty_cache()
    del L64
    torch.cuda.empty_cache()

    # the transposed problem L^T X = B (backward sweep over U = L^T), and the
    # upper problem U X = B with U = L^T given as an upper-triangular matrix
    # (read in place), invert + solve
    problems = ((0, "L X = B"), (T.FLAG_TRANSPOSE, "L^T X = B"),
                (T.FLAG_UPPER, "U X = B (U = L^T stored)"))
    for (n, k, prec) in ((16384, 16384, "f64"), (8192, 8192, "f64"), (8192, 8192, "f32")):
        L, B = gen.easy_system(n, k, args.seed)
        L64 = torch.from_numpy(L).to(dev)
        B64 = torch.from_numpy(B).to(dev)
        del L, B
        for flags, problem in problems:
            M = L64.t().contiguous() if flags == T.FLAG_UPPER else L64
            ms, info, _ = time_solves(T, torch, dev, M, B64, prec, 2048, flags, 3)
            del M
            tf = float(n) * n * k / (ms * 1e-3) / 1e12
            emit({"suite": "transposed", "n": n, "k": k, "precision": prec, "n0": int(info.n0),
                  "problem": problem, "ms": round(ms, 3),
                  "tflops_n2k": round(tf, 2), "frac_peak": round(tf / PEAK[prec], 4)})
            log(f"suite {problem} {prec} n=k={n}: {ms:.2f} ms {tf:.2f} TF")
        del L64, B64
        torch.cuda.empty_cache()

    # measured choice of n0 and tile policy (trsm_autotune) against the cost model
    for (n, k, prec) in ((8192, 8192, "f64"), (8192, 8192, "f32"), (16384, 128, "f64"),
                         (16384, 2048, "f64"), (2048, 64, "f64")):
        r = T.trsm_autotune(n, k, T.PRECISIONS[prec], 3, torch.cuda.current_stream().cuda_stream)
        emit({"suite": "autotune", "n": n, "k": k, "precision": prec, "n0": int(r.n0),
              "large_tiles": bool(r.flags & T.FLAG_LARGE_TILES), "ms": round(r.ms, 3),
              "model_n0": int(r.model_n0), "model_ms": round(r.model_ms, 3),
              "configurations": int(r.candidates)})
        log(f"suite autotune {prec} n={n} k={k}: n0={r.n0} flags={r.flags} {r.ms:.2f} ms "
            f"(model n0={r.model_n0} {r.model_ms:.2f} ms)")
    T.trsm_autotune_clear()
    torch.cuda.empty_cache()

    # serving with Cholesky factors: every request solves A X = B, A = L L^T
    res = serving_bench(args, torch, T, gen, dev, chol=True)
    emit({"suite": "serving_cholesky", **{k_: res[k_] for k_ in res if k_ != "rate_sweep"},
          "rate_sweep": res.get("rate_sweep")})
    torch.cuda.empty_cache()

    # blocked Cholesky and LU (no row exchanges) with inverted-block panel solves
    cholesky_bench(args, torch, T, gen, dev, emit)
    lu_bench(args, torch, T, gen, dev, emit)
    lu_piv_bench(args, torch, T, gen, dev, emit)

    # mixed precision at n = k = 16384 on the ill-conditioned factor (cond ~ 1e6)
    n = k = 16384
    L64 = gen.chol_lower_on(torch, dev, n, args.seed, ratio=1e-12)
    B64 = torch.from_numpy(gen.rhs(n, k, args.seed)).to(dev)
    ms64, _, X64 = time_solves(T, torch, dev, L64, B64, "f64", 0, 0, 3)
    nx = torch.linalg.norm(X64).item()
    for tol, prec in [(t_, p_) for t_ in (MIXED_TOL, 0.0) for p_ in ("bf16", "f16", "fp8")]:
        s = T.Solver.create(n, k, prec, 0, 0, device=dev, tolerance=tol)
        X = torch.empty_like(B64)
        inf = T.Info()
        stream = torch.cuda.current_stream().cuda_stream
        times = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.invert(L64)
            st = T.trsm_solve(s.plan, L64.data_ptr(), n, s.linv_ptr, B64.data_ptr(), k,
                              X.data_ptr(), k, s.workspace_ptr, stream, inf)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        diff = float(torch.linalg.norm(X - X64).item() / nx)
        ms = sorted(times)[1]
        emit({"suite": "mixed_hard", "n": n, "k": k, "precision": prec, "tolerance": tol,
              "status": T.status_string(st), "corrections": inf.iterations,
              "unrefined_error": inf.unrefined_error, "backward_error": inf.backward_error,
              "rel_diff_vs_f64_solve": diff, "ms": round(ms, 3), "f64_ms": round(ms64, 3)})
        log(f"suite mixed hard {prec} tolerance {tol:g}: {T.status_string(st)}, {inf.iterations} corrections, "
            f"{ms:.1f} ms (f64 {ms64:.1f} ms), diff vs f64 {diff:.2e}")
        s.close()
        del X
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--k", type=int, default=16384)
    ap.add_argument("--n0", type=int, default=0)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--lookahead", action="store_true",
                    help="two-stream lookahead sweep (per-launch timings then overlap)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--large-tiles", action="store_true",
                    help="128x128 tiles only (the tile policy trsm_autotune may pick)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="with --n0 0: use the cost model's n0 instead of trsm_autotune")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-factors", type=int, default=256)
    ap.add_argument("--serve-n0", type=int, default=0,
                    help="server block size (0: the batch autotuner's choice for the mix; >= n: each "
                         "factor fully inverted at registration; 64: persistent sweeps)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.5,
                    help="Poisson arrival rate as a fraction of the measured saturation rate")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device-to-device 3 times (reference "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--suite", action="store_true",
                    help="instead of the headline step, run the workload sweeps (one JSON line each)")
    ap.add_argument("--cholesky", action="store_true",
                    help="instead of the headline step, run only the Cholesky sweep of the suite")
    ap.add_argument("--lu", action="store_true",
                    help="instead of the headline step, run only the LU (no row exchanges) sweep")
    ap.add_argument("--lu-piv", action="store_true",
                    help="instead of the headline step, run only the LU with partial pivoting sweep")
    ap.add_argument("--chol-n", type=int, default=0, help="--cholesky / --lu: this n only")
    ap.add_argument("--chol-nb", type=int, default=None,
                    help="--cholesky / --lu: this block size only")
    args = ap.parse_args()

    if args.suite or args.cholesky or args.lu or args.lu_piv:
        import torch
        from paper_1612_01855_amd import inputs as gen
        from paper_1612_01855_amd import trsm as T
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        if args.cholesky or args.lu or args.lu_piv:
            bench_fn = cholesky_bench if args.cholesky else lu_bench if args.lu else lu_piv_bench
            bench_fn(args, torch, T, gen, torch.device("cuda:0"),
                     lambda rec: print(json.dumps(rec), flush=True))
        else:
            run_suite(args, torch, T, gen, torch.device("cuda:0"))
        return

    if args.calibrate_copy:
        import torch
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nbytes, "copies": 3}))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the solve is measured on one MI355X).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1612_01855_amd import inputs as gen
    from paper_1612_01855_amd import trsm as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n, k = args.n, args.k
    log(f"generating L ({n}x{n}) and B ({n}x{k}), seed {args.seed}")
    L, B = gen.easy_system(n, k, args.seed)
    dt = torch.float32 if args.precision == "f32" else torch.float64
    Ld = torch.from_numpy(L).to(dev, dt)
    Bd = torch.from_numpy(B).to(dev, dt)
    Xd = torch.empty_like(Bd)
    torch.cuda.synchronize()

    tune = None
    if args.n0 == 0 and not args.no_autotune:
        # n0 and the tile policy measured for this workload (plans made with
        # n0 = 0 then use the recorded choice)
        t0 = time.perf_counter()
        r = T.trsm_autotune(n, k, T.PRECISIONS[args.precision], 3,
                            torch.cuda.current_stream(dev).cuda_stream)
        tune = {"n0": int(r.n0), "large_tiles": bool(r.flags & T.FLAG_LARGE_TILES),
                "ms": round(r.ms, 3), "model_n0": int(r.model_n0),
                "model_ms": round(r.model_ms, 3), "configurations": int(r.candidates),
                "seconds": round(time.perf_counter() - t0, 1)}
        log(f"autotune: n0={r.n0} flags={r.flags} {r.ms:.2f} ms (cost model n0={r.model_n0} "
            f"{r.model_ms:.2f} ms), {r.candidates} configurations in {tune['seconds']} s")
        torch.cuda.empty_cache()
    flags = (T.FLAG_LOOKAHEAD if args.lookahead else 0) | (T.FLAG_LARGE_TILES if args.large_tiles else 0)
    solver = T.Solver.create(n, k, args.precision, args.n0, flags, device=dev)
    info = solver.info
    stream = torch.cuda.current_stream(dev)
    log(f"plan: n0={info.n0} m={info.m} (paper rule n0={info.n0_paper_rule}); "
        f"Linv {info.linv_bytes / 2**20:.0f} MiB, workspace {info.workspace_bytes / 2**20:.0f} MiB")

    def step():
        solver.invert(Ld)
        solver.solve(Ld, Bd, Xd)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    st, idx = solver.last_error()
    assert st == T.OK, f"singular diagonal at {idx}"

    T.trsm_plan_set_timing(solver.plan, True)
    T.trsm_plan_timing(solver.plan)           # clear
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    launches, gemm_ms, gemm_flops = T.trsm_plan_timing(solver.plan)
    T.trsm_plan_set_timing(solver.plan, False)
    ms_step = ms_total / args.steps
    flops_step = float(n) * n * k
    tflops = flops_step / (ms_step * 1e-3) / 1e12
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, {tflops:.2f} TFLOP/s (n^2 k)")

    # after the timed region: per-step distribution with the inversion and
    # the sweep bracketed separately (hipEvents on the solve stream)
    inv_ms, sol_ms, stp_ms = [], [], []
    for _ in range(max(args.steps, 10)):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        solver.invert(Ld)
        e[1].record(stream)
        solver.solve(Ld, Bd, Xd)
        e[2].record(stream)
        torch.cuda.synchronize()
        inv_ms.append(e[0].elapsed_time(e[1]))
        sol_ms.append(e[1].elapsed_time(e[2]))
        stp_ms.append(e[0].elapsed_time(e[2]))
    step_stats = {"runs": len(stp_ms), "step_ms_median": round(float(np.median(stp_ms)), 3),
                  "step_ms_p90": round(float(np.percentile(stp_ms, 90)), 3),
                  "invert_ms_median": round(float(np.median(inv_ms)), 3),
                  "solve_ms_median": round(float(np.median(sol_ms)), 3)}
    log(f"per step: median {step_stats['step_ms_median']} ms (p90 {step_stats['step_ms_p90']}), "
        f"invert {step_stats['invert_ms_median']} ms, solve {step_stats['solve_ms_median']} ms")

    workload = f"trsm_{args.precision}_n{n}_k{k}"
    # achieved: the step's n^2 k flops (the metric's count; the inversion's
    # extra flops are not credited) over the summed durations of all of the
    # step's product launches (inversion and sweep), timed with hipEvents on
    # the solve stream
    launches_step = max(launches // args.steps, 1)
    gemm_ms_step = gemm_ms / args.steps
    achieved = flops_step / (gemm_ms_step * 1e-3) / 1e12 if gemm_ms > 0 else 0.0
    peak = PEAK[args.precision]
    traffic = traffic_from_profiles(workload, info.n0, bool(info.flags & T.FLAG_LARGE_TILES))
    roofline = {"bound": "mfma", "kernel": "gemm_kernel (all product launches of a step)",
                "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "launches_per_step": launches_step,
                "avg_launch_ms": round(gemm_ms / max(launches, 1), 4),
                "algorithmic_flops_per_launch": flops_step / launches_step,
                "executed_flops_per_step": gemm_flops / args.steps}

    # correctness of the benchmarked X: binary64 residual on the GPU
    check = {}
    if args.precision == "f64":
        R = torch.empty_like(Bd)
        ws = torch.empty(T.trsm_residual_workspace_bytes(n, k), dtype=torch.uint8, device=dev)
        rn, xn, rmax = T.trsm_residual(n, k, Ld.data_ptr(), n, Xd.data_ptr(), k, Bd.data_ptr(), k,
                                       R.data_ptr(), k, ws.data_ptr(), stream.cuda_stream)
        lnorm = float(torch.linalg.norm(torch.tril(Ld)).item())
        check = {"backward_error": rn / (lnorm * xn)}
        del R, ws
        log(f"backward error {check['backward_error']:.2e}")

    mixed = {}
    if not args.no_mixed and args.precision == "f64":
        # refinement to the 1e-12 relative error the comparison asks for, then
        # to binary64's backward-error level (tolerance 0)
        mixed = {"tolerance": MIXED_TOL, "binary64_level": {}}
        for tol in (MIXED_TOL, 0.0):
            dest = mixed if tol > 0 else mixed["binary64_level"]
            for prec in ("bf16", "f16", "fp8"):
                try:
                    s2 = T.Solver.create(n, k, prec, args.n0, 0, device=dev, tolerance=tol)
                    Xm = torch.empty_like(Bd)
                    s2.invert(Ld)
                    inf = T.Info()
                    s2.solve(Ld, Bd, Xm, info=inf)         # warm
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    reps = 2
                    for _ in range(reps):
                        s2.invert(Ld)
                        s2.solve(Ld, Bd, Xm, info=inf)
                    torch.cuda.synchronize()
                    ms = (time.perf_counter() - t0) * 1e3 / reps
                    diff = float(torch.linalg.norm(Xm - Xd).item() / torch.linalg.norm(Xd).item())
                    dest[prec] = {"ms_per_solve": round(ms, 3),
                                  "tflops_n2k": round(flops_step / (ms * 1e-3) / 1e12, 3),
                                  "speedup_vs_f64": round(ms_step / ms, 3),
                                  "corrections": inf.iterations, "converged": bool(inf.converged),
                                  "status": T.status_string(s2.last_status),
                                  # of the last residual computed (with a tolerance the
                                  # final correction is added after it)
                                  "backward_error_last_residual": inf.backward_error,
                                  "unrefined_error_est": inf.unrefined_error,
                                  "rel_diff_vs_f64_solve": diff}
                    if tol > 0:
                        dest[prec]["within_tolerance"] = bool(diff <= tol)
                    log(f"mixed {prec} (tolerance {tol:g}): {ms:.2f} ms/solve, "
                        f"{inf.iterations} corrections, diff {diff:.1e}")
                    del Xm
                    s2.close()
                    torch.cuda.empty_cache()
                except Exception as e:  # report, never hide
                    dest[prec] = {"error": str(e)}
        ok = [v["speedup_vs_f64"] for pr, v in mixed.items()
              if pr in ("bf16", "f16", "fp8") and "error" not in v and v["within_tolerance"]]
        mixed["best_speedup_vs_f64_within_tolerance"] = max(ok) if ok else None

    serving = None
    if not args.no_serving and args.precision == "f64":
        del Xd
        torch.cuda.empty_cache()
        Xd = None
        serving = serving_bench(args, torch, T, gen, dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a column sample")
        cpu = cpu_baseline(L, B.astype(np.float32).astype(np.float64) if args.precision == "f32" else B)
        log(f"oracle: {cpu['value'] * 1e3:.2f} GFLOP/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "k": k, "n0": info.n0, "m": info.m,
                   "n0_paper_rule": info.n0_paper_rule, "precision": args.precision,
                   "L": "diag U[1,2], strict lower U[-1,1]/n", "B": "N(0,1)", "seed": args.seed,
                   "step": "trsm_invert_diag + trsm_solve (right-looking sweep"
                           + (", two-stream lookahead)" if args.lookahead else ")"),
                   "inversion_flops_per_step": info.inv_flops,
                   "tile_policy": "128x128 only" if info.flags & T.FLAG_LARGE_TILES
                   else "64x64 + split K for products with few tiles",
                   "n0_source": "fixed" if args.n0 else ("autotune" if tune else "cost model"),
                   "autotune": tune},
        "roofline": roofline,
        "step_stats": step_stats,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "serving": serving,
        "check": check,
    }
    print(json.dumps(out), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
