#!/usr/bin/env python3
"""Benchmark of the repeated SpMV y <- A x on the n = 10^6 irregular matrix.

Workload: the 1,000,000 x 1,000,000 binary64 CSR matrix with about 2*10^7
nonzeros (Zipf(2.0) row and column degrees, max 5,000, 30% of the nonzeros in
64 hidden diagonal blocks), K = 64 parts.  Following the paper's protocol
(Section 5.2: 3 warm-up calls, then 100 calls with the same matrix), every
timed product uses a fresh x from a pool of 103 seeded vectors that are
resident in HBM before timing starts; products run in the reordered space of
each form (Section 3), so permutations are outside the timed region.

A step is one product.  The JSON line reports the fastest reordered or split
form; every form's rate, the plain-CSR rate on the same GPU, the stream-read
ceiling and the partitioner's time are reported beside it.

Effective bytes per product (each array once):
  12 nnz + 4 (m + 1) + 8 n + 8 m.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def kernel_source_sha256():
    from paper_1203_2739_amd.rocprof_summary import kernel_source_sha256 as h
    return h()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(m, n, nnz):
    return 12 * nnz + 4 * (m + 1) + 8 * n + 8 * m


def time_form(spx, torch, P, form, xs, y, warmup, steps):
    """Returns (mean ms per product, mean ms of the SpMV kernel alone).

    Whole products are timed in one pass bracketed by two events; the kernel
    alone is timed in a second pass with an event pair around every launch,
    so the per-launch events do not weigh on the first figure."""
    stream = torch.cuda.current_stream()
    split = form.startswith("split")

    def product(i):
        if split:
            spx.split_prepare_y(P, y)
            return spx.spmv_split(P, xs[i], y, accumulate=2)
        return spx.spmv(P, xs[i], y)

    for i in range(warmup):
        product(i % xs.shape[0])
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for s in range(steps):
        product((warmup + s) % xs.shape[0])
    t1.record(stream)
    torch.cuda.synchronize()
    total = t0.elapsed_time(t1) / steps

    k_start = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    k_end = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for s in range(steps):
        i = (warmup + s) % xs.shape[0]
        if split:
            spx.split_prepare_y(P, y)
            k_start[s].record(stream)
            spx.spmv_split(P, xs[i], y, accumulate=2)
            k_end[s].record(stream)
        else:
            k_start[s].record(stream)
            spx.spmv(P, xs[i], y)
            k_end[s].record(stream)
    torch.cuda.synchronize()
    kern = float(np.mean([a.elapsed_time(b) for a, b in zip(k_start, k_end)]))
    return total, kern


FLUSH_BYTES = 512 << 20  # twice the 256 MB Infinity Cache, 128 times an XCD's L2


def time_cold(spx, torch, P, form, xs, y, steps=20):
    """Mean ms of one product (the split: zeroing of its shared rows plus the
    product) right after a read of FLUSH_BYTES that evicts the L2s and the
    Infinity Cache, so that the matrix, x and y come from HBM."""
    stream = torch.cuda.current_stream()
    flush = torch.zeros(FLUSH_BYTES // 8, dtype=torch.float64, device="cuda")
    sink = torch.empty(spx.stream_sink_len(FLUSH_BYTES), dtype=torch.float64, device="cuda")
    ev = []
    for s in range(steps):
        spx.stream_read(flush, FLUSH_BYTES, sink)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        if form.startswith("split"):
            spx.split_prepare_y(P, y)
            spx.spmv_split(P, xs[s % xs.shape[0]], y, accumulate=2)
        else:
            spx.spmv(P, xs[s % xs.shape[0]], y)
        b.record(stream)
        ev.append((a, b))
    torch.cuda.synchronize()
    del flush, sink
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def stream_ceiling(spx, torch, nbytes=1 << 30, reps=20):
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    sink = torch.empty(spx.stream_sink_len(nbytes), dtype=torch.float64, device="cuda")
    for _ in range(3):
        spx.stream_read(src, nbytes, sink)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        spx.stream_read(src, nbytes, sink)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, sink
    return nbytes / (ms * 1e-3) / 1e9


CPU_SO = os.path.join(ROOT, "bench_cpu.so")


def build_cpu_leg():
    """Compile the multi-core host product (bench_cpu.c) with OpenMP."""
    tmp = CPU_SO + ".tmp"
    import subprocess
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                           os.path.join(ROOT, "bench_cpu.c")])
    os.replace(tmp, CPU_SO)
    return CPU_SO


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, xs_host, budget_s=12.0, max_products=100):
    """Host CSR products on the full matrix, on a bounded number of products.

    The oracle's C product runs single-threaded (its index arrays are
    converted to the int64 it reads once, outside the timed loop); the
    OpenMP product of bench_cpu.c runs on every host core with int32
    indices.  Both sum each row left to right, so their results are
    identical; the byte count is the same algorithmic one as the GPU's."""
    import ctypes
    import oracle as orc
    nb = alg_bytes(A.m, A.n, A.nnz)
    P = ctypes.c_void_p
    rp64 = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    ci64 = np.ascontiguousarray(A.colidx, dtype=np.int64)
    vals = np.ascontiguousarray(A.vals, dtype=np.float64)
    y1 = np.empty(A.m)
    f = orc.lib().orc_spmv

    def one(x, y):
        rc = f(ctypes.c_int64(A.m), rp64.ctypes.data_as(P), ci64.ctypes.data_as(P), vals.ctypes.data_as(P),
               x.ctypes.data_as(P), y.ctypes.data_as(P))
        assert rc == 0

    def timed(fn, budget):
        fn(0)  # warm-up: pages and caches
        done, t0 = 0, time.perf_counter()
        while done < max_products and time.perf_counter() - t0 < budget:
            fn(done)
            done += 1
        return (time.perf_counter() - t0) / done, done

    xs = [np.ascontiguousarray(xs_host[i % xs_host.shape[0]]) for i in range(min(xs_host.shape[0], 103))]
    dt1, n1 = timed(lambda i: one(xs[i % len(xs)], y1), budget_s)
    out = {"value": round(nb / dt1 / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": f"{n1} products of the full n={A.n} matrix after one warm-up (the oracle's C loop, "
                     f"one thread, int64 indices converted once; {dt1 * 1e3:.1f} ms each)",
           "gflops": round(2 * A.nnz / dt1 / 1e9, 3), "cpu_model": cpu_model(),
           "host_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()}
    try:
        if not os.path.exists(CPU_SO):
            build_cpu_leg()
        C = ctypes.CDLL(CPU_SO)
    except Exception as e:  # no compiler on the host: report the oracle leg only
        out["all_cores"] = {"error": str(e)[:200]}
        return out
    rp32 = np.ascontiguousarray(A.rowptr, dtype=np.int32)
    ci32 = np.ascontiguousarray(A.colidx, dtype=np.int32)
    yp = np.empty(A.m)

    def par(i):
        rc = C.cpu_csr_spmv(ctypes.c_int32(A.m), rp32.ctypes.data_as(P), ci32.ctypes.data_as(P),
                            vals.ctypes.data_as(P), xs[i % len(xs)].ctypes.data_as(P), yp.ctypes.data_as(P))
        assert rc == 0

    dtp, npar = timed(par, budget_s)
    one(xs[(npar - 1) % len(xs)], y1)
    assert np.array_equal(y1, yp), "the OpenMP product differs from the oracle's"
    out["all_cores"] = {"value": round(nb / dtp / 1e9, 3), "unit": "GB/s", "cores": int(C.cpu_threads()),
                        "kind": "openmp static row blocks, int32 indices (bench_cpu.c)",
                        "sample": f"{npar} products ({dtp * 1e3:.2f} ms each); result equal to the oracle's",
                        "gflops": round(2 * A.nnz / dtp / 1e9, 3)}
    return out


def plan_sha256(rp, cp, parts, nleaves):
    """Hash of the layout a reordered plan hands the kernel: the row and
    column permutations, the part boundaries (SB, DB) or the part of each
    nonzero (split), and the number of leaves."""
    h = hashlib.sha256()
    for a in (rp, cp, parts):
        h.update(np.ascontiguousarray(a, dtype=np.int64).tobytes())
    h.update(str(int(nleaves)).encode())
    return h.hexdigest()


def tune_list(t):
    """A schedule dict as the bench line's tune list."""
    return [t.get("wg_size", 0), t.get("nnz_per_block", 0), t.get("blocks_per_tile", 1),
            t.get("window_entries", -1) or -1, t.get("tiles_per_group", 0), t.get("wave_blocks", 0),
            t.get("pipeline", 0), t.get("scan_reduce", 0), t.get("sort_gathers", 0), t.get("compact_index", 0)]


def schedule_name(tune):
    """Short name of a schedule [wg, nnz_per_block, blocks_per_tile, window,
    tiles_per_group, wave_blocks, pipeline, scan_reduce, sort_gathers,
    compact_index]: threads x nonzeros per thread (per lane for wave blocks,
    marked w; s for scan row sums, g for gather-sorted blocks, c for 16-bit
    indices, p for pipelined tiles), then tiles per row group (t) and the LDS
    window (W) when used."""
    wg, nb, _, win, tpg, wave, pipe, scan, srt, cpt = (list(tune) + [0] * 10)[:10]
    name = (f"{wg}x{nb // (64 if wave else wg)}" + ("w" if wave else "") + ("s" if scan else "")
            + ("g" if srt else "") + ("c" if cpt else "") + ("p" if pipe else ""))
    if tpg:
        name += f"t{tpg}"
    if win and win > 0:
        name += f"W{win}"
    return name


def kernel_name(tune):
    """The kernel that runs a schedule (tune list as in tune_list)."""
    wg, nb, bpt, win, tpg, wave, pipe, scan, srt, cpt = (list(tune) + [0] * 10)[:10]
    if cpt:
        return "spmv_compact"
    if wave:
        return "spmv_waves"
    if pipe:
        return "spmv_pipe"
    if srt:
        return "spmv_sorted_scan" if scan else "spmv_sorted"
    return "spmv_scan" if scan else "spmv_blocks"


def measured_traffic(form, nnz, sched, plan):
    """HBM bytes per launch of the SpMV kernel of this form from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated against a copy of
    known size), or None when the summary is missing, is for another matrix,
    schedule or plan layout, or the kernel source changed after the counters
    were taken."""
    from paper_1203_2739_amd.rocprof_summary import kernel_source_sha256
    path = os.path.join(ROOT, "profiles", f"spmv_c2_{form}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and parts[0].endswith(":"):
            kv[parts[0][:-1]] = parts[1]
    if (kv.get("kernel_source_sha256") != kernel_source_sha256() or int(kv.get("nnz", -1)) != nnz
            or kv.get("schedule") != sched or kv.get("plan_sha256") != plan):
        return None
    return int(kv["traffic_bytes_per_launch"])


def load_c2(n):
    from synth import gen_c2
    cache = os.environ.get("SPX_C2_CACHE")
    if cache and os.path.exists(cache):
        z = np.load(cache)
        from synth import CSR
        return CSR(int(z["m"]), int(z["n"]), z["rowptr"], z["colidx"], z["vals"],
                   {"block_frac": float(z["block_frac"])})
    A = gen_c2(n=n)
    if cache:
        np.savez(cache, m=A.m, n=A.n, rowptr=A.rowptr, colidx=A.colidx, vals=A.vals,
                 block_frac=A.info["block_frac"])
    return A


def time_calls(torch, fn, warmup, steps):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def main_precision(args, torch, spx, emit=True):
    """Precision mode on the SPD matrix A = offdiag(B + B^T) + diag(row sums + 1)
    built from the block generator at n = 5*10^5: product rates per stored
    precision, product errors against the binary64 oracle, and the refined CG
    solve of A x = A 1 to relative residual 1e-10."""
    import oracle as orc
    from synth import gen_c3_spd, gen_vectors
    torch.cuda.set_device(0)
    t = time.time()
    A = gen_c3_spd(seed=3, n=500_000)
    log(f"SPD matrix n={A.n} nnz={A.nnz} ({time.time() - t:.1f} s)")
    M = spx.from_csr(A)
    P = spx.plan_plain(M)
    spx.plan_add_lowp(P, "f32")
    spx.plan_add_lowp(P, "bf16")
    x64 = gen_vectors(3000, A.n, 1)[0]
    xd = torch.from_numpy(x64).cuda()
    x32 = xd.float()
    y = torch.empty(A.m, dtype=torch.float64, device="cuda")
    y32 = torch.empty(A.m, dtype=torch.float32, device="cuda")
    # every precision runs the schedule the library's autotuner picks for its
    # own product (binary64 may take gather-sorted blocks, the low precisions
    # may not); a solve runs the schedule of its inner precision
    ref = orc.spmv(A, x64)
    den = orc.abs_rowsum(A, x64)
    out = {"products": {}, "solves": {}}
    vb = {"f64": 8, "f32": 4, "bf16": 2}
    sched = {}
    for prec in ("f64", "f32", "bf16"):
        if prec == "f64":
            sched[prec], _ = spx.plan_autotune(P, xd, y, reps=10, precision="f64")
        else:
            sched[prec], _ = spx.plan_autotune(P, x32, y32, reps=10, precision=prec)
        if prec == "f64":
            ms = time_calls(torch, lambda: spx.spmv(P, xd, y), args.warmup, args.steps)
            got = y.cpu().numpy()
            xb = 8
        else:
            ms = time_calls(torch, lambda: spx.spmv_lowp(P, prec, x32, y32), args.warmup, args.steps)
            got = y32.double().cpu().numpy()
            xb = 4
        nb = A.nnz * (4 + vb[prec]) + 4 * (A.m + 1) + xb * (A.n + A.m)
        err = np.abs(got - ref) / np.maximum(den, 1e-300)
        out["products"][prec] = {"ms": round(ms, 5), "GBs": round(nb / (ms * 1e-3) / 1e9, 1),
                                 "bytes": nb, "max_rel_err_vs_f64_oracle": float(err.max()),
                                 "median_rel_err_vs_f64_oracle": float(np.median(err))}
        log(prec, json.dumps(out["products"][prec]))
    b = orc.spmv(A, np.ones(A.n))
    bd = torch.from_numpy(b).cuda()
    for prec, itol in (("f64", 1e-10), ("f32", 1e-3), ("bf16", 1e-2)):
        spx.plan_retune(P, sched[prec])
        xs = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        st = spx.cg_ir(P, prec, bd, xs, tol=1e-10, inner_tol=itol, max_outer=60, max_inner=5000)
        xh = xs.cpu().numpy()
        res = np.linalg.norm(b - orc.spmv(A, xh)) / np.linalg.norm(b)
        st.update({"inner_tol": itol, "oracle_rel_residual": float(res),
                   "max_abs_err_vs_ones": float(np.max(np.abs(xh - 1.0)))})
        out["solves"][prec] = st
        log(prec, json.dumps(st))
    f64 = out["products"]["f64"]["ms"]
    line = {
        "metric": "precision-mode SpMV GB/s and refined-CG time to 1e-10",
        "value": out["products"]["f32"]["GBs"], "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": out["products"]["f32"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"SPD n={A.n} from the block generator, nnz={A.nnz}; "
                               "binary32 values, binary32 accumulation"},
        "schedule": {p: schedule_name(tune_list(t)) for p, t in sched.items()},
        "speedup_vs_f64_product": {p: round(f64 / out["products"][p]["ms"], 3) for p in ("f32", "bf16")},
        "speedup_vs_f64_cg": {p: round(out["solves"]["f64"]["seconds"] / out["solves"][p]["seconds"], 3)
                              for p in ("f32", "bf16")},
        **out,
    }
    if emit:
        print(json.dumps(line), flush=True)
    return line


def main_batched(args, torch, spx, emit=True):
    """The uneven batch: 256 matrices (n log-uniform in [10^3, 2*10^5], mean
    degree U[5, 50], Zipf(2.2) rows) with 1, 8 or 32 right-hand sides each,
    run as one persistent launch replayed from a HIP graph with the
    autotuned schedule, against one plain SpMV launch per matrix and
    right-hand side."""
    import oracle as orc
    from synth import gen_c4_one
    count = 256
    t = time.time()
    mats, ks = [], []
    for j in range(count):
        A, k = gen_c4_one(j)
        mats.append(A)
        ks.append(k)
        if j % 32 == 31:
            log(f"generated {j + 1}/{count} ({time.time() - t:.0f} s)")
    tot_nnz = sum(A.nnz for A in mats)
    plans = [spx.plan_plain(spx.from_csr(A)) for A in mats]
    rng = np.random.default_rng(4444)
    X, Y, Xc, Yc = [], [], [], []
    for A, k in zip(mats, ks):
        x = torch.from_numpy(rng.uniform(-1, 1, (A.n, k))).cuda()
        X.append(x[:, 0].contiguous() if k == 1 else x)
        Y.append(torch.empty((A.m,) if k == 1 else (A.m, k), dtype=torch.float64, device="cuda"))
        Xc.append(x.t().contiguous())  # columns for the plain launches
        Yc.append(torch.empty((k, A.m), dtype=torch.float64, device="cuda"))
    log(f"batch of {count}: nnz={tot_nnz}, right-hand sides {sum(ks)} ({time.time() - t:.0f} s)")
    B = spx.Batch(plans, ks)
    B.bind(X, Y)
    best = B.autotune(reps=3)
    log("autotune", json.dumps(best))
    inf = B.info()
    B.capture()
    ms_graph = time_calls(torch, B.replay, args.warmup, args.steps)
    ms_run = time_calls(torch, B.run, args.warmup, args.steps)

    def plain_all():
        for P, xc, yc, k in zip(plans, Xc, Yc, ks):
            for c in range(k):
                spx.spmv(P, xc[c], yc[c])
    ms_plain = time_calls(torch, plain_all, 1, max(3, args.steps // 10))
    # parity on a sample of members (every 32nd), against the oracle
    B.replay()
    torch.cuda.synchronize()
    worst = 0.0
    for j in range(0, count, 32):
        A = mats[j]
        x = X[j].cpu().numpy().reshape(A.n, -1)
        y = Y[j].cpu().numpy().reshape(A.m, -1)
        ref = orc.spmm(A, x)
        bound = orc.spmm(type(A)(A.m, A.n, A.rowptr, A.colidx, np.abs(A.vals)), np.abs(x))
        worst = max(worst, float(np.max(np.abs(y - ref) / np.maximum(bound, 1e-300))))
    gbs = inf["bytes"] / (ms_graph * 1e-3) / 1e9
    line = {
        "metric": "batched SpMV effective GB/s, one persistent graph launch vs plain CSR launches",
        "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_graph, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"256 uneven matrices, nnz={tot_nnz}, 1/8/32 right-hand sides"},
        "speedup_vs_plain": round(ms_plain / ms_graph, 3),
        "ms_plain_launches": round(ms_plain, 4), "ms_single_launch": round(ms_run, 4),
        "plain_launches": int(sum(ks)), "items": inf["nitems"], "grid": inf["grid"],
        "bytes": inf["bytes"], "autotune": best,
        "sample_max_rel_err": worst, "pct_of_peak": round(100 * gbs / PEAK_HBM_GBS, 2),
    }
    if emit:
        print(json.dumps(line), flush=True)
    return line


def extension_summaries(args, torch, spx):
    """The precision and batched workloads, run after the main measurement
    and reported in its line: their own metrics, rates and checks."""
    p = main_precision(args, torch, spx, emit=False)
    b = main_batched(args, torch, spx, emit=False)
    return {
        "precision": {"metric": p["metric"], "config": p["config"], "unit": "GB/s",
                      "GBs": {k: v["GBs"] for k, v in p["products"].items()},
                      "ms": {k: v["ms"] for k, v in p["products"].items()},
                      "max_rel_err_vs_f64_oracle": {k: v["max_rel_err_vs_f64_oracle"]
                                                    for k, v in p["products"].items()},
                      "schedule": p["schedule"], "speedup_vs_f64_product": p["speedup_vs_f64_product"],
                      "solve_seconds": {k: round(v["seconds"], 4) for k, v in p["solves"].items()},
                      "solve_converged": {k: v["converged"] for k, v in p["solves"].items()},
                      "speedup_vs_f64_cg": p["speedup_vs_f64_cg"]},
        "batched": {k: b[k] for k in ("metric", "config", "value", "unit", "ms_per_step", "speedup_vs_plain",
                                      "ms_plain_launches", "plain_launches", "bytes", "sample_max_rel_err",
                                      "pct_of_peak")},
    }


def main_locality(args, torch, spx):
    """Temporal against spatial locality of the x accesses (Sec. 1, the
    paper's claim that temporal locality matters more for irregular
    matrices): four n x n matrices with 20 nonzeros per row whose columns are
    uniform over x (random), scattered inside a window of 16,384 columns that
    slides with the row (temporal only), one run of 20 consecutive columns at
    a random place (spatial only), or that run at the diagonal (both).  Each
    is timed with plain CSR under row blocks (512x4), gather-sorted blocks
    (512x4) and the library's autotuned schedule (or the --tune schedule
    alone)."""
    from synth import LOCALITY_KINDS, gen_locality, gen_vectors
    n = args.n
    npool = min(max(args.steps + args.warmup, 3), 103)
    xs = torch.from_numpy(gen_vectors(2000, n, npool)).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    res = {}
    for kind in LOCALITY_KINDS:
        t = time.time()
        L = gen_locality(kind, n=n)
        P = spx.plan_plain(spx.from_csr(L))
        nb = alg_bytes(L.m, L.n, L.nnz)
        r = {"nnz": L.nnz, "bytes": nb}
        if args.tune:
            f = [int(v) for v in args.tune.split(",")]
            keys = ["wg_size", "nnz_per_block", "blocks_per_tile", "window_entries", "tiles_per_group", "wave_blocks",
                    "pipeline", "scan_reduce", "sort_gathers", "compact_index"]
            scheds = {schedule_name(f): dict(zip(keys, f))}
        else:
            scheds = {"512x4": dict(wg_size=512), "512x4g": dict(wg_size=512, sort_gathers=1)}
        for name, tune in scheds.items():
            spx.plan_retune(P, tune)
            _, kms = time_form(spx, torch, P, "plain", xs, y, args.warmup, args.steps)
            r[name] = {"kernel_ms": round(kms, 5), "GBs": round(nb / (kms * 1e-3) / 1e9, 1)}
        if not args.tune and not args.no_autotune:
            best, _ = spx.plan_autotune(P, xs[0], y, reps=10)
            _, kms = time_form(spx, torch, P, "plain", xs, y, args.warmup, args.steps)
            r["autotuned"] = {"schedule": schedule_name(tune_list(best)), "kernel_ms": round(kms, 5),
                              "GBs": round(nb / (kms * 1e-3) / 1e9, 1)}
        log(f"{kind} ({time.time() - t:.0f} s): {json.dumps(r)}")
        res[kind] = r
    head = "autotuned" if "autotuned" in res["temporal"] else next(iter(scheds))
    line = {
        "metric": "SpMV GB/s by locality of the x accesses (random, temporal only, spatial only, both)",
        "value": res["temporal"][head]["GBs"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["temporal"][head]["kernel_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"n={n}, 20 nonzeros per row; temporal window 16384 columns"},
        "spatial_over_temporal": round(res["temporal"][head]["kernel_ms"] / res["spatial"][head]["kernel_ms"], 3),
        "kinds": res,
    }
    print(json.dumps(line), flush=True)


def main_selector(args, torch, spx):
    """Learned selector: every one of the 24 choices timed on matrices of the
    four families (n log-uniform in [n_lo, n_hi]); the network is trained on
    the training matrices with the library's kernels and evaluated on held-out
    ones by regret against exhaustive timing, beside the best fixed choice."""
    from paper_1203_2739_amd import selector
    from synth import gen_family
    rng = np.random.default_rng(5555)
    N = args.train + args.test
    fams = ["F1", "F2", "F3", "F4"]
    sizes = [int(round(np.exp(rng.uniform(np.log(args.n_lo), np.log(args.n_hi))))) for _ in range(N)]
    lo, hi = (int(v) for v in args.index_range.split(":")) if args.index_range else (0, N)
    tree_file = lambda i: os.path.join(args.trees or args.save_trees, f"sel_{i:05d}.npz")  # noqa: E731
    if args.save_trees:
        # the three K = 256 partitions of every matrix, on the host only
        os.makedirs(args.save_trees, exist_ok=True)
        t = time.time()
        for i in range(lo, hi):
            if os.path.exists(tree_file(i)):
                continue
            tr = selector.partition_trees(gen_family(fams[i % 4], 9000 + i, sizes[i]), seed=i)
            np.savez_compressed(tree_file(i), sb=tr["sb"].astype(np.uint8), db=tr["db"].astype(np.uint16),
                                split=tr["split"].astype(np.uint8), seconds=tr["seconds"])
            log(f"trees {i + 1}/{hi} n={sizes[i]} ({tr['seconds']:.1f} s, {time.time() - t:.0f} s in all)")
        return
    if args.selector_data:
        zs = [np.load(f) for f in args.selector_data.split(",")]
        F, T, tpart, nbytes = (np.concatenate([z[k] for z in zs]) for k in ("F", "T", "tpart", "nbytes"))
        assert F.shape[0] == N
    else:
        mats, T, tpart = [], [], []
        t = time.time()
        for i in range(lo, hi):
            A = gen_family(fams[i % 4], 9000 + i, sizes[i])
            trees = None
            if args.trees:
                with np.load(tree_file(i)) as z:
                    trees = {f: z[f].astype(np.int32) for f in ("sb", "db", "split")}
                    trees["seconds"] = float(z["seconds"])
            times, tp = selector.measure(A, seed=i, trees=trees)
            mats.append(A)
            T.append(times)
            tpart.append(tp)
            if i % 5 == 4:
                log(f"measured {i + 1}/{N} ({time.time() - t:.0f} s)")
        T = np.stack(T)
        F = selector.feature_matrix(mats)
        nbytes = np.array([alg_bytes(A.m, A.n, A.nnz) for A in mats])
        if args.save_selector_data:
            np.savez(args.save_selector_data, F=F, T=T, tpart=np.array(tpart), nbytes=nbytes)
        if args.index_range:
            return
    tr, te = np.arange(args.train), np.arange(args.train, N)
    norm = selector.Normalizer(F[tr])
    labels = T.argmin(axis=1)
    t0 = time.time()
    theta, chosen_settings, tried = selector.fit(F[tr], T[tr], norm)
    ttrain = time.time() - t0
    chosen = selector.predict(theta, F[te], norm)
    fixed = selector.best_fixed(T[tr])
    r_net = selector.regret(T[te], chosen)
    r_fix = selector.regret(T[te], np.full(te.size, fixed))
    r_plain = selector.regret(T[te], np.zeros(te.size, int))

    def stats(r):
        return {"mean": round(float(r.mean()), 4), "median": round(float(np.median(r)), 4),
                "p90": round(float(np.quantile(r, 0.9)), 4)}
    nb = nbytes[te]
    gbs = lambda tt: float(np.mean(nb / (tt * 1e-3) / 1e9))  # noqa: E731
    sel_t = T[te, chosen]
    line = {
        "metric": "learned selector regret vs exhaustive autotune (held-out), end-to-end GB/s",
        "value": round(gbs(sel_t), 1), "unit": "GB/s", "n_gpus": 1, "steps": 10, "warmup": 2,
        "ms_per_step": round(float(sel_t.mean()), 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.train} training + {args.test} held-out matrices of families F1-F4, "
                               f"n in [{args.n_lo}, {args.n_hi}], 24 choices"},
        "regret_network": stats(r_net), "regret_best_fixed": stats(r_fix),
        "best_fixed_choice": selector.choice_name(fixed), "regret_plain_default": stats(r_plain),
        "GBs_exhaustive": round(gbs(T[te].min(axis=1)), 1), "GBs_best_fixed": round(gbs(T[te, fixed]), 1),
        "GBs_plain": round(gbs(T[te, 0]), 1),
        "train_accuracy": round(float(np.mean(selector.predict(theta, F[tr], norm) == labels[tr])), 3),
        "test_accuracy": round(float(np.mean(chosen == labels[te])), 3),
        "label_counts": {selector.choice_name(c): int(k) for c, k in zip(*np.unique(labels, return_counts=True))},
        "settings_chosen_on_validation": chosen_settings,
        "validation_regret_best": min(t["val_regret"] for t in tried),
        "train_seconds": round(ttrain, 1),
        "partition_seconds_mean": round(float(np.mean(tpart)), 2),
    }
    print(json.dumps(line), flush=True)


def stored_rows(P):
    """(row pointers over the stored rows, their column indices) of any plan:
    the reordered CSR, or for the split the per-leaf slots."""
    if P.info()["form_name"] == "split":
        S = P.export_split()
        return S["slot_ptr"], S["colidx"]
    rp, col, _ = P.export_csr()
    return rp, col


def gather_requests(P, line_entries=16, max_nnz=None):
    """Model of the L1 -> L2 requests of a plan's x gathers: distinct cache
    lines (line_entries binary64 entries each; 16 for 128-byte lines) per
    gather instruction of 16 lanes (a quarter wave) and of 64 lanes (a wave),
    over the multi-row blocks of the plan's schedule, per gathered nonzero.
    Row order follows spmv_blocks: thread t of a block loads the 4
    consecutive entries from the aligned start zb + 4 t (+ 4 WG per further
    round) and the j-th gather of its lanes reads the j-th of them; the
    entries of the first aligned group that precede the block are gathered
    too.  Gather-sorted order follows spmv_sorted: the block's own entries
    sorted by column, the j-th gather of a quarter wave reading 16
    consecutive sorted entries and a wave covering four such runs, 64
    entries apart.  Long-row segments are left out.  Returns a dict of the
    four ratios and the counted nonzeros.  Host only."""
    _, col = stored_rows(P)
    bd, _ = P.export_sched()
    inf = P.info()
    wg, npt = inf["wg_size"], inf["nnz_per_block"] // max(inf["wg_size"], 1)
    line = col.astype(np.int64) // line_entries
    req = {"row16": 0, "row64": 0, "sorted16": 0, "sorted64": 0}
    cnt = {"row": 0, "sorted": 0}

    def distinct(L, group):
        # L: (instructions, lanes) line ids, -1 for lanes without an entry
        L = np.sort(L.reshape(-1, group), axis=1)
        new = np.ones(L.shape, bool)
        new[:, 1:] = L[:, 1:] != L[:, :-1]
        return int(np.count_nonzero(new & (L >= 0)))

    for s0, s1, z0, z1 in bd:
        if s1 < 0 or z1 <= z0:
            continue
        zb = z0 & ~3
        # row order: entry zb + 4 g + j for 16-byte group g = u WG + t
        ng = (z1 - zb + 3) // 4
        G = np.full(npt // 4 * wg * 4, -1, np.int64)
        G[:z1 - zb] = line[zb:z1]
        G = G.reshape(npt // 4, wg // 64, 64, 4)      # round, wave, lane, j
        R = G.transpose(0, 1, 3, 2)                     # instruction (round, wave, j) x lane
        req["row16"] += distinct(R, 16)
        req["row64"] += distinct(R, 64)
        cnt["row"] += z1 - zb
        # gather-sorted order: chunks of 64 sorted entries, quarter q of a
        # wave reading chunk 4 w + q, its j-th gather entries 16 j .. 16 j + 15
        S = np.sort(line[z0:z1])
        nc = (S.size + 63) // 64
        nw = (nc + 3) // 4
        C = np.full(nw * 4 * 64, -1, np.int64)
        C[:S.size] = S
        C = C.reshape(nw, 4, 4, 16)                     # wave, chunk (quarter), j, lane
        Q = C.transpose(0, 2, 1, 3)                     # instruction (wave, j) x (quarter, lane)
        req["sorted16"] += distinct(Q, 16)
        req["sorted64"] += distinct(Q, 64)
        cnt["sorted"] += S.size
        if max_nnz is not None and cnt["sorted"] >= max_nnz:
            break
    out = {k: round(float(v) / max(int(cnt["row" if k.startswith("row") else "sorted"]), 1), 4)
           for k, v in req.items()}
    out["nnz_counted"] = int(cnt["sorted"])
    return out


def block_fill(P):
    """Share of a schedule's load slots that its blocks fill: the entries
    every block (or long-row segment) loads from its aligned start, over the
    blocks' capacity (nnz_per_block each).  Host only."""
    bd, _ = P.export_sched()
    cap = P.info()["nnz_per_block"]
    load = (bd[:, 3].astype(np.int64) - (bd[:, 2] & ~3)).sum()
    return round(float(load) / max(bd.shape[0] * cap, 1), 4)


def reduction_chain(P):
    """Median over the multi-row blocks of a lane-group schedule of the
    dependent LDS reads of its longest row: ceil(length / lanes), a row
    being summed by 2^floor(log2(WG / rows)) lanes, at most 64.  Host only."""
    bd, _ = P.export_sched()
    rp = stored_rows(P)[0].astype(np.int64)
    wg = P.info()["wg_size"]
    chain = []
    for s0, s1, _, _ in bd[bd[:, 1] >= 0]:
        nr = int(s1 - s0)
        longest = int((rp[s0 + 1:s1 + 1] - rp[s0:s1]).max())
        lanes = 1
        while lanes * 2 <= wg // nr and lanes < 64:
            lanes *= 2
        chain.append(-(-longest // lanes))
    return float(np.median(chain)) if chain else 0.0


def main_gather_model(args, spx):
    """Modeled gather requests per nonzero of the DB form (K = 64) of the
    n = 10^6 matrix in row order and in gather-sorted order, for the
    workgroup row blocks of 2048 and 4096 entries (the latter as the
    gather-sorted kernel cuts them) and the scan's fuller blocks of 4096
    entries, and of the split at 1024 x 4 gather-sorted; block fill and
    reduction chain of plain CSR; host only, no GPU."""
    A = load_c2(args.n)
    M = spx.from_csr(A, device=False)
    P, _, _, _ = spx.reorder_db(M, args.K, 0, args.seed, tune=dict(wg_size=512, nnz_per_block=2048))
    rows = []
    for tune in (dict(wg_size=512, nnz_per_block=2048), dict(wg_size=1024, nnz_per_block=4096, sort_gathers=1),
                 dict(wg_size=1024, nnz_per_block=4096, scan_reduce=1)):
        spx.plan_retune(P, tune)
        r = gather_requests(P, max_nnz=args.model_nnz)
        r["schedule"] = schedule_name(tune_list(tune))
        r["form"] = "db"
        rows.append(r)
        log(f"gather model {r}")
    # the split (128 KB leaves) under the schedule its autotuning keeps
    tune = dict(wg_size=1024, nnz_per_block=4096, sort_gathers=1)
    P, _, _, _ = spx.split(M, args.K, args.window_bytes, args.seed, tune=tune)
    r = gather_requests(P, max_nnz=args.model_nnz)
    r["schedule"] = schedule_name(tune_list(tune))
    r["form"] = "split"
    rows.append(r)
    log(f"gather model {r}")
    # how full the blocks of plain CSR are with and without the scan's rule
    fill = {}
    for tune in (dict(wg_size=512, nnz_per_block=2048), dict(wg_size=512, nnz_per_block=2048, scan_reduce=1)):
        fill[schedule_name(tune_list(tune))] = block_fill(spx.plan_plain(M, tune=tune))
    chain = reduction_chain(spx.plan_plain(M, tune=dict(wg_size=512, nnz_per_block=2048)))
    log(f"plain CSR block fill {fill}, median reduction chain at 512x4 {chain}")
    line = {"workload": "gather request model", "K": args.K, "n": args.n, "line_bytes": 128,
            "rows": rows, "plain_block_fill": fill, "plain_median_reduction_chain": chain}
    print(json.dumps(line))
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="plain,sbfs,srcm,shp_rn,sb,db,split,split_unit,banded",
                    help="sbfs, srcm, shp_rn: breadth-first and reverse Cuthill-McKee orders of the "
                         "bipartite graph and the row-net model (Section 5.1); split: row nets weigh 32 column nets; split_unit: all nets weigh 1 "
                         "(Corollary 4); banded: plain CSR of the banded stand-in (same rows, columns next to "
                         "the diagonal)")
    ap.add_argument("--K", type=int, default=64)
    ap.add_argument("--window-bytes", type=int, default=131072,
                    help="leaf window budget of the split (x plus y entries, bytes)")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tune", default="",
                    help="wg,nnz_per_block[,blocks_per_tile,window_entries,tiles_per_group,wave_blocks,pipeline,"
                         "scan_reduce,sort_gathers,compact_index]")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the precision and batched workloads that the default run reports beside the SpMV")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default schedule")
    ap.add_argument("--cold", action="store_true",
                    help="also time 20 products per form, each after a 512 MB read that empties the caches")
    ap.add_argument("--workload", default="spmv",
                    choices=["spmv", "precision", "batched", "selector", "locality", "gather_model"],
                    help="spmv: repeated products on the n=10^6 matrix (default); precision: "
                         "binary32/bfloat16 products and refined CG on the n=5*10^5 SPD matrix")
    ap.add_argument("--train", type=int, default=60, help="selector: training matrices")
    ap.add_argument("--test", type=int, default=30, help="selector: held-out matrices")
    ap.add_argument("--n-lo", type=int, default=20000, help="selector: smallest n")
    ap.add_argument("--n-hi", type=int, default=150000, help="selector: largest n")
    ap.add_argument("--selector-data", default="",
                    help="selector: load features and timings from this .npz instead of measuring")
    ap.add_argument("--save-selector-data", default="", help="selector: save features and timings here")
    ap.add_argument("--index-range", default="",
                    help="selector: measure only matrices a:b of the sequence (with --save-selector-data)")
    ap.add_argument("--save-trees", default="",
                    help="selector: compute the three K = 256 partitions of every matrix on the host (no GPU) "
                         "into this folder, then stop")
    ap.add_argument("--trees", default="",
                    help="selector: take the partitions from this folder (written by --save-trees) instead of "
                         "partitioning during the measurement")
    ap.add_argument("--model-nnz", type=int, default=4_000_000,
                    help="gather_model: nonzeros of the first blocks counted")
    ap.add_argument("--only-stream", action="store_true",
                    help="run only the 1 GiB stream read and copy kernels (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: a run over several GPUs is not supported "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1203_2739_amd as spx
    from synth import gen_vectors

    if args.workload == "gather_model":
        spx.set_num_threads(min(16, os.cpu_count() or 1))
        return main_gather_model(args, spx)  # host only
    if args.workload == "selector" and args.save_trees:
        spx.set_num_threads(min(16, os.cpu_count() or 1))
        return main_selector(args, torch, spx)  # host partitions only
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "precision":
        return main_precision(args, torch, spx)
    if args.workload == "batched":
        return main_batched(args, torch, spx)
    if args.workload == "selector":
        return main_selector(args, torch, spx)
    if args.workload == "locality":
        return main_locality(args, torch, spx)
    if args.only_stream:
        nbytes = 1 << 30
        src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
        dst = torch.empty_like(src)
        sink = torch.empty(spx.stream_sink_len(nbytes), dtype=torch.float64, device="cuda")
        for _ in range(5):
            spx.stream_read(src, nbytes, sink)
            spx.stream_copy(src, dst, nbytes)
        torch.cuda.synchronize()
        print(json.dumps({"stream_read_GBs": round(stream_ceiling(spx, torch), 1), "bytes": nbytes}))
        return
    spx.set_num_threads(min(16, os.cpu_count() or 1))

    t = time.time()
    A = load_c2(args.n)
    log(f"matrix n={A.n} nnz={A.nnz} block_frac={A.info.get('block_frac', 0):.3f} "
        f"({time.time() - t:.1f} s)")
    npool = max(args.steps + args.warmup, 3)
    npool = min(npool, 103)
    xs_host = gen_vectors(2000, A.n, npool)
    xs = torch.from_numpy(xs_host).cuda()
    y = torch.zeros(A.m, dtype=torch.float64, device="cuda")
    M = spx.from_csr(A)
    nb = alg_bytes(A.m, A.n, A.nnz)

    tune = None
    if args.tune:
        f = [int(v) for v in args.tune.split(",")]
        keys = ["wg_size", "nnz_per_block", "blocks_per_tile", "window_entries", "tiles_per_group", "wave_blocks",
                "pipeline", "scan_reduce", "sort_gathers", "compact_index"]
        tune = dict(zip(keys, f))

    results = {}
    for form in [f for f in args.forms.split(",") if f]:
        t = time.time()
        if form == "plain":
            P = spx.plan_plain(M, tune=tune)
            xf = xs
        elif form in ("sbfs", "srcm"):
            rp, cp = (spx.order_bfs if form == "sbfs" else spx.order_rcm)(M)
            parts = np.zeros(1, np.int32)
            P = spx.plan_from_perm(M, rp, cp, tune=tune)
            xf = torch.empty_like(xs)
            for i in range(npool):
                spx.permute_x(P, xs[i], xf[i])
        elif form == "banded":
            from synth import gen_banded_like
            P = spx.plan_plain(spx.from_csr(gen_banded_like(A)), tune=tune)
            xf = xs
        else:
            fn = {"sb": spx.reorder_sb, "db": spx.reorder_db, "split": spx.split, "shp_rn": spx.reorder_rn,
                  "split_unit": lambda *a, **k: spx.split(*a, row_net_cost=1, **k)}[form]
            wb = args.window_bytes if form.startswith("split") else 0
            P, rp, cp, parts = fn(M, args.K, wb, args.seed, tune=tune)
            xf = torch.empty_like(xs)
            for i in range(npool):
                spx.permute_x(P, xs[i], xf[i])
        prep = time.time() - t
        if tune is None and not args.no_autotune:
            # schedule autotuning by the library (as OSKI tunes its kernel):
            # ten products per candidate schedule, the fastest is kept
            t = time.time()
            _, _, cand = spx.plan_autotune(P, xf[0], y, reps=10, report=True)
            log(f"{form}: autotune {time.time() - t:.1f} s, ms per candidate "
                + " ".join(f"{schedule_name(tune_list(c))}={v:.4f}" for c, v in zip(spx.autotune_candidates(), cand)))
        inf = P.info()
        plan_key = "identity" if form in ("plain", "banded") else plan_sha256(rp, cp, parts, inf["nleaves"])
        total_ms, kern_ms = time_form(spx, torch, P, form, xf, y, args.warmup, args.steps)
        r = {"ms_per_step": round(total_ms, 5), "kernel_ms": round(kern_ms, 5),
             "GBs": round(nb / (total_ms * 1e-3) / 1e9, 1),
             "kernel_GBs": round(nb / (kern_ms * 1e-3) / 1e9, 1),
             "GFLOPs": round(2 * A.nnz / (total_ms * 1e-3) / 1e9, 1),
             "prep_s": round(prep, 2), "partition_s": round(inf["partition_seconds"], 2),
             "nleaves": inf["nleaves"], "ntiles": inf["ntiles"], "nslots": inf["nslots"],
             "sum_lambda_col": inf["sum_lambda_col"], "sum_lambda_row": inf["sum_lambda_row"],
             "border_row_nnz": inf["border_row_nnz"], "bytes_matrix": inf["bytes_matrix"],
             "tune": [inf["wg_size"], inf["nnz_per_block"], inf["blocks_per_tile"],
                      inf["window_entries"], inf["tiles_per_group"], inf["wave_blocks"], inf["pipeline"],
                      inf["scan_reduce"], inf["sort_gathers"], inf["compact_index"]],
             "window_nnz": inf["window_nnz"],
             "plan_sha256": plan_key}
        if inf["compact_index"]:
            # 16-bit indices: the kernel has 2 bytes fewer to read per such nonzero
            nb_c = nb - 2 * inf["nnz_compact"]
            r.update({"nnz_compact": inf["nnz_compact"], "alg_bytes": nb_c,
                      "kernel_GBs_alg": round(nb_c / (kern_ms * 1e-3) / 1e9, 1)})
        if args.cold:
            cold_ms = time_cold(spx, torch, P, form, xf, y)
            r["cold_ms_per_step"] = round(cold_ms, 5)
            r["cold_GBs"] = round(nb / (cold_ms * 1e-3) / 1e9, 1)
        results[form] = r
        log(form, json.dumps(r))
        if form not in ("plain", "banded"):
            del xf
        del P
        torch.cuda.empty_cache()

    if "plain" in results:
        # Table 3's method: the reordering overhead (partition, ordering and
        # plan building on the host) in units of one plain CSR product on the
        # same GPU, and the number of products after which the faster form
        # has paid it back
        tp = results["plain"]["ms_per_step"]
        for k, r in results.items():
            if k in ("plain", "banded"):
                continue
            # Table 2's normalized time: the form's time over plain CSR's
            r["normalized_time"] = round(r["ms_per_step"] / tp, 3)
            over_ms = 1e3 * r["prep_s"]
            r["overhead_plain_products"] = round(over_ms / tp, 1)
            gain = tp - r["ms_per_step"]
            r["amortization_products"] = round(over_ms / gain) if gain > 0 else None
    # the headline is the best of the paper's proposed forms (Sections 3 and
    # 4); the comparison orderings and the banded stand-in are reported beside
    reord = {k: v for k, v in results.items() if k in ("sb", "db", "split", "split_unit")} or results
    best = max(reord, key=lambda k: reord[k]["GBs"])
    hb = results[best]
    out = {
        "metric": "SpMV effective HBM GB/s (% of peak) + GFLOP/s, reordered/split vs plain CSR",
        "value": hb["GBs"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hb["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"n={A.n} irregular Zipf(2.0) matrix, nnz={A.nnz}, "
                               f"64 hidden blocks; form {best}, K={args.K}",
                   "form": best, "K": args.K, "nnz": A.nnz, "m": A.m, "n": A.n},
        "pct_of_peak": round(100 * hb["GBs"] / PEAK_HBM_GBS, 2),
        "gflops": hb["GFLOPs"],
        "forms": results,
    }
    if "plain" in results:
        out["speedup_vs_plain"] = round(results["plain"]["ms_per_step"] / hb["ms_per_step"], 3)
    # with 16-bit indices the algorithmic bytes are the ones that layout reads
    ach = hb.get("kernel_GBs_alg", hb["kernel_GBs"])
    out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                       "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                       "traffic": measured_traffic(best, A.nnz, schedule_name(hb["tune"]), hb["plan_sha256"]),
                       "kernel": f"{kernel_name(hb['tune'])} ({best}, {schedule_name(hb['tune'])})",
                       "alg_bytes_per_launch": hb.get("alg_bytes", nb), "kernel_source_sha256": kernel_source_sha256()}
    if not args.no_stream:
        out["stream_read_GBs"] = round(stream_ceiling(spx, torch), 1)
        out["pct_of_stream_ceiling"] = round(100 * hb["GBs"] / out["stream_read_GBs"], 2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, xs_host)
    if not args.no_extensions:
        out["extensions"] = extension_summaries(args, torch, spx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
