"""Summaries of rocprofv3 output for the SpMV kernels.

  python -m paper_1203_2739_amd.rocprof_summary stats  <kernel_stats.csv>
  python -m paper_1203_2739_amd.rocprof_summary pmc    <counter_collection.csv> [name filter] [runs]
  python -m paper_1203_2739_amd.rocprof_summary traffic <out dir> <form> <kernel filter> <nnz> <alg bytes> <plan sha256> <tune> <schedule>

``traffic`` writes the summary that ``bench.py`` reads for roofline.traffic
(profiles/spmv_c2_<form>_traffic.txt):
<out dir> holds the five runs listed in the summary (prof, pmcf, pmcw, calf,
calw); FETCH_SIZE and WRITE_SIZE of the SpMV kernel are scaled by what they
read for a copy kernel of 1 GiB.  <plan sha256> is the ``plan_sha256`` that
the profiled bench runs print for the form: the figures hold for that plan
layout only.

``stats`` lists kernels by total time with call count and mean duration.
``pmc`` lists, per kernel and grid size, the mean per-dispatch value of each
collected counter (FETCH_SIZE and WRITE_SIZE are in KiB per dispatch); with
[runs], per consecutive run of the matching dispatches instead.
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys
from collections import defaultdict

SRCS = [os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f)
        for f in ("kernels.hip", "plan.cpp", "sched_limits.h")]


def kernel_source_sha256() -> str:
    """Hash of the kernel source and of the plan builder that lays out what it
    reads: counter figures are valid for these sources only."""
    h = hashlib.sha256()
    for path in SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name: str, width: int = 70) -> str:
    name = name.split("(")[0] if name.startswith("void ") else name
    return name if len(name) <= width else name[:width - 3] + "..."


def stats(path: str):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print(f"{'kernel':72s} {'calls':>6s} {'mean us':>10s} {'total ms':>10s} {'%':>6s}")
    for r in rows:
        print(f"{short(r['Name']):72s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")


def pmc(path: str, filt: str = "", groups: int = 0):
    """Mean counters per (kernel, grid); with groups > 0, the matching
    dispatches in dispatch order are cut into that many consecutive runs of
    equal length (one per configuration a script ran in turn) and each run is
    averaged on its own."""
    acc = defaultdict(lambda: defaultdict(list))
    seq = defaultdict(lambda: defaultdict(float))
    for r in csv.DictReader(open(path)):
        k = r["Kernel_Name"]
        if filt and filt not in k:
            continue
        acc[(k, r.get("Grid_Size", ""))][r["Counter_Name"]].append(float(r["Counter_Value"]))
        seq[int(r.get("Dispatch_Id", 0))][r["Counter_Name"]] += float(r["Counter_Value"])
    if groups > 0:
        ids = sorted(seq)
        size = len(ids) // groups
        for g in range(groups):
            part = ids[g * size:(g + 1) * size]
            names = sorted({c for i in part for c in seq[i]})
            vals = [f"{c}={sum(seq[i][c] for i in part) / len(part):.1f}" for c in names]
            print(f"run {g} (dispatches {part[0]}..{part[-1]}, n={len(part)}): " + ", ".join(vals))
        return
    for (k, g), cs in sorted(acc.items(), key=lambda kv: kv[0]):
        parts = [f"{c}={sum(v) / len(v):.1f} (n={len(v)})" for c, v in sorted(cs.items())]
        print(f"{short(k)} grid={g}: " + ", ".join(parts))


def _mean_by_kernel(path, filt):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if filt in r["Kernel_Name"]:
            acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic(out, form, filt, nnz, alg, plan, tune, sched, src_sha=None):
    """Writes profiles/spmv_c2_<form>_traffic.txt from the five runs in <out>;
    <tune> is the bench.py --tune argument the runs used and <sched> its
    schedule name (bench.schedule_name); <src_sha> the kernel_source_sha256
    the profiled bench run printed (the sources it ran), by default the hash
    of the sources here."""
    copy_kib = (1 << 30) / 1024
    calf = list(_mean_by_kernel(os.path.join(out, "calf", "pmc_counter_collection.csv"), "stream_copy").values())[0]
    calw = list(_mean_by_kernel(os.path.join(out, "calw", "pmc_counter_collection.csv"), "stream_copy").values())[0]
    ff, fw = copy_kib / calf, copy_kib / calw
    fe = _mean_by_kernel(os.path.join(out, "pmcf", "pmc_counter_collection.csv"), filt)
    wr = _mean_by_kernel(os.path.join(out, "pmcw", "pmc_counter_collection.csv"), filt)
    (kname, f_kib), = fe.items()
    w_kib = wr[kname]
    st = [r for r in csv.DictReader(open(os.path.join(out, "prof", "run_kernel_stats.csv"))) if filt in r["Name"]][0]
    fb, wb = f_kib * 1024 * ff, w_kib * 1024 * fw
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        f"spmv_c2_{form}_traffic.txt")
    args = f"--forms {form} --tune {tune} --no-cpu-baseline --no-stream --no-extensions"
    with open(path, "w") as o:
        o.write(f"""SpMV kernel ({form} form) on the n=10^6 irregular matrix (nnz={nnz}), K=64, schedule {sched}
(the one bench.py's autotuning picked: threads x nonzeros per thread, w = wave blocks, s = scan row sums, g = gather-sorted blocks, p = pipelined tiles,
t = tiles per row group, W = LDS window entries).

Commands (run from /tmp with TMPDIR=/tmp; R = repository root, OUT = output directory):
  rocprofv3 --kernel-trace --stats --output-format csv -d OUT/prof -o run -- python3 R/bench.py {args} --steps 20 --warmup 3
  rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/pmcf -o pmc -- python3 R/bench.py {args} --steps 5 --warmup 1
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/pmcw -o pmc -- python3 R/bench.py {args} --steps 5 --warmup 1
  rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/calf -o pmc -- python3 R/bench.py --only-stream
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/calw -o pmc -- python3 R/bench.py --only-stream
  python -m paper_1203_2739_amd.rocprof_summary traffic OUT {form} "{filt}" {nnz} {alg} {plan} {tune} {sched} {src_sha or kernel_source_sha256()}

Kernel trace (--stats): {st['Name'][:100]}
  calls {st['Calls']}, mean {float(st['AverageNs']) / 1e3:.2f} us, min {float(st['MinNs']) / 1e3:.2f} us, max {float(st['MaxNs']) / 1e3:.2f} us

Calibration on stream_copy_kernel of 1 GiB (reads 1 GiB, writes 1 GiB):
  FETCH_SIZE {calf:.1f} KiB per dispatch -> factor {ff:.4f}
  WRITE_SIZE {calw:.1f} KiB per dispatch -> factor {fw:.4f}

Counters per dispatch of the SpMV kernel (mean over dispatches):
  FETCH_SIZE {f_kib:.1f} KiB -> {fb / 1e6:.1f} MB calibrated
  WRITE_SIZE {w_kib:.1f} KiB -> {wb / 1e6:.1f} MB calibrated
  algorithmic bytes per product (12 nnz + 4 (m+1) + 8 n + 8 m): {alg / 1e6:.1f} MB
  traffic / algorithmic = {(fb + wb) / alg:.2f}

nnz: {nnz}
schedule: {sched}
kernel_source_sha256: {src_sha or kernel_source_sha256()}
plan_sha256: {plan}
traffic_bytes_per_launch: {int(fb + wb)}
""")
    print(open(path).read())


if __name__ == "__main__":
    if len(sys.argv) >= 10 and sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), int(sys.argv[6]), sys.argv[7],
                sys.argv[8], sys.argv[9], sys.argv[10] if len(sys.argv) > 10 else None)
        sys.exit(0)
    if len(sys.argv) < 3 or sys.argv[1] not in ("stats", "pmc"):
        print(__doc__)
        sys.exit(2)
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    else:
        pmc(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "", int(sys.argv[4]) if len(sys.argv) > 4 else 0)
