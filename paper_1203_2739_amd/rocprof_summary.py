"""Summaries of rocprofv3 output for the SpMV kernels.

  python -m paper_1203_2739_amd.rocprof_summary stats  <kernel_stats.csv>
  python -m paper_1203_2739_amd.rocprof_summary pmc    <counter_collection.csv> [name filter]

``stats`` lists kernels by total time with call count and mean duration.
``pmc`` lists, per kernel and grid size, the mean per-dispatch value of each
collected counter (FETCH_SIZE and WRITE_SIZE are in KiB per dispatch).
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys
from collections import defaultdict

SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "kernels.hip")


def kernel_source_sha256() -> str:
    """Hash of the kernel source: counter figures are valid for this source only."""
    with open(SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


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


def pmc(path: str, filt: str = ""):
    acc = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        k = r["Kernel_Name"]
        if filt and filt not in k:
            continue
        acc[(k, r.get("Grid_Size", ""))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    for (k, g), cs in sorted(acc.items(), key=lambda kv: kv[0]):
        parts = [f"{c}={sum(v) / len(v):.1f} (n={len(v)})" for c, v in sorted(cs.items())]
        print(f"{short(k)} grid={g}: " + ", ".join(parts))


if __name__ == "__main__":
    if len(sys.argv) < 3 or sys.argv[1] not in ("stats", "pmc"):
        print(__doc__)
        sys.exit(2)
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    else:
        pmc(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "")
