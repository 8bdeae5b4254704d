"""Host-side pieces of the measurement: the algorithmic byte count, the
lookup of committed counter summaries, the refusal of several GPUs, and the
rocprofv3 summary tool on small hand-made CSV files."""
import csv
import os
import subprocess
import sys

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_alg_bytes():
    import bench
    # 12 bytes per nonzero, 4 per row pointer, x read once and y written once
    assert bench.alg_bytes(3, 5, 7) == 12 * 7 + 4 * 4 + 8 * 5 + 8 * 3


def test_traffic_lookup_checks_source_schedule_matrix_and_plan():
    import bench
    from paper_1203_2739_amd.rocprof_summary import kernel_source_sha256
    keys = ("nnz", "schedule", "kernel_source_sha256", "plan_sha256", "traffic_bytes_per_launch")
    import glob
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "spmv_c2_*_traffic.txt")))
    for path in paths:
        form = os.path.basename(path)[len("spmv_c2_"):-len("_traffic.txt")]
        kv = {k: v.strip() for k, v in (line.split(": ", 1) for line in open(path).read().splitlines()
                                        if ": " in line and line.split(": ", 1)[0] in keys)}
        nnz, sched, plan = int(kv["nnz"]), kv["schedule"], kv.get("plan_sha256", "")
        got = bench.measured_traffic(form, nnz, sched, plan)
        if kv["kernel_source_sha256"] == kernel_source_sha256() and plan:
            assert got == int(kv["traffic_bytes_per_launch"])
        else:
            assert got is None
        assert bench.measured_traffic(form, nnz + 1, sched, plan) is None
        assert bench.measured_traffic(form, nnz, "1x1", plan) is None
        assert bench.measured_traffic(form, nnz, sched, "0" * 64) is None
    assert bench.measured_traffic("no_such_form", 1, "1x1", "0" * 64) is None


def test_schedule_names():
    import bench
    assert bench.schedule_name([512, 2048, 1, -1, 0, 0]) == "512x4"
    assert bench.schedule_name([256, 256, 4, -1, 0, 1]) == "256x4w"
    assert bench.schedule_name([1024, 256, 1, 15360, 32, 1]) == "1024x4wt32W15360"
    assert bench.schedule_name([512, 2048, 1, 16384, 32, 0]) == "512x4t32W16384"
    assert bench.schedule_name([512, 2048, 1, -1, 0, 0, 0, 1]) == "512x4s"
    assert bench.schedule_name([512, 2048, 1, -1, 128, 0, 1, 0]) == "512x4pt128"
    assert bench.schedule_name([512, 2048, 1, -1, 0, 0, 0, 0, 1]) == "512x4g"
    assert bench.kernel_name([1024, 4096, 1, -1, 0, 0, 0, 0, 1]) == "spmv_sorted"
    assert bench.kernel_name([512, 2048, 1, -1, 0, 0, 0, 1, 1]) == "spmv_sorted_scan"
    assert bench.kernel_name([256, 256, 4, -1, 0, 1]) == "spmv_waves"
    assert bench.schedule_name([256, 1024, 1, -1, 0, 0, 0, 0, 0, 1]) == "256x4c"
    assert bench.kernel_name([256, 1024, 1, -1, 0, 0, 0, 0, 0, 1]) == "spmv_compact"


def test_plan_hash_sees_every_part_of_the_layout():
    import bench
    rp, cp, parts = np.arange(5), np.array([2, 0, 1]), np.array([0, 2, 5])
    h = bench.plan_sha256(rp, cp, parts, 1)
    assert h == bench.plan_sha256(rp.astype(np.int32), cp, parts, 1)
    assert h != bench.plan_sha256(rp[::-1], cp, parts, 1)
    assert h != bench.plan_sha256(rp, cp[[1, 0, 2]], parts, 1)
    assert h != bench.plan_sha256(rp, cp, np.array([0, 3, 5]), 1)
    assert h != bench.plan_sha256(rp, cp, parts, 2)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def test_rocprof_summary_tool(tmp_path, capsys):
    from paper_1203_2739_amd import rocprof_summary as rs
    stats = tmp_path / "k.csv"
    write_csv(stats, [{"Name": "kernA", "Calls": 2, "TotalDurationNs": 3000, "AverageNs": 1500, "Percentage": 75,
                       "MinNs": 1000, "MaxNs": 2000},
                      {"Name": "kernB", "Calls": 1, "TotalDurationNs": 1000, "AverageNs": 1000, "Percentage": 25,
                       "MinNs": 1000, "MaxNs": 1000}])
    rs.stats(str(stats))
    out = capsys.readouterr().out.splitlines()
    assert out[1].startswith("kernA") and "1.50" in out[1]
    pmc = tmp_path / "p.csv"
    write_csv(pmc, [{"Kernel_Name": "kernA", "Grid_Size": 64, "Counter_Name": "FETCH_SIZE", "Counter_Value": 10,
                     "Dispatch_Id": 1},
                    {"Kernel_Name": "kernA", "Grid_Size": 64, "Counter_Name": "FETCH_SIZE", "Counter_Value": 30,
                     "Dispatch_Id": 2}])
    rs.pmc(str(pmc), "kern")
    assert "FETCH_SIZE=20.0 (n=2)" in capsys.readouterr().out


def test_cpu_baseline_legs_agree_and_report_cores():
    """Both host legs run on a small matrix: the oracle on one thread and
    the OpenMP product on every core give identical results (checked inside)
    and report their thread counts and the CPU model."""
    import bench
    from synth import gen_c1, gen_vectors
    bench.build_cpu_leg()
    A = gen_c1()
    xs = gen_vectors(9, A.n, 4)
    out = bench.cpu_baseline(A, xs, budget_s=0.5, max_products=5)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["value"] > 0
    assert out["cpu_model"] and out["host_cpus"] >= 1
    assert out["all_cores"]["cores"] >= 1 and out["all_cores"]["value"] > 0


def test_locality_matrices():
    """The locality workload's matrices: 20 distinct sorted columns per row;
    random spans all of x, temporal stays inside its sliding window and
    reuses columns across nearby rows while a row's own columns are spread,
    spatial and band are runs of 20 consecutive columns (band at the
    diagonal)."""
    from synth import LOCALITY_KINDS, gen_locality
    n, deg, w = 50_000, 20, 4096
    mats = {k: gen_locality(k, seed=3, n=n, deg=deg, window=w) for k in LOCALITY_KINDS}
    rows = np.arange(n)
    for k, A in mats.items():
        assert A.m == A.n == n and A.nnz == n * deg
        c = A.colidx.reshape(n, deg).astype(np.int64)
        assert np.all(np.diff(c, axis=1) > 0) and c.min() >= 0 and c.max() < n, k
    ct = mats["temporal"].colidx.reshape(n, deg).astype(np.int64)
    lo = rows * (n - w) // n
    assert np.all(ct >= lo[:, None]) and np.all(ct < (lo + w)[:, None])
    # temporal: the 100 rows around any row read far fewer distinct columns
    # than entries; spatial: a row's 20 entries fit 2 or 3 lines of 16 entries
    blk = ct[1000:1100].reshape(-1)
    assert np.unique(blk).size < 0.9 * blk.size
    for k in ("spatial", "band"):
        c = mats[k].colidx.reshape(n, deg).astype(np.int64)
        assert np.all(c[:, -1] - c[:, 0] == deg - 1)
        assert np.all(np.apply_along_axis(lambda r: np.unique(r >> 4).size, 1, c[:200]) <= 3)
    cb = mats["band"].colidx.reshape(n, deg).astype(np.int64)
    assert np.all(np.abs(cb[:, deg // 2] - rows) <= deg)
    # spatial runs start anywhere: no reuse of columns between neighbouring rows
    cs = mats["spatial"].colidx.reshape(n, deg).astype(np.int64)
    assert np.mean(np.abs(cs[1:, 0] - cs[:-1, 0]) > deg) > 0.99


def test_gather_request_model_on_a_hand_counted_block():
    """32 rows of 64 nonzeros, all on columns 0..63 (four 128-byte lines of
    x); the 8 row groups give 8 blocks of 4 rows (256 entries) at 512 x 4.
    Row order: the j-th gather of quarter wave q reads columns 4 m + j of
    row q (m < 16), four lines; the four quarters read the same four lines,
    so a wave instruction needs 4 and a quarter 4: 0.25 and 0.0625 requests
    per nonzero.  Sorted order: every column four times; 16 consecutive
    sorted entries cover columns 4 a .. 4 a + 3, one line, and the four
    runs of a wave instruction (columns 16 q + 4 j ..) four lines: 0.0625
    both ways."""
    import bench
    import paper_1203_2739_amd as spx
    m = 32
    rowptr = np.arange(0, 64 * m + 1, 64, dtype=np.int32)
    colidx = np.tile(np.arange(64, dtype=np.int32), m)
    M = spx.csr_create_host(m, 64, rowptr, colidx, np.ones(64 * m))
    P = spx.plan_plain(M, tune=dict(wg_size=512, nnz_per_block=2048))
    bd, _ = P.export_sched()
    assert bd.shape[0] == 8 and np.all(bd[:, 1] - bd[:, 0] == 4)
    r = bench.gather_requests(P)
    assert r["nnz_counted"] == 64 * m
    assert (r["row16"], r["row64"], r["sorted16"], r["sorted64"]) == (0.25, 0.0625, 0.0625, 0.0625)
    assert bench.block_fill(P) == 256 / 2048
    # 4 rows of 64 in a block of 512 threads: 128 lanes a row, capped at 64,
    # so one read of the row's partial sums
    assert bench.reduction_chain(P) == 1.0
    # the split's per-leaf storage is read through its slots
    Ps, _, _, _ = spx.split(M, 2, 0, 0, tune=dict(wg_size=512, nnz_per_block=2048))
    rs = bench.gather_requests(Ps)
    assert rs["nnz_counted"] == 64 * m and 0 < rs["sorted64"] <= rs["row16"] <= 1
    assert bench.reduction_chain(Ps) >= 1
    # one request per nonzero when every entry has a line of its own
    M2 = spx.csr_create_host(m, 64 * 16, rowptr, (colidx * 16).astype(np.int32), np.ones(64 * m))
    r2 = bench.gather_requests(spx.plan_plain(M2, tune=dict(wg_size=512, nnz_per_block=2048)))
    assert (r2["row16"], r2["row64"]) == (1.0, 0.25)


def test_gather_model_workload_runs_on_the_host():
    """bench.py --workload gather_model needs no GPU: at n = 20,000 it prints
    one JSON line with the DB rows, the split row and the block measures,
    every sorted figure at most its row-order one."""
    import json
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "gather_model", "--n", "20000",
                        "--model-nnz", "100000"], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert [(x["form"], x["schedule"]) for x in line["rows"]] == [
        ("db", "512x4"), ("db", "1024x4g"), ("db", "1024x4s"), ("split", "1024x4g")]
    for x in line["rows"]:
        assert 0 < x["sorted64"] <= x["sorted16"] <= x["row16"] <= 1 and x["row64"] <= x["row16"]
    assert 0 < line["plain_block_fill"]["512x4"] < line["plain_block_fill"]["512x4s"] <= 1
    assert line["plain_median_reduction_chain"] >= 1
