"""GPU parity of the SpMV forms against the CPU oracle, through the C ABI.

Binary64 results must satisfy |y - y_ref| <= 1e-12 * sum_j |a_ij x_j| per
entry; with small-integer values and inputs every summation order is exact,
so those cases are compared bit for bit.
"""
import numpy as np
import pytest

from gpu_util import assert_close_rowwise, dev, host, integer_problem
from synth import CSR, gen_c1, gen_uniform_zipf, gen_vectors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
spx = pytest.importorskip("paper_1203_2739_amd")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_plain(A, x, tune=None):
    M = spx.from_csr(A)
    P = spx.plan_plain(M, tune=tune)
    xd = dev(x)
    yd = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
    spx.spmv(P, xd, yd)
    return host(yd)


def run_reordered(A, x, form, K, window_bytes=0, tune=None, seed=0):
    M = spx.from_csr(A)
    fn = {"sb": spx.reorder_sb, "db": spx.reorder_db, "split": spx.split, "rn": spx.reorder_rn}[form]
    P, rp, cp, part = fn(M, K, window_bytes, seed, tune=tune)
    xh = dev(x[cp])
    yh = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
    if form == "split":
        spx.spmv_split(P, xh, yh)
    else:
        spx.spmv(P, xh, yh)
    return host(yh), rp, cp, part, P


TUNES = [None,
         dict(wg_size=64),
         dict(wg_size=512, blocks_per_tile=3),
         dict(reduce_iters=1, wg_size=256),
         dict(blocks_per_tile=2, xcd_remap=-1),
         dict(wg_size=128, nnz_per_block=1024, reduce_iters=7, blocks_per_tile=200),
         dict(wg_size=128, nnz_per_block=1024, xcd_remap=-1),
         dict(wg_size=256, tiles_per_group=5),
         dict(wg_size=1024, tiles_per_group=4, window_entries=15360),
         dict(wg_size=256, wave_blocks=1),
         dict(wg_size=512, wave_blocks=1, nnz_per_block=512, reduce_iters=5),
         dict(wg_size=512, wave_blocks=1, tiles_per_group=3, xcd_remap=-1),
         dict(wg_size=512, wave_blocks=1, blocks_per_tile=3),
         dict(wg_size=512, pipeline=1, tiles_per_group=7),
         dict(wg_size=256, pipeline=1, blocks_per_tile=5, nnz_per_block=2048, reduce_iters=4),
         dict(wg_size=1024, pipeline=1, tiles_per_group=2, xcd_remap=-1),
         dict(wg_size=128, scan_reduce=1),
         dict(wg_size=512, scan_reduce=1),
         dict(wg_size=1024, scan_reduce=1, xcd_remap=-1),
         dict(wg_size=256, scan_reduce=1, reduce_iters=1),
         dict(wg_size=128, sort_gathers=1),
         dict(wg_size=512, sort_gathers=1),
         dict(wg_size=256, sort_gathers=1, xcd_remap=-1, reduce_iters=3),
         dict(wg_size=512, nnz_per_block=4096, sort_gathers=1),
         dict(wg_size=1024, sort_gathers=1),
         dict(wg_size=256, sort_gathers=1, scan_reduce=1, xcd_remap=-1),
         dict(wg_size=1024, sort_gathers=1, scan_reduce=1),
         dict(wg_size=512, nnz_per_block=4096, sort_gathers=1, scan_reduce=1),
         dict(wg_size=256, compact_index=1),
         dict(wg_size=512, compact_index=1, xcd_remap=-1, reduce_iters=5)]
SCAN_TUNES = [t for t in TUNES if t and t.get("scan_reduce")]
SORTED_TUNES = [t for t in TUNES if t and t.get("sort_gathers")]


@pytest.mark.parametrize("ti", range(len(TUNES)))
def test_plain_c1(orc, ti):
    A = gen_c1()
    x = gen_vectors(101, A.n)[0]
    y = run_plain(A, x, TUNES[ti])
    assert_close_rowwise(y, orc.spmv(A, x), orc.abs_rowsum(A, x), "plain C1")


def test_plain_c1_integer_exact(orc):
    A, x = integer_problem(gen_c1(), 5)
    assert np.array_equal(run_plain(A, x), orc.spmv(A, x))
    for t in SCAN_TUNES + SORTED_TUNES:
        assert np.array_equal(run_plain(A, x, t), orc.spmv(A, x)), t


@pytest.mark.parametrize("form", ["sb", "db", "split", "rn"])
@pytest.mark.parametrize("K", [1, 8])
def test_reordered_c1(orc, form, K):
    A = gen_c1()
    x = gen_vectors(102, A.n)[0]
    y, rp, cp, part, P = run_reordered(A, x, form, K)
    assert_close_rowwise(y, orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp], f"{form} C1")
    if form == "split":
        ys = orc.split_spmv(A, part, K, x)
        assert_close_rowwise(y, ys[rp], orc.abs_rowsum(A, x)[rp], "split vs part order")


@pytest.mark.parametrize("form", ["sb", "db", "split", "rn"])
def test_reordered_c1_integer_exact(orc, form):
    A, x = integer_problem(gen_c1(), 9)
    y, rp, cp, part, P = run_reordered(A, x, form, 8)
    assert np.array_equal(y, orc.spmv(A, x)[rp])
    for t in (SCAN_TUNES[1], SORTED_TUNES[1], SORTED_TUNES[-1]):
        y, rp, cp, part, P = run_reordered(A, x, form, 8, tune=t)
        assert np.array_equal(y, orc.spmv(A, x)[rp]), t


WINDOW_TUNES = [dict(window_entries=4096, blocks_per_tile=64, wg_size=128),
                dict(window_entries=4096, blocks_per_tile=64, wg_size=256),
                dict(window_entries=8192, blocks_per_tile=32),
                dict(window_entries=16384, blocks_per_tile=16),
                dict(window_entries=16384, wg_size=512, blocks_per_tile=32),
                dict(window_entries=16384, wg_size=512, tiles_per_group=1),
                dict(window_entries=15360, wg_size=1024, tiles_per_group=1),
                dict(window_entries=4096, wg_size=256, tiles_per_group=1),
                dict(window_entries=15360, wg_size=1024, tiles_per_group=1, wave_blocks=1),
                dict(window_entries=8192, wg_size=256, tiles_per_group=1, wave_blocks=1),
                dict(window_entries=8192, wg_size=512, blocks_per_tile=64, wave_blocks=1, nnz_per_block=512),
                dict(window_entries=16384, wg_size=512, tiles_per_group=1, pipeline=1),
                dict(window_entries=8192, wg_size=256, blocks_per_tile=40, pipeline=1)]


@pytest.mark.parametrize("form", ["sb", "db", "split"])
@pytest.mark.parametrize("wi", range(len(WINDOW_TUNES)))
def test_windows_c1(orc, form, wi):
    """LDS x windows (leaves refined to the window budget, tiles of several
    blocks) give the same products."""
    A = gen_c1()
    x = gen_vectors(103, A.n)[0]
    t = WINDOW_TUNES[wi]
    wb = t["window_entries"] * 8
    y, rp, cp, part, P = run_reordered(A, x, form, 4, window_bytes=wb, tune=t)
    inf = P.info()
    assert inf["window_entries"] > 0 and inf["window_nnz"] > 0
    assert_close_rowwise(y, orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp], f"{form} window")
    Ai, xi = integer_problem(A, 4)
    yi, rp, _, _, _ = run_reordered(Ai, xi, form, 4, window_bytes=wb, tune=t)
    assert np.array_equal(yi, orc.spmv(Ai, xi)[rp])


def test_split_accumulate(orc):
    A = gen_c1()
    x = gen_vectors(104, A.n)[0]
    y0 = gen_vectors(105, A.m)[0]
    M = spx.from_csr(A)
    P, rp, cp, part = spx.split(M, 8, 0, 0)
    yd = dev(y0[rp])
    spx.spmv_split(P, dev(x[cp]), yd, accumulate=1)
    ref = orc.split_spmv(A, part, 8, x, y0)
    bound = orc.abs_rowsum(A, x) + np.abs(y0)
    assert_close_rowwise(host(yd), ref[rp], bound[rp], "split accumulate")


@pytest.mark.parametrize("form", ["sb", "db", "split"])
def test_permute_roundtrip(orc, form):
    A = gen_c1()
    x = gen_vectors(106, A.n)[0]
    M = spx.from_csr(A)
    fn = {"sb": spx.reorder_sb, "db": spx.reorder_db, "split": spx.split}[form]
    P, rp, cp, _ = fn(M, 8, 0, 0)
    xd = dev(x)
    xh = torch.empty_like(xd)
    spx.permute_x(P, xd, xh)
    assert np.array_equal(host(xh), x[cp])
    yh = torch.empty(A.m, dtype=torch.float64, device="cuda")
    spx.spmv(P, xh, yh)
    y = torch.empty_like(yh)
    spx.unpermute_y(P, yh, y)
    assert_close_rowwise(host(y), orc.spmv(A, x), orc.abs_rowsum(A, x), "P A Q (Q^T x) = P (A x)")


def odd_matrix(seed, m, n, long_len=0, empty_frac=0.3):
    """Rectangular, many empty rows, optionally one very long row."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, 12, size=m)
    deg[rng.random(m) < empty_frac] = 0
    if long_len:
        deg[m // 3] = long_len
    deg = np.minimum(deg, n)
    rows = np.repeat(np.arange(m), deg)
    cols = np.concatenate([np.sort(rng.choice(n, d, replace=False)) for d in deg]) if deg.sum() else np.zeros(0, int)
    rp = np.zeros(m + 1, np.int64)
    np.cumsum(deg, out=rp[1:])
    return CSR(m, n, rp, cols.astype(np.int32), rng.uniform(-1, 1, rows.size))


@pytest.mark.parametrize("shape", [(1, 1), (1, 50000), (777, 3), (5000, 20000), (20000, 5000)])
@pytest.mark.parametrize("long_len", [0, 3000, 20000])
def test_edge_shapes(orc, shape, long_len):
    m, n = shape
    A = odd_matrix(m * 7 + n, m, n, long_len=long_len if n >= long_len else 0)
    x = gen_vectors(107, n)[0]
    for ti in (0, 1, 3, 5, TUNES.index(SCAN_TUNES[0]), TUNES.index(SCAN_TUNES[-1]), len(TUNES) - 1):
        y = run_plain(A, x, TUNES[ti])
        assert_close_rowwise(y, orc.spmv(A, x), orc.abs_rowsum(A, x), f"plain {shape} {long_len}")
    if A.nnz:
        for form in ("sb", "db", "split"):
            y, rp, cp, _, _ = run_reordered(A, x, form, 4)
            assert_close_rowwise(y, orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp], f"{form} {shape}")


def test_empty_matrices(orc):
    for m, n in [(0, 0), (0, 5), (5, 0), (7, 9), (3000, 10)]:
        A = CSR(m, n, np.zeros(m + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
        M = spx.from_csr(A)
        for t in [None] + SCAN_TUNES[:1] + SORTED_TUNES[:1] + SORTED_TUNES[-1:]:
            P = spx.plan_plain(M, tune=t)
            yd = torch.full((max(m, 1),), np.nan, dtype=torch.float64, device="cuda")
            xd = torch.ones(max(n, 1), dtype=torch.float64, device="cuda")
            spx.spmv(P, xd, yd)
            if m:
                assert np.all(host(yd)[:m] == 0.0), t
        if m and n:
            P, rp, cp, _ = spx.split(M, 2, 0, 0)
            yd[:] = float("nan")
            spx.spmv_split(P, xd, yd)
            assert np.all(host(yd)[:m] == 0.0)


def test_rows_at_block_capacity(orc):
    """Rows whose lengths straddle the staging capacity (NT - 3, NT, NT + 1)
    and the long-row threshold."""
    lens = [1021, 1022, 1024, 1025, 2045, 2046, 2048, 2049, 1, 0, 4093, 4096, 8190, 3, 0, 0, 2]
    n = 9000
    rng = np.random.default_rng(3)
    cols = np.concatenate([np.sort(rng.choice(n, d, replace=False)) for d in lens])
    rp = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    A = CSR(len(lens), n, rp, cols.astype(np.int32), rng.uniform(-1, 1, cols.size))
    x = gen_vectors(108, n)[0]
    for t in TUNES:
        y = run_plain(A, x, t)
        assert_close_rowwise(y, orc.spmv(A, x), orc.abs_rowsum(A, x), f"capacity {t}")


def test_larger_irregular(orc):
    """Several thousand tiles, Zipf rows up to 5,000 nonzeros."""
    A = gen_uniform_zipf(31, 200_000, 4_000_000, 5000, diagonal=True)
    x = gen_vectors(109, A.n)[0]
    y = run_plain(A, x)
    assert_close_rowwise(y, orc.spmv(A, x), orc.abs_rowsum(A, x), "zipf 200k")
    y, rp, cp, part, P = run_reordered(A, x, "split", 16)
    assert_close_rowwise(y, orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp], "zipf 200k split")
    y, rp, cp, part, P = run_reordered(A, x, "db", 16, window_bytes=8192 * 8,
                                       tune=dict(window_entries=8192, blocks_per_tile=16))
    assert_close_rowwise(y, orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp], "zipf 200k db window")
    for t in SORTED_TUNES + SCAN_TUNES:
        y = run_plain(A, x, t)
        assert_close_rowwise(y, orc.spmv(A, x), orc.abs_rowsum(A, x), f"zipf 200k {t}")
    y, rp, cp, part, P = run_reordered(A, x, "split", 16, tune=SORTED_TUNES[1])
    assert_close_rowwise(y, orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp], "zipf 200k split sorted")


def test_rows_cut_into_segments(orc):
    """Rows longer than one block are summed by several workgroups whose
    partial sums the last one adds up, in plain, split and accumulating split
    products, twice in a row (the arrival counters reset themselves)."""
    lens = [3, 70000, 0, 1, 140000, 65536, 65537, 2, 1021, 5]
    n = 150000
    rng = np.random.default_rng(5)
    cols = np.concatenate([np.sort(rng.choice(n, d, replace=False)) for d in lens])
    rp = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    A = CSR(len(lens), n, rp, cols.astype(np.int32), rng.uniform(-1, 1, cols.size))
    x = gen_vectors(110, n)[0]
    ref, den = orc.spmv(A, x), orc.abs_rowsum(A, x)
    for t in (None, dict(wg_size=64), dict(wg_size=512), dict(blocks_per_tile=3), dict(wg_size=256, scan_reduce=1),
              dict(wg_size=512, sort_gathers=1), dict(wg_size=512, sort_gathers=1, scan_reduce=1)):
        M = spx.from_csr(A)
        P = spx.plan_plain(M, tune=t)
        assert P.info()["nlong_rows"] >= 4
        xd = dev(x)
        for rep in range(2):
            yd = torch.full((A.m,), 7.0, dtype=torch.float64, device="cuda")
            spx.spmv(P, xd, yd)
            assert_close_rowwise(host(yd), ref, den, f"segments plain {t} {rep}")
        y, rp, cp, part, P = run_reordered(A, x, "split", 2, tune=t)
        assert_close_rowwise(y, ref[rp], den[rp], f"segments split {t}")
        xh = torch.empty_like(xd)
        spx.permute_x(P, xd, xh)
        yh = dev(np.full(A.m, 0.5))
        spx.spmv_split(P, xh, yh, accumulate=1)
        assert_close_rowwise(host(yh) - 0.5, ref[rp], den[rp] + 1.0, f"segments split acc {t}")
        yh.fill_(np.nan)
        spx.split_prepare_y(P, yh)
        spx.spmv_split(P, xh, yh, accumulate=2)
        # rows owned by one leaf are stored, so no NaN survives
        assert_close_rowwise(host(yh), ref[rp], den[rp], f"segments split prezeroed {t}")


def test_stream_probe():
    nbytes = 64 << 20
    src = torch.arange(nbytes // 8, dtype=torch.float64, device="cuda")
    sink = torch.zeros(spx.stream_sink_len(nbytes), dtype=torch.float64, device="cuda")
    spx.stream_read(src, nbytes, sink)
    assert abs(host(sink).sum() - host(src).sum()) <= 1e-9 * abs(host(src).sum())
    dst = torch.zeros_like(src)
    spx.stream_copy(src, dst, nbytes)
    assert torch.equal(dst, src)


def test_split_deterministic_and_retune(orc):
    """Split products stay within tolerance after retunes that change which
    slots are long (the long-slot scratch is rebuilt), over repeated calls
    (the arrival counters reset themselves)."""
    A = gen_uniform_zipf(41, 30_000, 600_000, 3000, diagonal=True)
    x = gen_vectors(111, A.n)[0]
    M = spx.from_csr(A)
    P, rp, cp, part = spx.split(M, 8, 0, 4)
    xd = dev(x)
    xh = torch.empty_like(xd)
    spx.permute_x(P, xd, xh)
    ref, den = orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp]
    for t in (None, dict(wg_size=512), dict(wg_size=64), dict(reduce_iters=2, wg_size=256),
              dict(wg_size=512, scan_reduce=1), dict(wg_size=512, sort_gathers=1), dict(wg_size=128)):
        spx.plan_retune(P, t)
        outs = []
        for rep in range(3):
            yh = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
            spx.spmv_split(P, xh, yh)
            outs.append(host(yh))
        for o in outs:
            assert_close_rowwise(o, ref, den, f"split retune {t}")


@pytest.mark.parametrize("form", ["sb", "db", "split"])
@pytest.mark.parametrize("K", [3, 17])
def test_products_from_random_partitions(orc, form, K):
    """Products of plans built from arbitrary partitions (random parts, so
    borders are large and parts uneven) match the oracle."""
    A = gen_c1()
    rng = np.random.default_rng(K)
    if form == "split":
        parts = rng.integers(0, K, A.nnz).astype(np.int32)
    else:
        parts = rng.integers(0, K + (1 if form == "db" else 0), A.m).astype(np.int32)
    M = spx.from_csr(A)
    P, rp, cp = spx.plan_from_parts(M, form, K, parts)
    x = gen_vectors(112, A.n)[0]
    xd = dev(x)
    xh = torch.empty_like(xd)
    spx.permute_x(P, xd, xh)
    yh = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
    spx.spmv(P, xh, yh)
    assert_close_rowwise(host(yh), orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp], f"{form} K={K}")


@pytest.mark.parametrize("name", ["bfs", "rcm"])
def test_comparison_orderings_c1(orc, name):
    """Products on the sBFS and sRCM orders (Section 5.1) in their reordered
    space, against the oracle: within the per-entry bound, and bit for bit
    on small integers."""
    A = gen_c1()
    M = spx.from_csr(A)
    rp, cp = getattr(spx, "order_" + name)(M)
    P = spx.plan_from_perm(M, rp, cp)
    x = gen_vectors(107, A.n)[0]
    xd = dev(x)
    xh = torch.empty_like(xd)
    spx.permute_x(P, xd, xh)
    yh = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
    spx.spmv(P, xh, yh)
    assert_close_rowwise(host(yh), orc.spmv(A, x)[rp], orc.abs_rowsum(A, x)[rp], name)
    y = torch.empty_like(yh)
    spx.unpermute_y(P, yh, y)
    assert_close_rowwise(host(y), orc.spmv(A, x), orc.abs_rowsum(A, x), name + " unpermuted")
    Ai, xi = integer_problem(A, 12)
    Mi = spx.from_csr(Ai)
    Pi = spx.plan_from_perm(Mi, rp, cp)
    yi = torch.empty(A.m, dtype=torch.float64, device="cuda")
    spx.spmv(Pi, dev(xi[cp]), yi)
    assert np.array_equal(host(yi), orc.spmv(Ai, xi)[rp])


@pytest.mark.parametrize("kind", ["random", "temporal", "spatial", "band"])
def test_locality_matrices(orc, kind):
    """The locality workload's patterns (n = 60,000) under row blocks,
    gather-sorted blocks and scan blocks match the oracle."""
    from synth import gen_locality
    A = gen_locality(kind, seed=9, n=60_000, window=4096)
    x = gen_vectors(112, A.n)[0]
    ref, den = orc.spmv(A, x), orc.abs_rowsum(A, x)
    for t in (dict(wg_size=512), dict(wg_size=1024, sort_gathers=1), dict(wg_size=256, scan_reduce=1),
              dict(wg_size=256, compact_index=1)):
        assert_close_rowwise(run_plain(A, x, t), ref, den, f"{kind} {t}")
    # banded rows: every block reads 16-bit indices, integer data exact
    if kind == "band":
        Ai, xi = integer_problem(A, 21)
        assert np.array_equal(run_plain(Ai, xi, dict(wg_size=512, compact_index=1)), orc.spmv(Ai, xi))
