"""Parity at full size, in the launch configurations the benchmark times.

The n = 10^6 irregular matrix (20 M nonzeros) as plain CSR, DB form at
K = 64 and split at K = 64 with 128 KB leaves, run through the same calls as
the benchmark (permute_x, split_prepare_y, accumulate = 2) under every
candidate schedule of the library's autotuner; the n = 5*10^5 SPD matrix in
binary64, binary32 and bfloat16 under the same schedules, and one refined
CG solve; all 256 members of the uneven batch with the autotuned schedule,
graph capture and replays.  Every output entry is compared with the
oracle's full product; permutations are checked bit for bit.
"""
import numpy as np
import pytest

from gpu_util import assert_close_rowwise, dev, host
from synth import CSR, gen_c3_spd, gen_vectors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
spx = pytest.importorskip("paper_1203_2739_amd")
bench = pytest.importorskip("bench")

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def is_permutation(p, n):
    return p.size == n and np.array_equal(np.sort(p), np.arange(n))


@pytest.fixture(scope="module")
def c2():
    A = bench.load_c2(1_000_000)
    x = gen_vectors(4242, A.n)[0]
    return A, x


@pytest.fixture(scope="module")
def c2_ref(orc, c2):
    A, x = c2
    return orc.spmv(A, x), orc.abs_rowsum(A, x)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("form", ["plain", "db", "split"])
def test_full_size_forms(orc, c2, c2_ref, form):
    A, x = c2
    ref, bound = c2_ref
    M = spx.from_csr(A)
    xd = dev(x)
    if form == "plain":
        P = spx.plan_plain(M)
        rp = np.arange(A.m)
        xh = xd
    else:
        fn = {"db": spx.reorder_db, "split": spx.split}[form]
        P, rp, cp, parts = fn(M, 64, 131072 if form == "split" else 0, 0)
        assert is_permutation(rp, A.m) and is_permutation(cp, A.n)
        xh = torch.empty_like(xd)
        spx.permute_x(P, xd, xh)
        assert np.array_equal(host(xh), x[cp])
        if form == "split":
            assert parts.size == A.nnz and parts.min() >= 0 and parts.max() < 64
    for tune in spx.autotune_candidates():
        spx.plan_retune(P, tune)
        y = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
        if form == "split":
            spx.split_prepare_y(P, y)
            spx.spmv_split(P, xh, y, accumulate=2)
        else:
            spx.spmv(P, xh, y)
        yh = host(y)
        assert not np.isnan(yh).any(), f"{form} {tune}: unwritten rows"
        assert_close_rowwise(yh, ref[rp], bound[rp], f"{form} {tune}")
    # the schedule the library's autotuner keeps gives the same products
    y = torch.empty(A.m, dtype=torch.float64, device="cuda")
    chosen, _ = spx.plan_autotune(P, xh, y, reps=3)
    y.fill_(np.nan)
    if form == "split":
        spx.spmv_split(P, xh, y)
    else:
        spx.spmv(P, xh, y)
    assert_close_rowwise(host(y), ref[rp], bound[rp], f"{form} autotuned {chosen}")


@pytest.fixture(scope="module")
def spd():
    A = gen_c3_spd(seed=3, n=500_000)
    M = spx.from_csr(A)
    P = spx.plan_plain(M)
    spx.plan_add_lowp(P, "f32")
    spx.plan_add_lowp(P, "bf16")
    return A, P


@pytest.mark.timeout(600)
def test_full_size_precision_products(orc, spd):
    """Every entry of the binary64, binary32 and bfloat16 products of the SPD
    matrix under every low-precision candidate schedule: binary64 within the
    per-entry bound of the sum order (its rows reach about 10^4 nonzeros, so
    gamma of the row length, not 1e-12, bounds it), the low precisions within
    the binary32 summation bound of the oracle's binary32 product of the same
    rounded values.  Gather-sorted and 16-bit-index schedules run binary64
    only."""
    A, P = spd
    x = gen_vectors(3000, A.n, 1)[0]
    x32 = x.astype(np.float32)
    deg = np.diff(A.rowptr).astype(np.float64)
    ref64, bound64 = orc.spmv(A, x), orc.abs_rowsum(A, x)
    g64 = np.maximum(1e-12, 1.01 * deg * 2.0 ** -53 / (1 - deg * 2.0 ** -53))
    f = orc.to_f32(A.vals)
    h = orc.f32_to_bf16(f)
    refs = {"f32": (orc.spmv_lowp(A, f, x32), f.astype(np.float64)),
            "bf16": (orc.spmv_lowp(A, None, x32, vals16=h), orc.bf16_bits_to_f32(h).astype(np.float64))}
    absq = {p: orc.abs_rowsum(CSR(A.m, A.n, A.rowptr, A.colidx, vq), x32.astype(np.float64))
            for p, (_, vq) in refs.items()}
    cands = [t for t in spx.autotune_candidates() if not t.get("tiles_per_group")]
    for tune in cands:
        spx.plan_retune(P, tune)
        y = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
        spx.spmv(P, dev(x), y)
        yh = host(y)
        assert np.all(np.abs(yh - ref64) <= g64 * bound64), f"f64 {tune}"
        if tune.get("sort_gathers") or tune.get("compact_index"):
            with pytest.raises(spx.SpxError):
                spx.spmv_lowp(P, "f32", dev(x32), torch.empty(A.m, dtype=torch.float32, device="cuda"))
            continue
        for prec, (ref, vq) in refs.items():
            y32 = torch.full((A.m,), np.nan, dtype=torch.float32, device="cuda")
            spx.spmv_lowp(P, prec, dev(x32), y32)
            got = host(y32).astype(np.float64)
            # both sides sum binary32 products of the same rounded values
            assert np.all(np.abs(got - ref.astype(np.float64)) <= 2.0 * (deg + 2) * U32 * absq[prec]), \
                f"{prec} {tune}"


@pytest.mark.timeout(300)
def test_full_size_refined_cg(orc, spd):
    """The benchmark's binary32 solve of A x = A 1 to relative residual 1e-10,
    under the schedule its autotuner picked there (512 threads)."""
    A, P = spd
    spx.plan_retune(P, dict(wg_size=512))
    b = orc.spmv(A, np.ones(A.n))
    xs = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st = spx.cg_ir(P, "f32", dev(b), xs, tol=1e-10, inner_tol=1e-3, max_outer=60, max_inner=5000)
    xh = host(xs)
    res = np.linalg.norm(b - orc.spmv(A, xh)) / np.linalg.norm(b)
    assert st["converged"] and res <= 2e-10, (st, res)
    # lambda_min(A) >= 1 (diagonal dominance with margin 1): ||x - 1|| <= ||b - A x||
    assert np.linalg.norm(xh - 1.0) <= np.linalg.norm(b - orc.spmv(A, xh)) * (1 + 1e-6)


@pytest.mark.timeout(900)
def test_full_size_batch_members(orc):
    """All 256 members of the uneven batch at full size, with the library's
    schedule search, graph capture and three replays (eager work and waits
    in between): every entry of every member and right-hand side against
    the oracle's product."""
    from synth import gen_c4_one
    mats, ks = [], []
    for j in range(256):
        A, k = gen_c4_one(j)
        mats.append(A)
        ks.append(k)
    assert set(ks) == {1, 8, 32}
    plans = [spx.plan_plain(spx.from_csr(A)) for A in mats]
    rng = np.random.default_rng(4444)
    X, Y, refs = [], [], []
    for A, k in zip(mats, ks):
        x = rng.uniform(-1, 1, (A.n, k))
        X.append(dev(x[:, 0].copy()) if k == 1 else dev(x))
        Y.append(torch.empty((A.m,) if k == 1 else (A.m, k), dtype=torch.float64, device="cuda"))
        absA = CSR(A.m, A.n, A.rowptr, A.colidx, np.abs(A.vals))
        refs.append((orc.spmm(A, x), orc.spmm(absA, np.abs(x))))
    B = spx.Batch(plans, ks)
    B.bind(X, Y)
    B.autotune(reps=3)
    B.capture()
    other = plans[0]
    xo = torch.ones(mats[0].n, dtype=torch.float64, device="cuda")
    yo = torch.empty(mats[0].m, dtype=torch.float64, device="cuda")
    for rep in range(3):
        for y in Y:
            y.fill_(np.nan)
        spx.spmv(other, xo, yo)  # eager work between replays
        torch.cuda.synchronize()
        B.replay()
        for i, (ref, bound) in enumerate(refs):
            y = host(Y[i]).reshape(mats[i].m, -1)
            assert np.all(np.abs(y - ref) <= 1e-12 * bound), f"replay {rep} member {i} k={ks[i]}"
