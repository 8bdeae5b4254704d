"""Parity at full size, in the launch configurations the benchmark times.

The n = 10^6 irregular matrix (20 M nonzeros) as plain CSR, DB form at
K = 64 and split at K = 64 with 128 KB leaves, run through the same calls as
the benchmark (permute_x, split_prepare_y, accumulate = 2) under every
schedule its autotuner may pick; the n = 5*10^5 SPD matrix in binary64,
binary32 and bfloat16 under the same schedules, and one refined CG solve;
every 8th member of the 256-matrix uneven batch with the benchmark's
schedule search, graph capture and replays.  The oracle computes sampled
outputs row by row: random rows, the longest rows and, for the split, rows
whose nonzeros lie in several parts.  Permutations are checked bit for bit.
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


def rows_of(A, rows):
    """The CSR matrix made of the given rows of A, in that order."""
    rows = np.asarray(rows, dtype=np.int64)
    lens = (A.rowptr[rows + 1] - A.rowptr[rows]).astype(np.int64)
    rp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    idx = np.repeat(A.rowptr[rows].astype(np.int64) - rp[:-1], lens) + np.arange(rp[-1])
    return CSR(rows.size, A.n, rp, A.colidx[idx], A.vals[idx])


def sample_rows(A, seed, extra=()):
    rng = np.random.default_rng(seed)
    deg = np.diff(A.rowptr)
    longest = np.argsort(deg, kind="stable")[-64:]
    picks = [rng.choice(A.m, 4096, replace=False), longest, np.array([0, A.m - 1])]
    picks += [np.asarray(e, dtype=np.int64) for e in extra]
    return np.unique(np.concatenate(picks))


def is_permutation(p, n):
    return p.size == n and np.array_equal(np.sort(p), np.arange(n))


@pytest.fixture(scope="module")
def c2():
    A = bench.load_c2(1_000_000)
    x = gen_vectors(4242, A.n)[0]
    return A, x


@pytest.mark.timeout(300)
@pytest.mark.parametrize("form", ["plain", "db", "split"])
def test_full_size_forms(orc, c2, form):
    A, x = c2
    M = spx.from_csr(A)
    xd = dev(x)
    extra = ()
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
            # rows whose nonzeros lie in more than one part: their sums are
            # accumulated from several leaves
            row_of = np.repeat(np.arange(A.m), np.diff(A.rowptr))
            first = parts[A.rowptr[:-1].clip(max=A.nnz - 1)]
            shared = np.unique(row_of[parts != first[row_of]])
            assert shared.size > 0
            extra = (np.random.default_rng(7).choice(shared, min(2048, shared.size), replace=False),)
    rows = sample_rows(A, 11, extra)
    sub = rows_of(A, rows)
    ref, bound = orc.spmv(sub, x), orc.abs_rowsum(sub, x)
    inv = np.empty(A.m, np.int64)
    inv[rp] = np.arange(A.m)
    for tune in bench.AUTOTUNE:
        spx.plan_retune(P, tune)
        y = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
        if form == "split":
            spx.split_prepare_y(P, y)
            spx.spmv_split(P, xh, y, accumulate=2)
        else:
            spx.spmv(P, xh, y)
        yh = host(y)
        assert not np.isnan(yh).any(), f"{form} {tune}: unwritten rows"
        assert_close_rowwise(yh[inv[rows]], ref, bound, f"{form} {tune}")


@pytest.fixture(scope="module")
def spd():
    A = gen_c3_spd(seed=3, n=500_000)
    M = spx.from_csr(A)
    P = spx.plan_plain(M)
    spx.plan_add_lowp(P, "f32")
    spx.plan_add_lowp(P, "bf16")
    return A, P


@pytest.mark.timeout(300)
def test_full_size_precision_products(orc, spd):
    A, P = spd
    x = gen_vectors(3000, A.n, 1)[0]
    x32 = x.astype(np.float32)
    rows = sample_rows(A, 12)
    sub = rows_of(A, rows)
    ref64, bound64 = orc.spmv(sub, x), orc.abs_rowsum(sub, x)
    f = orc.to_f32(sub.vals)
    h = orc.f32_to_bf16(f)
    refs = {"f32": (orc.spmv_lowp(sub, f, x32), f.astype(np.float64)),
            "bf16": (orc.spmv_lowp(sub, None, x32, vals16=h), orc.bf16_bits_to_f32(h).astype(np.float64))}
    deg = np.diff(sub.rowptr)
    for tune in bench.AUTOTUNE:
        spx.plan_retune(P, tune)
        y = torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda")
        spx.spmv(P, dev(x), y)
        assert_close_rowwise(host(y)[rows], ref64, bound64, f"f64 {tune}")
        for prec, (ref, vq) in refs.items():
            y32 = torch.full((A.m,), np.nan, dtype=torch.float32, device="cuda")
            spx.spmv_lowp(P, prec, dev(x32), y32)
            got = host(y32)[rows].astype(np.float64)
            # both sides sum binary32 products of the same rounded values
            absq = orc.abs_rowsum(CSR(sub.m, sub.n, sub.rowptr, sub.colidx, vq), x32.astype(np.float64))
            assert np.all(np.abs(got - ref.astype(np.float64)) <= 2.0 * (deg + 2) * U32 * absq), f"{prec} {tune}"


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


@pytest.mark.timeout(300)
def test_full_size_batch_members(orc):
    """Every 8th member of the 256-matrix uneven batch, at full size, with the
    benchmark's schedule search, graph capture and replays (eager work and
    waits in between); 512 sampled rows of every member and right-hand side
    against the oracle."""
    from synth import gen_c4_one
    mats, ks = [], []
    for j in range(0, 256, 8):
        A, k = gen_c4_one(j)
        mats.append(A)
        ks.append(k)
    assert set(ks) == {1, 8, 32}
    plans = [spx.plan_plain(spx.from_csr(A)) for A in mats]
    rng = np.random.default_rng(4444)
    X, Y, Xh = [], [], []
    for A, k in zip(mats, ks):
        x = rng.uniform(-1, 1, (A.n, k))
        Xh.append(x)
        X.append(dev(x[:, 0].copy()) if k == 1 else dev(x))
        Y.append(torch.empty((A.m,) if k == 1 else (A.m, k), dtype=torch.float64, device="cuda"))
    B = spx.Batch(plans, ks)
    B.bind(X, Y)
    B.autotune(reps=3)
    B.capture()
    samples = []
    for i, A in enumerate(mats):
        rows = np.unique(np.concatenate([np.random.default_rng(i).choice(A.m, min(512, A.m), replace=False),
                                         np.argsort(np.diff(A.rowptr), kind="stable")[-8:]]))
        sub = rows_of(A, rows)
        absub = CSR(sub.m, sub.n, sub.rowptr, sub.colidx, np.abs(sub.vals))
        samples.append((rows, orc.spmm(sub, Xh[i]), orc.spmm(absub, np.abs(Xh[i]))))
    other = plans[0]
    xo = torch.ones(mats[0].n, dtype=torch.float64, device="cuda")
    yo = torch.empty(mats[0].m, dtype=torch.float64, device="cuda")
    for rep in range(3):
        for y in Y:
            y.fill_(np.nan)
        spx.spmv(other, xo, yo)  # eager work between replays
        torch.cuda.synchronize()
        B.replay()
        for i, (rows, ref, bound) in enumerate(samples):
            y = host(Y[i]).reshape(mats[i].m, -1)[rows]
            assert np.all(np.abs(y - ref) <= 1e-12 * bound), f"replay {rep} member {8 * i} k={ks[i]}"
