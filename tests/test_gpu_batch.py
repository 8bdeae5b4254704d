"""Batched products through the C interface: every Y_i = A_i X_i of an
uneven batch against the oracle's storage-order products, for eager runs,
repeated runs, HIP graph replays and autotuned schedules."""
import numpy as np
import pytest

import paper_1203_2739_amd as spx
from gpu_util import TOL, dev, host
from synth import CSR, gen_c4_one, gen_uniform_zipf

pytestmark = pytest.mark.gpu


def long_rows_matrix(seed):
    rng = np.random.default_rng(seed)
    lens = [3, 2000, 0, 5, 130, 129, 128, 4100, 1, 64] + list(rng.integers(0, 40, 300))
    n = 6000
    cols = np.concatenate([np.sort(rng.choice(n, d, replace=False)) for d in lens])
    rp = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    return CSR(len(lens), n, rp, cols.astype(np.int32), rng.uniform(-1, 1, cols.size))


def make_batch(seed=0):
    """Members of the uneven batch at reduced size, plus matrices with rows
    longer than a block, an empty matrix and odd right-hand-side counts."""
    mats, ks = [], []
    for j in range(10):
        A, k = gen_c4_one(j, base_seed=7000 + seed, n_hi=20_000)
        mats.append(A)
        ks.append(k)
    mats += [long_rows_matrix(1), long_rows_matrix(2), long_rows_matrix(3),
             CSR(7, 9, np.zeros(8, np.int64), np.zeros(0, np.int32), np.zeros(0)),
             gen_uniform_zipf(77, 6000, 40000, 1500)]
    ks += [8, 1, 32, 8, 3]
    return mats, ks


def vectors(mats, ks, pad, seed):
    import torch
    rng = np.random.default_rng(seed)
    X, Y, Xh = [], [], []
    for A, k in zip(mats, ks):
        x = rng.uniform(-1, 1, (A.n, k))
        Xh.append(x)
        if k == 1:
            X.append(dev(x[:, 0].copy()))
            Y.append(torch.full((A.m,), np.nan, dtype=torch.float64, device="cuda"))
        else:
            xp = np.zeros((A.n, k + pad))
            xp[:, :k] = x
            X.append(dev(xp)[:, :k])
            Y.append(torch.full((A.m, k + pad), np.nan, dtype=torch.float64, device="cuda")[:, :k])
    return X, Y, Xh


def check(orc, mats, Xh, Y, what):
    for i, (A, x) in enumerate(zip(mats, Xh)):
        y = host(Y[i]).reshape(A.m, -1)
        ref = orc.spmm(A, x)
        absA = CSR(A.m, A.n, A.rowptr, A.colidx, np.abs(A.vals))
        bound = orc.spmm(absA, np.abs(x))
        err = np.abs(y - ref)
        assert np.all(err <= TOL * bound), f"{what}: matrix {i} k={x.shape[1]} worst {np.nanmax(err - TOL * bound)}"


def plans_of(mats):
    return [spx.plan_plain(spx.from_csr(A)) for A in mats]


@pytest.mark.parametrize("pad", [0, 3])
def test_batch_runs_match_oracle(orc, pad):
    mats, ks = make_batch()
    P = plans_of(mats)
    B = spx.Batch(P, ks)
    X, Y, Xh = vectors(mats, ks, pad, 5)
    B.bind(X, Y)
    for rep in range(2):  # the queue and the long-row counters reset themselves
        for y in Y:
            y.fill_(np.nan)
        B.run()
        check(orc, mats, Xh, Y, f"run {rep}")
    for cfg in (dict(order=1), dict(span_div=4), dict(reduce_iters=1), dict(order=1, span_div=2, reduce_iters=8)):
        B.configure(**cfg)
        for y in Y:
            y.fill_(np.nan)
        B.run()
        check(orc, mats, Xh, Y, f"config {cfg}")


def test_batch_graph_replays(orc):
    """The captured launch replayed several times with eager work and waits
    in between: every replay matches the oracle."""
    import torch
    mats, ks = make_batch(1)
    P = plans_of(mats)
    B = spx.Batch(P, ks)
    X, Y, Xh = vectors(mats, ks, 0, 6)
    B.bind(X, Y)
    B.capture()
    other = spx.plan_plain(spx.from_csr(mats[0]))
    xo = torch.ones(mats[0].n, dtype=torch.float64, device="cuda")
    yo = torch.empty(mats[0].m, dtype=torch.float64, device="cuda")
    for rep in range(4):
        for y in Y:
            y.fill_(np.nan)
        spx.spmv(other, xo, yo)  # eager work between replays
        torch.cuda.synchronize()
        B.replay()
        check(orc, mats, Xh, Y, f"replay {rep}")


def test_batch_autotune_and_one_shot(orc):
    mats, ks = make_batch(2)
    P = plans_of(mats)
    B = spx.Batch(P, ks)
    X, Y, Xh = vectors(mats, ks, 0, 7)
    B.bind(X, Y)
    best = B.autotune(reps=2)
    assert best["ms"] > 0 and best["order"] in (0, 1)
    for y in Y:
        y.fill_(np.nan)
    B.run()
    check(orc, mats, Xh, Y, "autotuned")
    X2, Y2, Xh2 = vectors(mats, ks, 2, 8)
    spx.spmv_batched(P, ks, X2, Y2)
    check(orc, mats, Xh2, Y2, "one shot")


def test_batch_errors():
    A = gen_uniform_zipf(3, 100, 500, 20)
    P = plans_of([A])
    with pytest.raises(spx.SpxError):
        spx.Batch(P, [65])
    B = spx.Batch(P, [1])
    with pytest.raises(spx.SpxError):
        B.run()  # not bound
    with pytest.raises(spx.SpxError):
        B.replay()  # not captured


@pytest.mark.parametrize("form", ["sb", "db"])
def test_batch_of_reordered_plans(orc, form):
    """Batched products of SB/DB plans run in each plan's reordered space."""
    import torch
    mats, ks = make_batch(3)
    mats, ks = mats[:6], ks[:6]
    fn = {"sb": spx.reorder_sb, "db": spx.reorder_db}[form]
    res = [fn(spx.from_csr(A), 4, 0, 1) for A in mats]
    P = [r[0] for r in res]
    X, Y, Xh = vectors(mats, ks, 1, 9)
    Xr = []
    for (p, rp, cp, _), x, k in zip(res, X, ks):
        Xr.append(x[torch.from_numpy(cp.astype(np.int64)).cuda()].contiguous())
    B = spx.Batch(P, ks)
    B.bind(Xr, Y)
    B.run()
    for i, (A, x) in enumerate(zip(mats, Xh)):
        rp = res[i][1]
        y = host(Y[i]).reshape(A.m, -1)
        ref = orc.spmm(A, x)[rp]
        bound = orc.spmm(CSR(A.m, A.n, A.rowptr, A.colidx, np.abs(A.vals)), np.abs(x))[rp]
        assert np.all(np.abs(y - ref) <= TOL * bound), f"{form} matrix {i}"


def test_batch_rejects_strided_single_rhs():
    import torch
    A = gen_uniform_zipf(4, 200, 1000, 20)
    P = plans_of([A])
    B = spx.Batch(P, [1])
    X = torch.zeros((A.n, 2), dtype=torch.float64, device="cuda")[:, :1]
    Y = torch.zeros((A.m, 1), dtype=torch.float64, device="cuda")
    with pytest.raises((spx.SpxError, ValueError)):
        B.bind([X], [Y])
