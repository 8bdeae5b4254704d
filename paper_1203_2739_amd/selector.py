"""Learned choice of the SpMV form, K and schedule.

The 24 choices are 6 schedules of plain CSR and the SB, DB and split forms
(Sections 3 and 4) at K = 8, 16, 32, 64, 128, 256.  For each training matrix
every choice is timed on the GPU (the label is the fastest), the 40 features
come from :func:`paper_1203_2739_amd.features`, and the 40 -> 64 -> 64 -> 24
network is trained by the library's own forward/backward and Adam kernels.
Exhaustive timing is the fallback and the reference for the regret
t(chosen) / t(best) - 1.

The reordered forms at every K come from one K = 256 recursive bisection per
model: bisection numbers parts so that part p of the K = 256 tree lies in
part p >> (8 - log2 K) of the tree cut at K (the row border of DB stays the
border), which gives the K-way partition that the same tree yields at that
depth without partitioning again.
"""
from __future__ import annotations

import time

import numpy as np

from . import (Plan, features, from_csr, mlp_adam, mlp_forward, mlp_loss_grad, plan_from_parts, plan_plain,
               reorder_db, reorder_sb, split, split_prepare_y, spmv, spmv_split, permute_x, MLP_PARAMS,
               NCHOICES, NFEATURES)

PLAIN_TILES = [dict(wg_size=128), dict(wg_size=64), dict(wg_size=256), dict(wg_size=128, nnz_per_block=1024),
               dict(reduce_iters=16), dict(wg_size=512)]
KS = [8, 16, 32, 64, 128, 256]
CHOICES = [("plain", t) for t in PLAIN_TILES] + [(f, k) for f in ("sb", "db", "split") for k in KS]
assert len(CHOICES) == NCHOICES


def choice_name(c):
    f, p = CHOICES[c]
    return f"plain{PLAIN_TILES.index(p)}" if f == "plain" else f"{f}{p}"


def _time_products(torch, run, warmup, steps):
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        run()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def measure(A, seed=0, warmup=2, steps=10):
    """Milliseconds per product of every choice on matrix A (a synth CSR),
    and the host seconds of the three partitions."""
    import torch
    M = from_csr(A)
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.uniform(-1, 1, A.n)).cuda()
    y = torch.empty(max(A.m, 1), dtype=torch.float64, device="cuda")
    times = np.zeros(NCHOICES)
    t0 = time.time()
    trees = {"sb": reorder_sb(M, 256, 0, seed)[0].export_parts()[0],
             "db": reorder_db(M, 256, 0, seed)[0].export_parts()[0],
             "split": split(M, 256, 0, seed)[0].export_parts()[0]}
    tpart = time.time() - t0
    for c, (form, p) in enumerate(CHOICES):
        if form == "plain":
            P = plan_plain(M, tune=p)
            times[c] = _time_products(torch, lambda: spmv(P, x, y), warmup, steps)
            continue
        a = trees[form]
        shift = 8 - int(np.log2(p))
        parts = np.where(a >= 256, p, a >> shift) if form == "db" else a >> shift
        P, rp, cp = plan_from_parts(M, form, p, parts.astype(np.int32))
        xh = torch.empty_like(x)
        permute_x(P, x, xh)
        if form == "split":
            def run(P=P, xh=xh):
                split_prepare_y(P, y)
                spmv_split(P, xh, y, accumulate=2)
        else:
            def run(P=P, xh=xh):
                spmv(P, xh, y)
        times[c] = _time_products(torch, run, warmup, steps)
    return times, tpart


def feature_matrix(mats):
    return np.stack([features(from_csr(A, device=False)) for A in mats]).astype(np.float32)


class Normalizer:
    """log1p of the non-negative features, then z-scores on the training set."""

    def __init__(self, F):
        G = np.log1p(np.maximum(F.astype(np.float64), 0.0))
        self.mu = G.mean(axis=0)
        self.sd = G.std(axis=0) + 1e-6

    def __call__(self, F):
        return ((np.log1p(np.maximum(F.astype(np.float64), 0.0)) - self.mu) / self.sd).astype(np.float32)


def init_theta(seed=0):
    """He-uniform weights, zero biases, in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((64, NFEATURES), (64, 64), (NCHOICES, 64)):
        lim = np.sqrt(6.0 / fan_in)
        parts += [rng.uniform(-lim, lim, fan_out * fan_in), np.zeros(fan_out)]
    th = np.concatenate(parts).astype(np.float32)
    assert th.size == MLP_PARAMS
    return th


def train(Xn, labels, epochs=400, batch=64, lr=3e-3, seed=0):
    """Adam on mean cross-entropy with the library's kernels; returns the
    parameters (device tensor) and the loss after every epoch."""
    import torch
    rng = np.random.default_rng(seed)
    theta = torch.from_numpy(init_theta(seed)).cuda()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    Xd = torch.from_numpy(np.ascontiguousarray(Xn, dtype=np.float32)).cuda()
    Ld = torch.from_numpy(np.ascontiguousarray(labels, dtype=np.int32)).cuda()
    N = Xd.shape[0]
    t = 0
    curve = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).cuda()
        tot = 0.0
        for s in range(0, N, batch):
            idx = perm[s:s + batch]
            xb = Xd[idx].contiguous()
            lb = Ld[idx].contiguous()
            mlp_loss_grad(theta, xb, lb, loss, grad)
            t += 1
            mlp_adam(theta, grad, m, v, t, lr=lr)
            tot += float(loss.item()) * idx.numel()
        curve.append(tot / N)
    return theta, curve


def predict(theta, Xn):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(Xn, dtype=np.float32)).cuda()
    logits = torch.empty((Xd.shape[0], NCHOICES), dtype=torch.float32, device="cuda")
    mlp_forward(theta, Xd, logits)
    return logits.argmax(dim=1).cpu().numpy()


def regret(times, chosen):
    """t(chosen) / t(best) - 1 per matrix."""
    best = times.min(axis=1)
    return times[np.arange(times.shape[0]), chosen] / best - 1.0


def best_fixed(times):
    """The single choice with the lowest mean regret on these matrices."""
    r = times / times.min(axis=1, keepdims=True) - 1.0
    return int(np.argmin(r.mean(axis=0)))


def augment(F, T, tol=0.02):
    """Training pairs for every choice within (1 + tol) of a matrix's fastest
    time, so that near-ties teach the set of good choices rather than one
    noisy argmin."""
    Xs, ls = [], []
    for i in range(T.shape[0]):
        good = np.flatnonzero(T[i] <= (1.0 + tol) * T[i].min())
        Xs.append(np.repeat(F[i:i + 1], good.size, axis=0))
        ls.append(good)
    return np.concatenate(Xs), np.concatenate(ls).astype(np.int32)


def fit(Fn, T, epochs=300, check_every=20, val_frac=0.2, tols=(0.0, 0.02), lrs=(1e-3, 3e-3), batch=32, seed=0):
    """Train on near-optimal labels with early stopping.  A held-back fifth of
    the training matrices picks the label tolerance, the learning rate and
    the epoch count (lowest mean regret); the network is then trained again
    on every training matrix with that choice.  Returns (theta, settings,
    validation regret of every setting tried)."""
    rng = np.random.default_rng(seed)
    N = T.shape[0]
    perm = rng.permutation(N)
    nv = max(1, int(round(val_frac * N)))
    va, tr = perm[:nv], perm[nv:]
    best, tried = None, []
    for tol in tols:
        X, lab = augment(Fn[tr], T[tr], tol)
        for lr in lrs:
            for ep in range(check_every, epochs + 1, check_every):
                theta, _ = train(X, lab, epochs=ep, batch=batch, lr=lr, seed=seed)
                r = float(regret(T[va], predict(theta, Fn[va])).mean())
                tried.append({"tol": tol, "lr": lr, "epochs": ep, "val_regret": round(r, 5)})
                if best is None or r < best[0]:
                    best = (r, tol, lr, ep)
    _, tol, lr, ep = best
    X, lab = augment(Fn, T, tol)
    theta, _ = train(X, lab, epochs=ep, batch=batch, lr=lr, seed=seed)
    return theta, {"tol": tol, "lr": lr, "epochs": ep}, tried
