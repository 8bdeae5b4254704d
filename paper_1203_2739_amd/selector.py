"""Learned choice of the SpMV form, K and schedule: training and evaluation.

The 24 choices (6 schedules of plain CSR, and the SB, DB and split forms of
Sections 3 and 4 at K = 8 .. 256) live in the library (spx_choice_info), as
do the exhaustive timing of every choice (spx_select_exhaustive: the label,
the fallback and the measure of the regret t(chosen) / t(best) - 1) and the
selection itself (spx_select / spx_select_features: features, normalisation,
network forward, argmax).  This module holds what is training: the
normalisation statistics of the training set, the label tolerance, and the
loop that trains the 40 -> 64 -> 64 -> 24 network with the library's
forward/backward and Adam kernels.
"""
from __future__ import annotations

import numpy as np

from . import (choice_info, features, from_csr, mlp_adam, mlp_loss_grad, partition_tree, select_exhaustive,
               select_exhaustive_trees, select_features, MLP_PARAMS, NCHOICES, NFEATURES)


def choice_name(c):
    form, K, tune = choice_info(c)
    return f"plain{c}" if form == "plain" else f"{form}{K}"


def measure(A, seed=0, reps=10, trees=None):
    """Milliseconds per product of every choice on matrix A (a synth CSR),
    timed by the library, and the host seconds of the three partitions.
    trees: the three K = 256 partitions computed beforehand (dict form ->
    parts, with their seconds under "seconds"), as partition_trees gives."""
    import torch
    M = from_csr(A)
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.uniform(-1, 1, A.n)).cuda()
    y = torch.empty(max(A.m, 1), dtype=torch.float64, device="cuda")
    if trees is not None:
        _, times = select_exhaustive_trees(M, trees, x, y, reps=reps)
        return times, float(trees["seconds"])
    _, times, tpart = select_exhaustive(M, x, y, reps=reps, seed=seed)
    return times, tpart


def partition_trees(A, seed=0):
    """The three K = 256 partitions of A (host only, no GPU) for measure."""
    M = from_csr(A, device=False)
    out, sec = {}, 0.0
    for f in ("sb", "db", "split"):
        out[f], s = partition_tree(M, f, seed)
        sec += s
    out["seconds"] = sec
    return out


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


def predict(theta, F, norm):
    """The library's choice for every row of raw features F (spx_select_features)."""
    return np.array([select_features(f, theta, norm.mu, norm.sd)[0] for f in F], dtype=np.int64)


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


def fit(F, T, norm, epochs=300, check_every=20, val_frac=0.2, tols=(0.0, 0.02), lrs=(1e-3, 3e-3), batch=32,
        seed=0):
    """Train on near-optimal labels with early stopping.  A held-back fifth of
    the training matrices (raw features F, normalised by norm) picks the
    label tolerance, the learning rate and the epoch count (lowest mean
    regret of the library's choice); the network is then trained again on
    every training matrix with that choice.  Returns (theta, settings,
    validation regret of every setting tried)."""
    Fn = norm(F)
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
                r = float(regret(T[va], predict(theta, F[va], norm)).mean())
                tried.append({"tol": tol, "lr": lr, "epochs": ep, "val_regret": round(r, 5)})
                if best is None or r < best[0]:
                    best = (r, tol, lr, ep)
    _, tol, lr, ep = best
    X, lab = augment(Fn, T, tol)
    theta, _ = train(X, lab, epochs=ep, batch=batch, lr=lr, seed=seed)
    return theta, {"tol": tol, "lr": lr, "epochs": ep}, tried
