"""Seeded generators for the synthetic sparse matrices used as workloads.

The paper evaluates on irregular matrices whose row and column degrees have a
coefficient of variation between about 0.2 and 250 (Section 5.1, Table 1).
Those matrices are not available here; the families below stand in for them.
Every generator is a pure function of its seed: it draws from
``numpy.random.Generator(PCG64(seed))`` in a fixed order.

Nothing in this module computes a matrix-vector product or any quantity the
SpMV method itself produces; it only builds (rowptr, colidx, vals) triples and
dense vectors.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    """A CSR matrix: int64 row pointers, int32 column indices, float64 values.

    Column indices are sorted ascending and unique inside every row.
    """

    m: int
    n: int
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray
    info: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_degrees(self) -> np.ndarray:
        return np.diff(self.rowptr)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _zipf_pmf(s: float, dmax: int) -> np.ndarray:
    k = np.arange(1, dmax + 1, dtype=np.float64)
    p = k ** (-float(s))
    return p / p.sum()


def _zipf_samples(rng, s, dmax, size):
    return rng.choice(int(dmax), size=int(size), p=_zipf_pmf(s, dmax)) + 1


def zipf_degrees(rng, s: float, dmax: int, size: int, target_total: int,
                 dmin: int = 1) -> np.ndarray:
    """Truncated-Zipf degrees rescaled so that their sum hits a target.

    z_i ~ Zipf(s) on [1, dmax]; d_i = clip(round(c * z_i), dmin, dmax) with the
    scale c found by bisection so that sum(d_i) is as close as possible to
    ``target_total``.  (A raw truncated Zipf(2) has mean 4.1 on [1, 500] and
    5.5 on [1, 5000], below the mean degrees the workloads ask for.)
    """
    z = _zipf_samples(rng, s, dmax, size).astype(np.float64)

    def total(c):
        return int(np.clip(np.rint(c * z), dmin, dmax).sum())

    lo, hi = 0.0, 1.0
    while total(hi) < target_total and hi < 1e9:
        hi *= 2.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if total(mid) < target_total:
            lo = mid
        else:
            hi = mid
    c = hi if abs(total(hi) - target_total) <= abs(total(lo) - target_total) else lo
    return np.clip(np.rint(c * z), dmin, dmax).astype(np.int64)


def _dedupe(rows, cols, n, redraw, forbid_diag=False, max_iter=200):
    """Redraw entries until every (row, col) pair is unique.

    ``redraw(idx, it)`` returns fresh columns for the entry positions ``idx``
    at retry ``it``.  The first occurrence of a pair (in position order) is
    kept.
    """
    for it in range(max_iter):
        key = rows.astype(np.int64) * np.int64(n) + cols.astype(np.int64)
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(rows.size, dtype=bool)
        dup[order[1:][ks[1:] == ks[:-1]]] = True
        if forbid_diag:
            dup |= rows == cols
        idx = np.flatnonzero(dup)
        if idx.size == 0:
            return cols
        cols[idx] = redraw(idx, it)
    return _fill_from_complement(rows, cols, n, forbid_diag)


def _fill_from_complement(rows, cols, n, forbid_diag):
    """Last resort for rows so dense that redrawing duplicates does not
    converge: their duplicate entries take columns the row does not use yet,
    drawn without replacement from a generator seeded by (n, row)."""
    key = rows.astype(np.int64) * np.int64(n) + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    dup = np.zeros(rows.size, dtype=bool)
    dup[order[1:][ks[1:] == ks[:-1]]] = True
    if forbid_diag:
        dup |= rows == cols
    for r in np.unique(rows[dup]):
        pos = np.flatnonzero(rows == r)
        bad = pos[dup[pos]]
        used = np.zeros(n, dtype=bool)
        used[cols[pos[~dup[pos]]]] = True
        if forbid_diag and r < n:
            used[r] = True
        free = np.flatnonzero(~used)
        if free.size < bad.size:
            raise RuntimeError("row degree exceeds the number of columns")
        rng = np.random.default_rng([int(n), int(r), 0x5EED])
        cols[bad] = rng.choice(free, size=bad.size, replace=False)
    return cols


def _to_csr(m, n, rows, cols, vals, info=None) -> CSR:
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    vals = vals[order].astype(np.float64)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return CSR(int(m), int(n), rowptr, cols, vals, dict(info or {}))


def _weighted_draw(rng, cdf, size, lo=None, hi=None):
    """Draw indices with probability proportional to the weights behind ``cdf``.

    With ``lo``/``hi`` (per-draw index ranges) each draw is restricted to
    columns [lo, hi).
    """
    total = cdf[-1]
    if lo is None:
        u = rng.random(size) * total
        idx = np.searchsorted(cdf, u, side="right")
        return np.minimum(idx, cdf.size - 1)
    base = np.where(lo > 0, cdf[np.maximum(lo - 1, 0)], 0.0)
    top = cdf[hi - 1]
    u = base + rng.random(size) * (top - base)
    idx = np.searchsorted(cdf, u, side="right")
    return np.clip(idx, lo, hi - 1)


def gen_uniform_zipf(seed: int, n: int, target_offdiag: int, dmax: int,
                     s: float = 2.0, diagonal: bool = True, m: int | None = None,
                     values: bool = True) -> CSR:
    """Zipf row degrees with uniformly random distinct column positions.

    Row i holds d_i distinct columns drawn uniformly (off the diagonal when a
    diagonal is added), plus the diagonal entry when ``diagonal``.
    """
    rng = _rng(seed)
    m = n if m is None else m
    cap = min(dmax, n - 1 if diagonal else n)
    deg = zipf_degrees(rng, s, cap, m, target_offdiag)
    rows = np.repeat(np.arange(m, dtype=np.int64), deg)
    cols = rng.integers(0, n, size=rows.size, dtype=np.int64)
    cols = _dedupe(rows, cols, n,
                   lambda idx, it: rng.integers(0, n, size=idx.size, dtype=np.int64),
                   forbid_diag=diagonal)
    if diagonal:
        d = np.arange(min(m, n), dtype=np.int64)
        rows = np.concatenate([rows, d])
        cols = np.concatenate([cols, d])
    vals = rng.uniform(-1.0, 1.0, size=rows.size) if values else np.ones(rows.size)
    return _to_csr(m, n, rows, cols, vals,
                   {"kind": "uniform_zipf", "seed": seed, "s": s, "dmax": dmax})


def gen_c1(seed: int = 1) -> CSR:
    """n = 10,000 square; Zipf(2.0) off-diagonal degrees on [1, 500] scaled to
    90,000 in total (about 100,000 nonzeros with the diagonal)."""
    A = gen_uniform_zipf(seed, 10_000, 90_000, 500, s=2.0, diagonal=True)
    A.info["config"] = "n=10000 zipf2.0 dmax500 +diag"
    return A


def gen_block_hidden(seed: int, n: int, mean_deg: float, nblocks: int,
                     block_frac: float, dmax: int = 5000, s: float = 2.0,
                     col_cap: int = 5000) -> CSR:
    """Irregular matrix with hidden diagonal blocks.

    * Row degrees: truncated Zipf(s) on [1, dmax] scaled to ``mean_deg``.
    * Column weights: the same law, assigned to columns in random order.
    * ``nblocks`` contiguous diagonal blocks (generator order).  Each row draws
      Binomial(d_i, block_frac) of its columns, proportionally to weight,
      inside its own block and the rest proportionally to weight over all
      columns.  Duplicates are redrawn; column degrees are capped at
      ``col_cap`` by redrawing excess entries on uncapped columns.
    * One random symmetric permutation hides the blocks.
    """
    rng = _rng(seed)
    deg = zipf_degrees(rng, s, dmax, n, int(round(mean_deg * n)))
    w = _zipf_samples(rng, s, dmax, n).astype(np.float64)
    w = w[rng.permutation(n)]
    bounds = np.linspace(0, n, nblocks + 1).round().astype(np.int64)
    blk_of = np.repeat(np.arange(nblocks, dtype=np.int64), np.diff(bounds))
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    in_blk = np.minimum(rng.binomial(deg, block_frac),
                        np.diff(bounds)[blk_of] // 2)
    # category per entry: the first in_blk[i] entries of row i are in-block
    start = np.repeat(np.cumsum(deg) - deg, deg)
    cat = (np.arange(rows.size, dtype=np.int64) - start) < np.repeat(in_blk, deg)
    blo = bounds[blk_of[rows]]
    bhi = bounds[blk_of[rows] + 1]

    def draw(idx, weights, it=0):
        # after a few weighted retries, remaining duplicates are redrawn
        # uniformly in the same range so that heavy rows terminate
        if it >= 8:
            weights = np.where(weights > 0, 1.0, 0.0)
        cdf = np.cumsum(weights)
        out = np.empty(idx.size, dtype=np.int64)
        c = cat[idx]
        g = ~c
        if g.any():
            out[g] = _weighted_draw(rng, cdf, int(g.sum()))
        if c.any():
            ii = idx[c]
            out[c] = _weighted_draw(rng, cdf, ii.size, blo[ii], bhi[ii])
        return out

    cols = draw(np.arange(rows.size, dtype=np.int64), w)
    wcur = w
    for _ in range(100):
        cols = _dedupe(rows, cols, n, lambda idx, it: draw(idx, wcur, it))
        cnt = np.bincount(cols, minlength=n)
        over = cnt > col_cap
        if not over.any():
            break
        # rank the entries of each over-full column randomly; redraw the excess
        sel = np.flatnonzero(over[cols])
        key = rng.random(sel.size)
        order = np.lexsort((key, cols[sel]))
        sel = sel[order]
        cs = cols[sel]
        first = np.searchsorted(cs, cs, side="left")
        rank = np.arange(sel.size) - first
        redo = sel[rank >= col_cap]
        wcur = np.where(cnt >= col_cap, 0.0, w)
        cols[redo] = draw(redo, wcur)
    else:
        raise RuntimeError("column cap not reached")
    vals = rng.uniform(-1.0, 1.0, size=rows.size)
    perm = rng.permutation(n).astype(np.int64)  # old index -> hidden index
    in_block = (cols >= blo) & (cols < bhi)
    info = {"kind": "block_hidden", "seed": seed, "nblocks": nblocks,
            "block_frac_target": block_frac,
            "block_frac": float(in_block.mean()) if rows.size else 0.0,
            "hidden_perm_seeded": True}
    A = _to_csr(n, n, perm[rows], perm[cols], vals, info)
    A.info["block_of_row"] = np.empty(n, dtype=np.int64)
    A.info["block_of_row"][perm] = blk_of
    return A


def gen_c2(seed: int = 2, n: int = 1_000_000) -> CSR:
    """n = 10^6, mean degree 20, Zipf(2.0) rows and columns (max 5,000), 30% of
    the nonzeros inside 64 hidden diagonal blocks."""
    A = gen_block_hidden(seed, n, 20.0, 64, 0.30)
    A.info["config"] = f"n={n} zipf2.0 dmax5000 64 hidden blocks 30%"
    return A


def gen_c3_spd(seed: int = 3, n: int = 500_000, mean_deg: float = 20.0):
    """Symmetric positive definite test matrix built from the block generator.

    B comes from :func:`gen_block_hidden`; A keeps the off-diagonal part of
    B + B^T and puts sum_{j != i} |(B + B^T)_ij| + 1 on the diagonal, so A is
    strictly diagonally dominant with margin 1 (hence SPD, smallest eigenvalue
    at least 1 by Gershgorin).
    """
    B = gen_block_hidden(seed, n, mean_deg, 64, 0.30, dmax=min(5000, n), col_cap=min(5000, n))
    rows = np.repeat(np.arange(n, dtype=np.int64), B.row_degrees())
    cols = B.colidx.astype(np.int64)
    r = np.concatenate([rows, cols])
    c = np.concatenate([cols, rows])
    v = np.concatenate([B.vals, B.vals])
    off = r != c
    r, c, v = r[off], c[off], v[off]
    key = r * n + c
    order = np.argsort(key, kind="stable")
    key, v = key[order], v[order]
    first = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
    vs = np.add.reduceat(v, first)
    ks = key[first]
    r, c = ks // n, ks % n
    absrow = np.bincount(r, weights=np.abs(vs), minlength=n)
    d = np.arange(n, dtype=np.int64)
    A = _to_csr(n, n, np.concatenate([r, d]), np.concatenate([c, d]),
                np.concatenate([vs, absrow + 1.0]),
                {"kind": "spd_from_block_hidden", "seed": seed,
                 "nnz_B": B.nnz})
    return A


def gen_c4_one(j: int, base_seed: int = 4000, n_lo: int = 1_000,
               n_hi: int = 200_000):
    """One matrix of the uneven batch: returns (CSR, nrhs).

    n = round(exp(U[ln n_lo, ln n_hi])), mean degree U[5, 50], Zipf(2.2) row
    degrees capped at min(n, 5000), uniform distinct columns, and a number of
    right-hand sides drawn from {1, 8, 32}.
    """
    rng = _rng(base_seed + j)
    n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
    mu = float(rng.uniform(5.0, 50.0))
    k = int(rng.choice(np.array([1, 8, 32])))
    A = gen_uniform_zipf(int(rng.integers(1 << 62)), n, int(round(mu * n)),
                         min(n, 5000), s=2.2, diagonal=False)
    A.info.update({"kind": "batch_member", "j": j, "mean_deg": mu, "nrhs": k})
    return A, k


def gen_c4_batch(count: int = 256, base_seed: int = 4000, **kw):
    return [gen_c4_one(j, base_seed, **kw) for j in range(count)]


def gen_vectors(seed: int, n: int, count: int = 1, k: int = 1) -> np.ndarray:
    """``count`` dense inputs of n rows and k columns, U[-1, 1].

    Returns shape (count, n) for k == 1, else (count, n, k) row-major.
    """
    rng = _rng(seed)
    if k == 1:
        return rng.uniform(-1.0, 1.0, size=(count, n))
    return rng.uniform(-1.0, 1.0, size=(count, n, k))


def gen_family(family: str, seed: int, n: int) -> CSR:
    """Matrix families used to train and test the selector.

    F1 Zipf power law; F2 banded with a relocated fraction; F3 hidden
    block-diagonal with a border; F4 2-D random geometric graph in random
    order.  Mean degrees are drawn in [5, 30].
    """
    rng = _rng(seed)
    mu = float(rng.uniform(5.0, 30.0))
    sub = int(rng.integers(1 << 62))
    if family == "F1":
        A = gen_block_hidden(sub, n, mu, 1, 0.0, dmax=min(5000, n))
    elif family == "F2":
        beta = int(round(np.exp(rng.uniform(np.log(2), np.log(1000)))))
        frac = float(rng.uniform(0.0, 0.2))
        r2 = _rng(sub)
        deg = np.minimum(r2.poisson(mu, size=n) + 1, 2 * beta + 1)
        rows = np.repeat(np.arange(n, dtype=np.int64), deg)

        def draw(idx, it=0):
            far = r2.random(idx.size) < frac
            off = r2.integers(-beta, beta + 1, size=idx.size)
            c = np.clip(rows[idx] + off, 0, n - 1)
            c[far] = r2.integers(0, n, size=int(far.sum()))
            return c

        cols = _dedupe(rows, draw(np.arange(rows.size)), n, draw)
        A = _to_csr(n, n, rows, cols, r2.uniform(-1, 1, rows.size),
                    {"bandwidth": beta, "relocated": frac})
    elif family == "F3":
        nb = int(rng.integers(8, 513))
        bfrac = float(rng.uniform(0.001, 0.05))
        r2 = _rng(sub)
        deg = np.clip(r2.poisson(mu, size=n), 1, None)
        bounds = np.linspace(0, n, nb + 1).round().astype(np.int64)
        blk = np.repeat(np.arange(nb), np.diff(bounds))
        deg = np.minimum(deg, np.diff(bounds)[blk])
        rows = np.repeat(np.arange(n, dtype=np.int64), deg)
        border_row = r2.random(n) < bfrac

        def draw(idx, it=0):
            r = rows[idx]
            lo, hi = bounds[blk[r]], bounds[blk[r] + 1]
            c = lo + (r2.random(idx.size) * (hi - lo)).astype(np.int64)
            g = border_row[r] | (r2.random(idx.size) < bfrac)
            c[g] = r2.integers(0, n, size=int(g.sum()))
            return c

        cols = _dedupe(rows, draw(np.arange(rows.size)), n, draw)
        perm = r2.permutation(n)
        A = _to_csr(n, n, perm[rows], perm[cols], r2.uniform(-1, 1, rows.size),
                    {"nblocks": nb, "border_frac": bfrac})
    elif family == "F4":
        from scipy.spatial import cKDTree
        r2 = _rng(sub)
        pts = r2.random((n, 2))
        radius = np.sqrt(mu / (np.pi * n))
        pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
        i, j = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
        d = np.arange(n, dtype=np.int64)
        rows = np.concatenate([i, j, d])
        cols = np.concatenate([j, i, d])
        perm = r2.permutation(n)
        A = _to_csr(n, n, perm[rows], perm[cols], r2.uniform(-1, 1, rows.size),
                    {"radius": float(radius)})
    else:
        raise ValueError(family)
    A.info.update({"family": family, "seed": seed, "mean_deg_target": mu})
    return A


def csr_sha256(A: CSR) -> str:
    h = hashlib.sha256()
    h.update(np.int64([A.m, A.n]).tobytes())
    h.update(np.ascontiguousarray(A.rowptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(A.colidx, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(A.vals, dtype=np.float64).tobytes())
    return h.hexdigest()


def gen_banded_like(A: CSR) -> CSR:
    """The banded stand-in of a matrix: the same row lengths and values, row
    i of length d holding the d consecutive columns that start at
    min(max(i - d // 2, 0), n - d).  Every row's entries sit next to its
    diagonal, so a product's reads of x stay inside a band as wide as the
    longest row: the rate it reaches is the kernel's rate without scattered
    gathers."""
    deg = np.diff(A.rowptr).astype(np.int64)
    assert deg.size == 0 or int(deg.max()) <= A.n, "a row longer than the matrix is wide"
    start = np.clip(np.arange(A.m, dtype=np.int64) - deg // 2, 0, np.maximum(A.n - deg, 0))
    off = np.arange(A.nnz, dtype=np.int64) - np.repeat(A.rowptr[:-1].astype(np.int64), deg)
    cols = (np.repeat(start, deg) + off).astype(np.int32)
    return CSR(A.m, A.n, A.rowptr, cols, A.vals, {"banded_like": True})


LOCALITY_KINDS = ("random", "temporal", "spatial", "band")


def gen_locality(kind: str, seed: int = 7, n: int = 1_000_000, deg: int = 20, window: int = 16384) -> CSR:
    """Square matrices of n rows with deg nonzeros each (values U[-1, 1]) that
    separate the two localities of the x accesses (Sec. 1): "random" draws a
    row's columns uniformly from all of x (neither locality); "temporal"
    draws them, distinct and scattered, from a window of `window` columns
    that slides with the row (row i: [i (n - window) / n, + window)), so
    nearby rows reuse the same x entries but a row's own columns rarely share
    a cache line; "spatial" gives each row one run of deg consecutive
    columns at a uniform random start, so a row's reads share lines but no
    entry is reused by nearby rows; "band" puts the run next to the diagonal
    (both localities)."""
    if kind not in LOCALITY_KINDS:
        raise ValueError(f"kind must be one of {LOCALITY_KINDS}")
    rng = _rng(seed)
    rows = np.arange(n, dtype=np.int64)
    if kind == "random":
        cols = rng.integers(0, n, (n, deg), dtype=np.int64)
        cols.sort(axis=1)
        # redraw duplicates inside a row until every row has deg distinct columns
        for _ in range(100):
            dup = np.zeros_like(cols, dtype=bool)
            dup[:, 1:] = cols[:, 1:] == cols[:, :-1]
            if not dup.any():
                break
            cols[dup] = rng.integers(0, n, int(dup.sum()), dtype=np.int64)
            cols.sort(axis=1)
        assert not (cols[:, 1:] == cols[:, :-1]).any()
    elif kind == "temporal":
        lo = rows * (n - window) // n
        # deg distinct offsets per row: a random permutation's first deg of window
        # entries would be costly, so draw and redraw duplicates as above
        off = rng.integers(0, window, (n, deg), dtype=np.int64)
        off.sort(axis=1)
        for _ in range(100):
            dup = np.zeros_like(off, dtype=bool)
            dup[:, 1:] = off[:, 1:] == off[:, :-1]
            if not dup.any():
                break
            off[dup] = rng.integers(0, window, int(dup.sum()), dtype=np.int64)
            off.sort(axis=1)
        assert not (off[:, 1:] == off[:, :-1]).any()
        cols = lo[:, None] + off
    elif kind == "spatial":
        start = rng.integers(0, n - deg + 1, n, dtype=np.int64)
        cols = start[:, None] + np.arange(deg, dtype=np.int64)[None, :]
    else:
        start = np.clip(rows - deg // 2, 0, n - deg)
        cols = start[:, None] + np.arange(deg, dtype=np.int64)[None, :]
    rowptr = np.arange(n + 1, dtype=np.int64) * deg
    vals = rng.uniform(-1.0, 1.0, n * deg)
    return CSR(n, n, rowptr, cols.reshape(-1).astype(np.int32), vals, {"locality": kind, "window": window})
