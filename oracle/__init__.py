"""CPU oracle for the SpMV hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library: the arithmetic lives in ``oracle.c`` (plain C, binary64, no fused
multiply-add) and in the numpy functions below, each written from the paper's
definitions (Akbudak, Kayaaslan, Aykanat, arXiv 1203.2739) or, for the parts
the paper leaves open, from the readings stated in each docstring.

Parity status per function (what pins it is in ``tests/test_oracle.py``):

* spmv / spmv_rows / spmm / permute_csr / split_spmv: pinned (dense products,
  integer-exact cases, scipy.sparse, invariants).
* lambda_cols / lambda_split / bounds: pinned (brute force over sets on tiny
  matrices, hidden block-diagonal closed form).
* canonical_* / split_gcsr / check_*: pinned (hand-worked examples and
  structural invariants).
* to_f32 / f32_to_bf16 / spmv_lowp: pinned (numpy / torch conversions,
  integer-exact sums).
* cg / ir_cg: pinned (numpy.linalg.solve on small SPD systems).
* mlp_*: pinned (central finite differences, torch.optim.Adam in float64).
* features: pinned (hand-computed values on small matrices).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fused multiply-add)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle call failed with {rc}")


# --------------------------------------------------------------------------
# Section 2.1 and Section 3: the product itself


def spmv(A, x):
    """y = A x, each row summed left to right in storage order (CSR scheme)."""
    rp, ci, v, x = _i64(A.rowptr), _i64(A.colidx), _f64(A.vals), _f64(x)
    y = np.empty(A.m, dtype=np.float64)
    _check(lib().orc_spmv(ctypes.c_int64(A.m), _p(rp), _p(ci), _p(v), _p(x), _p(y)))
    return y


def spmv_rows(A, x, rows):
    """Selected entries of A x and their bounds sum_j |a_ij x_j|."""
    rows = _i64(rows)
    rp, ci, v, x = _i64(A.rowptr), _i64(A.colidx), _f64(A.vals), _f64(x)
    y = np.empty(rows.size)
    a = np.empty(rows.size)
    _check(lib().orc_spmv_rows(ctypes.c_int64(rows.size), _p(rows), _p(rp), _p(ci),
                               _p(v), _p(x), _p(y), _p(a)))
    return y, a


def abs_rowsum(A, x):
    """sum_j |a_ij x_j| per row, the denominator of the per-entry bound."""
    rp, ci, v, x = _i64(A.rowptr), _i64(A.colidx), _f64(A.vals), _f64(x)
    out = np.empty(A.m)
    _check(lib().orc_abs_rowsum(ctypes.c_int64(A.m), _p(rp), _p(ci), _p(v), _p(x), _p(out)))
    return out


def spmm(A, X):
    """Y = A X for X of shape (n, k), every entry a storage-order row sum."""
    X = _f64(X)
    k = X.shape[1]
    rp, ci, v = _i64(A.rowptr), _i64(A.colidx), _f64(A.vals)
    Y = np.empty((A.m, k))
    _check(lib().orc_spmm(ctypes.c_int64(A.m), _p(rp), _p(ci), _p(v), ctypes.c_int64(k),
                          _p(X), ctypes.c_int64(k), _p(Y), ctypes.c_int64(k)))
    return Y


def permute_csr(A, row_perm, col_perm):
    """A_hat = P_r A P_c with perms stored new -> old (Section 3).

    Returns (rowptr, colidx, vals) of A_hat, columns ascending within rows.
    """
    rp, ci, v = _i64(A.rowptr), _i64(A.colidx), _f64(A.vals)
    orp = np.empty(A.m + 1, dtype=np.int64)
    oci = np.empty(A.nnz, dtype=np.int64)
    ov = np.empty(A.nnz)
    _check(lib().orc_permute_csr(ctypes.c_int64(A.m), ctypes.c_int64(A.n), _p(rp), _p(ci),
                                 _p(v), _p(_i64(row_perm)), _p(_i64(col_perm)),
                                 _p(orp), _p(oci), _p(ov)))
    return orp, oci, ov


def split_spmv(A, nz_part, K, x, y0=None):
    """y <- y + A^k x for k = 0..K-1 (Section 4), each A^k in CSR order.

    ``nz_part`` gives the part of every stored nonzero in A's CSR order.
    With ``y0`` None, y starts at zero.
    """
    rp, ci, v, x = _i64(A.rowptr), _i64(A.colidx), _f64(A.vals), _f64(x)
    y = np.zeros(A.m) if y0 is None else _f64(y0).copy()
    _check(lib().orc_split_spmv(ctypes.c_int64(A.m), _p(rp), _p(ci), _p(v),
                                _p(_i64(nz_part)), ctypes.c_int64(K), _p(x), _p(y),
                                ctypes.c_int(0 if y0 is None else 1)))
    return y


# --------------------------------------------------------------------------
# Eq. (3), Theorems 1-3 and Corollary 4


def lambda_cols(A, r2p, K):
    """lambda(c_j) over the row slices given by r2p; rows with r2p outside
    [0, K) are border rows and are left out (lambda' of Eq. 6)."""
    rp, ci = _i64(A.rowptr), _i64(A.colidx)
    lam = np.empty(A.n, dtype=np.int64)
    _check(lib().orc_lambda_cols(ctypes.c_int64(A.m), ctypes.c_int64(A.n), _p(rp), _p(ci),
                                 _p(_i64(r2p)), ctypes.c_int64(K), _p(lam)))
    return lam


def lambda_split(A, nz_part, K):
    """(lambda(r_i), lambda(c_j)) for the splitting given by nz_part."""
    rp, ci = _i64(A.rowptr), _i64(A.colidx)
    lr = np.empty(A.m, dtype=np.int64)
    lc = np.empty(A.n, dtype=np.int64)
    _check(lib().orc_lambda_split(ctypes.c_int64(A.m), ctypes.c_int64(A.n), _p(rp), _p(ci),
                                  _p(_i64(nz_part)), ctypes.c_int64(K), _p(lr), _p(lc)))
    return lr, lc


def bound_sb(A, r2p, K):
    """Theorem 1: sum_j lambda(c_j)."""
    return int(lambda_cols(A, r2p, K).sum())


def bound_db(A, r2p, K):
    """Theorem 2: sum_j lambda'(c_j) + sum over border rows of nnz(r_i)."""
    r2p = _i64(r2p)
    deg = np.diff(_i64(A.rowptr))
    border = (r2p < 0) | (r2p >= K)
    return int(lambda_cols(A, r2p, K).sum() + deg[border].sum())


def bound_split(A, nz_part, K):
    """Corollary 4: sum_i lambda(r_i) + sum_j lambda(c_j)."""
    lr, lc = lambda_split(A, nz_part, K)
    return int(lr.sum() + lc.sum())


# --------------------------------------------------------------------------
# Canonical orderings.  The paper fixes the block structure (Eq. 1-5) but not
# the order inside blocks; the reading used throughout is "grouped by class,
# ties broken by original index".


def _row_of(A):
    return np.repeat(np.arange(A.m, dtype=np.int64), np.diff(_i64(A.rowptr)))


def _sets_per_index(idx, lab, size):
    """For each index: number of distinct labels, and the smallest label."""
    cnt = np.zeros(size, dtype=np.int64)
    first = np.full(size, -1, dtype=np.int64)
    if idx.size:
        key = np.unique(idx.astype(np.int64) * (int(lab.max()) + 1) + lab)
        ii = key // (int(lab.max()) + 1)
        ll = key % (int(lab.max()) + 1)
        cnt = np.bincount(ii, minlength=size).astype(np.int64)
        firsts = np.r_[True, ii[1:] != ii[:-1]]
        first[ii[firsts]] = ll[firsts]
    return cnt, first


XCD_GROUPS = 8  # row groups of the order inside classes: one per XCD of the MI355X


def _group_of_start(start, nnz):
    """Row group of a stored row (slot) whose nonzeros start at storage
    offset ``start``: the stored matrix is cut into XCD_GROUPS runs of nearly
    equal nonzeros, floor(XCD_GROUPS * start / nnz)."""
    start = np.asarray(start, dtype=np.int64)
    if nnz <= 0:
        return np.zeros_like(start)
    return (XCD_GROUPS * start) // int(nnz)


def _reader_mask(cols, grp, n):
    """For every column, the set of row groups with a nonzero in it, as a
    number whose bit g is set when group g reads the column."""
    mask = np.zeros(n, dtype=np.int64)
    if cols.size:
        np.bitwise_or.at(mask, cols, np.left_shift(np.int64(1), grp.astype(np.int64)))
    return mask


def canonical_rowcol(A, r2p, r2leaf, K, nleaves=None):
    """Row and column orders of the SB form (Eq. 1) or DB form (Eq. 5).

    Inputs: r2p[i] in [0, K) for part rows and K for row-border rows (DB);
    r2leaf[i] the leaf of a part row (leaves numbered part-major).

    Rows: by part (border last), then by leaf, then by original index.
    Columns, classified by the non-border rows that touch them: a column touched
    by one leaf goes with that leaf, a column touched by several leaves of one
    part goes after that part's leaf columns, and every other column (touched
    by several parts, or by none) goes to the column border C_B at the end.
    Inside each of these classes columns go by the set of row groups that
    read them (as a number, ascending; the rows in their new order are cut
    into XCD_GROUPS runs of nearly equal nonzeros, border rows included),
    then by decreasing number of nonzeros (in A), then by original index.

    Returns dict(row_perm, col_perm, part_ptr[K+2], col_part_ptr[K+2],
    leaf_row_ptr, leaf_col_lo, leaf_col_hi, row_leaf, col_class).
    """
    r2p = _i64(r2p)
    r2leaf = _i64(r2leaf)
    m, n = A.m, A.n
    border = (r2p < 0) | (r2p >= K)
    grp = np.where(border, K, r2p)
    lf = np.where(border, 0, r2leaf)
    row_perm = np.lexsort((np.arange(m), lf, grp))
    rows = _row_of(A)
    cols = _i64(A.colidx)
    keep = ~border[rows]
    cr, cc = rows[keep], cols[keep]
    nleaf_c, leaf_c = _sets_per_index(cc, r2leaf[cr], n)
    npart_c, part_c = _sets_per_index(cc, r2p[cr], n)
    ck_part = np.where(npart_c == 1, part_c, K)
    ck_sub = np.where(nleaf_c == 1, 0, 1)
    ck_leaf = np.where(nleaf_c == 1, leaf_c, 0)
    ck_sub = np.where(ck_part == K, 0, ck_sub)
    ck_leaf = np.where(ck_part == K, 0, ck_leaf)
    cdeg = np.bincount(cols, minlength=n)
    rdeg = np.diff(_i64(A.rowptr))
    start_new = np.cumsum(rdeg[row_perm]) - rdeg[row_perm]
    rgrp = np.empty(m, dtype=np.int64)
    rgrp[row_perm] = _group_of_start(start_new, A.nnz)
    mask = _reader_mask(cols, rgrp[rows], n)
    col_perm = np.lexsort((np.arange(n), -cdeg, mask, ck_leaf, ck_sub, ck_part))
    part_ptr = np.searchsorted(grp[row_perm], np.arange(K + 2), side="left")
    part_ptr[K + 1] = m
    col_part_ptr = np.searchsorted(ck_part[col_perm], np.arange(K + 2), side="left")
    col_part_ptr[K + 1] = n
    if nleaves is None:
        nleaves = int(r2leaf[~border].max()) + 1 if (~border).any() else 0
    leaf_sorted = np.where(border, nleaves, r2leaf)[row_perm]
    leaf_row_ptr = np.searchsorted(leaf_sorted, np.arange(nleaves + 1), side="left")
    cls_leaf = np.where((ck_part < K) & (ck_sub == 0), ck_leaf, -1)[col_perm]
    leaf_col_lo = np.full(nleaves, 0, dtype=np.int64)
    leaf_col_hi = np.full(nleaves, 0, dtype=np.int64)
    for l in range(nleaves):
        w = np.flatnonzero(cls_leaf == l)
        if w.size:
            leaf_col_lo[l], leaf_col_hi[l] = w[0], w[-1] + 1
    return dict(row_perm=row_perm.astype(np.int64), col_perm=col_perm.astype(np.int64),
                part_ptr=part_ptr.astype(np.int64), col_part_ptr=col_part_ptr.astype(np.int64),
                leaf_row_ptr=leaf_row_ptr.astype(np.int64), leaf_col_lo=leaf_col_lo,
                leaf_col_hi=leaf_col_hi)


def canonical_split(A, nz_part, nz_leaf, K):
    """Row and column orders for the splitting (Section 4).

    Rows whose nonzeros all lie in one leaf come first, grouped by leaf; rows
    spread over several leaves follow, grouped by part (rows spread over
    several parts last); empty rows close the order.  Columns follow the same
    rule as :func:`canonical_rowcol` (classes, then the set of row groups that
    read them, then decreasing number of nonzeros, then original index); a
    nonzero's row group is that of its stored row (leaf, row) in the per-leaf
    storage of :func:`split_gcsr`, whose stored rows are cut into
    XCD_GROUPS runs of nearly equal nonzeros.

    Returns dict(row_perm, col_perm, row_shared_begin, row_empty_begin,
    col_part_ptr[K+2]).
    """
    nz_part = _i64(nz_part)
    nz_leaf = _i64(nz_leaf)
    m, n = A.m, A.n
    rows = _row_of(A)
    cols = _i64(A.colidx)
    nl_r, l_r = _sets_per_index(rows, nz_leaf, m)
    np_r, p_r = _sets_per_index(rows, nz_part, m)
    empty = nl_r == 0
    rk0 = np.where(empty, 2, np.where(nl_r == 1, 0, 1))
    rk1 = np.where(rk0 == 0, l_r, np.where(np_r == 1, p_r, K))
    rk1 = np.where(empty, 0, rk1)
    row_perm = np.lexsort((np.arange(m), rk1, rk0))
    row_shared_begin = int(np.sum(rk0 == 0))
    row_empty_begin = int(np.sum(rk0 <= 1))
    nl_c, l_c = _sets_per_index(cols, nz_leaf, n)
    np_c, p_c = _sets_per_index(cols, nz_part, n)
    ck_part = np.where(np_c == 1, p_c, K)
    ck_sub = np.where((ck_part < K) & (nl_c > 1), 1, 0)
    ck_leaf = np.where((ck_part < K) & (nl_c == 1), l_c, 0)
    cdeg = np.bincount(cols, minlength=n)
    # stored rows: (leaf, new row) pairs, leaf-major then by new row
    inv_r = np.empty(m, dtype=np.int64)
    inv_r[row_perm] = np.arange(m)
    nr = inv_r[rows]
    order = np.lexsort((nr, nz_leaf))
    key = nz_leaf[order] * max(m, 1) + nr[order]
    first = np.r_[True, key[1:] != key[:-1]] if key.size else np.zeros(0, bool)
    start_sorted = np.maximum.accumulate(np.where(first, np.arange(key.size), 0)) if key.size else key
    start = np.empty(key.size, dtype=np.int64)
    start[order] = start_sorted
    mask = _reader_mask(cols, _group_of_start(start, A.nnz), n)
    col_perm = np.lexsort((np.arange(n), -cdeg, mask, ck_leaf, ck_sub, ck_part))
    col_part_ptr = np.searchsorted(ck_part[col_perm], np.arange(K + 2), side="left")
    col_part_ptr[K + 1] = n
    return dict(row_perm=row_perm.astype(np.int64), col_perm=col_perm.astype(np.int64),
                row_shared_begin=row_shared_begin, row_empty_begin=row_empty_begin,
                col_part_ptr=col_part_ptr.astype(np.int64))


def split_gcsr(A, nz_leaf, nleaves, row_perm, col_perm):
    """The per-leaf GCSR storage of a splitting in reordered coordinates.

    Leaf l holds the nonzeros with nz_leaf == l.  Its stored rows ("slots")
    are its non-empty rows in ascending new index (the non-empty-row list of
    the GCSR format, Section 5.2); entries ascend by new column.  Returns
    dict(leaf_slot_ptr, slot_row, slot_ptr, colidx, vals), all concatenated
    in leaf order.
    """
    rows = _row_of(A)
    inv_r = np.empty(A.m, dtype=np.int64)
    inv_r[_i64(row_perm)] = np.arange(A.m)
    inv_c = np.empty(A.n, dtype=np.int64)
    inv_c[_i64(col_perm)] = np.arange(A.n)
    nr = inv_r[rows]
    nc = inv_c[_i64(A.colidx)]
    lf = _i64(nz_leaf)
    order = np.lexsort((nc, nr, lf))
    lf_s, nr_s = lf[order], nr[order]
    newslot = np.r_[True, (lf_s[1:] != lf_s[:-1]) | (nr_s[1:] != nr_s[:-1])] if order.size else np.zeros(0, bool)
    starts = np.flatnonzero(newslot)
    slot_row = nr_s[starts]
    slot_leaf = lf_s[starts]
    slot_ptr = np.r_[starts, order.size].astype(np.int64)
    leaf_slot_ptr = np.searchsorted(slot_leaf, np.arange(nleaves + 1), side="left")
    return dict(leaf_slot_ptr=leaf_slot_ptr.astype(np.int64), slot_row=slot_row,
                slot_ptr=slot_ptr, colidx=nc[order], vals=_f64(A.vals)[order])


# --------------------------------------------------------------------------
# Structural checks of the forms (Eq. 1-3, Eq. 5, Section 4)


def check_sb(rowptr, colidx, part_ptr, col_part_ptr, K, db=False):
    """Check a reordered CSR against the K-way SB form (Eq. 1) or DB form (Eq. 5).

    Every nonzero of a part row lies in that part's column slice C_k or in
    the column border C_B; columns of C_k are touched by part k only (their
    lambda, counted over part rows, is 1) and columns of C_B have lambda != 1.
    With ``db`` the rows from part_ptr[K] on form the row border R_B and may
    hold any column.  Returns a list of violated rules (empty when valid).
    """
    rowptr, colidx = _i64(rowptr), _i64(colidx)
    part_ptr, col_part_ptr = _i64(part_ptr), _i64(col_part_ptr)
    m = rowptr.size - 1
    n = int(col_part_ptr[-1])
    errs = []
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    rpart = np.searchsorted(part_ptr, rows, side="right") - 1
    cpart = np.searchsorted(col_part_ptr, colidx, side="right") - 1
    if not db and part_ptr[K] != m:
        errs.append("SB form has a row border")
    in_parts = rpart < K
    bad = in_parts & (cpart != rpart) & (cpart != K)
    if bad.any():
        errs.append(f"{int(bad.sum())} nonzeros outside A_kk and C_B")
    lam = np.zeros(n, dtype=np.int64)
    sel = in_parts
    if sel.any():
        key = np.unique(colidx[sel] * (K + 1) + rpart[sel])
        lam = np.bincount(key // (K + 1), minlength=n)
    colk = np.searchsorted(col_part_ptr, np.arange(n), side="right") - 1
    if ((colk < K) & (lam != 1)).any():
        errs.append("a column of some C_k is not touched by exactly one part")
    if ((colk == K) & (lam == 1)).any():
        errs.append("a column of C_B has connectivity 1")
    return errs


def check_split(A, nz_part, K):
    """A splitting is a partition of the stored nonzeros into K parts."""
    nz_part = _i64(nz_part)
    errs = []
    if nz_part.size != A.nnz:
        errs.append("nz_part length differs from nnz")
    elif nz_part.size and (nz_part.min() < 0 or nz_part.max() >= K):
        errs.append("part id out of range")
    return errs


# --------------------------------------------------------------------------
# Precision mode


def to_f32(v):
    v = _f64(v)
    out = np.empty(v.size, dtype=np.float32)
    _check(lib().orc_to_f32(ctypes.c_int64(v.size), _p(v), _p(out)))
    return out


def f32_to_bf16(v):
    v = np.ascontiguousarray(v, dtype=np.float32)
    out = np.empty(v.size, dtype=np.uint16)
    _check(lib().orc_f32_to_bf16(ctypes.c_int64(v.size), _p(v), _p(out)))
    return out


def bf16_bits_to_f32(h):
    return (np.ascontiguousarray(h, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def spmv_lowp(A, vals32, x32, vals16=None):
    """binary32-accumulated product with quantized values (left to right)."""
    rp, ci = _i64(A.rowptr), _i64(A.colidx)
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    v32 = np.ascontiguousarray(vals32 if vals32 is not None else np.zeros(1), dtype=np.float32)
    y = np.empty(A.m, dtype=np.float32)
    v16p = None
    if vals16 is not None:
        v16 = np.ascontiguousarray(vals16, dtype=np.uint16)
        v16p = _p(v16)
    _check(lib().orc_spmv_lowp(ctypes.c_int64(A.m), _p(rp), _p(ci), _p(v32), v16p,
                               _p(x32), _p(y)))
    return y


def cg(apply, b, tol, max_iter, x0=None, dtype=np.float64):
    """Conjugate gradients (Hestenes-Stiefel) in the given precision.

    Returns (x, iterations, relative residual of the recurrence).
    """
    b = np.asarray(b, dtype=dtype)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=dtype).copy()
    r = b - apply(x).astype(dtype) if x0 is not None else b.copy()
    p = r.copy()
    rr = dtype(np.dot(r, r))
    bn = np.sqrt(dtype(np.dot(b, b)))
    if bn == 0:
        return x, 0, 0.0
    it = 0
    while it < max_iter and np.sqrt(rr) > tol * bn:
        q = apply(p).astype(dtype)
        alpha = rr / dtype(np.dot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        rr_new = dtype(np.dot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr) / bn)


def ir_cg(apply64, apply_low, b, tol=1e-10, inner_tol=1e-3, max_outer=50,
          max_inner=1000):
    """Mixed-precision iterative refinement around an inner binary32 CG.

    x <- 0; r <- b - A x (binary64); while ||r|| / ||b|| > tol: solve A d = r
    approximately by CG in binary32 with the quantized matrix (to relative
    residual inner_tol), then x <- x + d and r <- b - A x in binary64.
    Returns (x, outer iterations, total inner iterations, final relative
    residual).
    """
    b = _f64(b)
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    outer = inner_total = 0
    rel = np.linalg.norm(r) / bn if bn else 0.0
    while rel > tol and outer < max_outer:
        scale = np.linalg.norm(r)
        d, it, _ = cg(lambda v: apply_low(v.astype(np.float32)),
                      (r / scale).astype(np.float32), inner_tol, max_inner,
                      dtype=np.float32)
        x = x + scale * d.astype(np.float64)
        r = b - apply64(x)
        rel = np.linalg.norm(r) / bn
        outer += 1
        inner_total += it
    return x, outer, inner_total, float(rel)


# --------------------------------------------------------------------------
# Selector network: 40 -> 64 -> 64 -> 24 multilayer perceptron, binary64.

MLP_SHAPES = [("W1", (64, 40)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (24, 64)), ("b3", (24,))]


def mlp_unflatten(theta):
    theta = _f64(theta)
    out, o = {}, 0
    for name, shp in MLP_SHAPES:
        sz = int(np.prod(shp))
        out[name] = theta[o:o + sz].reshape(shp)
        o += sz
    assert o == theta.size
    return out


def mlp_flatten(p):
    return np.concatenate([np.ravel(p[name]) for name, _ in MLP_SHAPES])


def mlp_forward(theta, X):
    """Linear-ReLU-Linear-ReLU-Linear; returns logits (batch x 24)."""
    p = mlp_unflatten(theta)
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    return h2 @ p["W3"].T + p["b3"]


def mlp_loss(theta, X, labels):
    """Mean softmax cross-entropy of the labels."""
    z = mlp_forward(theta, _f64(X))
    z = z - z.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z).sum(axis=1))
    return float(np.mean(lse - z[np.arange(z.shape[0]), labels]))


def mlp_grad(theta, X, labels):
    """(loss, gradient) by the chain rule through the three layers."""
    X = _f64(X)
    p = mlp_unflatten(theta)
    B = X.shape[0]
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"].T + p["b3"]
    zs = z3 - z3.max(axis=1, keepdims=True)
    e = np.exp(zs)
    sm = e / e.sum(axis=1, keepdims=True)
    loss = float(np.mean(np.log(e.sum(axis=1)) - zs[np.arange(B), labels]))
    d3 = sm.copy()
    d3[np.arange(B), labels] -= 1.0
    d3 /= B
    g = {"W3": d3.T @ h2, "b3": d3.sum(axis=0)}
    d2 = (d3 @ p["W3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    return loss, mlp_flatten(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba): returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# Selector features (a reading: the 40 inputs of the selector network are
# log1p(n), log1p(nnz), a 16-bin histogram of row degrees, a 16-bin histogram
# of column degrees and six structure statistics; the paper defines none of
# them, they describe what its Section 3-4 methods exploit: how far nonzeros
# lie from the diagonal and how much block structure there is).

def degree_bin(d):
    """Bin 0: degree 0; bin b in 1..15: 2^(b-1) <= d < 2^b; bin 15 also takes
    every degree >= 2^14."""
    d = np.asarray(d, dtype=np.int64)
    b = np.zeros(d.shape, dtype=np.int64)
    pos = d > 0
    b[pos] = np.minimum(np.floor(np.log2(d[pos])).astype(np.int64) + 1, 15)
    return b


def features(A):
    """The 40 features of an m x n CSR matrix, binary64 (to be stored in
    binary32):

      0 log1p(n)           1 log1p(nnz)
      2..17  fraction of rows in each degree bin (degree_bin)
      18..33 fraction of columns in each degree bin
      with u = |i/m - j/n| over the nonzeros (i, j):
      34 mean u            35 max u
      36 fraction of nonzeros with u <= 1/64
      37 fraction of nonzeros in a diagonal block of the 8 x 8 grid,
         floor(8 i / m) == floor(8 j / n)
      38 mean over non-empty rows of (last column - first column) / n
      39 coefficient of variation of the row degrees (std / mean; 0 when
         the mean is 0)
    Empty matrices give zeros for every statistic over nonzeros or rows.
    """
    m, n, nnz = A.m, A.n, A.nnz
    f = np.zeros(40)
    f[0] = np.log1p(n)
    f[1] = np.log1p(nnz)
    rdeg = np.diff(_i64(A.rowptr))
    cdeg = np.bincount(_i64(A.colidx), minlength=n) if n else np.zeros(0, np.int64)
    if m:
        f[2:18] = np.bincount(degree_bin(rdeg), minlength=16) / m
    if n:
        f[18:34] = np.bincount(degree_bin(cdeg), minlength=16) / n
    if nnz:
        i = np.repeat(np.arange(m, dtype=np.int64), rdeg)
        j = _i64(A.colidx)
        u = np.abs(i / m - j / n)
        f[34] = u.mean()
        f[35] = u.max()
        f[36] = np.mean(u <= 1.0 / 64.0)
        f[37] = np.mean((8 * i) // m == (8 * j) // n)
        ne = np.flatnonzero(rdeg > 0)
        rp = _i64(A.rowptr)
        f[38] = np.mean((j[rp[ne + 1] - 1] - j[rp[ne]]) / n)
    if m and rdeg.mean() > 0:
        f[39] = rdeg.std() / rdeg.mean()
    return f


# --------------------------------------------------------------------------
# Comparison orderings of Section 5.1 on the bipartite graph of A: vertices
# are rows 0..m-1 and columns m..m+n-1, an edge per nonzero.  Readings (the
# paper names the methods, not their start vertices or tie-breaks): sBFS
# visits components in order of their smallest vertex, breadth-first from
# it, neighbours by increasing number; sRCM starts each component (in order
# of its smallest vertex) at George and Liu's pseudo-peripheral vertex,
# searched from the component's least-degree vertex (smallest number on
# ties), visits unvisited neighbours by increasing (degree, number), and
# reverses the whole visit sequence.


def _bipartite(A):
    """CSR adjacency of the bipartite graph, neighbours ascending."""
    m, n = A.m, A.n
    rows = _row_of(A)
    cols = _i64(A.colidx) + m
    src = np.concatenate([rows, cols])
    dst = np.concatenate([cols, rows])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    off = np.zeros(m + n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=m + n), out=off[1:])
    return off, dst


def _levels(off, adj, start, visited):
    """Breadth-first search from start over vertices with visited False,
    level by level; each level lists the new vertices in the order their
    first visiting neighbour (earlier in the previous level, and earlier in
    its adjacency list) reaches them.  Marks them visited; returns the
    levels."""
    visited[start] = True
    levels = [np.array([start], dtype=np.int64)]
    while True:
        fr = levels[-1]
        lens = off[fr + 1] - off[fr]
        if lens.sum() == 0:
            break
        idx = np.repeat(off[fr] - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + np.arange(lens.sum())
        cand = adj[idx]
        cand = cand[~visited[cand]]
        if cand.size == 0:
            break
        _, first = np.unique(cand, return_index=True)
        new = cand[np.sort(first)]
        visited[new] = True
        levels.append(new)
    return levels


def order_bfs(A):
    """sBFS row and column orders (new -> old)."""
    m, n = A.m, A.n
    off, adj = _bipartite(A)
    visited = np.zeros(m + n, dtype=bool)
    seq = []
    for v in range(m + n):
        if not visited[v]:
            seq.extend(_levels(off, adj, v, visited))
    seq = np.concatenate(seq) if seq else np.zeros(0, np.int64)
    return seq[seq < m], seq[seq >= m] - m


def order_rcm(A):
    """sRCM row and column orders (new -> old)."""
    m, n = A.m, A.n
    off, adj = _bipartite(A)
    deg = np.diff(off)
    # every adjacency list sorted by (degree, number) for Cuthill-McKee
    owner = np.repeat(np.arange(m + n), deg)
    o2 = np.lexsort((adj, deg[adj], owner))
    adj_cm = adj[o2]
    done = np.zeros(m + n, dtype=bool)
    seq = []
    for v0 in range(m + n):
        if done[v0]:
            continue
        comp = np.concatenate(_levels(off, adj, v0, np.zeros(m + n, dtype=bool)))
        start = int(comp[np.lexsort((comp, deg[comp]))[0]])

        def last_level(s):
            lv = _levels(off, adj, s, np.zeros(m + n, dtype=bool))
            return len(lv), lv[-1]
        ecc, last = last_level(start)
        while True:
            cand = int(last[np.lexsort((last, deg[last]))[0]])
            e2, l2 = last_level(cand)
            if e2 <= ecc:
                break
            start, ecc, last = cand, e2, l2
        seq.extend(_levels(off, adj_cm, start, done))
    seq = np.concatenate(seq)[::-1] if seq else np.zeros(0, np.int64)
    return seq[seq < m], seq[seq >= m] - m
