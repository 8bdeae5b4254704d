"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests re-types an oracle formula: each compares the oracle with
an independent route to the same number (dense integer arithmetic, a library
routine, brute force over sets, a hand-worked example, a closed form).
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from synth import CSR, gen_c1, gen_uniform_zipf


def rand_csr(rng, m, n, density, integer=False, empty_rows=0.0):
    D = (rng.random((m, n)) < density).astype(np.float64)
    if empty_rows:
        D[rng.random(m) < empty_rows] = 0.0
    if integer:
        V = rng.integers(-8, 9, size=(m, n)).astype(np.float64)
        V[V == 0] = 1.0
    else:
        V = rng.uniform(-1, 1, size=(m, n))
    D = D * V
    return dense_to_csr(D), D


def dense_to_csr(D):
    m, n = D.shape
    r, c = np.nonzero(D)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m), out=rowptr[1:])
    return CSR(m, n, rowptr, c.astype(np.int32), D[r, c].astype(np.float64))


# ---------------------------------------------------------------- products

@settings(max_examples=60, deadline=None)
@given(st.integers(1, 30), st.integers(1, 30), st.floats(0.0, 1.0), st.integers(0, 2**31))
def test_spmv_integer_exact_vs_dense(orc, m, n, dens, seed):
    """Small integers make every summation order exact: the CSR row sums must
    equal the dense integer product bit for bit."""
    rng = np.random.default_rng(seed)
    A, D = rand_csr(rng, m, n, dens, integer=True)
    x = rng.integers(-8, 9, size=n)
    y = orc.spmv(A, x.astype(np.float64))
    ref = (D.astype(np.int64) @ x).astype(np.float64)
    assert np.array_equal(y, ref)


@settings(max_examples=40, deadline=None)
@given(st.integers(1, 40), st.integers(1, 40), st.integers(0, 2**31))
def test_spmv_float_vs_dense(orc, m, n, seed):
    rng = np.random.default_rng(seed)
    A, D = rand_csr(rng, m, n, 0.3)
    x = rng.uniform(-1, 1, n)
    y = orc.spmv(A, x)
    ref = D @ x
    bound = np.abs(D) @ np.abs(x)
    assert np.all(np.abs(y - ref) <= 1e-14 * bound + 1e-300)


def test_spmv_vs_scipy_c1(orc):
    import scipy.sparse as sp
    A = gen_c1()
    x = np.random.default_rng(5).uniform(-1, 1, A.n)
    S = sp.csr_matrix((A.vals, A.colidx, A.rowptr), shape=(A.m, A.n))
    y = orc.spmv(A, x)
    ref = S @ x
    bound = abs(S) @ np.abs(x)
    assert np.all(np.abs(y - ref) <= 1e-13 * bound)


def test_spmv_special_cases(orc):
    n = 7
    I = dense_to_csr(np.eye(n))
    x = np.arange(n, dtype=np.float64) - 3.5
    assert np.array_equal(orc.spmv(I, x), x)
    d = np.array([2.0, -1.0, 0.5, 4.0, 3.0, 1.0, -2.0])
    assert np.array_equal(orc.spmv(dense_to_csr(np.diag(d)), x), d * x)
    D = np.zeros((4, 5))
    D[1, 2] = 3.0
    y = orc.spmv(dense_to_csr(D), np.ones(5))
    assert np.array_equal(y, [0.0, 3.0, 0.0, 0.0])
    # an empty matrix
    E = CSR(0, 3, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert orc.spmv(E, np.ones(3)).size == 0


def test_spmv_is_left_to_right(orc):
    """Rounding reveals the summation order: (1 + 1e16) - 1e16 = 0 in binary64
    when summed in storage order."""
    A = CSR(1, 3, np.array([0, 3]), np.array([0, 1, 2], np.int32),
            np.array([1.0, 1e16, -1e16]))
    assert orc.spmv(A, np.ones(3))[0] == 0.0


def test_spmv_rows_and_abs(orc):
    rng = np.random.default_rng(3)
    A, D = rand_csr(rng, 50, 40, 0.2, integer=True)
    x = rng.integers(-4, 5, size=40).astype(np.float64)
    rows = np.array([0, 7, 49, 7])
    y, a = orc.spmv_rows(A, x, rows)
    assert np.array_equal(y, (D @ x)[rows])
    assert np.array_equal(a, (np.abs(D) @ np.abs(x))[rows])
    assert np.array_equal(orc.abs_rowsum(A, x), np.abs(D) @ np.abs(x))


def test_spmm_integer(orc):
    rng = np.random.default_rng(4)
    A, D = rand_csr(rng, 30, 20, 0.3, integer=True)
    X = rng.integers(-5, 6, size=(20, 8)).astype(np.float64)
    assert np.array_equal(orc.spmm(A, X), D @ X)


# ------------------------------------------------------------- permutation

@settings(max_examples=40, deadline=None)
@given(st.integers(1, 25), st.integers(1, 25), st.integers(0, 2**31))
def test_permute_matches_dense(orc, m, n, seed):
    """A_hat = P_r A P_c with new->old perms is the dense fancy-indexed matrix,
    and P A Q (Q^T x) = P (A x) exactly on integers (Section 3)."""
    rng = np.random.default_rng(seed)
    A, D = rand_csr(rng, m, n, 0.35, integer=True)
    rp_, cp_ = rng.permutation(m), rng.permutation(n)
    orp, oci, ov = orc.permute_csr(A, rp_, cp_)
    H = np.zeros((m, n))
    for i in range(m):
        for p in range(orp[i], orp[i + 1]):
            H[i, oci[p]] = ov[p]
        assert np.all(np.diff(oci[orp[i]:orp[i + 1]]) > 0)
    assert np.array_equal(H, D[rp_][:, cp_])
    x = rng.integers(-8, 9, size=n).astype(np.float64)
    Ah = CSR(m, n, orp, oci.astype(np.int32), ov)
    assert np.array_equal(orc.spmv(Ah, x[cp_]), orc.spmv(A, x)[rp_])


def test_permute_rejects_non_bijection(orc):
    A, _ = rand_csr(np.random.default_rng(0), 4, 4, 0.5)
    with pytest.raises(ValueError):
        orc.permute_csr(A, np.arange(4), np.array([0, 1, 1, 2]))


# ------------------------------------------------------------------- split

@settings(max_examples=40, deadline=None)
@given(st.integers(1, 30), st.integers(1, 30), st.integers(1, 9), st.integers(0, 2**31))
def test_split_sum_equals_product(orc, m, n, K, seed):
    """sum_k A^k x = A x for any nonzero-disjoint splitting (Section 4);
    exact on integers."""
    rng = np.random.default_rng(seed)
    A, D = rand_csr(rng, m, n, 0.4, integer=True)
    part = rng.integers(0, K, size=A.nnz)
    x = rng.integers(-8, 9, size=n).astype(np.float64)
    assert np.array_equal(orc.split_spmv(A, part, K, x), D @ x)
    y0 = rng.integers(-8, 9, size=m).astype(np.float64)
    assert np.array_equal(orc.split_spmv(A, part, K, x, y0), y0 + D @ x)


def test_split_accumulates_part_by_part(orc):
    """y <- y + A^k x is applied for k = 1..K in turn (Section 4): in binary64
    (1e16 - 1e16) + 1 = 1 when the two large entries form A^1, while storage
    order would give (1 + 1e16) - 1e16 = 0."""
    A = CSR(1, 3, np.array([0, 3]), np.array([0, 1, 2], np.int32),
            np.array([1.0, 1e16, -1e16]))
    part = np.array([1, 0, 0])
    assert orc.split_spmv(A, part, 2, np.ones(3))[0] == 1.0
    assert orc.split_spmv(A, np.array([0, 0, 0]), 1, np.ones(3))[0] == 0.0


def test_split_rejects_bad_part(orc):
    A, _ = rand_csr(np.random.default_rng(0), 5, 5, 0.6)
    with pytest.raises(ValueError):
        orc.split_spmv(A, np.full(A.nnz, 3), 3, np.ones(5))


# ---------------------------------------------------------- connectivities

def brute_lambda_cols(D, r2p, K):
    m, n = D.shape
    return np.array([len({r2p[i] for i in range(m) if D[i, j] != 0 and 0 <= r2p[i] < K})
                     for j in range(n)])


@settings(max_examples=40, deadline=None)
@given(st.integers(1, 20), st.integers(1, 20), st.integers(1, 6), st.integers(0, 2**31))
def test_lambda_cols_brute(orc, m, n, K, seed):
    rng = np.random.default_rng(seed)
    A, D = rand_csr(rng, m, n, 0.3)
    r2p = rng.integers(0, K + 1, size=m)  # value K marks a border row
    lam = orc.lambda_cols(A, r2p, K)
    assert np.array_equal(lam, brute_lambda_cols(D, r2p, K))
    deg = (D != 0).sum(axis=1)
    assert orc.bound_db(A, r2p, K) == lam.sum() + deg[r2p == K].sum()


@settings(max_examples=40, deadline=None)
@given(st.integers(1, 20), st.integers(1, 20), st.integers(1, 6), st.integers(0, 2**31))
def test_lambda_split_brute(orc, m, n, K, seed):
    rng = np.random.default_rng(seed)
    A, D = rand_csr(rng, m, n, 0.3)
    part = rng.integers(0, K, size=A.nnz)
    rows = np.repeat(np.arange(m), np.diff(A.rowptr))
    lr, lc = orc.lambda_split(A, part, K)
    for i in range(m):
        assert lr[i] == len(set(part[rows == i]))
    for j in range(n):
        assert lc[j] == len(set(part[A.colidx == j]))
    assert orc.bound_split(A, part, K) == lr.sum() + lc.sum()


def test_lambda_hidden_block_diagonal(orc):
    """A pure block-diagonal matrix split along its blocks has every column
    in exactly one row slice: sum_j lambda(c_j) = n (Theorem 1 closed form)."""
    rng = np.random.default_rng(9)
    K, bs = 4, 6
    D = np.zeros((K * bs, K * bs))
    for k in range(K):
        blk = rng.uniform(-1, 1, (bs, bs)) * (rng.random((bs, bs)) < 0.5)
        np.fill_diagonal(blk, 1.0)
        D[k * bs:(k + 1) * bs, k * bs:(k + 1) * bs] = blk
    p = rng.permutation(K * bs)
    Dh = D[p][:, p]
    A = dense_to_csr(Dh)
    r2p = (np.arange(K * bs) // bs)[p]
    assert orc.bound_sb(A, r2p, K) == K * bs
    # every row in its own part of size one gives the column degrees
    assert orc.bound_sb(A, np.arange(K * bs), K * bs) == A.nnz


def test_bounds_hand_worked():
    """Hand-worked 4x5 example (Eq. 3, Theorem 1, Theorem 2, Corollary 4).

        row0: c0 c1          part 0
        row1: c1 c2          part 0
        row2: c2 c3 c4       part 1
        row3: c0 c4          part 1 (DB: border row)

    SB (parts {0,1},{2,3}): lambda = c0:2 c1:1 c2:2 c3:1 c4:1 -> sum 7.
    DB with row 3 in R_B: lambda' = c0:1 c1:1 c2:2 c3:1 c4:1 = 6, plus
    nnz(row3) = 2 -> 8.
    Split with parts [0,0 | 0,1 | 1,1,1 | 0,1] (storage order):
    lambda(r) = 1,2,1,2 -> 6; lambda(c): c0 {0}, c1 {0}, c2 {1}, c3 {1},
    c4 {1} -> 5; total 11.
    """
    import oracle as orc
    D = np.zeros((4, 5))
    for i, cs in enumerate([[0, 1], [1, 2], [2, 3, 4], [0, 4]]):
        D[i, cs] = 1.0
    A = dense_to_csr(D)
    assert orc.bound_sb(A, [0, 0, 1, 1], 2) == 7
    assert orc.bound_db(A, [0, 0, 1, 2], 2) == 8
    assert orc.bound_split(A, [0, 0, 0, 1, 1, 1, 1, 0, 1], 2) == 11


# -------------------------------------------------------- canonical orders

def test_canonical_rowcol_hand_worked(orc):
    """Canonical orders of the SB and DB forms worked by hand (Eq. 1 and
    Eq. 5 fix the blocks; inside them: class, then the set of row groups
    reading a column, then decreasing count, then index).

    8 x 6 matrix, 16 nonzeros, parts {r0..r3}, {r4..r7}, one leaf each:
      r0: c0 c1 | r1: c1 | r2: c0 c1 c2 | r3: c2 | r4: c3 c4 | r5: c3 c5 |
      r6: c4 c5 | r7: c2 c4 c5
    Row starts 0 2 3 6 7 9 11 13 give row groups floor(8 s / 16) =
    0 1 1 3 3 4 5 6.  Reader sets (bit g for group g): c0 {0,1} = 3,
    c1 {0,1} = 3, c2 {1,3,6} = 74, c3 {3,4} = 24, c4 {3,5,6} = 104,
    c5 {4,5,6} = 112.  SB classes: C_1 = {c0, c1}, C_2 = {c3, c4, c5},
    C_B = {c2}.  In C_1 the sets tie, so the count decides (c1: 3 before
    c0: 2, against index order); in C_2 the sets decide (c3 before c4, c5,
    against count order)."""
    D = np.zeros((8, 6))
    for i, cs in enumerate([[0, 1], [1], [0, 1, 2], [2], [3, 4], [3, 5], [4, 5], [2, 4, 5]]):
        D[i, cs] = 1.0
    A = dense_to_csr(D)
    c = orc.canonical_rowcol(A, [0, 0, 0, 0, 1, 1, 1, 1], [0, 0, 0, 0, 1, 1, 1, 1], 2)
    assert list(c["row_perm"]) == list(range(8))
    assert list(c["col_perm"]) == [1, 0, 3, 4, 5, 2]
    assert list(c["part_ptr"]) == [0, 4, 8, 8]
    assert list(c["col_part_ptr"]) == [0, 2, 5, 6]
    orp, oci, _ = orc.permute_csr(A, c["row_perm"], c["col_perm"])
    assert orc.check_sb(orp, oci, c["part_ptr"], c["col_part_ptr"], 2) == []
    # DB with r7 in the row border R_B: c2 is then read by part 0 only among
    # part rows (C_1), while its reader set still counts r7's group (74):
    # C_1 = c1 c0 (set 3) then c2 (set 74); C_2 = c3 c4 c5; C_B empty
    c = orc.canonical_rowcol(A, [0, 0, 0, 0, 1, 1, 1, 2], [0, 0, 0, 0, 1, 1, 1, 0], 2)
    assert list(c["row_perm"]) == list(range(8))
    assert list(c["col_perm"]) == [1, 0, 2, 3, 4, 5]
    assert list(c["col_part_ptr"]) == [0, 3, 6, 6]
    orp, oci, _ = orc.permute_csr(A, c["row_perm"], c["col_perm"])
    assert orc.check_sb(orp, oci, c["part_ptr"], c["col_part_ptr"], 2, db=True) == []
    assert orc.check_sb(orp, oci, c["part_ptr"], c["col_part_ptr"], 2, db=False) != []
    # 4 x 5 matrix, 9 nonzeros: r0: c0 c1 | r1: c1 c2 | r2: c2 c3 c4 | r3: c0 c4,
    # parts {r0, r1}, {r2, r3}; groups 0 1 3 6; sets c0 65, c1 3, c2 10, c3 8,
    # c4 72: C_1 = c1 | C_2 = c3 c4 | C_B = c2 c0 (sets 10 < 65, against index)
    D = np.zeros((4, 5))
    for i, cs in enumerate([[0, 1], [1, 2], [2, 3, 4], [0, 4]]):
        D[i, cs] = 1.0
    c = orc.canonical_rowcol(dense_to_csr(D), [0, 0, 1, 1], [0, 0, 1, 1], 2)
    assert list(c["col_perm"]) == [1, 3, 4, 2, 0]


def test_check_sb_flags_violation(orc):
    """A nonzero of part 0 in part 1's column slice breaks Eq. 1."""
    D = np.zeros((4, 4))
    D[0, 0] = D[1, 1] = D[2, 2] = D[3, 3] = 1.0
    D[0, 2] = 1.0
    A = dense_to_csr(D)
    errs = orc.check_sb(A.rowptr, A.colidx, [0, 2, 4, 4], [0, 2, 4, 4], 2)
    assert errs


@settings(max_examples=25, deadline=None)
@given(st.integers(2, 30), st.integers(2, 30), st.integers(1, 5), st.integers(0, 2**31))
def test_canonical_rowcol_random_partition(orc, m, n, K, seed):
    """Any row partition yields a valid SB form after the canonical orders."""
    rng = np.random.default_rng(seed)
    A, _ = rand_csr(rng, m, n, 0.25)
    r2p = rng.integers(0, K, size=m)
    leaves_per = 2
    r2leaf = r2p * leaves_per + rng.integers(0, leaves_per, size=m)
    c = orc.canonical_rowcol(A, r2p, r2leaf, K, nleaves=K * leaves_per)
    assert sorted(c["row_perm"]) == list(range(m))
    assert sorted(c["col_perm"]) == list(range(n))
    orp, oci, _ = orc.permute_csr(A, c["row_perm"], c["col_perm"])
    assert orc.check_sb(orp, oci, c["part_ptr"], c["col_part_ptr"], K) == []
    # leaf-exclusive column ranges hold only columns of that leaf's rows
    inv = np.empty(m, np.int64)
    inv[c["row_perm"]] = np.arange(m)
    rows = np.repeat(np.arange(m), np.diff(orp))
    for l in range(K * leaves_per):
        lo, hi = c["leaf_col_lo"][l], c["leaf_col_hi"][l]
        sel = (oci >= lo) & (oci < hi)
        rl, rh = c["leaf_row_ptr"][l], c["leaf_row_ptr"][l + 1]
        assert np.all((rows[sel] >= rl) & (rows[sel] < rh))


def test_canonical_split_and_gcsr(orc):
    """The per-leaf GCSR of a splitting stores every nonzero once; summing
    the leaves back gives A_hat (Section 4, nonzero-disjoint parts)."""
    rng = np.random.default_rng(11)
    A, D = rand_csr(rng, 25, 30, 0.25)
    K = 3
    part = rng.integers(0, K, size=A.nnz)
    leaf = part * 2 + rng.integers(0, 2, size=A.nnz)
    c = orc.canonical_split(A, part, leaf, K)
    assert sorted(c["row_perm"]) == list(range(25))
    g = orc.split_gcsr(A, leaf, 2 * K, c["row_perm"], c["col_perm"])
    H = np.zeros_like(D)
    for s in range(g["slot_row"].size):
        for p in range(g["slot_ptr"][s], g["slot_ptr"][s + 1]):
            assert H[g["slot_row"][s], g["colidx"][p]] == 0
            H[g["slot_row"][s], g["colidx"][p]] = g["vals"][p]
    assert np.array_equal(H, D[c["row_perm"]][:, c["col_perm"]])
    # rows spread over several leaves are exactly those from row_shared_begin
    rows = np.repeat(np.arange(25), np.diff(A.rowptr))
    nleaf = np.array([len(set(leaf[rows == i])) for i in range(25)])
    inv = np.empty(25, np.int64)
    inv[c["row_perm"]] = np.arange(25)
    rb, re_ = c["row_shared_begin"], c["row_empty_begin"]
    assert np.all((inv[nleaf > 1] >= rb) & (inv[nleaf > 1] < re_))
    assert np.all(inv[nleaf == 1] < rb)
    assert np.all(inv[nleaf == 0] >= re_)


def _split_example():
    """8 x 8 matrix split into K = 2 parts with two leaves each (part 0:
    leaves 0, 1; part 1: leaves 2, 3).  Entries (row, column, leaf):"""
    entries = [(0, 0, 2), (0, 3, 2), (0, 6, 2), (0, 7, 2),      # row 0: leaf 2 only
               (1, 2, 3), (1, 3, 2), (1, 6, 3), (1, 7, 3),      # row 1: leaves 2, 3 (part 1)
               (3, 0, 0), (3, 4, 3),                            # row 3: parts 0 and 1
               (4, 1, 0), (4, 5, 0),                            # row 4: leaf 0 only
               (5, 2, 1), (5, 5, 0),                            # row 5: leaves 0, 1 (part 0)
               (6, 4, 1),                                       # row 6: leaf 1 only
               (7, 4, 3), (7, 7, 3)]                            # row 7: leaf 3 only; row 2 empty
    D = np.zeros((8, 8))
    leafD = np.full((8, 8), -1)
    for r, c, l in entries:
        D[r, c] = 10 * r + c + 1
        leafD[r, c] = l
    A = dense_to_csr(D)
    rows = np.repeat(np.arange(8), np.diff(A.rowptr))
    leaf = leafD[rows, A.colidx]
    return A, leaf // 2, leaf


def test_canonical_split_hand_worked(orc):
    """Exact orders of the split (Section 4; inside the forms rows and
    columns go by class, columns then by the set of row groups that read
    them, then by decreasing count, then by index), worked by hand on
    _split_example.

    Rows: single-leaf rows by leaf (r4 | r6 | r0 | r7), not by index; then
    rows shared by leaves of one part, by part (r5 of part 0 before r1 of
    part 1), before the row shared by both parts (r3); the empty row r2 last.

    Stored rows, leaf-major (new row numbers: r4 0, r6 1, r0 2, r7 3, r5 4,
    r1 5, r3 6, r2 7) start at offsets 0 2 3 | 4 5 | 6 10 | 11 13 16 of the
    17 nonzeros: row groups floor(8 s / 17) = 0 0 1 | 1 2 | 2 4 | 5 6 7.
    Columns (class; reader set; count): c1 (leaf 0; 1; 1), c5 (leaf 0; 1; 2),
    c3 (leaf 2; 20; 2), c6 (part 1 shared; 68; 2), c7 (part 1 shared; 100; 3),
    c0 (border; 6; 2), c2 (border; 68; 2), c4 (border; 162; 3).  Order:
    c5 c1 (sets tie: count) | c3 | c6 c7 (sets, against count) | c0 c2 c4."""
    A, part, leaf = _split_example()
    c = orc.canonical_split(A, part, leaf, 2)
    assert list(c["row_perm"]) == [4, 6, 0, 7, 5, 1, 3, 2]
    assert c["row_shared_begin"] == 4 and c["row_empty_begin"] == 7
    assert list(c["col_perm"]) == [5, 1, 3, 6, 7, 0, 2, 4]
    assert list(c["col_part_ptr"]) == [0, 2, 5, 8]
    # per-leaf GCSR in the new coordinates (columns: c5->0, c1->1, c3->2,
    # c6->3, c7->4, c0->5, c2->6, c4->7), each leaf's non-empty rows
    # ascending, entries by new column
    g = orc.split_gcsr(A, leaf, 4, c["row_perm"], c["col_perm"])
    assert list(g["leaf_slot_ptr"]) == [0, 3, 5, 7, 10]
    assert list(g["slot_row"]) == [0, 4, 6, 1, 4, 2, 5, 3, 5, 6]
    assert list(g["slot_ptr"]) == [0, 2, 3, 4, 5, 6, 10, 11, 13, 16, 17]
    assert list(g["colidx"]) == [0, 1, 0, 5, 7, 6, 2, 3, 4, 5, 2, 4, 7, 3, 4, 6, 7]
    assert list(g["vals"]) == [46, 42, 56, 31, 65, 53, 4, 7, 8, 1, 14, 78, 75, 17, 18, 13, 35]


# ------------------------------------------------------------ precision

def test_quantization_vs_libraries(orc):
    import torch
    rng = np.random.default_rng(2)
    v = np.concatenate([rng.uniform(-1, 1, 5000), rng.standard_normal(5000) * 1e30,
                        [0.0, -0.0, 1.0, 3.0e38, 1e-40, 1 + 2.0**-24, 1 + 3 * 2.0**-24]])
    f = orc.to_f32(v)
    assert np.array_equal(f.view(np.uint32), v.astype(np.float32).view(np.uint32))
    h = orc.f32_to_bf16(f)
    ref = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(h, ref)
    # ties to even: 1 + 2^-8 is halfway between bf16 1.0 and 1 + 2^-7
    t = np.array([1 + 2.0**-8, 1 + 3 * 2.0**-8], dtype=np.float32)
    assert list(orc.f32_to_bf16(t)) == [0x3F80, 0x3F82]


def test_lowp_spmv_integer_exact(orc):
    rng = np.random.default_rng(6)
    A, D = rand_csr(rng, 60, 50, 0.3, integer=True)
    x = rng.integers(-8, 9, size=50)
    f = orc.to_f32(A.vals)
    y32 = orc.spmv_lowp(A, f, x.astype(np.float32))
    y16 = orc.spmv_lowp(A, None, x.astype(np.float32), vals16=orc.f32_to_bf16(f))
    ref = (D.astype(np.int64) @ x).astype(np.float32)
    assert np.array_equal(y32, ref) and np.array_equal(y16, ref)


def test_lowp_spmv_rounds_in_binary32_left_to_right(orc):
    """The precision mode accumulates in binary32 (the reading for values
    stored in binary32 or bfloat16), product by product in storage order.

    Row 0: values (1, 2^24, -2^24) on x = 1.  In binary32, 1 + 2^24 is a tie
    that rounds to the even 2^24, and the row then cancels to 0; a binary64
    accumulator, or any order that adds 2^24 - 2^24 first, gives 1.
    Row 1: (1 + 2^-23)^2 = 1 + 2^-22 + 2^-46 is rounded to 1 + 2^-22 as a
    binary32 product, so subtracting 1 + 2^-22 leaves 0; a product kept in
    binary64 leaves 2^-46."""
    e = 2.0 ** -23
    D = np.array([[1.0, 2.0 ** 24, -(2.0 ** 24), 0.0],
                  [0.0, 0.0, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 0.0]])
    A = dense_to_csr(D)
    x = np.ones(4, dtype=np.float32)
    y = orc.spmv_lowp(A, orc.to_f32(A.vals), x)
    assert y[0] == 0.0
    # bfloat16 holds 1 and 2^24 exactly: the same cancellation
    y16 = orc.spmv_lowp(A, None, x, vals16=orc.f32_to_bf16(orc.to_f32(A.vals)))
    assert y16[0] == 0.0
    # row 1 of a second matrix: a * x with a = x = 1 + 2^-23, then -(1 + 2^-22) * 1
    B = CSR(1, 2, np.array([0, 2]), np.array([0, 1], dtype=np.int32),
            np.array([1.0 + e, -(1.0 + 2 * e)]))
    xb = np.array([1.0 + e, 1.0], dtype=np.float32)
    yb = orc.spmv_lowp(B, orc.to_f32(B.vals), xb)
    assert yb[0] == 0.0
    assert (1.0 + e) * (1.0 + e) - (1.0 + 2 * e) == 2.0 ** -46  # what binary64 would keep


def spd(rng, n, density=0.2):
    B = rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < density)
    S = B + B.T
    np.fill_diagonal(S, 0.0)
    np.fill_diagonal(S, np.abs(S).sum(axis=1) + 1.0)
    return S


def test_cg_and_ir_cg_vs_solve(orc):
    rng = np.random.default_rng(8)
    S = spd(rng, 80)
    A = dense_to_csr(S)
    xs = np.ones(80)
    b = S @ xs
    x, it, rel = orc.cg(lambda v: orc.spmv(A, v), b, 1e-12, 500)
    ref = np.linalg.solve(S, b)
    assert np.max(np.abs(x - ref)) < 1e-9
    f = orc.to_f32(A.vals)
    x2, outer, inner, rel2 = orc.ir_cg(lambda v: orc.spmv(A, v),
                                      lambda v: orc.spmv_lowp(A, f, v), b, tol=1e-10)
    assert rel2 <= 1e-10
    assert np.linalg.norm(b - S @ x2) / np.linalg.norm(b) <= 1e-10
    assert np.max(np.abs(x2 - ref)) < 1e-8
    assert outer >= 2  # binary32 alone cannot reach 1e-10


# ------------------------------------------------------------------- MLP

def test_mlp_gradient_finite_differences(orc):
    rng = np.random.default_rng(12)
    theta = rng.standard_normal(8344) * 0.2
    X = rng.standard_normal((7, 40))
    lab = rng.integers(0, 24, size=7)
    loss, g = orc.mlp_grad(theta, X, lab)
    assert abs(loss - orc.mlp_loss(theta, X, lab)) < 1e-12
    h = 1e-6
    idx = np.concatenate([rng.choice(8344, 60, replace=False), [0, 2559, 2560, 8343]])
    for i in idx:
        e = np.zeros(8344)
        e[i] = h
        fd = (orc.mlp_loss(theta + e, X, lab) - orc.mlp_loss(theta - e, X, lab)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_mlp_forward_and_adam_vs_torch(orc):
    import torch
    rng = np.random.default_rng(13)
    theta = rng.standard_normal(8344) * 0.2
    X = rng.standard_normal((5, 40))
    lab = rng.integers(0, 24, size=5)
    p = orc.mlp_unflatten(theta)
    net = torch.nn.Sequential(torch.nn.Linear(40, 64), torch.nn.ReLU(),
                              torch.nn.Linear(64, 64), torch.nn.ReLU(),
                              torch.nn.Linear(64, 24)).double()
    with torch.no_grad():
        for layer, (w, b) in zip([net[0], net[2], net[4]],
                                 [("W1", "b1"), ("W2", "b2"), ("W3", "b3")]):
            layer.weight.copy_(torch.from_numpy(p[w]))
            layer.bias.copy_(torch.from_numpy(p[b]))
    z = net(torch.from_numpy(X))
    assert np.allclose(z.detach().numpy(), orc.mlp_forward(theta, X), rtol=0, atol=1e-12)
    opt = torch.optim.Adam(net.parameters(), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(8344)
    v = np.zeros(8344)
    th = theta.copy()
    for t in range(1, 4):
        opt.zero_grad()
        loss = torch.nn.functional.cross_entropy(net(torch.from_numpy(X)), torch.from_numpy(lab))
        loss.backward()
        _, g = orc.mlp_grad(th, X, lab)
        tg = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                             net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                             net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])
        assert np.allclose(g, tg, rtol=1e-10, atol=1e-13)
        opt.step()
        th, m, v = orc.adam_step(th, g, m, v, t)
    tp = np.concatenate([net[0].weight.detach().numpy().ravel(), net[0].bias.detach().numpy(),
                         net[2].weight.detach().numpy().ravel(), net[2].bias.detach().numpy(),
                         net[4].weight.detach().numpy().ravel(), net[4].bias.detach().numpy()])
    assert np.allclose(th, tp, rtol=0, atol=1e-12)


# --------------------------------------------------------------- features

def test_features_closed_forms(orc):
    from synth import CSR
    n = 64
    eye = CSR(n, n, np.arange(n + 1), np.arange(n, dtype=np.int32), np.ones(n))
    f = orc.features(eye)
    assert f[0] == np.log1p(64) and f[1] == np.log1p(64)
    assert f[3] == 1.0 and f[19] == 1.0 and f[2:18].sum() == 1.0  # every degree is 1: bin 1
    assert f[34] == 0.0 and f[35] == 0.0 and f[36] == 1.0 and f[37] == 1.0 and f[38] == 0.0 and f[39] == 0.0
    # anti-diagonal: u = |i - (n-1-i)| / n = |2i - n + 1| / n, mean (n/2) / n for even n
    anti = CSR(n, n, np.arange(n + 1), np.arange(n - 1, -1, -1, dtype=np.int32), np.ones(n))
    g = orc.features(anti)
    assert abs(g[34] - 0.5) < 1e-15 and abs(g[35] - (n - 1) / n) < 1e-15
    assert g[36] == 2 / 64  # |2i - 63| <= 1 only for i = 31, 32
    # diagonal 8x8 grid blocks: i in block i//8, j = 63 - i in block 7 - i//8: never equal
    assert g[37] == 0.0
    # one dense row of 64 plus empty rows: row degrees [64, 0 x 63]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = n
    dense = CSR(n, n, rp, np.arange(n, dtype=np.int32), np.ones(n))
    h = orc.features(dense)
    assert h[2] == 63 / 64 and h[2 + 7] == 1 / 64  # 64 = 2^6 -> bin 7
    assert h[19] == 1.0                            # every column has degree 1
    assert abs(h[38] - 63 / 64) < 1e-15             # one non-empty row spanning columns 0..63
    assert abs(h[39] - np.sqrt(63.0)) < 1e-12       # std/mean of [64, 0 x 63] = sqrt(63)
    # empty matrix
    e = orc.features(CSR(5, 3, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0)))
    assert e[1] == 0.0 and e[2] == 1.0 and e[18] == 1.0 and np.all(e[34:] == 0.0)


def test_degree_bins_edges(orc):
    d = np.array([0, 1, 2, 3, 4, 7, 8, 2**13, 2**14 - 1, 2**14, 10**6])
    assert list(orc.degree_bin(d)) == [0, 1, 2, 2, 3, 3, 4, 14, 14, 15, 15]


# ------------------------------------------------- comparison orderings (Sec. 5.1)

def test_bfs_order_vs_scipy_breadth_first():
    """sBFS on a connected matrix is scipy's breadth-first order of the
    bipartite graph (rows 0..m-1, columns m..m+n-1) from vertex 0, whose
    neighbours it takes in ascending order; on several components each
    starts at its smallest vertex."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import breadth_first_order, connected_components
    import oracle as orc
    for A in (gen_c1(), gen_uniform_zipf(7, 3000, 9000, 50)):
        m, n = A.m, A.n
        S = sp.csr_matrix((np.ones(A.nnz), A.colidx, A.rowptr), shape=(m, n))
        G = sp.bmat([[None, S], [S.T, None]]).tocsr()
        G.sort_indices()
        ncomp, lab = connected_components(G, directed=False)
        seq = []
        for comp in range(ncomp):
            v = int(np.flatnonzero(lab == comp)[0])
            seq.append(breadth_first_order(G, v, directed=False, return_predecessors=False))
        seq = np.concatenate([seq[i] for i in np.argsort([s.min() for s in seq])])
        r, c = orc.order_bfs(A)
        assert np.array_equal(r, seq[seq < m]) and np.array_equal(c, seq[seq >= m] - m)


def test_bfs_and_rcm_hand_worked(orc):
    """Two 3 x 3 matrices worked by hand (vertices r0 r1 r2 = 0 1 2, c0 c1
    c2 = 3 4 5).

    First: r0: c1 | r1: c0 c2 | r2: c2.  Components {0, 4}, {1, 3, 5, 2}.
    BFS: 0 4 | 1 3 5 2.  RCM: component {0, 4} starts at 0; component
    {1, 2, 3, 5} at its least-degree vertex 2 (degrees 2: 1, 3: 1; 2 < 3),
    whose last level {3} does not reach further; Cuthill-McKee 0 4 | 2 5 1 3,
    reversed 3 1 5 2 4 0.

    Second: r0: c1 | r1: c0 c1 | r2: c1 c2, a path c0-r1-c1-r2-c2 with r0
    hanging from c1.  The least-degree vertex 0 has eccentricity 3 (4
    levels); from the least-degree vertex 3 of its last level {3, 5} the
    search has 5 levels, so George and Liu's search moves to 3, and from 5
    (last level of 3) it stays at 5 levels: start 3.  Cuthill-McKee 3 1 4
    0 2 5 (0 before 2: degree 1 < 2), reversed 5 2 0 4 1 3.  Starting at 0
    instead would give 5 3 2 1 4 0."""
    A = CSR(3, 3, np.array([0, 1, 3, 4]), np.array([1, 0, 2, 2], np.int32), np.ones(4))
    r, c = orc.order_bfs(A)
    assert list(r) == [0, 1, 2] and list(c) == [1, 0, 2]
    r, c = orc.order_rcm(A)
    assert list(r) == [1, 2, 0] and list(c) == [0, 2, 1]
    B = CSR(3, 3, np.array([0, 1, 3, 5]), np.array([1, 0, 1, 1, 2], np.int32), np.ones(5))
    r, c = orc.order_bfs(B)
    assert list(r) == [0, 1, 2] and list(c) == [1, 0, 2]
    r, c = orc.order_rcm(B)
    assert list(r) == [2, 0, 1] and list(c) == [2, 1, 0]


def test_rcm_recovers_a_hidden_band(orc):
    """A banded matrix (bandwidth 3) hidden by random row and column
    permutations: the sRCM orders bring every nonzero back within a few
    positions of the diagonal of the reordered matrix (the envelope
    reduction RCM exists for), while the hidden order spreads them."""
    rng = np.random.default_rng(3)
    n = 400
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(max(0, i - 3), min(n, i + 4)):
            D[i, j] = 1.0
    pr, pc = rng.permutation(n), rng.permutation(n)
    A = dense_to_csr(D[pr][:, pc])
    r, c = orc.order_rcm(A)
    assert sorted(r) == list(range(n)) and sorted(c) == list(range(n))
    orp, oci, _ = orc.permute_csr(A, r, c)
    rows = np.repeat(np.arange(n), np.diff(orp))
    assert np.max(np.abs(rows - oci)) <= 8
    rows0 = np.repeat(np.arange(n), np.diff(A.rowptr))
    assert np.max(np.abs(rows0 - A.colidx)) > 100
