// Plan construction: canonical row/column orders of the SB, DB and split
// forms, the reordered storage, and the kernel schedule.
//
// Orders (the paper fixes the block structure of Eq. 1 and Eq. 5 but not the
// order inside a block): rows by part, then by leaf, then by original index,
// with the row border R_B last (DB).  A column touched (by part rows) from a
// single leaf goes with that leaf; one touched from several leaves of a
// single part follows that part's leaf columns; every other column -- touched
// from several parts, or from none -- forms the column border C_B at the end.
// Inside a class, columns go by the set of row groups (kXcdGroups runs of
// the stored rows with nearly equal nonzeros, one per XCD) that read them,
// then by decreasing count, then by index.
// The split orders rows the same way over the leaves of their nonzeros, with
// rows spread over several leaves after all single-leaf rows and empty rows
// last, so that the rows needing atomic accumulation form one range.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <future>
#include <numeric>

#include "spx_internal.h"

namespace spx {

// Row group of a stored row whose nonzeros start at storage offset `start`:
// the stored matrix is cut into kXcdGroups runs of nearly equal nonzeros.
static inline int32_t group_of_start(int64_t start, int64_t nnz) {
    return nnz > 0 ? (int32_t)((kXcdGroups * start) / nnz) : 0;
}

namespace {

// Stable counting sort of 0..cnt-1 by bucket.
std::vector<int32_t> counting_order(const std::vector<int32_t> &bucket, int32_t nb) {
    std::vector<int64_t> off((size_t)nb + 1, 0);
    for (int32_t b : bucket) off[b + 1]++;
    for (int32_t b = 0; b < nb; ++b) off[b + 1] += off[b];
    std::vector<int32_t> out(bucket.size());
    for (size_t i = 0; i < bucket.size(); ++i) out[off[bucket[i]]++] = (int32_t)i;
    return out;
}

template <class F>
void parallel_for(int64_t n, F f) {
    int32_t T = num_threads();
    if (n < 4096 || T <= 1) {
        f(0, n);
        return;
    }
    std::vector<std::future<void>> futs;
    int64_t chunk = (n + T - 1) / T;
    for (int32_t t = 0; t < T; ++t) {
        int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
        if (lo >= hi) break;
        futs.push_back(std::async(std::launch::async, [&f, lo, hi] { f(lo, hi); }));
    }
    for (auto &x : futs) x.get();
}

// Column classes from (row-of-nonzero labels).  leaf_of/part_of give the
// labels of every nonzero of A that counts (label < 0: ignored).
struct ColClass {
    std::vector<int32_t> first_leaf, first_part;
    std::vector<uint8_t> multi_leaf, multi_part;
};

// Columns by class (leaf, part-shared, border); inside a class by the set of
// row groups that read them (mask[j], bit g for group g, ascending as a
// number), then by decreasing number of nonzeros, then by original index.
// The kernel runs the blocks of row group g on XCD g, so a cache line of x
// then holds entries read by the same XCDs, and among those the entries
// gathered most often share lines.
std::vector<int32_t> column_order(const CsrHost &A, int32_t K, int32_t nleaves,
                                  const std::vector<int32_t> &leaf_lo_of_part,
                                  const ColClass &cc, const std::vector<uint8_t> &mask,
                                  int32_t &border_begin) {
    const int32_t n = A.n;
    std::vector<int32_t> bucket(n);
    for (int32_t j = 0; j < n; ++j) {
        int32_t p = cc.first_part[j];
        if (p < 0 || cc.multi_part[j]) bucket[j] = nleaves + K;
        else if (cc.multi_leaf[j]) bucket[j] = leaf_lo_of_part[p + 1] + p;
        else bucket[j] = cc.first_leaf[j] + p;
    }
    std::vector<int64_t> deg((size_t)n, 0);
    for (int64_t q = 0; q < A.nnz; ++q) deg[A.colidx[q]]++;
    std::vector<int32_t> by_deg(n);
    std::iota(by_deg.begin(), by_deg.end(), 0);
    std::sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) {
        if (mask[a] != mask[b]) return mask[a] < mask[b];
        if (deg[a] != deg[b]) return deg[a] > deg[b];
        return a < b;
    });
    // stable counting sort of the degree order by class
    std::vector<int64_t> off((size_t)nleaves + K + 2, 0);
    for (int32_t j = 0; j < n; ++j) off[bucket[j] + 1]++;
    for (int32_t b = 0; b <= nleaves + K; ++b) off[b + 1] += off[b];
    std::vector<int32_t> order(n);
    for (int32_t j : by_deg) order[off[bucket[j]]++] = j;
    border_begin = n;
    for (int32_t t = 0; t < n; ++t)
        if (bucket[order[t]] == nleaves + K) { border_begin = t; break; }
    return order;
}

void leaf_column_ranges(spx_plan_s &P, const std::vector<int32_t> &col_perm,
                        const ColClass &cc) {
    P.leaf_col_lo.assign(P.nleaves, 0);
    P.leaf_col_hi.assign(P.nleaves, 0);
    std::vector<uint8_t> seen(P.nleaves, 0);
    for (int32_t t = 0; t < (int32_t)col_perm.size(); ++t) {
        int32_t j = col_perm[t];
        if (cc.first_part[j] < 0 || cc.multi_part[j] || cc.multi_leaf[j]) continue;
        int32_t l = cc.first_leaf[j];
        if (!seen[l]) { seen[l] = 1; P.leaf_col_lo[l] = t; }
        P.leaf_col_hi[l] = t + 1;
    }
}

void permuted_rows(spx_plan_s &P, const CsrHost &A, const std::vector<int32_t> &inv_col) {
    int32_t m = A.m;
    P.slot_ptr.assign((size_t)m + 1, 0);
    for (int32_t i = 0; i < m; ++i) {
        int32_t r = P.row_perm[i];
        P.slot_ptr[i + 1] = P.slot_ptr[i] + (A.rowptr[r + 1] - A.rowptr[r]);
    }
    P.colidx.resize(A.nnz);
    P.vals.resize(A.nnz);
    parallel_for(m, [&](int64_t lo, int64_t hi) {
        std::vector<std::pair<int32_t, int32_t>> buf;
        for (int64_t i = lo; i < hi; ++i) {
            int32_t r = P.row_perm[i];
            buf.clear();
            for (int32_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p)
                buf.emplace_back(inv_col[A.colidx[p]], p);
            std::sort(buf.begin(), buf.end());
            int32_t o = P.slot_ptr[i];
            for (size_t t = 0; t < buf.size(); ++t) {
                P.colidx[o + t] = buf[t].first;
                P.vals[o + t] = A.vals[buf[t].second];
            }
        }
    });
}

}  // namespace

void plan_plain(spx_plan_s &P, const CsrHost &A) {
    P.form = SPX_FORM_PLAIN;
    P.K = 1;
    P.m = A.m;
    P.n = A.n;
    P.nnz = A.nnz;
    P.slot_ptr = A.rowptr;
    P.colidx = A.colidx;
    P.vals = A.vals;
    P.nleaves = 1;
    P.leaf_slot_ptr = {0, A.m};
    P.leaf_col_lo = {0};
    P.leaf_col_hi = {0};
    P.part_ptr = {0, A.m};
    P.row_border_begin = A.m;
    P.row_empty_begin = A.m;
    P.col_border_begin = A.n;
}

// A_hat = P_r A P_c for orders given by the caller (new -> old), stored in
// CSR with columns ascending inside rows; one leaf, no parts.
void plan_from_perm(spx_plan_s &P, const CsrHost &A, const int32_t *row_perm, const int32_t *col_perm) {
    auto t0 = std::chrono::steady_clock::now();
    P.form = SPX_FORM_ORDER;
    P.K = 1;
    P.m = A.m;
    P.n = A.n;
    P.nnz = A.nnz;
    P.row_perm.assign(row_perm, row_perm + A.m);
    P.col_perm.assign(col_perm, col_perm + A.n);
    std::vector<int32_t> inv_col(A.n);
    for (int32_t t = 0; t < A.n; ++t) inv_col[P.col_perm[t]] = t;
    permuted_rows(P, A, inv_col);
    P.nleaves = 1;
    P.leaf_slot_ptr = {0, A.m};
    P.leaf_col_lo = {0};
    P.leaf_col_hi = {0};
    P.part_ptr = {0, A.m};
    P.row_border_begin = A.m;
    P.row_empty_begin = A.m;
    P.col_border_begin = A.n;
    P.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void plan_from_rowparts(spx_plan_s &P, const CsrHost &A, const PartitionResult &r, bool db) {
    auto t0 = std::chrono::steady_clock::now();
    int32_t m = A.m, n = A.n, K = P.K;
    P.m = m;
    P.n = n;
    P.nnz = A.nnz;
    P.form = db ? SPX_FORM_DB : SPX_FORM_SB;
    P.part_a = r.part;
    P.part_b = r.leaf;
    P.nleaves = r.nleaves;
    int32_t L = r.nleaves;
    // leaves are numbered part-major: first leaf of every part
    std::vector<int32_t> leaf_part(L, 0);
    for (int32_t i = 0; i < m; ++i)
        if (r.part[i] < K) leaf_part[r.leaf[i]] = r.part[i];
    std::vector<int32_t> leaf_lo_of_part(K + 1, 0);
    {
        std::vector<int32_t> cnt(K + 1, 0);
        for (int32_t l = 0; l < L; ++l) cnt[leaf_part[l] + 1]++;
        for (int32_t k = 0; k < K; ++k) leaf_lo_of_part[k + 1] = leaf_lo_of_part[k] + cnt[k + 1];
    }
    // rows: by leaf (border rows last), stable
    std::vector<int32_t> rb(m);
    for (int32_t i = 0; i < m; ++i) rb[i] = (r.part[i] >= K) ? L : r.leaf[i];
    P.row_perm = counting_order(rb, L + 1);
    // columns
    ColClass cc;
    cc.first_leaf.assign(n, -1);
    cc.first_part.assign(n, -1);
    cc.multi_leaf.assign(n, 0);
    cc.multi_part.assign(n, 0);
    for (int32_t i = 0; i < m; ++i) {
        if (r.part[i] >= K) continue;
        int32_t p = r.part[i], l = r.leaf[i];
        for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
            int32_t j = A.colidx[q];
            if (cc.first_part[j] < 0) { cc.first_part[j] = p; cc.first_leaf[j] = l; }
            else {
                if (cc.first_part[j] != p) cc.multi_part[j] = 1;
                if (cc.first_leaf[j] != l) cc.multi_leaf[j] = 1;
            }
        }
    }
    // row groups of the rows in their new order (border rows included)
    std::vector<uint8_t> mask(n, 0);
    {
        int64_t run = 0;
        for (int32_t t = 0; t < m; ++t) {
            const int32_t i = P.row_perm[t];
            const uint8_t bit = (uint8_t)(1u << group_of_start(run, A.nnz));
            for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) mask[A.colidx[q]] |= bit;
            run += A.rowptr[i + 1] - A.rowptr[i];
        }
    }
    int32_t cb = n;
    P.col_perm = column_order(A, K, L, leaf_lo_of_part, cc, mask, cb);
    P.col_border_begin = cb;
    std::vector<int32_t> inv_col(n);
    for (int32_t t = 0; t < n; ++t) inv_col[P.col_perm[t]] = t;
    permuted_rows(P, A, inv_col);
    // parts and leaves in the new row order
    P.part_ptr.assign(K + 2, 0);
    for (int32_t i = 0; i < m; ++i) P.part_ptr[std::min(r.part[i], K) + 1]++;
    for (int32_t k = 0; k <= K; ++k) P.part_ptr[k + 1] += P.part_ptr[k];
    P.row_border_begin = P.part_ptr[K];
    P.row_empty_begin = m;
    P.leaf_slot_ptr.assign(L + 1, 0);
    for (int32_t i = 0; i < m; ++i)
        if (r.part[i] < K) P.leaf_slot_ptr[r.leaf[i] + 1]++;
    for (int32_t l = 0; l < L; ++l) P.leaf_slot_ptr[l + 1] += P.leaf_slot_ptr[l];
    leaf_column_ranges(P, P.col_perm, cc);
    // Theorem 1 / Theorem 2 quantities
    std::vector<int32_t> mark(n, -1);
    int64_t lam = 0, bnnz = 0;
    for (int32_t t = 0; t < m; ++t) {
        int32_t i = P.row_perm[t];
        if (r.part[i] >= K) {
            bnnz += A.rowptr[i + 1] - A.rowptr[i];
            continue;
        }
        for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
            int32_t j = A.colidx[q];
            if (mark[j] != r.part[i]) { mark[j] = r.part[i]; ++lam; }
        }
    }
    P.sum_lambda_col = lam;
    P.border_row_nnz = db ? bnnz : 0;
    P.cut = r.cut;
    P.partition_seconds = r.seconds;
    P.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void plan_from_split(spx_plan_s &P, const CsrHost &A, const PartitionResult &r) {
    auto t0 = std::chrono::steady_clock::now();
    int32_t m = A.m, n = A.n, K = P.K;
    int64_t nnz = A.nnz;
    P.m = m;
    P.n = n;
    P.nnz = nnz;
    P.form = SPX_FORM_SPLIT;
    P.part_a = r.part;
    P.part_b = r.leaf;
    P.nleaves = r.nleaves;
    int32_t L = r.nleaves;
    std::vector<int32_t> leaf_part(L, 0);
    for (int64_t p = 0; p < nnz; ++p) leaf_part[r.leaf[p]] = r.part[p];
    std::vector<int32_t> leaf_lo_of_part(K + 1, 0);
    {
        std::vector<int32_t> cnt(K + 1, 0);
        for (int32_t l = 0; l < L; ++l) cnt[leaf_part[l] + 1]++;
        for (int32_t k = 0; k < K; ++k) leaf_lo_of_part[k + 1] = leaf_lo_of_part[k] + cnt[k + 1];
    }
    // row classes
    std::vector<int32_t> rb(m);
    for (int32_t i = 0; i < m; ++i) {
        int32_t fl = -1, fp = -1;
        bool ml = false, mp = false;
        for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
            if (fl < 0) { fl = r.leaf[q]; fp = r.part[q]; }
            else {
                if (r.leaf[q] != fl) ml = true;
                if (r.part[q] != fp) mp = true;
            }
        }
        if (fl < 0) rb[i] = L + K + 1;
        else if (!ml) rb[i] = fl;
        else rb[i] = L + (mp ? K : fp);
    }
    P.row_perm = counting_order(rb, L + K + 2);
    P.row_border_begin = m;
    P.row_empty_begin = m;
    for (int32_t t = 0; t < m; ++t) {
        int32_t b = rb[P.row_perm[t]];
        if (b >= L && P.row_border_begin == m) P.row_border_begin = t;
        if (b == L + K + 1) { P.row_empty_begin = t; break; }
    }
    if (P.row_empty_begin < P.row_border_begin) P.row_border_begin = P.row_empty_begin;
    // column classes
    ColClass cc;
    cc.first_leaf.assign(n, -1);
    cc.first_part.assign(n, -1);
    cc.multi_leaf.assign(n, 0);
    cc.multi_part.assign(n, 0);
    for (int64_t q = 0; q < nnz; ++q) {
        int32_t j = A.colidx[q];
        if (cc.first_part[j] < 0) { cc.first_part[j] = r.part[q]; cc.first_leaf[j] = r.leaf[q]; }
        else {
            if (cc.first_part[j] != r.part[q]) cc.multi_part[j] = 1;
            if (cc.first_leaf[j] != r.leaf[q]) cc.multi_leaf[j] = 1;
        }
    }
    std::vector<int32_t> inv_col(n), inv_row(m);
    for (int32_t t = 0; t < m; ++t) inv_row[P.row_perm[t]] = t;
    std::vector<int32_t> row_of(nnz);
    for (int32_t i = 0; i < m; ++i)
        for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) row_of[q] = i;
    std::vector<int64_t> loff((size_t)L + 1, 0);
    for (int64_t q = 0; q < nnz; ++q) loff[r.leaf[q] + 1]++;
    for (int32_t l = 0; l < L; ++l) loff[l + 1] += loff[l];
    std::vector<int64_t> key(nnz);
    std::vector<int32_t> src(nnz);
    // stored rows (leaf, new row), leaf-major then by new row: the storage
    // offset of each stored row gives the row group of its nonzeros
    {
        std::vector<int64_t> fill(loff.begin(), loff.end() - 1);
        for (int64_t q = 0; q < nnz; ++q) {
            int64_t o = fill[r.leaf[q]]++;
            key[o] = ((int64_t)inv_row[row_of[q]] << 32) | (uint32_t)q;
            src[o] = (int32_t)q;
        }
    }
    parallel_for(L, [&](int64_t lo, int64_t hi) {
        for (int64_t l = lo; l < hi; ++l) std::sort(key.begin() + loff[l], key.begin() + loff[l + 1]);
    });
    std::vector<uint8_t> mask(n, 0);
    for (int32_t l = 0; l < L; ++l) {
        int64_t start = loff[l];
        for (int64_t o = loff[l]; o < loff[l + 1]; ++o) {
            if (o > loff[l] && (key[o] >> 32) != (key[o - 1] >> 32)) start = o;
            const int32_t q = (int32_t)(key[o] & 0xffffffff);
            mask[A.colidx[q]] |= (uint8_t)(1u << group_of_start(start, nnz));
        }
    }
    int32_t cb = n;
    P.col_perm = column_order(A, K, L, leaf_lo_of_part, cc, mask, cb);
    P.col_border_begin = cb;
    for (int32_t t = 0; t < n; ++t) inv_col[P.col_perm[t]] = t;
    // per-leaf GCSR: nonzeros grouped by leaf, then by (new row, new col)
    {
        std::vector<int64_t> fill(loff.begin(), loff.end() - 1);
        for (int64_t q = 0; q < nnz; ++q) {
            int64_t o = fill[r.leaf[q]]++;
            key[o] = ((int64_t)inv_row[row_of[q]] << 32) | (uint32_t)inv_col[A.colidx[q]];
            src[o] = (int32_t)q;
        }
    }
    parallel_for(L, [&](int64_t lo, int64_t hi) {
        std::vector<std::pair<int64_t, int32_t>> buf;
        for (int64_t l = lo; l < hi; ++l) {
            buf.clear();
            for (int64_t o = loff[l]; o < loff[l + 1]; ++o) buf.emplace_back(key[o], src[o]);
            std::sort(buf.begin(), buf.end());
            for (size_t t = 0; t < buf.size(); ++t) {
                key[loff[l] + t] = buf[t].first;
                src[loff[l] + t] = buf[t].second;
            }
        }
    });
    P.colidx.resize(nnz);
    P.vals.resize(nnz);
    P.slot_ptr.clear();
    P.slot_row.clear();
    P.leaf_slot_ptr.assign(L + 1, 0);
    for (int32_t l = 0; l < L; ++l) {
        int64_t prev = -1;
        for (int64_t o = loff[l]; o < loff[l + 1]; ++o) {
            int64_t row = key[o] >> 32;
            if (row != prev) {
                P.slot_ptr.push_back((int32_t)o);
                P.slot_row.push_back((int32_t)row);
                prev = row;
            }
            P.colidx[o] = (int32_t)(key[o] & 0xffffffff);
            P.vals[o] = A.vals[src[o]];
        }
        P.leaf_slot_ptr[l + 1] = (int32_t)P.slot_row.size();
    }
    P.slot_ptr.push_back((int32_t)nnz);
    P.part_ptr.clear();
    leaf_column_ranges(P, P.col_perm, cc);
    // Corollary 4 quantities for the K parts
    std::vector<int64_t> poff((size_t)K + 1, 0);
    for (int64_t q = 0; q < nnz; ++q) poff[r.part[q] + 1]++;
    for (int32_t k = 0; k < K; ++k) poff[k + 1] += poff[k];
    std::vector<int32_t> byp(nnz);
    {
        std::vector<int64_t> fill(poff.begin(), poff.end() - 1);
        for (int64_t q = 0; q < nnz; ++q) byp[fill[r.part[q]]++] = (int32_t)q;
    }
    std::vector<int32_t> mr(m, -1), mc(n, -1);
    int64_t lr = 0, lc = 0;
    for (int64_t t = 0; t < nnz; ++t) {
        int32_t q = byp[t], k = r.part[q];
        if (mr[row_of[q]] != k) { mr[row_of[q]] = k; ++lr; }
        if (mc[A.colidx[q]] != k) { mc[A.colidx[q]] = k; ++lc; }
    }
    P.sum_lambda_row = lr;
    P.sum_lambda_col = lc;
    P.cut = r.cut;
    P.partition_seconds = r.seconds;
    P.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ----------------------------------------------------------------- schedule

// Densest range of at most W consecutive column indices among the stored
// nonzeros [z0, z1): its first column, its length and the nonzeros it
// serves (0, 0, 0 when empty).
static void densest_window(const std::vector<int32_t> &colidx, int64_t z0, int64_t z1, int32_t W,
                           std::vector<int32_t> &buf, int32_t &lo, int32_t &len, int64_t &served) {
    lo = len = 0;
    served = 0;
    buf.assign(colidx.begin() + z0, colidx.begin() + z1);
    std::sort(buf.begin(), buf.end());
    size_t bi = 0, bj = 0, j = 0;
    for (size_t i = 0; i < buf.size(); ++i) {
        while (j < buf.size() && buf[j] < (int64_t)buf[i] + W) ++j;
        if ((int64_t)(j - i) > served) {
            served = (int64_t)(j - i);
            bi = i;
            bj = j;
        }
    }
    if (served > 0) {
        lo = buf[bi];
        len = buf[bj - 1] + 1 - lo;
    }
}

// Tiles per row group: the blocks [xb[g], xb[g+1]) of group g are cut into
// T runs of nearly equal nonzeros (fewer when the group has fewer blocks),
// each with the densest window of at most W columns among its nonzeros,
// kept when it serves at least half as many gathers as it holds entries.
static void group_tiles(spx_plan_s &P, const std::vector<int32_t> &xb, int32_t T, int32_t W) {
    P.tiles.clear();
    P.window_nnz = 0;
    P.window_bytes_fill = 0;
    auto bnz = [&](int32_t b) { return (int64_t)P.blk_desc[4 * (size_t)b + 3] - P.blk_desc[4 * (size_t)b + 2]; };
    for (int g = 0; g < kXcdGroups; ++g) {
        const int32_t b0 = xb[g], b1 = xb[g + 1];
        if (b0 >= b1) continue;
        int64_t total = 0;
        for (int32_t b = b0; b < b1; ++b) total += bnz(b);
        int64_t acc = 0;
        int32_t start = b0, t = 1;
        for (int32_t b = b0; b < b1; ++b) {
            acc += bnz(b);
            // close the tile once it reaches t/T of the group's nonzeros
            if (b + 1 < b1 && acc * T >= total * t) {
                P.tiles.insert(P.tiles.end(), {start, b + 1, 0, 0});
                start = b + 1;
                while (acc * T >= total * t) ++t;
            }
        }
        P.tiles.insert(P.tiles.end(), {start, b1, 0, 0});
    }
    if (W <= 0) return;
    const int32_t nt = (int32_t)(P.tiles.size() / 4);
    std::vector<int64_t> served(nt, 0);
    parallel_for(nt, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> buf;
        for (int64_t t = lo; t < hi; ++t) {
            int32_t *tl = &P.tiles[4 * (size_t)t];
            const int64_t z0 = P.blk_desc[4 * (size_t)tl[0] + 2], z1 = P.blk_desc[4 * (size_t)(tl[1] - 1) + 3];
            int32_t wlo, wlen;
            int64_t sv;
            densest_window(P.colidx, z0, z1, W, buf, wlo, wlen, sv);
            if (sv > 0 && 2 * sv >= (int64_t)wlen) {
                tl[2] = wlo;
                tl[3] = wlen;
                served[t] = sv;
            }
        }
    });
    for (int32_t t = 0; t < nt; ++t) {
        P.window_nnz += served[t];
        P.window_bytes_fill += 8 * (int64_t)P.tiles[4 * (size_t)t + 3];
    }
}


// Gather-sorted storage (sort_gathers): the nonzeros of every multi-row
// block sorted by column (ties by position) at a 64-aligned offset, each
// index carrying in its upper bits (from bit pack_shift(nnz_per_block)) the
// nonzero's offset in row order from the block's 4-aligned start,
// interleaved in chunks of 64 sorted entries
// (stored entry 64 k + 4 l + j holds sorted entry 64 k + 16 j + l) and the
// last chunk padded with all-ones indices and zero values.  Long-slot
// segments stay in the stored order.  Empty without sort_gathers.
static void gather_sorted_storage(spx_plan_s &P) {
    P.colidx_sorted.clear();
    P.vals_sorted.clear();
    P.sorted_ofs.clear();
    if (!P.tune.sort_gathers) return;
    const int sh = pack_shift(P.tune.nnz_per_block);
    if ((int64_t)P.n > ((int64_t)1 << sh))
        fail(SPX_EUNSUPPORTED, "sort_gathers: too many columns for the block's offsets (at most 2^(32 - "
                               "log2 nnz_per_block))");
    const int64_t nb = (int64_t)(P.blk_desc.size() / 4);
    P.sorted_ofs.assign((size_t)nb, -1);
    int64_t total = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t *d = &P.blk_desc[4 * (size_t)b];
        if (d[1] < 0) continue;
        P.sorted_ofs[(size_t)b] = (int32_t)total;
        total += (d[3] - d[2] + 63) & ~63;
    }
    if (total > INT32_MAX) fail(SPX_EUNSUPPORTED, "gather-sorted copy too large");
    P.colidx_sorted.assign((size_t)total, 0xFFFFFFFFu);
    P.vals_sorted.assign((size_t)total, 0.0);
    parallel_for(nb, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> idx;
        for (int64_t b = lo; b < hi; ++b) {
            const int32_t *d = &P.blk_desc[4 * (size_t)b];
            if (d[1] < 0) continue;
            const int32_t z0 = d[2], z1 = d[3], zb = z0 & ~3;
            const size_t so = (size_t)P.sorted_ofs[(size_t)b];
            idx.resize((size_t)(z1 - z0));
            std::iota(idx.begin(), idx.end(), z0);
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int32_t u, int32_t v) { return P.colidx[u] < P.colidx[v]; });
            for (int32_t s = 0; s < z1 - z0; ++s) {
                const int32_t src = idx[(size_t)s];
                const size_t dst = so + (size_t)(s & ~63) + 4 * (size_t)(s & 15) + (size_t)((s >> 4) & 3);
                P.colidx_sorted[dst] = (uint32_t)P.colidx[src] | ((uint32_t)(src - zb) << sh);
                P.vals_sorted[dst] = P.vals[src];
            }
        }
    });
}

// Compact indices (compact_index): every multi-row block whose columns lie
// within 65,536 of its smallest column keeps 16-bit offsets from that column
// (blk_cbase) at the stored positions of its nonzeros; other blocks keep
// blk_cbase = -1 and the 32-bit indices.  Empty otherwise.
static void compact_index_storage(spx_plan_s &P) {
    P.colidx16.clear();
    P.blk_cbase.clear();
    P.nnz_compact = 0;
    if (!P.tune.compact_index) return;
    const int64_t nb = (int64_t)(P.blk_desc.size() / 4);
    P.colidx16.assign(P.colidx.size(), 0);
    P.blk_cbase.assign((size_t)nb, -1);
    std::vector<int64_t> count((size_t)nb, 0);
    parallel_for(nb, [&](int64_t lo, int64_t hi) {
        for (int64_t b = lo; b < hi; ++b) {
            const int32_t *d = &P.blk_desc[4 * (size_t)b];
            if (d[1] < 0 || d[3] <= d[2]) continue;
            int32_t cmin = P.colidx[d[2]], cmax = cmin;
            for (int32_t z = d[2]; z < d[3]; ++z) {
                cmin = std::min(cmin, P.colidx[z]);
                cmax = std::max(cmax, P.colidx[z]);
            }
            if (cmax - cmin > 65535) continue;
            P.blk_cbase[(size_t)b] = cmin;
            for (int32_t z = d[2]; z < d[3]; ++z) P.colidx16[(size_t)z] = (uint16_t)(P.colidx[z] - cmin);
            count[(size_t)b] = d[3] - d[2];
        }
    });
    for (int64_t c : count) P.nnz_compact += c;
}

// Lanes the kernel gives to each row of a block of nr rows: the largest
// power of two <= wg / nr, at most a wave.
static int32_t lanes_per_row(int32_t wg, int32_t nr) {
    int32_t q = wg / nr, g = 1;
    while (g * 2 <= q && g < 64) g *= 2;
    return g;
}

// Row blocks and tiles.  A multi-row block holds whole consecutive slots of
// one unit (a leaf, or the rows outside all leaves) while (i) its nonzeros
// span at most nnz_per_block entries from the 4-aligned start, (ii) it has at most
// wg slots and (iii) ceil(longest / lanes_per_row) <= reduce_iters (not
// with scan_reduce, whose row sums do not depend on row lengths).  A slot
// that cannot form a block alone is a long slot: it is cut at 4-aligned
// offsets into segments of one load round each (at most nnz_per_block
// entries from the aligned start).  Descriptors are {first slot, end slot,
// first nonzero, end nonzero}; a segment of long slot number l has end slot
// -1 - l, and long_seg_ptr[l] is the first of its partial-sum entries.  A tile is a run of at least blocks_per_tile blocks
// of one unit, with an optional LDS x window.
void build_schedule(spx_plan_s &P) {
    const Tune &T = P.tune;
    const int64_t span = T.nnz_per_block;
    // the scan kernel's row sums take the same steps whatever the row lengths
    const int32_t iters = T.scan ? INT32_MAX : T.reduce_iters;
    const int32_t bt = block_threads(T);
    P.blk_slot.clear();
    P.blk_desc.clear();
    P.tiles.clear();
    P.long_seg_ptr.assign(1, 0);
    P.window_nnz = 0;
    P.window_bytes_fill = 0;
    std::vector<std::pair<int32_t, int32_t>> units;
    std::vector<int32_t> unit_leaf;
    const int32_t nslots = (int32_t)P.slot_ptr.size() - 1;
    const int64_t nnz_all = nslots > 0 ? P.slot_ptr[nslots] : 0;
    // first slot of every row group; blocks and tiles never cross a group
    std::vector<int32_t> gfirst(kXcdGroups + 1, nslots);
    gfirst[0] = 0;
    for (int g = 1; g < kXcdGroups; ++g) {
        int32_t lo = 0, hi = nslots;  // first slot whose group is >= g
        while (lo < hi) {
            int32_t mid = lo + (hi - lo) / 2;
            if (group_of_start(P.slot_ptr[mid], nnz_all) >= g) hi = mid;
            else lo = mid + 1;
        }
        gfirst[g] = lo;
    }
    auto add_unit = [&](int32_t s0, int32_t s1, int32_t leaf) {
        for (int g = 0; g < kXcdGroups && s0 < s1; ++g) {
            const int32_t cut = gfirst[g + 1];
            if (cut > s0 && cut < s1) {
                units.emplace_back(s0, cut);
                unit_leaf.push_back(leaf);
                s0 = cut;
            }
        }
        units.emplace_back(s0, s1);
        unit_leaf.push_back(leaf);
    };
    for (int32_t l = 0; l < P.nleaves; ++l) add_unit(P.leaf_slot_ptr[l], P.leaf_slot_ptr[l + 1], l);
    int32_t covered = P.nleaves ? P.leaf_slot_ptr[P.nleaves] : 0;
    if (covered < nslots) add_unit(covered, nslots, -1);
    // a slot too long for a block of its own
    auto is_long = [&](int64_t len) {
        return len > span - 3 || (len + 63) / 64 > iters;
    };
    std::vector<int32_t> cols;
    for (size_t u = 0; u < units.size(); ++u) {
        int32_t s0 = units[u].first, s1 = units[u].second;
        if (s0 >= s1) continue;
        int32_t first_blk = (int32_t)(P.blk_desc.size() / 4);
        int32_t b_slo = s0, nr = 0;
        int64_t lmax = 0;
        auto close = [&](int32_t s_hi) {
            if (nr > 0)
                P.blk_desc.insert(P.blk_desc.end(), {b_slo, s_hi, P.slot_ptr[b_slo], P.slot_ptr[s_hi]});
            b_slo = s_hi;
            nr = 0;
            lmax = 0;
        };
        for (int32_t s = s0; s < s1; ++s) {
            const int64_t ps = P.slot_ptr[s], pe = P.slot_ptr[s + 1], len = pe - ps;
            if (is_long(len)) {
                close(s);
                // segments end on 4-aligned offsets: each is one load round
                const int32_t lr = (int32_t)P.long_seg_ptr.size() - 1;
                int32_t nseg = 0;
                for (int64_t z = ps, e = (ps & ~(int64_t)3) + span; z < pe; z = e, e += span, ++nseg)
                    P.blk_desc.insert(P.blk_desc.end(), {s, -1 - lr, (int32_t)z, (int32_t)std::min<int64_t>(e, pe)});
                P.long_seg_ptr.push_back(P.long_seg_ptr.back() + nseg);
                b_slo = s + 1;
                continue;
            }
            const int64_t zb = P.slot_ptr[b_slo] & ~(int64_t)3;
            const int64_t lm = std::max(lmax, len);
            const int32_t g = lanes_per_row(bt, nr + 1);
            if (nr > 0 && (pe - zb > span || nr + 1 > bt || (lm + g - 1) / g > iters)) close(s);
            ++nr;
            lmax = std::max(lmax, len);
        }
        close(s1);
        int32_t last_blk = (int32_t)(P.blk_desc.size() / 4);
        // window of this unit
        int32_t wlo = 0, wlen = 0;
        // tiles of blocks_per_tile blocks; wave blocks default to one per wave
        int32_t B = std::max(1, T.blocks_per_tile);
        if (T.wave_blocks && T.blocks_per_tile <= 1) B = T.wg / 64;
        int32_t l = unit_leaf[u];
        if (T.window_entries > 0 && T.tiles_per_group == 0 && l >= 0 && last_blk > first_blk) {
            int64_t z0 = P.slot_ptr[s0], z1 = P.slot_ptr[s1];
            cols.assign(P.colidx.begin() + z0, P.colidx.begin() + z1);
            std::sort(cols.begin(), cols.end());
            int64_t best = 0;
            size_t bi = 0, bj = 0, j = 0;
            for (size_t i = 0; i < cols.size(); ++i) {
                while (j < cols.size() && cols[j] < (int64_t)cols[i] + T.window_entries) ++j;
                if ((int64_t)(j - i) > best) {
                    best = (int64_t)(j - i);
                    bi = i;
                    bj = j;
                }
            }
            int32_t est_tiles = std::max(1, (last_blk - first_blk + B - 1) / B);
            if (best > 0) {
                int32_t lo = cols[bi], hi = cols[bj - 1] + 1;
                // the window pays when the gathers it serves outnumber the
                // entries loaded to fill it
                if (2 * best >= (int64_t)est_tiles * (hi - lo)) {
                    wlo = lo;
                    wlen = hi - lo;
                    P.window_nnz += best;
                }
            }
        }
        for (int32_t b = first_blk; b < last_blk; b += B) {
            P.tiles.insert(P.tiles.end(), {b, std::min(b + B, last_blk), wlo, wlen});
            if (wlen > 0) P.window_bytes_fill += (int64_t)wlen * 8;
        }
    }
    int32_t nb = (int32_t)(P.blk_desc.size() / 4);
    P.blk_slot.resize((size_t)nb + 1);
    for (int32_t b = 0; b < nb; ++b) P.blk_slot[b] = P.blk_desc[4 * (size_t)b];
    P.blk_slot[nb] = nslots;
    // first block and first tile of every row group
    auto group_ptr = [&](bool by_tile, std::vector<int32_t> &ptr) {
        const int32_t nu = by_tile ? (int32_t)(P.tiles.size() / 4) : nb;
        ptr.assign(kXcdGroups + 1, nu);
        ptr[0] = 0;
        int32_t g = 0;
        for (int32_t u = 0; u < nu; ++u) {
            const int32_t b = by_tile ? P.tiles[4 * (size_t)u] : u;
            const int32_t ug = group_of_start(P.slot_ptr[P.blk_desc[4 * (size_t)b]], nnz_all);
            while (g < ug) ptr[++g] = u;
        }
    };
    group_ptr(false, P.xcd_blk_ptr);
    if (T.tiles_per_group > 0) group_tiles(P, P.xcd_blk_ptr, T.tiles_per_group, T.window_entries);
    group_ptr(true, P.xcd_tile_ptr);
    gather_sorted_storage(P);
    compact_index_storage(P);
}

}  // namespace spx
