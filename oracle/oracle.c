/*
 * CPU oracle for the SpMV hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference implementations of what the GPU
 * path computes, written from the definitions in Akbudak, Kayaaslan and
 * Aykanat, "Analyzing and enhancing OSKI for sparse matrix-vector
 * multiplication" (arXiv 1203.2739).  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library.  It shares
 * no code, header or table with the HIP library.
 *
 * Conventions: every index array is int64; values are IEEE double; every sum
 * is accumulated left to right in storage order.  Build with
 * -O2 -ffp-contract=off so that a*b+c is never fused.
 *
 * Every function returns 0 on success and a negative number on bad input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Section 2.1 (CSR scheme): y_i = sum over the stored nonzeros of row i of
 * nonzero[p] * x[colIndex[p]], p from rowStart[i] to rowStart[i+1]-1.      */
int orc_spmv(int64_t m, const int64_t *rowptr, const int64_t *colidx,
             const double *vals, const double *x, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            s = s + vals[p] * x[colidx[p]];
        y[i] = s;
    }
    return 0;
}

/* Same definition for a list of rows only (spot checks of large products),
 * also returning sum_j |a_ij x_j| for the per-entry error bound.           */
int orc_spmv_rows(int64_t nr, const int64_t *rows, const int64_t *rowptr,
                  const int64_t *colidx, const double *vals, const double *x,
                  double *y, double *absy)
{
    for (int64_t t = 0; t < nr; ++t) {
        int64_t i = rows[t];
        double s = 0.0, a = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            double v = vals[p] * x[colidx[p]];
            s = s + v;
            a = a + (v < 0 ? -v : v);
        }
        y[t] = s;
        if (absy) absy[t] = a;
    }
    return 0;
}

/* sum_j |a_ij x_j| for every row (denominator of the per-entry bound).     */
int orc_abs_rowsum(int64_t m, const int64_t *rowptr, const int64_t *colidx,
                   const double *vals, const double *x, double *out)
{
    for (int64_t i = 0; i < m; ++i) {
        double a = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            double v = vals[p] * x[colidx[p]];
            a = a + (v < 0 ? -v : v);
        }
        out[i] = a;
    }
    return 0;
}

/* Several right-hand sides: Y (m x k, row stride ldy) = A X (n x k, ldx).  */
int orc_spmm(int64_t m, const int64_t *rowptr, const int64_t *colidx,
             const double *vals, int64_t k, const double *X, int64_t ldx,
             double *Y, int64_t ldy)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < k; ++c) {
            double s = 0.0;
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                s = s + vals[p] * X[colidx[p] * ldx + c];
            Y[i * ldy + c] = s;
        }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Section 3 (reordered product): A_hat = P_r A P_c.  With permutations
 * stored new -> old, A_hat[i', j'] = A[row_perm[i'], col_perm[j']]; the
 * result is written in CSR with column indices ascending inside each row.  */
static int cmp_pair(const void *a, const void *b)
{
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    return (x[0] > y[0]) - (x[0] < y[0]);
}

int orc_permute_csr(int64_t m, int64_t n, const int64_t *rowptr,
                    const int64_t *colidx, const double *vals,
                    const int64_t *row_perm, const int64_t *col_perm,
                    int64_t *out_rowptr, int64_t *out_colidx, double *out_vals)
{
    int64_t *inv_col = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t maxdeg = 0;
    if (!inv_col) return -2;
    for (int64_t j = 0; j < n; ++j) inv_col[j] = -1;
    for (int64_t j = 0; j < n; ++j) {
        if (col_perm[j] < 0 || col_perm[j] >= n || inv_col[col_perm[j]] >= 0) {
            free(inv_col);
            return -1;
        }
        inv_col[col_perm[j]] = j;
    }
    for (int64_t i = 0; i < m; ++i) {
        int64_t d = rowptr[i + 1] - rowptr[i];
        if (d > maxdeg) maxdeg = d;
    }
    /* pairs of (new column, position of the entry in A) */
    int64_t *buf = (int64_t *)malloc(sizeof(int64_t) * 2 * (maxdeg > 0 ? maxdeg : 1));
    if (!buf) { free(inv_col); return -2; }
    out_rowptr[0] = 0;
    for (int64_t ip = 0; ip < m; ++ip) {
        int64_t i = row_perm[ip];
        if (i < 0 || i >= m) { free(buf); free(inv_col); return -1; }
        int64_t d = rowptr[i + 1] - rowptr[i];
        for (int64_t t = 0; t < d; ++t) {
            buf[2 * t] = inv_col[colidx[rowptr[i] + t]];
            buf[2 * t + 1] = rowptr[i] + t;
        }
        qsort(buf, (size_t)d, 2 * sizeof(int64_t), cmp_pair);
        int64_t o = out_rowptr[ip];
        for (int64_t t = 0; t < d; ++t) {
            out_colidx[o + t] = buf[2 * t];
            out_vals[o + t] = vals[buf[2 * t + 1]];
        }
        out_rowptr[ip + 1] = o + d;
    }
    free(buf);
    free(inv_col);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Section 4 (multiple-SpMxV framework): y <- y + A^k x for k = 1..K, the
 * products of each A^k accumulated into y on the fly.  A^k holds the stored
 * nonzeros p with nz_part[p] == k (parts numbered 0..K-1 here); each A^k is
 * traversed in CSR order.  With accumulate == 0, y starts at zero.          */
int orc_split_spmv(int64_t m, const int64_t *rowptr, const int64_t *colidx,
                   const double *vals, const int64_t *nz_part, int64_t K,
                   const double *x, double *y, int accumulate)
{
    int64_t nnz = rowptr[m];
    int64_t *cnt = (int64_t *)calloc((size_t)(K + 1), sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
    int64_t *row_of = (int64_t *)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
    if (!cnt || !order || !row_of) { free(cnt); free(order); free(row_of); return -2; }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) row_of[p] = i;
    for (int64_t p = 0; p < nnz; ++p) {
        if (nz_part[p] < 0 || nz_part[p] >= K) {
            free(cnt); free(order); free(row_of);
            return -1;
        }
        cnt[nz_part[p] + 1]++;
    }
    for (int64_t k = 0; k < K; ++k) cnt[k + 1] += cnt[k];
    for (int64_t p = 0; p < nnz; ++p) order[cnt[nz_part[p]]++] = p;  /* stable */
    if (!accumulate)
        for (int64_t i = 0; i < m; ++i) y[i] = 0.0;
    for (int64_t t = 0; t < nnz; ++t) {
        int64_t p = order[t];
        y[row_of[p]] = y[row_of[p]] + vals[p] * x[colidx[p]];
    }
    free(cnt); free(order); free(row_of);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Eq. (3): lambda(c_j) = number of row slices R_k holding a nonzero of
 * column j.  r2p[i] in [0, K) is the part of row i; any other value marks a
 * row of the row border R_B of the DB form (Eq. 5), which is left out, so
 * the same routine yields lambda'(c_j) of A'_SB.                            */
int orc_lambda_cols(int64_t m, int64_t n, const int64_t *rowptr,
                    const int64_t *colidx, const int64_t *r2p, int64_t K,
                    int64_t *lam)
{
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t *cnt = (int64_t *)calloc((size_t)(K + 1), sizeof(int64_t));
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    if (!mark || !cnt || !rows) { free(mark); free(cnt); free(rows); return -2; }
    for (int64_t j = 0; j < n; ++j) { mark[j] = -1; lam[j] = 0; }
    int64_t nin = 0;
    for (int64_t i = 0; i < m; ++i)
        if (r2p[i] >= 0 && r2p[i] < K) { cnt[r2p[i] + 1]++; nin++; }
    for (int64_t k = 0; k < K; ++k) cnt[k + 1] += cnt[k];
    for (int64_t i = 0; i < m; ++i)
        if (r2p[i] >= 0 && r2p[i] < K) rows[cnt[r2p[i]]++] = i;
    /* rows now grouped by part: count each part once per column */
    for (int64_t t = 0; t < nin; ++t) {
        int64_t i = rows[t], k = r2p[i];
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int64_t j = colidx[p];
            if (mark[j] != k) { mark[j] = k; lam[j]++; }
        }
    }
    free(mark); free(cnt); free(rows);
    return 0;
}

/* Section 4.1: lambda(r_i) and lambda(c_j) = number of parts A^k holding a
 * nonzero of row i / column j, for the splitting given by nz_part.          */
int orc_lambda_split(int64_t m, int64_t n, const int64_t *rowptr,
                     const int64_t *colidx, const int64_t *nz_part, int64_t K,
                     int64_t *lam_r, int64_t *lam_c)
{
    int64_t nnz = rowptr[m];
    int64_t *mr = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    int64_t *mc = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t *cnt = (int64_t *)calloc((size_t)(K + 1), sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
    int64_t *row_of = (int64_t *)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
    if (!mr || !mc || !cnt || !order || !row_of) {
        free(mr); free(mc); free(cnt); free(order); free(row_of);
        return -2;
    }
    for (int64_t i = 0; i < m; ++i) { mr[i] = -1; lam_r[i] = 0; }
    for (int64_t j = 0; j < n; ++j) { mc[j] = -1; lam_c[j] = 0; }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) row_of[p] = i;
    for (int64_t p = 0; p < nnz; ++p) {
        if (nz_part[p] < 0 || nz_part[p] >= K) {
            free(mr); free(mc); free(cnt); free(order); free(row_of);
            return -1;
        }
        cnt[nz_part[p] + 1]++;
    }
    for (int64_t k = 0; k < K; ++k) cnt[k + 1] += cnt[k];
    for (int64_t p = 0; p < nnz; ++p) order[cnt[nz_part[p]]++] = p;
    for (int64_t t = 0; t < nnz; ++t) {
        int64_t p = order[t], k = nz_part[p], i = row_of[p], j = colidx[p];
        if (mr[i] != k) { mr[i] = k; lam_r[i]++; }
        if (mc[j] != k) { mc[j] = k; lam_c[j]++; }
    }
    free(mr); free(mc); free(cnt); free(order); free(row_of);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Precision mode.  IEEE binary64 -> binary32 with round-to-nearest-even is
 * the C conversion under the default rounding mode.  binary32 -> bfloat16
 * keeps the upper 16 bits after rounding to nearest, ties to even.          */
int orc_to_f32(int64_t cnt, const double *in, float *out)
{
    for (int64_t t = 0; t < cnt; ++t) out[t] = (float)in[t];
    return 0;
}

int orc_f32_to_bf16(int64_t cnt, const float *in, uint16_t *out)
{
    for (int64_t t = 0; t < cnt; ++t) {
        uint32_t u;
        memcpy(&u, &in[t], 4);
        if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
            out[t] = (uint16_t)((u >> 16) | 0x0040u);   /* quiet NaN */
            continue;
        }
        uint32_t lsb = (u >> 16) & 1u;
        u = u + 0x7fffu + lsb;
        out[t] = (uint16_t)(u >> 16);
    }
    return 0;
}

static float bf16_to_f32(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* Low-precision product: quantized values (binary32, or bfloat16 when
 * vals16 is given), binary32 x, binary32 accumulation in storage order.    */
int orc_spmv_lowp(int64_t m, const int64_t *rowptr, const int64_t *colidx,
                  const float *vals32, const uint16_t *vals16, const float *x,
                  float *y)
{
    for (int64_t i = 0; i < m; ++i) {
        float s = 0.0f;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            float a = vals16 ? bf16_to_f32(vals16[p]) : vals32[p];
            s = s + a * x[colidx[p]];
        }
        y[i] = s;
    }
    return 0;
}
