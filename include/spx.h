/*
 * spx -- cache-aware sparse matrix-vector products for AMD MI355X (gfx950).
 *
 * C interface of the library.  The operations follow Akbudak, Kayaaslan and
 * Aykanat, "Analyzing and enhancing OSKI for sparse matrix-vector
 * multiplication" (arXiv 1203.2739):
 *
 *   - the CSR product y <- A x (Section 2.1, the CSR scheme);
 *   - the single-SpMxV framework: the product on A_hat = P_r A P_c in
 *     singly-bordered form (Section 3.1, Eq. 1-3) or doubly-bordered form
 *     (Section 3.2, Eq. 5), computed in reordered space, y_hat <- A_hat x_hat;
 *   - the multiple-SpMxV framework: y <- y + A^k x for k = 1..K over a
 *     nonzero-disjoint splitting A = A^1 + ... + A^K (Section 4).
 *
 * General rules
 *   - Every function returns SPX_OK (0) or a negative status; no C++
 *     exception crosses this interface.  spx_last_error() returns a
 *     thread-local message describing the last failure of the calling thread.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device allocations (for example the data_ptr() of a torch tensor on
 *     cuda:0).  Host input arrays are copied; the library never keeps them.
 *   - Index arrays are int32; a matrix may hold at most 2^31 - 64 nonzeros.
 *   - Streams are hipStream_t passed as void* (NULL = the null stream).
 *     Products are asynchronous on that stream; a launch failure is reported
 *     by the call that launches (SPX_EHIP).
 *   - Handles are immutable after creation apart from spx_plan_retune,
 *     spx_plan_add_lowp and the batch calls that change a batch.  A plan
 *     owns a little scratch memory (partial sums and arrival counters of rows
 *     too long for one block), so products of one plan must not overlap in
 *     time: order them on one stream.  Different plans run independently.
 *   - Input and output vectors of one call must not overlap.
 */
#ifndef SPX_H
#define SPX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t spx_status;

#define SPX_OK 0
#define SPX_EINVAL (-1)       /* invalid argument or malformed matrix        */
#define SPX_ENOMEM (-2)       /* host or device allocation failed            */
#define SPX_EHIP (-3)         /* a HIP runtime call failed                   */
#define SPX_ENOTCONV (-4)     /* iterative solver hit its iteration limit    */
#define SPX_EUNSUPPORTED (-5) /* the operation does not apply to this handle */
#define SPX_ENODEVICE (-6)    /* the handle has no device copy               */

typedef struct spx_mat_s *spx_mat;   /* a CSR matrix (host copy, optionally on the device) */
typedef struct spx_plan_s *spx_plan; /* a matrix in one of the forms, ready to multiply    */

/* Plan forms. */
#define SPX_FORM_PLAIN 0 /* CSR in the original order                       */
#define SPX_FORM_SB 1    /* singly-bordered block-diagonal form, Eq. 1      */
#define SPX_FORM_DB 2    /* doubly-bordered block-diagonal form, Eq. 5      */
#define SPX_FORM_SPLIT 3 /* nonzero-disjoint splitting, Section 4           */
#define SPX_FORM_ORDER 4 /* CSR in a given row and column order (sBFS, sRCM) */

/* Kernel schedule.  Any field set to 0 takes the library default.
 *   wg_size          threads per workgroup: 64, 128 (default), 256, 512 (or
 *                    1024, see tiles_per_group and scan_reduce)
 *   nnz_per_block    nonzeros one workgroup stages per block: 4 * wg_size
 *                    (default; 8 * wg_size for wg_size 64) or 8 * wg_size
 *                    (every thread loads 4 or 8 consecutive nonzeros)
 *   blocks_per_tile  least number of row blocks one workgroup processes in
 *                    sequence (default 1; a tile never crosses a leaf); the
 *                    tile's x window is loaded into LDS once per tile
 *   window_entries   largest LDS x window in binary64 entries (0 = default:
 *                    none, -1 = none); at most 16384; windows are contiguous
 *                    column ranges chosen per leaf
 *   xcd_remap        1 = map consecutive tiles to the same XCD (default),
 *                    -1 = hardware dispatch order
 *   reduce_iters     bound on the strided per-row reduction loop inside a
 *                    block, 1..64 (default 64); smaller bounds make blocks of
 *                    mixed row lengths hold fewer rows
 *   tiles_per_group  0 (default): tiles as above.  T > 0: each of the 8 row
 *                    groups (runs of the stored rows with nearly equal
 *                    nonzeros, one per XCD) is cut into T tiles of nearly
 *                    equal nonzeros across leaves, each run by one workgroup
 *                    with its own LDS x window (the densest column range of
 *                    at most window_entries among the tile's nonzeros, kept
 *                    when it serves at least half as many gathers as it
 *                    holds entries); blocks_per_tile is then ignored.  With
 *                    T near the number of workgroups resident on an XCD the
 *                    launch is persistent and each window is loaded once.
 *                    wg_size 1024 is available only in this mode with a
 *                    window (at most 15360 entries), or with wave_blocks.
 *   wave_blocks      0 (default): a row block is run by a whole workgroup.
 *                    1: blocks are sized for one 64-lane wave (at most 64
 *                    slots, nnz_per_block = 256 or 512, i.e. 4 or 8
 *                    nonzeros per lane, default 256) and each wave of a
 *                    workgroup runs the blocks of the workgroup's tile in
 *                    turn with no workgroup barrier after the window load;
 *                    wg_size 256, 512 or 1024; tiles hold blocks_per_tile
 *                    blocks (default wg_size / 64) or come from
 *                    tiles_per_group.
 *   pipeline         0 (default) or 1: workgroup blocks in tiles (given by
 *                    tiles_per_group or blocks_per_tile > 1), each
 *                    workgroup issuing the index and value loads of its
 *                    tile's next block before reducing the current one, so
 *                    that a round of loads is always in flight; not with
 *                    wave_blocks.  wg_size 256, 512 (4 or 8 nonzeros per
 *                    thread for 256, 4 for 512) or 1024 (4); windows of up
 *                    to 8192 (256 threads) or 16384 (512) entries.
 *   scan_reduce      0 (default) or 1: one workgroup per block, and the
 *                    rows of a block are summed by a segmented scan over
 *                    its products (every thread holds 4 or 8 consecutive
 *                    products; the thread holding a row's last nonzero
 *                    writes the row) instead of by lane groups per row;
 *                    blocks are then cut by nonzeros and rows only
 *                    (reduce_iters is ignored).  wg_size 128, 256, 512 or
 *                    1024 with 4 nonzeros per thread; no tiles, windows,
 *                    wave_blocks or pipeline.
 *   sort_gathers     0 (default) or 1: binary64 products from a second
 *                    device copy in which the nonzeros of every multi-row
 *                    block are sorted by column, each index carrying the
 *                    nonzero's row-order offset in its upper
 *                    ceil(log2 nnz_per_block) bits; the x gathers of a
 *                    quarter wave then read 16 consecutive columns of the
 *                    block, so lanes that hit one cache line share one
 *                    request, more often the larger the block.  wg_size
 *                    128, 256, 512 or 1024 with 4 nonzeros per thread, 256
 *                    or 512 with 8; at most 2^(32 - ceil(log2
 *                    nnz_per_block)) columns (SPX_EUNSUPPORTED otherwise);
 *                    no tiles, windows, wave_blocks or pipeline; with
 *                    scan_reduce (wg_size 256, 512 or 1024 with 4 per
 *                    thread, 256 or 512 with 8)
 *                    the products go to their row-order slots and the rows
 *                    are summed by the scan, so that blocks are cut by
 *                    nonzeros and rows only; not for the precision mode.
 *   compact_index    0 (default) or 1: a block whose columns lie within
 *                    65,536 of its smallest column reads 16-bit offsets
 *                    from that column (a second index copy, 2 bytes per
 *                    nonzero instead of 4; Sec. 2.1 compresses indices for
 *                    the same reason) and other blocks the 32-bit indices;
 *                    binary64 workgroup row blocks only (wg_size 128, 256
 *                    or 512, 4 per thread), not with the options above.
 * Only some (wg_size, nnz_per_block, window) combinations have a kernel;
 * others fail with SPX_EUNSUPPORTED.                                         */
typedef struct spx_tune_s {
    int32_t wg_size;
    int32_t nnz_per_block;
    int32_t blocks_per_tile;
    int32_t window_entries;
    int32_t xcd_remap;
    int32_t reduce_iters;
    int32_t tiles_per_group;
    int32_t wave_blocks;
    int32_t pipeline;
    int32_t scan_reduce;
    int32_t sort_gathers;
    int32_t compact_index;
} spx_tune;

/* Plan summary.  The lambda sums are the right-hand sides of Theorem 1
 * (SB: sum_j lambda(c_j)), Theorem 2 (DB: sum_j lambda'(c_j) and
 * sum over R_B of nnz(r_i)) and Corollary 4 (split: sum_i lambda(r_i) and
 * sum_j lambda(c_j)), computed for the K top-level parts.                 */
typedef struct spx_plan_info_s {
    int32_t form, K, m, n;
    int64_t nnz;
    int32_t nleaves, nblocks, ntiles, nslots;
    int32_t row_border_begin; /* DB: first row of R_B; split: first row shared by leaves */
    int32_t row_empty_begin;  /* split: first row holding no nonzero (m otherwise) */
    int32_t col_border_begin; /* SB/DB/split: first column of the column border C_B */
    int32_t wg_size, nnz_per_block, blocks_per_tile, window_entries;
    int64_t sum_lambda_col;   /* Thm 1 / Thm 2 first term / Cor 4 column term */
    int64_t sum_lambda_row;   /* Cor 4 row term (split), 0 otherwise */
    int64_t border_row_nnz;   /* Thm 2 second term (DB), 0 otherwise */
    int64_t cut_connectivity; /* sum over nets of cost * (lambda - 1) at the top level */
    int64_t bytes_matrix;     /* device bytes streamed per product: values, indices, slot tables */
    int64_t bytes_window;     /* LDS window fill bytes per product (read from x) */
    int64_t window_nnz;       /* nonzeros whose x entry is read from an LDS window */
    double partition_seconds; /* host time of the partitioner */
    double plan_seconds;      /* host time of ordering and table building */
    int32_t reduce_iters;     /* bound on the per-row reduction loop of a block */
    int32_t nlong_rows;       /* slots too long for one block, run as one-round segments */
    int32_t tiles_per_group;  /* tiles of every row group (0: tiles follow leaves) */
    int32_t wave_blocks;      /* 1: blocks sized for and run by single waves */
    int32_t pipeline;         /* 1: pipelined tiles */
    int32_t scan_reduce;      /* 1: rows summed by a segmented scan per block */
    int32_t sort_gathers;     /* 1: blocks stored sorted by column for the x gathers */
    int32_t compact_index;    /* 1: 16-bit block-local column indices where they fit */
    int64_t nnz_compact;      /* nonzeros read through 16-bit indices (compact_index) */
} spx_plan_info;

const char *spx_last_error(void);
const char *spx_version(void);

/* Number of host threads the partitioner may use (>= 1).  Results do not
 * depend on it.  With SPX_DEBUG set in the environment the partitioner
 * prints the sizes and times of its coarsening levels to stderr. */
spx_status spx_set_num_threads(int32_t nthreads);

/* ----------------------------------------------------------------------
 * Matrices (Section 2.1: CSR arrays nonzero, colIndex, rowStart).
 *
 * rowptr[m+1], colidx[nnz], vals[nnz] are host arrays.  They must satisfy
 * rowptr[0] = 0, rowptr non-decreasing, rowptr[m] = nnz, 0 <= colidx < n and
 * column indices strictly increasing inside every row; otherwise SPX_EINVAL.
 * m, n >= 0.  spx_csr_upload also copies the matrix to the current HIP
 * device on `stream` and returns after the copy completed;
 * spx_csr_create_host keeps a host copy only (its plans can be built,
 * inspected and exported, not multiplied: SPX_ENODEVICE).
 */
spx_status spx_csr_upload(int32_t m, int32_t n, int64_t nnz, const int32_t *rowptr,
                          const int32_t *colidx, const double *vals, void *stream,
                          spx_mat *out);
spx_status spx_csr_create_host(int32_t m, int32_t n, int64_t nnz, const int32_t *rowptr,
                               const int32_t *colidx, const double *vals, spx_mat *out);
/* spx_mat_destroy frees the matrix (the upload has completed by the time
 * spx_csr_upload returns); plans built from it stay valid. */
void spx_mat_destroy(spx_mat A);

/* ----------------------------------------------------------------------
 * Plans.  A plan keeps what it needs of the matrix; destroying the matrix
 * first is allowed.  `tune` may be NULL.
 *
 * spx_plan_plain: the CSR product in the original order (Section 2.1).
 *
 * spx_reorder_sb: K-way columnwise SB form (Section 3.1, Eq. 1) found by
 *   recursive bisection of the column-net hypergraph of A (rows = vertices
 *   weighted by nnz, columns = unit-cost nets, connectivity cutsize), which
 *   minimizes the bound of Theorem 1.  K >= 1.
 * spx_reorder_db: K-way DB form (Section 3.2, Eq. 5) found by recursive
 *   bisection of the row-column-net hypergraph (nonzeros = vertices; column
 *   nets of cost 1 under the connectivity metric and split when cut; row nets
 *   of cost nnz(r_i) under the cut-net metric, removed together with their
 *   vertices when cut, which sends the row to R_B), minimizing the bound of
 *   Theorem 2.
 * spx_split: nonzero-disjoint splitting into K parts (Section 4.1) by
 *   recursive bisection of the row-column-net hypergraph with the
 *   connectivity metric on row and column nets.  Corollary 4 weighs a cut
 *   row and a cut column alike; here a row net costs 32 and a column net 1,
 *   because a row shared by one more part costs a binary64 atomic add on the
 *   GPU while a shared column costs an x read that usually hits L2.
 *   Products then run as y <- y + A^k x.
 *
 *   window_bytes > 0 continues the bisection inside each part until every
 *   leaf's x subvector (split: x and y subvectors) fits window_bytes; leaves
 *   are the units whose x window is staged in LDS.  0 stops at the K parts.
 *   seed makes the randomized partitioner reproducible; the result does not
 *   depend on the thread count.
 *
 *   Outputs (caller-allocated host arrays, each may be NULL):
 *     row_perm[m], col_perm[n]: new -> old, so that
 *       A_hat[i', j'] = A[row_perm[i'], col_perm[j']],
 *       x_hat[j'] = x[col_perm[j']], y[row_perm[i']] = y_hat[i'].
 *     part_ptr: SB [K+1], DB [K+2]: first reordered row of each part; for DB
 *       part_ptr[K] .. part_ptr[K+1] is the row border R_B.
 *     nz_part[nnz] (split): part of every nonzero, in A's CSR order.
 *   Orders (the paper leaves them open): rows by part, then leaf, then
 *   original index, R_B last; columns of one leaf, then columns shared by
 *   leaves of one part, then the column border C_B; inside each of these
 *   classes by decreasing number of nonzeros, then by original index.
 *   For the split, rows touched by a single leaf come first (by leaf), rows
 *   shared by leaves follow, empty rows last.
 */
spx_status spx_plan_plain(spx_mat A, const spx_tune *tune, spx_plan *out);
spx_status spx_reorder_sb(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed,
                          int32_t *row_perm, int32_t *col_perm, int32_t *part_ptr,
                          const spx_tune *tune, spx_plan *out);
spx_status spx_reorder_db(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed,
                          int32_t *row_perm, int32_t *col_perm, int32_t *part_ptr,
                          const spx_tune *tune, spx_plan *out);
spx_status spx_split(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed,
                     int32_t *row_perm, int32_t *col_perm, int32_t *nz_part,
                     const spx_tune *tune, spx_plan *out);
/* spx_reorder_rn (sHP_RN, Section 5.1, the row-net model of Yzelman and
 * Bisseling): the columns of A are partitioned into K parts by recursive
 * bisection of the row-net hypergraph (columns are vertices weighted
 * nnz + 1, rows are nets; connectivity cutsize); a row whose columns lie in
 * one part joins that part, a row reaching several parts goes to the row
 * border R_B (the cut nets; the paper's method places them between the
 * parts, here they follow all parts).  The result has the DB block
 * structure of Eq. 5 and is stored as a DB plan: part_ptr[K+2] as for
 * spx_reorder_db.  No leaves below the K parts. */
spx_status spx_reorder_rn(spx_mat A, int32_t K, uint64_t seed, int32_t *row_perm, int32_t *col_perm,
                          int32_t *part_ptr, const spx_tune *tune, spx_plan *out);
/* spx_split_ex: spx_split with the cost of a row net of the row-column-net
 * model given relative to a column net (1..2^20).  Corollary 4 bounds the
 * misses of the split by the cut rows and cut columns alike: cost 1 is that
 * objective as written.  spx_split uses 32: on the GPU a row shared by one
 * more part costs a zeroed y entry and a binary64 atomic add, a shared
 * column one more x read that usually hits L2. */
spx_status spx_split_ex(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed, int32_t row_net_cost,
                        int32_t *row_perm, int32_t *col_perm, int32_t *nz_part, const spx_tune *tune,
                        spx_plan *out);

/* spx_plan_from_parts: the SB form (Section 3.1, Eq. 1), DB form (Section
 * 3.2, Eq. 5) or split (Section 4) for a partition given by the caller
 * instead of the library's partitioner (the leaves are the parts):
 * SB parts[m] in 0..K-1 (row i in row slice parts[i]); DB parts[m] in 0..K
 * (K = the row border R_B); split parts[nnz] in 0..K-1 (the part of each
 * nonzero, in A's CSR order).  row_perm / col_perm as for spx_reorder_sb
 * (may be NULL).  SPX_EINVAL for an index out of range. */
spx_status spx_plan_from_parts(spx_mat A, int32_t form, int32_t K, const int32_t *parts,
                               const spx_tune *tune, int32_t *row_perm, int32_t *col_perm,
                               spx_plan *out);
/* Comparison orderings of the single-SpMxV framework (Section 5.1), on the
 * bipartite graph of A (row i = vertex i, column j = vertex m + j, an edge
 * per nonzero): the visit order of the row vertices is the row order, that
 * of the column vertices the column order.  Outputs are host arrays
 * row_perm[m] and col_perm[n] (new -> old).
 * spx_order_bfs (sBFS): components in order of their smallest vertex,
 *   breadth-first from it, neighbours by increasing vertex number.
 * spx_order_rcm (sRCM): reverse Cuthill-McKee; each component (in order of
 *   its smallest vertex) starts at the pseudo-peripheral vertex of George
 *   and Liu's search begun at its least-degree vertex; neighbours by
 *   increasing degree, then number; the whole visit sequence is reversed.
 * spx_plan_from_perm: plan of form SPX_FORM_ORDER holding A_hat =
 *   A[row_perm][:, col_perm] in CSR (columns ascending in every row), run
 *   like a plain plan in the reordered space (spx_permute_x,
 *   spx_unpermute_y).  SPX_EINVAL when a permutation is not a bijection. */
spx_status spx_order_bfs(spx_mat A, int32_t *row_perm, int32_t *col_perm);
spx_status spx_order_rcm(spx_mat A, int32_t *row_perm, int32_t *col_perm);
spx_status spx_plan_from_perm(spx_mat A, const int32_t *row_perm, const int32_t *col_perm, const spx_tune *tune,
                              spx_plan *out);
/* Rebuild the kernel schedule (row blocks, tiles, windows) of a plan without
 * repartitioning.  Not thread-safe against products running on the plan. */
spx_status spx_plan_retune(spx_plan P, const spx_tune *tune);
/* spx_plan_autotune: pick the plan's schedule by measurement, as OSKI tunes
 * its kernel to the matrix by timing it (Section 5.2).  Every candidate
 * schedule of the library (spx_autotune_candidate) is installed in turn and
 * timed over `reps` products (after two warm-up products) of x into y on
 * `stream` with HIP events.  precision SPX_PREC_F64: binary64 products, x
 * and y binary64 device vectors of n and m entries (a split product
 * includes zeroing its shared rows, accumulate = 0).  SPX_PREC_F32 /
 * SPX_PREC_BF16: the low-precision product of spx_spmv_lowp on binary32
 * vectors, over the candidates without tiles (spx_plan_add_lowp first).
 * The plan keeps the fastest schedule; *chosen (may be NULL) receives it
 * and *ms (may be NULL) its mean milliseconds per product; cand_ms (host,
 * one entry per candidate, may be NULL) receives every candidate's mean
 * milliseconds (-1 for candidates the precision does not run).  y is
 * overwritten.  Synchronizes the device between candidates; not
 * thread-safe against other products on the plan.  SPX_ENODEVICE for a
 * host-only plan, SPX_EINVAL for reps < 1 or a NULL vector. */
/* spx_autotune_candidate: the number of candidate schedules of
 * spx_plan_autotune; when 0 <= i < that number and out is not NULL, *out
 * receives candidate i (in the order they are tried). */
int32_t spx_autotune_candidate(int32_t i, spx_tune *out);
spx_status spx_plan_autotune(spx_plan P, int32_t precision, const void *x, void *y, int32_t reps,
                             spx_tune *chosen, float *ms, float *cand_ms, void *stream);
/* spx_plan_destroy frees the plan's host and device memory.  Work queued
 * on a stream that reads the plan (products, permutations, batches built on
 * it) must have completed first: synchronize that stream before destroying. */
void spx_plan_destroy(spx_plan P);
spx_status spx_plan_info_get(spx_plan P, spx_plan_info *info);

/* ----------------------------------------------------------------------
 * Products (device vectors, binary64).
 *
 * spx_spmv: y <- A x for the plain form; y_hat <- A_hat x_hat in reordered
 *   space for SB/DB (Section 3); for a split plan the same as
 *   spx_spmv_split with accumulate = 0.  x has n entries, y has m.
 * spx_spmv_split: y <- y + A^k x for k = 1..K (Section 4) in the split's
 *   reordered space.  accumulate = 0: y starts at zero (the call zeroes the
 *   rows shared by several leaves and the rows without nonzeros, then stores
 *   the rows owned by one leaf and adds the per-leaf sums of shared rows
 *   with binary64 atomics); accumulate = 1: the products are added to the
 *   incoming y; accumulate = 2: as 0, but the caller has already zeroed the
 *   rows [row_border_begin, m) (spx_split_prepare_y), so only the product
 *   kernel runs.  The atomic adds make the rounding of shared rows vary from
 *   run to run within the error bound of reordered summation.
 * spx_split_prepare_y: y[i] = 0 for the rows i >= row_border_begin.
 * Products of one plan use the plan's scratch memory (partial sums and
 * arrival counters of rows too long for one block): products of the same
 * plan must not overlap in time; order them on one stream.
 * spx_permute_x: x_hat[j'] = x[col_perm[j']] (Section 3).
 * spx_unpermute_y: y[row_perm[i']] = y_hat[i'].
 *   Both return SPX_EUNSUPPORTED for the plain form.
 */
spx_status spx_spmv(spx_plan P, const double *x, double *y, void *stream);
spx_status spx_spmv_split(spx_plan P, const double *x, double *y, int32_t accumulate,
                          void *stream);
spx_status spx_split_prepare_y(spx_plan P, double *y, void *stream);
spx_status spx_permute_x(spx_plan P, const double *x, double *x_hat, void *stream);
spx_status spx_unpermute_y(spx_plan P, const double *y_hat, double *y, void *stream);

/* ----------------------------------------------------------------------
 * Precision mode.  Not part of the paper, whose products are binary64
 * throughout: values are stored in binary32 or bfloat16, indices stay
 * int32, x, y and the accumulation are binary32.  A conjugate-gradient solve
 * on that product is wrapped in binary64 iterative refinement, in which only
 * the residual r = b - A x (with the binary64 values) and the update
 * x <- x + d are binary64.
 *
 * spx_plan_add_lowp: rounds the plan's stored values to binary32 (nearest,
 *   ties to even) and, for SPX_PREC_BF16, the binary32 values further to
 *   bfloat16 (nearest, ties to even, NaN kept quiet); keeps a host copy and,
 *   for a device plan, a device copy.  Plain, SB and DB plans only
 *   (SPX_EUNSUPPORTED for a split).
 * spx_plan_export_lowp: the rounded values (float[nnz] or uint16_t[nnz]
 *   bfloat16 bit patterns) in the plan's storage order.
 * spx_spmv_lowp: y <- A_low x with binary32 device vectors x[n], y[m], in the
 *   plan's (reordered) space; schedules without an LDS window, row blocks
 *   untiled, not gather-sorted (SPX_EUNSUPPORTED otherwise).  Each row is summed in
 *   binary32 in a tree order, so against the exact sum of the rounded
 *   products a row of length m_i errs by at most about m_i 2^-24 times
 *   sum_j |a_ij x_j|.
 * spx_cg_ir: solves A x = b for a symmetric positive definite matrix in a
 *   plain plan (SPX_EUNSUPPORTED for other forms, whose row and column
 *   permutations differ); b, x are device binary64 vectors.  x <- 0, r <- b; while
 *   ||r|| / ||b|| > tol and fewer than max_outer refinements: run CG in the
 *   given precision on A_low d = r / ||r|| to relative residual inner_tol
 *   (at most max_inner iterations), x <- x + ||r|| d, r <- b - A x.
 *   The host reads the inner residual every 8 iterations, so an inner
 *   solve may take up to 7 iterations past the first that meets inner_tol.
 *   SPX_PREC_F64 runs the inner CG in binary64 with the binary64 product
 *   under any schedule; the other precisions need a schedule that
 *   spx_spmv_lowp runs.
 *   Returns SPX_ENOTCONV (with stats filled and x the last iterate) if the
 *   tolerance was not reached.  Allocates its workspace on every call.
 */
#define SPX_PREC_F64 0
#define SPX_PREC_F32 1
#define SPX_PREC_BF16 2

typedef struct spx_cg_stats_s {
    int32_t outer;        /* refinement steps                          */
    int32_t inner;        /* CG iterations over all refinement steps    */
    double rel_residual;  /* final ||b - A x|| / ||b||, binary64        */
    double seconds;       /* wall time of the solve                     */
} spx_cg_stats;

spx_status spx_plan_add_lowp(spx_plan P, int32_t precision);
spx_status spx_plan_export_lowp(spx_plan P, int32_t precision, void *vals);
spx_status spx_spmv_lowp(spx_plan P, int32_t precision, const float *x, float *y, void *stream);
spx_status spx_cg_ir(spx_plan P, int32_t precision, const double *b, double *x, double tol,
                     double inner_tol, int32_t max_outer, int32_t max_inner, spx_cg_stats *stats,
                     void *stream);

/* ----------------------------------------------------------------------
 * Batched products.  Not part of the paper: Y_i = A_i X_i for many plain, SB
 * or DB plans at once, X_i n_i x k_i and Y_i m_i x k_i row-major binary64
 * device arrays (leading dimensions ldx[i] >= k_i, ldy[i] >= k_i; k_i = 1
 * needs unit strides), 1 <= k_i <= 64.  One persistent launch runs every
 * block of every matrix: workgroups take items from a queue (reset by a
 * kernel, so the launch can be captured in a HIP graph and replayed).  Each
 * entry of Y is a sum over its row's nonzeros in a fixed tree order, so the
 * binary64 bound of spx_spmv applies per column.
 *
 * spx_batch_create: the batch over count plans with nrhs[i] right-hand
 *   sides; the plans must outlive the batch.
 * spx_batch_bind: the device arrays X[i], Y[i] and their leading dimensions
 *   (copied; rebinding drops a captured graph).
 * spx_batch_run: one launch on the stream.  Runs of one batch must not
 *   overlap in time (they share the queue and the long-row scratch).
 * spx_batch_capture / spx_batch_replay: capture one run in a HIP graph on
 *   the batch's own stream, then launch the graph on any stream.
 * spx_batch_autotune: times every schedule candidate (item order, block
 *   capacity divisor for several right-hand sides, reduction bound for one)
 *   on the bound arrays, `reps` runs each, keeps the fastest and reports it.
 *   It overwrites Y.
 * spx_batch_configure: sets a schedule explicitly.
 * spx_spmv_batched: create, bind, run, wait and destroy in one call.
 */
typedef struct spx_batch_s *spx_batch;

typedef struct spx_batch_config_s {
    int32_t order;        /* 0: matrices by decreasing work; 1: all blocks by decreasing work */
    int32_t span_div;     /* k > 1: item capacity max(64, 4096 / span_div) nonzeros, 1..64    */
    int32_t reduce_iters; /* k = 1: per-row reduction loop bound, 1..64                        */
    float ms;             /* autotune: mean time of one run of the chosen schedule             */
} spx_batch_config;

spx_status spx_batch_create(int32_t count, const spx_plan *plans, const int32_t *nrhs, spx_batch *out);
/* spx_batch_destroy frees the batch, its work queue and its captured graph;
 * as for plans, runs and replays queued on a stream must have completed. */
void spx_batch_destroy(spx_batch B);
spx_status spx_batch_bind(spx_batch B, const double *const *X, const int64_t *ldx, double *const *Y,
                          const int64_t *ldy);
spx_status spx_batch_run(spx_batch B, void *stream);
spx_status spx_batch_capture(spx_batch B);
spx_status spx_batch_replay(spx_batch B, void *stream);
spx_status spx_batch_autotune(spx_batch B, int32_t reps, spx_batch_config *best, void *stream);
spx_status spx_batch_configure(spx_batch B, const spx_batch_config *cfg);
spx_status spx_batch_info(spx_batch B, int32_t *nitems, int64_t *bytes, int32_t *grid);
spx_status spx_spmv_batched(int32_t count, const spx_plan *plans, const int32_t *nrhs,
                            const double *const *X, const int64_t *ldx, double *const *Y,
                            const int64_t *ldy, void *stream);

/* ----------------------------------------------------------------------
 * Learned selector.  Not part of the paper, which picks the form by
 * measurement: a 40 -> 64 -> 64 -> 24 perceptron (ReLU hidden layers,
 * softmax over 24 choices of form, K and schedule) predicts the fastest
 * choice from 40 matrix features.
 *
 * spx_features: out[40] (host) for a matrix: log1p(n), log1p(nnz), the
 *   fractions of rows (out[2..17]) and of columns (out[18..33]) whose degree
 *   falls in bin 0 (degree 0) or bin b = floor(log2 d) + 1 (capped at 15),
 *   and, with u = |i/m - j/n| over the nonzeros: mean u, max u, the fraction
 *   with u <= 1/64, the fraction inside the diagonal blocks of an 8 x 8 grid
 *   (floor(8i/m) = floor(8j/n)), the mean over non-empty rows of (last
 *   column - first column)/n, and std/mean of the row degrees.
 * spx_mlp_forward: logits[B x 24] for features X[B x 40] (device, binary32,
 *   row-major); theta[8344] holds W1 (64 x 40), b1, W2 (64 x 64), b2,
 *   W3 (24 x 64), b3, each row-major, in that order.
 * spx_mlp_loss_grad: mean softmax cross-entropy of labels[B] (device int32
 *   in 0..23) into *loss and its gradient into grad[8344] (device).  The
 *   labels are device memory and are not checked on the host: a label
 *   outside 0..23 reads no memory and turns the loss and the gradient NaN.
 * spx_mlp_adam: one Adam step (Kingma and Ba) on theta with moments m, v
 *   (device, 8344 each), step number t >= 1.
 * The network calls keep a per-thread device workspace sized for the
 * largest B seen.
 */
#define SPX_NFEATURES 40
#define SPX_NCHOICES 24
#define SPX_MLP_PARAMS 8344

spx_status spx_features(spx_mat A, float *out);
spx_status spx_mlp_forward(const float *theta, const float *X, int32_t B, float *logits, void *stream);
spx_status spx_mlp_loss_grad(const float *theta, const float *X, const int32_t *labels, int32_t B,
                             float *loss, float *grad, void *stream);
spx_status spx_mlp_adam(float *theta, const float *grad, float *m, float *v, int32_t t, float lr,
                        float beta1, float beta2, float eps, void *stream);
/* spx_mlp_loss_grad_noalloc: spx_mlp_loss_grad for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training or
 * serving loops, harnesses that forbid hipMalloc): the same kernels, with
 * their workspace in a fixed device array of the library instead of an
 * allocation, so the call allocates nothing.  B must be in 1..512
 * (SPX_EINVAL otherwise).  Every GPU holds its own copy of the array until
 * the process ends, and every call on a GPU shares it: calls that overlap
 * on one GPU (different streams or threads) race.  Nothing in the
 * workspace needs to start at zero. */
spx_status spx_mlp_loss_grad_noalloc(const float *theta, const float *X, const int32_t *labels, int32_t B,
                                     float *loss, float *grad, void *stream);

/* Selection among the 24 choices (the paper picks the ordering by measuring
 * it, Section 5.2; here a trained network picks and measurement is the
 * fallback).  Choice c < 6: plain CSR with schedule c (workgroup 128, 64,
 * 256, 128 with 8 nonzeros per thread, 128 with reduce_iters 16, 512);
 * 6 <= c < 24: form SB, DB, split for (c - 6) / 6 = 0, 1, 2 at
 * K = 8, 16, 32, 64, 128, 256 for (c - 6) % 6, default schedule.  The K-way
 * partitions of one form all come from one K = 256 recursive bisection of
 * that form's model (seed `seed`): part p of it lies in part
 * p >> (8 - log2 K), the DB row border stays the border.
 *
 * spx_choice_info: form (SPX_FORM_*), K and schedule of choice c (any
 *   output may be NULL); SPX_EINVAL outside 0..23.
 * spx_select: the choice the network picks for A: the 40 features of
 *   spx_features, each mapped to (log1p(max(f, 0)) - mu[t]) / sd[t] (mu, sd:
 *   host, 40 binary64 each, the training set's statistics), the network
 *   forward with theta (device, 8344 binary32) on `stream`, and the largest
 *   logit (first on ties) into *choice; logits (host, 24, may be NULL)
 *   receives the logits.  Synchronizes `stream`.
 * spx_select_features: the same from features f (host, 40) already
 *   computed by spx_features.
 * spx_plan_for_choice: the plan of choice c for A (partitioning at K = 256
 *   and coarsening for the reordered forms); row_perm[m] / col_perm[n]
 *   (host, may be NULL) receive its permutations (identity for plain).
 * spx_select_exhaustive: the fallback and the yardstick of the network's
 *   regret: every choice is built and timed over `reps` products (two
 *   warm-up products first) of x (device, n binary64) into y (device, m,
 *   overwritten; split products include zeroing their shared rows) on
 *   `stream`; the reordered forms multiply x permuted by their column
 *   order.  ms (host, 24, may be NULL) receives the milliseconds per
 *   product of every choice, *choice the fastest, *partition_seconds (may
 *   be NULL) the host time of the three K = 256 partitions.  SPX_ENODEVICE
 *   for a host-only matrix.
 * spx_partition_tree: the K = 256 recursive bisection that the reordered
 *   choices of `form` (SPX_FORM_SB, _DB or _SPLIT) are cut from (the
 *   column-net model, Sec. 3.1; the enhanced row-column-net model, Sec. 3.2;
 *   the row-column-net model, Sec. 4.1), on the host, also for host-only
 *   matrices: parts (host) receives r2p[m] in 0..255 (SB), r2p[m] in 0..256
 *   with 256 for R_B (DB), or nz_part[nnz] in 0..255 in A's CSR order
 *   (split); *seconds (may be NULL) its host time.
 * spx_select_exhaustive_trees: spx_select_exhaustive with the three trees
 *   given (as spx_partition_tree returns them for the same A), so that the
 *   partitioning can run apart from the timing; values out of range fail
 *   with SPX_EINVAL. */
spx_status spx_choice_info(int32_t choice, int32_t *form, int32_t *K, spx_tune *tune);
spx_status spx_select(spx_mat A, const float *theta, const double *mu, const double *sd, int32_t *choice,
                      float *logits, void *stream);
spx_status spx_select_features(const float *f, const float *theta, const double *mu, const double *sd,
                               int32_t *choice, float *logits, void *stream);
spx_status spx_plan_for_choice(spx_mat A, int32_t choice, uint64_t seed, int32_t *row_perm, int32_t *col_perm,
                               spx_plan *out);
spx_status spx_select_exhaustive(spx_mat A, const double *x, double *y, int32_t reps, uint64_t seed, float *ms,
                                 int32_t *choice, double *partition_seconds, void *stream);
spx_status spx_partition_tree(spx_mat A, int32_t form, uint64_t seed, int32_t *parts, double *seconds);
spx_status spx_select_exhaustive_trees(spx_mat A, const int32_t *tree_sb, const int32_t *tree_db,
                                       const int32_t *tree_split, const double *x, double *y, int32_t reps,
                                       float *ms, int32_t *choice, void *stream);

/* ----------------------------------------------------------------------
 * Inspection (host arrays, caller-allocated; any pointer may be NULL).
 *
 * spx_plan_export_csr: the stored matrix of a plain/SB/DB plan in CSR:
 *   rowptr[m+1], colidx[nnz], vals[nnz] (A itself for plain, A_hat else);
 *   SPX_EUNSUPPORTED for a split plan.
 * spx_plan_export_split: the per-leaf GCSR storage of a split plan in
 *   reordered coordinates (GCSR = CSR plus the list of non-empty rows,
 *   Section 5.2): leaf_slot_ptr[nleaves+1], slot_row[nslots],
 *   slot_ptr[nslots+1], colidx[nnz], vals[nnz]; SPX_EUNSUPPORTED for the
 *   other forms.
 * spx_plan_export_parts: the partition itself.  SB/DB: r2p[m] (part of each
 *   original row, K for R_B) and r2leaf[m] (leaf, -1 for R_B).  Split:
 *   nz_part[nnz] and nz_leaf[nnz] in A's CSR order.
 * spx_plan_export_perm: row_perm[m], col_perm[n] (identity for plain).
 * spx_plan_export_sched: blk_desc[4*nblocks] = {first slot starting in the
 *   block, end of those slots, first nonzero, end nonzero} per row block (a
 *   row may continue from one block into the next of the same tile) and
 *   tiles[4*ntiles] = {first block, end block, window first column, window
 *   length} per tile.
 * spx_plan_export_gather_order: the gather-sorted copy of a plan tuned with
 *   sort_gathers: *len entries in all, ofs[nblocks] (offset of every
 *   multi-row block, -1 for long-slot segments), colidx[len] (column |
 *   row-order offset << (32 - ceil(log2 nnz_per_block)), all ones for
 *   padding: chunk k of a block holds
 *   sorted entry 64 k + 16 j + l at 64 k + 4 l + j) and vals[len];
 *   SPX_EUNSUPPORTED for other schedules.
 * spx_plan_export_compact: the 16-bit indices of a plan tuned with
 *   compact_index, colidx16[nnz] at the stored positions (offsets from the
 *   block's cbase; zero where a block keeps 32-bit indices) and
 *   cbase[nblocks] (-1 for such blocks and long-slot segments);
 *   SPX_EUNSUPPORTED for other schedules.
 */
spx_status spx_plan_export_csr(spx_plan P, int32_t *rowptr, int32_t *colidx, double *vals);
spx_status spx_plan_export_split(spx_plan P, int32_t *leaf_slot_ptr, int32_t *slot_row,
                                 int32_t *slot_ptr, int32_t *colidx, double *vals);
spx_status spx_plan_export_parts(spx_plan P, int32_t *a, int32_t *b);
spx_status spx_plan_export_perm(spx_plan P, int32_t *row_perm, int32_t *col_perm);
spx_status spx_plan_export_sched(spx_plan P, int32_t *blk_desc, int32_t *tiles);
spx_status spx_plan_export_gather_order(spx_plan P, int64_t *len, int32_t *ofs, uint32_t *colidx, double *vals);
spx_status spx_plan_export_compact(spx_plan P, uint16_t *colidx16, int32_t *cbase);

/* ----------------------------------------------------------------------
 * Measurement helpers.
 *
 * spx_stream_read: reads `bytes` bytes of device memory at `src` with 16-byte
 *   streaming loads and writes one binary64 per workgroup to `sink`
 *   (sink holds at least spx_stream_sink_len(bytes) entries); the achieved
 *   bandwidth of this kernel is the read ceiling the SpMV kernels are
 *   compared with.  bytes must be a multiple of 16.
 * spx_stream_copy: dst <- src, `bytes` a multiple of 16 (a plain copy of
 *   known size, used to calibrate memory-traffic counters).
 */
int64_t spx_stream_sink_len(int64_t bytes);
spx_status spx_stream_read(const void *src, int64_t bytes, double *sink, void *stream);
spx_status spx_stream_copy(const void *src, void *dst, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPX_H */
