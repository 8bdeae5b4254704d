// Launchers of the HIP kernels (internal to libspx).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sched_limits.h"

namespace spx {

// Arguments of the row-block kernel.  Slots are rows (plain/SB/DB) or the
// (leaf, row) pairs of a split; slot_row maps a split slot to its row.  V is
// the stored value type (double, float, or uint16_t bfloat16 bit patterns),
// A the type of x, y and the accumulation.
template <class V, class A>
struct SpmvArgsT {
    const int32_t *slot_ptr;  // [nslots+1] nonzero offsets
    const int32_t *slot_row;  // [nslots]   split only
    const int32_t *colidx;    // padded to a multiple of 4 plus 16
    const V *vals;            // padded likewise
    const A *x;
    A *y;
    const int32_t *blk_desc;  // 4 per block: first slot, end slot, first nonzero, end nonzero
    const int32_t *tiles;     // 4 per tile: first block, end block, window lo, window len
    int32_t ntiles;           // workgroups: tiles, or blocks when not tiled
    int32_t shared_begin;     // split: rows >= this are accumulated atomically
    int32_t accumulate;       // split: add to y for rows owned by one leaf
    int32_t xcd_remap;        // 1: workgroup w runs unit xcd_ptr[w % 8] + w / 8 of row group w % 8
    int32_t n;                // columns
    int32_t xcd_ptr[kXcdGroups + 1];  // first unit (tile or block) of every row group
    const int32_t *scol;          // gather-sorted copy (sort_gathers): packed indices, interleaved chunks
    const V *sval;                // its values
    const int32_t *sofs;          // its 64-aligned offset of every multi-row block
    const uint16_t *c16;          // compact_index: 16-bit offsets from cbase[block], padded like colidx
    const int32_t *cbase;         // smallest column of every block, -1 where the 32-bit indices serve
    const int32_t *long_seg_ptr;  // [nlong+1] partial-sum entries of each long slot
    double *partials;             // one per long-slot segment
    uint32_t *counters;           // one per long slot, zero between products
};
using SpmvArgs = SpmvArgsT<double, double>;

// Batched products: one matrix of the batch (device pointers).  X is n x k
// row-major with leading dimension ldx, Y m x k with ldy.
struct BatchMat {
    const int32_t *slot_ptr;
    const int32_t *colidx;
    const double *vals;
    const double *X;
    double *Y;
    int64_t ldx, ldy;
    int32_t k;                    // right-hand sides, 1..64
    int32_t span;                 // nonzeros per long-row segment (k > 1 items)
    const int32_t *long_seg_ptr;  // per long row: first partial index
    double *partials;             // k per long-row segment
    uint32_t *counters;           // per long row, zero between launches
};
struct BatchArgs {
    const BatchMat *mats;
    const int32_t *items;  // 5 per item: matrix, first slot, end slot (or -1 - long row), first nz, end nz
    int32_t nitems;
    uint32_t *queue;       // reset by launch_batch before the persistent kernel
};
constexpr int kBatchWG = 256;
// Queue reset then the persistent kernel on `grid` workgroups.
hipError_t launch_batch(const BatchArgs &b, int grid, hipStream_t s);
int batch_grid();  // workgroups that are resident at once on the device

// One workgroup of wg threads per tile (tiled) or per block (not tiled);
// ntiles counts workgroups.  npt = nonzeros staged per thread.  The kernel
// kind: Blocks, the row-block kernel (rows summed from LDS by power-of-two
// lane groups); Waves, the wave-block kernel (tiles of wave-sized blocks,
// each wave of a workgroup running its own blocks; npt is then the nonzeros
// per lane); Pipe, the pipelined-tile kernel (a workgroup per tile, the next
// block's loads issued before the current block is reduced); Scan, one
// workgroup per block with rows summed by a segmented scan over the block.
bool spmv_variant_exists(int wg, int npt, int window_entries, int *wmax_out, Kind k = Kind::Blocks);
hipError_t launch_spmv(const SpmvArgs &a, int wg, int npt, int window_entries, bool tiled, bool split,
                       hipStream_t s, Kind k = Kind::Blocks);
// Low-precision products (binary32 or bfloat16 values, binary32 x, y and
// accumulation): any kind without a window; row blocks untiled.
bool spmv_lowp_variant_exists(int wg, int npt, Kind k);
hipError_t launch_spmv_f32(const SpmvArgsT<float, float> &a, int wg, int npt, bool split, hipStream_t s,
                           Kind k = Kind::Blocks);
hipError_t launch_spmv_bf16(const SpmvArgsT<uint16_t, float> &a, int wg, int npt, bool split, hipStream_t s,
                            Kind k = Kind::Blocks);
// Precision-mode vector kernels (see spx_cg_ir).  Dot products write their
// result to *out (device) using part[dot_groups(n)] as scratch.
int dot_groups(int64_t n);
template <class T>
hipError_t launch_dot(const T *a, const T *b, int64_t n, T *part, T *out, hipStream_t s);
template <class T>
hipError_t launch_cg_start(const double *r, double inv_scale, T *rl, T *p, T *d, int64_t n, hipStream_t s);
template <class T>
hipError_t launch_cg_update(const T *rr, const T *pq, T *d, T *r, const T *p, const T *q, int64_t n, hipStream_t s);
template <class T>
hipError_t launch_cg_direction(const T *rr, const T *rr_new, T *p, const T *r, int64_t n, hipStream_t s);
template <class T>
hipError_t launch_ir_update(double *x, const T *d, double scale, int64_t n, hipStream_t s);
hipError_t launch_residual(const double *b, const double *ax, double *r, int64_t n, hipStream_t s);
hipError_t launch_to_f32(const double *x, float *out, int64_t n, hipStream_t s);
hipError_t launch_fill(double *y, int64_t lo, int64_t hi, double v, hipStream_t s);
hipError_t launch_gather(const double *x, const int32_t *perm, double *out, int64_t n, hipStream_t s);
hipError_t launch_scatter(const double *yhat, const int32_t *perm, double *y, int64_t m, hipStream_t s);
int64_t stream_grid(int64_t bytes);
hipError_t launch_stream_read(const void *src, int64_t bytes, double *sink, hipStream_t s);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);

}  // namespace spx
