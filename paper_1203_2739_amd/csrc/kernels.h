// Launchers of the HIP kernels (internal to libspx).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sched_limits.h"

namespace spx {

// Arguments of the tiled CSR kernel.  Slots are rows (plain/SB/DB) or the
// (leaf, row) pairs of a split; slot_row maps a split slot to its row.
struct SpmvArgs {
    const int32_t *slot_ptr;  // [nslots+1] nonzero offsets
    const int32_t *slot_row;  // [nslots]   split only
    const int32_t *colidx;    // padded to a multiple of 4 plus 16
    const double *vals;       // padded likewise
    const double *x;
    double *y;
    const int32_t *blk_desc;  // 4 per block: first slot, end slot, first nonzero, end nonzero
    const int32_t *tiles;     // 4 per tile: first block, end block, window lo, window len
    int32_t ntiles;
    int32_t shared_begin;     // split: rows >= this are accumulated atomically
    int32_t accumulate;       // split: add to y for rows owned by one leaf
    int32_t xcd_remap;
    int32_t n;                // columns (no gathers when 0)
};

// wg = 64 * waves per workgroup; each wave owns one tile, ntiles counts
// workgroups.
bool spmv_variant_exists(int wg, int window_entries, int *wmax_out);
hipError_t launch_spmv(const SpmvArgs &a, int wg, int window_entries, bool split, hipStream_t s);
hipError_t launch_fill(double *y, int64_t lo, int64_t hi, double v, hipStream_t s);
hipError_t launch_gather(const double *x, const int32_t *perm, double *out, int64_t n, hipStream_t s);
hipError_t launch_scatter(const double *yhat, const int32_t *perm, double *y, int64_t m, hipStream_t s);
int64_t stream_grid(int64_t bytes);
hipError_t launch_stream_read(const void *src, int64_t bytes, double *sink, hipStream_t s);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);

}  // namespace spx
