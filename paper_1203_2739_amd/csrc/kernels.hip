// HIP kernels of libspx for gfx950 (CDNA4, wave64).
//
// The SpMV is bound by HBM streaming of the matrix (12 bytes per binary64
// nonzero against 2 flops), so the kernels are organised around memory:
//
//  * A workgroup processes a tile: a run of row blocks of one leaf.  A row
//    block is a range of consecutive slots (rows, or the non-empty rows of a
//    split leaf) whose nonzeros fit the staging buffer.
//  * Phase 1 streams the block's column indices and values with 16-byte
//    non-temporal loads starting at a 4-aligned nonzero (every lane fetches
//    4 consecutive nonzeros per load triple), gathers x -- from the tile's
//    LDS window when the column falls inside it, else through L2 -- and
//    stores the products in LDS.
//  * Phase 2 reduces the products row by row: each row gets a power-of-two
//    group of lanes (the block's thread count divided by its row count,
//    capped at a wave) that sum strided products and combine them with DPP
//    (lane distance 1, 2), ds_swizzle (4, 8, 16) and a cross-half permute (32).
//  * A block made of a single slot (a long row) is reduced by the whole
//    workgroup: every lane accumulates in registers, then waves combine in
//    LDS.
//  * Tiles are assigned to XCDs in contiguous chunks: the hardware hands out
//    workgroups to the 8 XCDs round robin, so workgroup b runs tile
//    start(b mod 8) + b div 8.  The tiles of a part then run on one XCD and
//    its x entries stay in that XCD's L2, the GPU counterpart of a part that
//    "fits into the cache" (Section 3, Theorem 1).
//  * Split products (y <- y + A^k x, Section 4) store rows owned by a single
//    leaf directly and add rows shared by several leaves with binary64
//    atomics after the shared range was zeroed.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace spx {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

namespace {

__device__ __forceinline__ double xor_lanes(double v, int off) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    switch (off) {
    case 1:
        lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
        break;
    case 2:
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
        break;
    case 4:
        lo = __builtin_amdgcn_ds_swizzle(lo, 0x101F);
        hi = __builtin_amdgcn_ds_swizzle(hi, 0x101F);
        break;
    case 8:
        lo = __builtin_amdgcn_ds_swizzle(lo, 0x201F);
        hi = __builtin_amdgcn_ds_swizzle(hi, 0x201F);
        break;
    case 16:
        lo = __builtin_amdgcn_ds_swizzle(lo, 0x401F);
        hi = __builtin_amdgcn_ds_swizzle(hi, 0x401F);
        break;
    default: {
        int src = ((int)(threadIdx.x & 63) ^ 32) << 2;
        lo = __builtin_amdgcn_ds_bpermute(src, lo);
        hi = __builtin_amdgcn_ds_bpermute(src, hi);
    }
    }
    return __hiloint2double(hi, lo);
}

// Sum over aligned groups of g lanes (g a power of two, at most 64); every
// lane of the group receives the total.  Must be reached by the whole wave.
__device__ __forceinline__ double group_sum(double v, int g) {
    for (int off = 1; off < g; off <<= 1) v += xor_lanes(v, off);
    return v;
}

__device__ __forceinline__ int remap_tile(int bid, int ntiles, int on) {
    if (!on) return bid;
    int x = bid & 7, i = bid >> 3;
    int per = ntiles >> 3, rem = ntiles & 7;
    return x * per + (x < rem ? x : rem) + i;
}

template <bool SPLIT>
__device__ __forceinline__ void store_row(double *__restrict__ y, const int32_t *__restrict__ slot_row,
                                          int32_t slot, double v, int32_t shared_begin,
                                          int32_t accumulate) {
    if (SPLIT) {
        int32_t row = slot_row[slot];
        if (row >= shared_begin) {
            unsafeAtomicAdd(&y[row], v);
        } else {
            y[row] = accumulate ? y[row] + v : v;
        }
    } else {
        y[slot] = v;
    }
}

template <int WMAX>
__device__ __forceinline__ double xval(const double *__restrict__ x, const double *sw, int32_t c,
                                       int32_t wlo, int32_t wlen) {
    if (WMAX > 0) {
        uint32_t o = (uint32_t)(c - wlo);
        if (o < (uint32_t)wlen) return sw[o];
    }
    return x[c];
}

}  // namespace

// ---------------------------------------------------------------------------
// Wave-level SpMV.  Every wave owns a tile: a run of chunks of at most 253
// nonzeros (loads start at a 4-aligned nonzero, so a chunk spans at most
// 256 = 4 per lane) in which at most 256 rows start.  A row may continue
// from one chunk into the next of the same tile; its partial sum is carried
// in scalar registers.  Waves never wait for each other: the only workgroup
// barrier follows the load of the group's shared LDS x window.

constexpr int kRowPtrPerLane = (kChunkRows + 1 + 63) / 64;

struct Stage {
    int32_t s_lo, s_hi, z_lo, z_hi;
    v4i cc;
    v2d va, vb;
    int32_t rp[kRowPtrPerLane];
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Every load is issued unconditionally (out-of-range lanes read a clamped,
// valid address; their values are masked later), so the number of loads in
// flight is known at compile time and waiting for the oldest ones does not
// drain the younger prefetches.
__device__ __forceinline__ void issue_chunk(const SpmvArgs &a, v4i d, int lane, Stage &st) {
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.colidx);
    const v2d *__restrict__ v2 = reinterpret_cast<const v2d *>(a.vals);
    // the descriptor is uniform across the wave: keep it in scalar registers
    st.s_lo = __builtin_amdgcn_readfirstlane(d.x);
    st.s_hi = __builtin_amdgcn_readfirstlane(d.y);
    st.z_lo = __builtin_amdgcn_readfirstlane(d.z);
    st.z_hi = __builtin_amdgcn_readfirstlane(d.w);
    const int32_t nr = st.s_hi - st.s_lo;
    const int32_t zb = st.z_lo & ~3;
    const int32_t G = (st.z_hi - zb + 3) >> 2;
    const int32_t g = min(lane, G > 0 ? G - 1 : 0);
    st.cc = __builtin_nontemporal_load(&c4[(zb >> 2) + g]);
    st.va = __builtin_nontemporal_load(&v2[(zb >> 1) + 2 * g]);
    st.vb = __builtin_nontemporal_load(&v2[(zb >> 1) + 2 * g + 1]);
#pragma unroll
    for (int k = 0; k < kRowPtrPerLane; ++k) st.rp[k] = a.slot_ptr[st.s_lo + min(lane + 64 * k, nr)];
}

// Wave-private LDS.
struct WaveSmem {
    uint32_t flag[8];             // row-start bits of the 256 staged nonzeros
    int32_t row[256];             // slot id at each row start
    int32_t ptr[64 * kRowPtrPerLane];
};

// One chunk.  Gathers of x for the staged nonzeros are issued first, then
// the loads of the next chunk, so both latencies overlap.  Lane t holds the
// products of nonzeros 4t .. 4t+3.  Rows starting in the chunk are marked in
// LDS; a lane finishes the rows lying inside it and keeps the sum before its
// first row start (head) and of its last open row (tail); a segmented scan
// over the 64 lanes finishes the rows spanning lanes; the row still open at
// the end of the chunk is carried to the next chunk (cv, cr).
template <bool SPLIT, int WMAX>
__device__ __forceinline__ void run_chunk(const SpmvArgs &a, v4i dn, int lane, Stage &cur,
                                          Stage &nxt, WaveSmem &ws, const double *swin,
                                          int32_t wlo, int32_t wlen, double &cv, int32_t &cr) {
    const double *__restrict__ x = a.x;
    const int32_t s_lo = cur.s_lo, z_lo = cur.z_lo, z_hi = cur.z_hi;
    const int32_t nr = cur.s_hi - s_lo;
    const int32_t zb = z_lo & ~3;

    double xv[4];
    if (a.n > 0) {
        xv[0] = xval<WMAX>(x, swin, cur.cc.x, wlo, wlen);
        xv[1] = xval<WMAX>(x, swin, cur.cc.y, wlo, wlen);
        xv[2] = xval<WMAX>(x, swin, cur.cc.z, wlo, wlen);
        xv[3] = xval<WMAX>(x, swin, cur.cc.w, wlo, wlen);
    } else {
        xv[0] = xv[1] = xv[2] = xv[3] = 0.0;
    }
    issue_chunk(a, dn, lane, nxt);

#pragma unroll
    for (int k = 0; k < kRowPtrPerLane; ++k) {
        int32_t i = lane + 64 * k;
        if (i <= nr) ws.ptr[i] = cur.rp[k] - zb;
    }
    if (lane < 8) ws.flag[lane] = 0u;
    const int32_t z = zb + 4 * lane;
    double p[4];
    p[0] = (z + 0 >= z_lo && z + 0 < z_hi) ? cur.va.x * xv[0] : 0.0;
    p[1] = (z + 1 >= z_lo && z + 1 < z_hi) ? cur.va.y * xv[1] : 0.0;
    p[2] = (z + 2 >= z_lo && z + 2 < z_hi) ? cur.vb.x * xv[2] : 0.0;
    p[3] = (z + 3 >= z_lo && z + 3 < z_hi) ? cur.vb.y * xv[3] : 0.0;
    wave_sync();
    // mark the first nonzero of every non-empty row; empty rows are zero
    for (int32_t r = lane; r < nr; r += 64) {
        int32_t lo = ws.ptr[r], hi = ws.ptr[r + 1];
        if (lo == hi) {
            store_row<SPLIT>(a.y, a.slot_row, s_lo + r, 0.0, a.shared_begin, a.accumulate);
        } else {
            atomicOr(&ws.flag[lo >> 5], 1u << (lo & 31));
            ws.row[lo] = s_lo + r;
        }
    }
    const bool row_ends = ws.ptr[nr] + zb <= z_hi;  // no row continues past the chunk
    wave_sync();
    const uint32_t f = (ws.flag[lane >> 3] >> ((lane & 7) * 4)) & 0xFu;
    double head = 0.0, tail = 0.0;
    int32_t trow = -1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if ((f >> e) & 1u) {
            if (trow >= 0) store_row<SPLIT>(a.y, a.slot_row, trow, tail, a.shared_begin, a.accumulate);
            trow = ws.row[4 * lane + e];
            tail = p[e];
        } else if (trow >= 0) {
            tail += p[e];
        } else {
            head += p[e];
        }
    }
    // segmented inclusive scan of (open row, partial sum) over the lanes
    double v = trow >= 0 ? tail : head;
    int32_t rw = trow;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        double vo = __shfl_up(v, off);
        int32_t ro = __shfl_up(rw, off);
        if (lane >= off && rw < 0) {
            v += vo;
            rw = ro;
        }
    }
    if (rw < 0) {
        v += cv;
        rw = cr;
    }
    double av = __shfl_up(v, 1);
    int32_t ar = __shfl_up(rw, 1);
    if (lane == 0) {
        av = cv;
        ar = cr;
    }
    if (f != 0u && ar >= 0) store_row<SPLIT>(a.y, a.slot_row, ar, av + head, a.shared_begin, a.accumulate);
    const int32_t t_end = (z_hi - zb - 1) >> 2;  // lane of the chunk's last nonzero (uniform)
    if (t_end >= 0) {
        double ov = f != 0u ? tail : av + head;
        int32_t orow = f != 0u ? trow : ar;
        if (row_ends) {
            if (lane == t_end && orow >= 0)
                store_row<SPLIT>(a.y, a.slot_row, orow, ov, a.shared_begin, a.accumulate);
            cv = 0.0;
            cr = -1;
        } else {
            cv = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(ov), t_end),
                                  __builtin_amdgcn_readlane(__double2loint(ov), t_end));
            cr = __builtin_amdgcn_readlane(orow, t_end);
        }
    }
    wave_sync();
}

template <int WPG, bool SPLIT, int WMAX>
__global__ __launch_bounds__(64 * WPG) void spmv_waves(SpmvArgs a) {
    __shared__ WaveSmem wsm[WPG];
    __shared__ double swin[WMAX > 0 ? WMAX : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int group = remap_tile(blockIdx.x, a.ntiles, a.xcd_remap);
    const v4i *__restrict__ tiles = reinterpret_cast<const v4i *>(a.tiles);
    const v4i *__restrict__ desc = reinterpret_cast<const v4i *>(a.blk_desc);
    const v4i t4 = tiles[group * WPG + wave];
    const int32_t b0 = __builtin_amdgcn_readfirstlane(t4.x);
    const int32_t b1 = __builtin_amdgcn_readfirstlane(t4.y);
    int32_t wlo = 0, wlen = 0;
    Stage s0, s1;
    if (b0 < b1) issue_chunk(a, desc[b0], lane, s0);
    if (WMAX > 0) {
        // the tiles of a group share one LDS x window
        const v4i g4 = tiles[group * WPG];
        wlo = __builtin_amdgcn_readfirstlane(g4.z);
        wlen = __builtin_amdgcn_readfirstlane(g4.w);
        for (int i = threadIdx.x; i < wlen; i += 64 * WPG) swin[i] = a.x[wlo + i];
        __syncthreads();
    }
    if (b0 >= b1) return;
    WaveSmem &ws = wsm[wave];
    double cv = 0.0;
    int32_t cr = -1;
    // two register stages alternate so that no load result is copied
    for (int32_t b = b0; b < b1; b += 2) {
        v4i dn = desc[b + 1 < b1 ? b + 1 : b];
        run_chunk<SPLIT, WMAX>(a, dn, lane, s0, s1, ws, swin, wlo, wlen, cv, cr);
        if (b + 1 >= b1) break;
        dn = desc[b + 2 < b1 ? b + 2 : b + 1];
        run_chunk<SPLIT, WMAX>(a, dn, lane, s1, s0, ws, swin, wlo, wlen, cv, cr);
    }
}

__global__ void fill_kernel(double *__restrict__ y, int64_t lo, int64_t hi, double v) {
    int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < hi) y[i] = v;
}

__global__ void gather_kernel(const double *__restrict__ x, const int32_t *__restrict__ perm,
                              double *__restrict__ out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = x[perm[i]];
}

__global__ void scatter_kernel(const double *__restrict__ yhat, const int32_t *__restrict__ perm,
                               double *__restrict__ y, int64_t m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) y[perm[i]] = yhat[i];
}

constexpr int kStreamWG = 256;
constexpr int kStreamUnroll = 16;

__global__ __launch_bounds__(kStreamWG) void stream_read_kernel(const v2d *__restrict__ src,
                                                                int64_t n16,
                                                                double *__restrict__ sink) {
    int64_t base = (int64_t)blockIdx.x * kStreamWG * kStreamUnroll + threadIdx.x;
    v2d acc = {0.0, 0.0};
    v2d t[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        int64_t i = base + (int64_t)u * kStreamWG;
        t[u] = i < n16 ? __builtin_nontemporal_load(&src[i]) : v2d{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) acc += t[u];
    __shared__ double red[kStreamWG];
    red[threadIdx.x] = acc.x + acc.y;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < kStreamWG; ++i) s += red[i];
        sink[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kStreamWG) void stream_copy_kernel(const v2d *__restrict__ src,
                                                                v2d *__restrict__ dst, int64_t n16) {
    int64_t base = (int64_t)blockIdx.x * kStreamWG * kStreamUnroll + threadIdx.x;
    v2d t[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        int64_t i = base + (int64_t)u * kStreamWG;
        if (i < n16) t[u] = __builtin_nontemporal_load(&src[i]);
    }
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        int64_t i = base + (int64_t)u * kStreamWG;
        if (i < n16) __builtin_nontemporal_store(t[u], &dst[i]);
    }
}

// ----------------------------------------------------------------- launchers

namespace {
template <int WPG, int WMAX>
hipError_t launch_variant(const SpmvArgs &a, bool split, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    // a.ntiles counts workgroups here: WPG tiles each
    if (split)
        hipLaunchKernelGGL((spmv_waves<WPG, true, WMAX>), dim3(a.ntiles), dim3(64 * WPG), 0, s, a);
    else
        hipLaunchKernelGGL((spmv_waves<WPG, false, WMAX>), dim3(a.ntiles), dim3(64 * WPG), 0, s, a);
    return hipGetLastError();
}
}  // namespace

struct Variant {
    int wg, wmax;
    hipError_t (*fn)(const SpmvArgs &, bool, hipStream_t);
};

static const Variant kVariants[] = {
    {64, 0, launch_variant<1, 0>},
    {128, 0, launch_variant<2, 0>},
    {256, 0, launch_variant<4, 0>},
    {256, 4096, launch_variant<4, 4096>},
    {256, 8192, launch_variant<4, 8192>},
    {512, 12288, launch_variant<8, 12288>},
};

bool spmv_variant_exists(int wg, int window_entries, int *wmax_out) {
    int best = -1;
    for (const Variant &v : kVariants) {
        if (v.wg != wg) continue;
        if (window_entries <= 0 ? v.wmax == 0 : v.wmax >= window_entries) {
            if (best < 0 || v.wmax < best) best = v.wmax;
        }
    }
    if (best < 0) return false;
    if (wmax_out) *wmax_out = best;
    return true;
}

hipError_t launch_spmv(const SpmvArgs &a, int wg, int window_entries, bool split, hipStream_t s) {
    int wmax = 0;
    if (!spmv_variant_exists(wg, window_entries, &wmax)) return hipErrorInvalidValue;
    for (const Variant &v : kVariants)
        if (v.wg == wg && v.wmax == wmax) return v.fn(a, split, s);
    return hipErrorInvalidValue;
}

hipError_t launch_fill(double *y, int64_t lo, int64_t hi, double v, hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    int64_t n = hi - lo;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, lo, hi, v);
    return hipGetLastError();
}

hipError_t launch_gather(const double *x, const int32_t *perm, double *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, perm, out, n);
    return hipGetLastError();
}

hipError_t launch_scatter(const double *yhat, const int32_t *perm, double *y, int64_t m, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, yhat, perm, y, m);
    return hipGetLastError();
}

int64_t stream_grid(int64_t bytes) {
    int64_t n16 = bytes / 16;
    return (n16 + (int64_t)kStreamWG * kStreamUnroll - 1) / ((int64_t)kStreamWG * kStreamUnroll);
}

hipError_t launch_stream_read(const void *src, int64_t bytes, double *sink, hipStream_t s) {
    int64_t g = stream_grid(bytes);
    if (g <= 0) return hipSuccess;
    hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)g), dim3(kStreamWG), 0, s,
                       reinterpret_cast<const v2d *>(src), bytes / 16, sink);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s) {
    int64_t g = stream_grid(bytes);
    if (g <= 0) return hipSuccess;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)g), dim3(kStreamWG), 0, s,
                       reinterpret_cast<const v2d *>(src), reinterpret_cast<v2d *>(dst), bytes / 16);
    return hipGetLastError();
}

}  // namespace spx
