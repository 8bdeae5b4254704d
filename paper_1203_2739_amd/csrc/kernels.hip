// HIP kernels of libspx for gfx950 (CDNA4, wave64).
//
// The SpMV is bound by HBM streaming of the matrix (12 bytes per binary64
// nonzero against 2 flops), so the kernels are organised around memory:
//
//  * One workgroup runs one row block (or, when tiles are requested, a run of
//    blocks of one leaf sharing an LDS x window).  A block is a range of
//    whole consecutive slots (rows, or the non-empty rows of a split leaf)
//    whose nonzeros fit one load round: every thread fetches 4 or 8
//    consecutive nonzeros with 16-byte non-temporal loads from a 4-aligned
//    start, so the workgroup issues all of its HBM traffic at once.
//  * Products go to LDS; each row is then summed by a power-of-two group of
//    lanes with DPP (lane distance 1, 2), ds_swizzle (4, 8, 16) and a
//    cross-half permute (32).
//  * A slot too long for one block is cut into one-round segments whose
//    partial sums are combined by the last segment to finish.
//  * Blocks are assigned to XCDs in contiguous chunks: the hardware hands out
//    workgroups to the 8 XCDs round robin, so workgroup b runs block
//    start(b mod 8) + b div 8.  Consecutive blocks of a part then run on one
//    XCD and share its x entries in that XCD's L2, the GPU counterpart of a
//    part that fits into the cache (Section 3, Theorem 1).
//  * Split products (y <- y + A^k x, Section 4) store rows owned by a single
//    leaf directly and add the per-leaf sums of rows shared by several leaves
//    with binary64 atomics onto the zeroed shared range (measured faster than
//    writing per-leaf sums and folding them in a second kernel, whose reads
//    of the sums are scattered).
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

__device__ __forceinline__ int remap_tile(int bid, int ntiles, int on) {
    if (!on) return bid;
    int x = bid & 7, i = bid >> 3;
    int per = ntiles >> 3, rem = ntiles & 7;
    return x * per + (x < rem ? x : rem) + i;
}

// Writes the sum of one slot: an atomic add for a row shared by several
// leaves of a split (onto the zeroed entry), an add for a split product that
// accumulates, a plain store otherwise.
template <bool SPLIT>
__device__ __forceinline__ void store_row(const SpmvArgs &a, int32_t slot, double v) {
    double *__restrict__ y = a.y;
    const int32_t row = SPLIT ? a.slot_row[slot] : slot;
    if (SPLIT && row >= a.shared_begin) {
        unsafeAtomicAdd(&y[row], v);
    } else if (SPLIT && a.accumulate) {
        y[row] += v;
    } else {
        y[row] = v;
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

// Sum over aligned groups of g lanes (g a power of two, at most 64); every
// lane of the group receives the total.  Must be reached by the whole wave.
__device__ __forceinline__ double group_sum_unrolled(double v, int g) {
    if (g > 1) v += xor_lanes(v, 1);
    if (g > 2) v += xor_lanes(v, 2);
    if (g > 4) v += xor_lanes(v, 4);
    if (g > 8) v += xor_lanes(v, 8);
    if (g > 16) v += xor_lanes(v, 16);
    if (g > 32) v += xor_lanes(v, 32);
    return v;
}

// One multi-row block: whole slots [d.x, d.y) with nonzeros [d.z, d.w).
template <int WG, int NPT, bool SPLIT, int WMAX>
__device__ __forceinline__ void multi_row_block(const SpmvArgs &a, const v4i d, double *sprod, int32_t *sptr,
                                                const double *swin, int32_t wlo, int32_t wlen) {
    const int tid = threadIdx.x;
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.colidx);
    const v2d *__restrict__ v2 = reinterpret_cast<const v2d *>(a.vals);
    const int32_t zb = d.z & ~3;
    const int32_t nr = d.y - d.x;
    const int32_t G = (d.w - zb + 3) >> 2;
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid + u * WG;
        if (gi < G) {
            const v4i cc = __builtin_nontemporal_load(&c4[(zb >> 2) + gi]);
            const v2d va = __builtin_nontemporal_load(&v2[(zb >> 1) + 2 * gi]);
            const v2d vb = __builtin_nontemporal_load(&v2[(zb >> 1) + 2 * gi + 1]);
            v2d *sp = reinterpret_cast<v2d *>(&sprod[4 * gi]);
            sp[0] = v2d{va.x * xval<WMAX>(a.x, swin, cc.x, wlo, wlen), va.y * xval<WMAX>(a.x, swin, cc.y, wlo, wlen)};
            sp[1] = v2d{vb.x * xval<WMAX>(a.x, swin, cc.z, wlo, wlen), vb.y * xval<WMAX>(a.x, swin, cc.w, wlo, wlen)};
        }
    }
    for (int i = tid; i <= nr; i += WG) sptr[i] = a.slot_ptr[d.x + i] - zb;
    __syncthreads();
    // lanes per row: the largest power of two <= WG / nr, at most 64
    const int q = WG / nr;
    const int lg = q >= 64 ? 6 : 31 - __builtin_clz(q);
    const int g = 1 << lg;
    const int grp = tid >> lg, lane = tid & (g - 1);
    double sum = 0.0;
    if (grp < nr) {
        const int k1 = sptr[grp + 1];
        for (int k = sptr[grp] + lane; k < k1; k += g) sum += sprod[k];
    }
    sum = group_sum_unrolled(sum, g);
    if (grp < nr && lane == 0) store_row<SPLIT>(a, d.x + grp, sum);
}

// One segment [d.z, d.w) of long slot d.x: one load round like a multi-row
// block, summed in registers and across waves.  A slot cut into several
// segments combines them without atomics on y: each segment stores its
// partial sum, and the workgroup that arrives last (counted by an atomic
// counter) adds the partials in segment order, writes the slot and resets
// the counter for the next product.
template <int WG, int NPT, bool SPLIT, int WMAX>
__device__ __forceinline__ void long_row_segment(const SpmvArgs &a, const v4i d, double *swave,
                                                 const double *swin, int32_t wlo, int32_t wlen) {
    const int tid = threadIdx.x;
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.colidx);
    const v2d *__restrict__ v2 = reinterpret_cast<const v2d *>(a.vals);
    const int32_t zb = d.z & ~3;
    const int32_t G = (d.w - zb + 3) >> 2;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid + u * WG;
        if (gi < G) {
            const int32_t k0 = zb + 4 * gi;
            const v4i cc = __builtin_nontemporal_load(&c4[(zb >> 2) + gi]);
            const v2d va = __builtin_nontemporal_load(&v2[(zb >> 1) + 2 * gi]);
            const v2d vb = __builtin_nontemporal_load(&v2[(zb >> 1) + 2 * gi + 1]);
            const double p0 = va.x * xval<WMAX>(a.x, swin, cc.x, wlo, wlen);
            const double p1 = va.y * xval<WMAX>(a.x, swin, cc.y, wlo, wlen);
            const double p2 = vb.x * xval<WMAX>(a.x, swin, cc.z, wlo, wlen);
            const double p3 = vb.y * xval<WMAX>(a.x, swin, cc.w, wlo, wlen);
            acc += (k0 >= d.z) ? p0 : 0.0;
            acc += (k0 + 1 >= d.z && k0 + 1 < d.w) ? p1 : 0.0;
            acc += (k0 + 2 >= d.z && k0 + 2 < d.w) ? p2 : 0.0;
            acc += (k0 + 3 >= d.z && k0 + 3 < d.w) ? p3 : 0.0;
        }
    }
    acc = group_sum_unrolled(acc, 64);
    if ((tid & 63) == 0) swave[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double part = 0.0;
#pragma unroll
        for (int w = 0; w < WG / 64; ++w) part += swave[w];
        const int32_t lr = -1 - d.y;
        const int32_t base = a.long_seg_ptr[lr];
        const int32_t nseg = a.long_seg_ptr[lr + 1] - base;
        if (nseg == 1) {
            store_row<SPLIT>(a, d.x, part);
        } else {
            const int32_t seg = (zb - (a.slot_ptr[d.x] & ~3)) / (NPT * WG);
            // The partial goes to the device-coherent level (an agent-scope
            // atomic store writes through the XCD's L2) and must have landed
            // before the counter moves: wait for the store to complete.  An
            // acquire/release fence would also write back and invalidate the
            // whole L2 of the XCD, discarding the cached x entries.
            __hip_atomic_store(&a.partials[base + seg], part, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): expcnt and lgkmcnt left unconstrained
            const uint32_t done =
                __hip_atomic_fetch_add(&a.counters[lr], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (done == (uint32_t)nseg - 1) {
                double sum = 0.0;
                for (int32_t k = 0; k < nseg; ++k)
                    sum += __hip_atomic_load(&a.partials[base + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.counters[lr], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                store_row<SPLIT>(a, d.x, sum);
            }
        }
    }
}

// TILED = false: workgroup i runs block remap(i), no window.  TILED = true:
// workgroup i runs the blocks of tile remap(i) with the tile's LDS window.
template <int WG, int NPT, bool SPLIT, int WMAX, bool TILED>
__global__ __launch_bounds__(WG) void spmv_blocks(SpmvArgs a) {
    __shared__ double sprod[NPT * WG];
    __shared__ int32_t sptr[WG + 1];
    __shared__ double swave[WG / 64];
    __shared__ double swin[WMAX > 0 ? WMAX : 1];
    const int tid = threadIdx.x;
    const int id = remap_tile(blockIdx.x, a.ntiles, a.xcd_remap);
    if (!TILED) {
        const v4i d = reinterpret_cast<const v4i *>(a.blk_desc)[id];
        if (d.y >= 0) multi_row_block<WG, NPT, SPLIT, 0>(a, d, sprod, sptr, swin, 0, 0);
        else long_row_segment<WG, NPT, SPLIT, 0>(a, d, swave, swin, 0, 0);
        return;
    }
    const v4i tl = reinterpret_cast<const v4i *>(a.tiles)[id];
    const int32_t wlo = tl.z;
    const int32_t wlen = WMAX > 0 ? tl.w : 0;
    if (WMAX > 0 && wlen > 0) {
        for (int i = tid; i < wlen; i += WG) swin[i] = a.x[wlo + i];
        __syncthreads();
    }
    for (int b = tl.x; b < tl.y; ++b) {
        const v4i d = reinterpret_cast<const v4i *>(a.blk_desc)[b];
        if (d.y >= 0) multi_row_block<WG, NPT, SPLIT, WMAX>(a, d, sprod, sptr, swin, wlo, wlen);
        else long_row_segment<WG, NPT, SPLIT, WMAX>(a, d, swave, swin, wlo, wlen);
        __syncthreads();
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
template <int WG, int NPT, int WMAX>
hipError_t launch_variant(const SpmvArgs &a, bool split, bool tiled, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (WMAX == 0 && !tiled) {
        if (split)
            hipLaunchKernelGGL((spmv_blocks<WG, NPT, true, 0, false>), dim3(a.ntiles), dim3(WG), 0, s, a);
        else
            hipLaunchKernelGGL((spmv_blocks<WG, NPT, false, 0, false>), dim3(a.ntiles), dim3(WG), 0, s, a);
    } else {
        if (split)
            hipLaunchKernelGGL((spmv_blocks<WG, NPT, true, WMAX, true>), dim3(a.ntiles), dim3(WG), 0, s, a);
        else
            hipLaunchKernelGGL((spmv_blocks<WG, NPT, false, WMAX, true>), dim3(a.ntiles), dim3(WG), 0, s, a);
    }
    return hipGetLastError();
}
}  // namespace

struct Variant {
    int wg, npt, wmax;
    hipError_t (*fn)(const SpmvArgs &, bool, bool, hipStream_t);
};

static const Variant kVariants[] = {
    {64, 8, 0, launch_variant<64, 8, 0>},
    {128, 4, 0, launch_variant<128, 4, 0>},
    {128, 8, 0, launch_variant<128, 8, 0>},
    {256, 4, 0, launch_variant<256, 4, 0>},
    {512, 4, 0, launch_variant<512, 4, 0>},
    {128, 4, 4096, launch_variant<128, 4, 4096>},
    {128, 4, 8192, launch_variant<128, 4, 8192>},
    {128, 4, 16384, launch_variant<128, 4, 16384>},
    {256, 4, 4096, launch_variant<256, 4, 4096>},
    {256, 4, 8192, launch_variant<256, 4, 8192>},
    {256, 4, 16384, launch_variant<256, 4, 16384>},
    {512, 4, 16384, launch_variant<512, 4, 16384>},
};

bool spmv_variant_exists(int wg, int npt, int window_entries, int *wmax_out) {
    int best = -1;
    for (const Variant &v : kVariants) {
        if (v.wg != wg || v.npt != npt) continue;
        if (window_entries <= 0 ? v.wmax == 0 : v.wmax >= window_entries) {
            if (best < 0 || v.wmax < best) best = v.wmax;
        }
    }
    if (best < 0) return false;
    if (wmax_out) *wmax_out = best;
    return true;
}

hipError_t launch_spmv(const SpmvArgs &a, int wg, int npt, int window_entries, bool tiled, bool split,
                       hipStream_t s) {
    int wmax = 0;
    if (!spmv_variant_exists(wg, npt, window_entries, &wmax)) return hipErrorInvalidValue;
    for (const Variant &v : kVariants)
        if (v.wg == wg && v.npt == npt && v.wmax == wmax) return v.fn(a, split, tiled, s);
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
