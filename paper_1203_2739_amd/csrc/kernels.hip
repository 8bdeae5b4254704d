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

template <int WG, int IPT, bool SPLIT, int WMAX>
__global__ __launch_bounds__(WG) void spmv_tiles(SpmvArgs a) {
    constexpr int NT = WG * IPT;
    constexpr int GPT = IPT / 4;  // 4-nonzero groups per thread per step
    __shared__ double sprod[NT];
    __shared__ double swin[WMAX > 0 ? WMAX : 1];
    __shared__ double sred[WG / 64];

    const int tid = threadIdx.x;
    const int tile = remap_tile(blockIdx.x, a.ntiles, a.xcd_remap);
    const int32_t b0 = a.tiles[4 * tile + 0];
    const int32_t b1 = a.tiles[4 * tile + 1];
    const int32_t wlo = a.tiles[4 * tile + 2];
    const int32_t wlen = WMAX > 0 ? a.tiles[4 * tile + 3] : 0;
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.colidx);
    const v2d *__restrict__ v2 = reinterpret_cast<const v2d *>(a.vals);
    const double *__restrict__ x = a.x;

    if (WMAX > 0 && wlen > 0) {
        for (int i = tid; i < wlen; i += WG) swin[i] = x[wlo + i];
        __syncthreads();
    }

    for (int32_t b = b0; b < b1; ++b) {
        const int32_t s_lo = a.blk_slot[b];
        const int32_t s_hi = a.blk_slot[b + 1];
        const int32_t z_lo = a.slot_ptr[s_lo];
        const int32_t z_hi = a.slot_ptr[s_hi];
        const int32_t nr = s_hi - s_lo;

        if (nr == 1) {
            // a single row: whole-workgroup reduction in registers
            double acc = 0.0;
            const int32_t gbeg = z_lo >> 2, gend = (z_hi + 3) >> 2;
            for (int32_t gb = gbeg; gb < gend; gb += WG * GPT) {
                v4i cc[GPT];
                v2d va[GPT], vb[GPT];
#pragma unroll
                for (int k = 0; k < GPT; ++k) {
                    int32_t g = gb + tid + k * WG;
                    if (g < gend) {
                        cc[k] = __builtin_nontemporal_load(&c4[g]);
                        va[k] = __builtin_nontemporal_load(&v2[2 * g]);
                        vb[k] = __builtin_nontemporal_load(&v2[2 * g + 1]);
                    }
                }
#pragma unroll
                for (int k = 0; k < GPT; ++k) {
                    int32_t g = gb + tid + k * WG;
                    if (g < gend) {
                        int32_t z = 4 * g;
                        double vv[4] = {va[k].x, va[k].y, vb[k].x, vb[k].y};
                        int32_t ci[4] = {cc[k].x, cc[k].y, cc[k].z, cc[k].w};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (z + e >= z_lo && z + e < z_hi)
                                acc += vv[e] * xval<WMAX>(x, swin, ci[e], wlo, wlen);
                    }
                }
            }
            acc = group_sum(acc, 64);
            if ((tid & 63) == 0) sred[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < WG / 64; ++w) s += sred[w];
                store_row<SPLIT>(a.y, a.slot_row, s_lo, s, a.shared_begin, a.accumulate);
            }
            __syncthreads();
            continue;
        }

        // phase 1: stream the block, products to LDS
        const int32_t zb = z_lo & ~3;
        const int32_t G = (z_hi - zb + 3) >> 2;  // <= NT / 4 by construction
        {
            v4i cc[GPT];
            v2d va[GPT], vb[GPT];
#pragma unroll
            for (int k = 0; k < GPT; ++k) {
                int32_t g = tid + k * WG;
                if (g < G) {
                    cc[k] = __builtin_nontemporal_load(&c4[(zb >> 2) + g]);
                    va[k] = __builtin_nontemporal_load(&v2[(zb >> 1) + 2 * g]);
                    vb[k] = __builtin_nontemporal_load(&v2[(zb >> 1) + 2 * g + 1]);
                }
            }
#pragma unroll
            for (int k = 0; k < GPT; ++k) {
                int32_t g = tid + k * WG;
                if (g < G) {
                    int32_t z = zb + 4 * g;
                    double p0 = (z + 0 >= z_lo && z + 0 < z_hi) ? va[k].x * xval<WMAX>(x, swin, cc[k].x, wlo, wlen) : 0.0;
                    double p1 = (z + 1 >= z_lo && z + 1 < z_hi) ? va[k].y * xval<WMAX>(x, swin, cc[k].y, wlo, wlen) : 0.0;
                    double p2 = (z + 2 >= z_lo && z + 2 < z_hi) ? vb[k].x * xval<WMAX>(x, swin, cc[k].z, wlo, wlen) : 0.0;
                    double p3 = (z + 3 >= z_lo && z + 3 < z_hi) ? vb[k].y * xval<WMAX>(x, swin, cc[k].w, wlo, wlen) : 0.0;
                    v2d *sp = reinterpret_cast<v2d *>(&sprod[4 * g]);
                    sp[0] = v2d{p0, p1};
                    sp[1] = v2d{p2, p3};
                }
            }
        }
        __syncthreads();

        // phase 2: one power-of-two lane group per row
        int gsz = WG / nr;
        gsz = gsz >= 64 ? 64 : gsz;
        gsz = gsz < 1 ? 1 : (1 << (31 - __builtin_clz(gsz)));
        const int ngroups = WG / gsz;
        const int grp = tid / gsz, lane = tid & (gsz - 1);
        for (int32_t rb = 0; rb < nr; rb += ngroups) {
            int32_t r = rb + grp;
            double s = 0.0;
            if (r < nr) {
                int32_t lo = a.slot_ptr[s_lo + r] - zb;
                int32_t hi = a.slot_ptr[s_lo + r + 1] - zb;
                for (int32_t k = lo + lane; k < hi; k += gsz) s += sprod[k];
            }
            s = group_sum(s, gsz);
            if (r < nr && lane == 0)
                store_row<SPLIT>(a.y, a.slot_row, s_lo + r, s, a.shared_begin, a.accumulate);
        }
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
template <int WG, int IPT, int WMAX>
hipError_t launch_variant(const SpmvArgs &a, bool split, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (split)
        hipLaunchKernelGGL((spmv_tiles<WG, IPT, true, WMAX>), dim3(a.ntiles), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((spmv_tiles<WG, IPT, false, WMAX>), dim3(a.ntiles), dim3(WG), 0, s, a);
    return hipGetLastError();
}
}  // namespace

struct Variant {
    int wg, ipt, wmax;
    hipError_t (*fn)(const SpmvArgs &, bool, hipStream_t);
};

static const Variant kVariants[] = {
    {256, 4, 0, launch_variant<256, 4, 0>},
    {256, 8, 0, launch_variant<256, 8, 0>},
    {512, 4, 0, launch_variant<512, 4, 0>},
    {512, 8, 0, launch_variant<512, 8, 0>},
    {1024, 4, 0, launch_variant<1024, 4, 0>},
    {256, 8, 4096, launch_variant<256, 8, 4096>},
    {512, 4, 8192, launch_variant<512, 4, 8192>},
    {512, 8, 8192, launch_variant<512, 8, 8192>},
    {1024, 4, 12288, launch_variant<1024, 4, 12288>},
};

bool spmv_variant_exists(int wg, int ipt, int window_entries, int *wmax_out) {
    int best = -1;
    for (const Variant &v : kVariants) {
        if (v.wg != wg || v.ipt != ipt) continue;
        if (window_entries <= 0 ? v.wmax == 0 : v.wmax >= window_entries) {
            if (best < 0 || v.wmax < best) best = v.wmax;
        }
    }
    if (best < 0) return false;
    if (wmax_out) *wmax_out = best;
    return true;
}

hipError_t launch_spmv(const SpmvArgs &a, int wg, int ipt, int window_entries, bool split,
                       hipStream_t s) {
    int wmax = 0;
    if (!spmv_variant_exists(wg, ipt, window_entries, &wmax)) return hipErrorInvalidValue;
    for (const Variant &v : kVariants)
        if (v.wg == wg && v.ipt == ipt && v.wmax == wmax) return v.fn(a, split, s);
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
