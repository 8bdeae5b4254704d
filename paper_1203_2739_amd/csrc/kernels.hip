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

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace spx {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

namespace {

// Value of the lane `off` positions away in an xor pattern (off a power of two
// up to 32): DPP quad permutes for 1 and 2, ds_swizzle for 4 to 16, a
// cross-half permute for 32.
__device__ __forceinline__ int xor_lanes_i(int v, int off) {
    switch (off) {
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    case 4: return __builtin_amdgcn_ds_swizzle(v, 0x101F);
    case 8: return __builtin_amdgcn_ds_swizzle(v, 0x201F);
    case 16: return __builtin_amdgcn_ds_swizzle(v, 0x401F);
    default: return __builtin_amdgcn_ds_bpermute(((int)(threadIdx.x & 63) ^ 32) << 2, v);
    }
}

__device__ __forceinline__ double xor_lanes(double v, int off) {
    return __hiloint2double(xor_lanes_i(__double2hiint(v), off), xor_lanes_i(__double2loint(v), off));
}

__device__ __forceinline__ float xor_lanes(float v, int off) {
    return __int_as_float(xor_lanes_i(__float_as_int(v), off));
}

// Unit (tile or block) of workgroup bid: with the XCD mapping on, the
// hardware's round-robin dispatch puts workgroup bid on XCD bid % 8, which
// runs the units of row group bid % 8 in order; -1 when that group has no
// unit left for this workgroup.
template <class V, class A>
__device__ __forceinline__ int unit_of(const SpmvArgsT<V, A> &a, int bid) {
    if (!a.xcd_remap) return bid;
    const int x = bid & (kXcdGroups - 1), i = bid / kXcdGroups;
    const int u = a.xcd_ptr[x] + i;
    return u < a.xcd_ptr[x + 1] ? u : -1;
}

// Writes the sum of one slot: an atomic add for a row shared by several
// leaves of a split (onto the zeroed entry), an add for a split product that
// accumulates, a plain store otherwise.
template <bool SPLIT, class V, class A>
__device__ __forceinline__ void store_row(const SpmvArgsT<V, A> &a, int32_t slot, A v) {
    A *__restrict__ y = a.y;
    const int32_t row = SPLIT ? a.slot_row[slot] : slot;
    if (SPLIT && row >= a.shared_begin) {
        unsafeAtomicAdd(&y[row], v);
    } else if (SPLIT && a.accumulate) {
        y[row] += v;
    } else {
        y[row] = v;
    }
}

template <int WMAX, class A>
__device__ __forceinline__ A xval(const A *__restrict__ x, const A *sw, int32_t c, int32_t wlo, int32_t wlen) {
    if (WMAX > 0) {
        uint32_t o = (uint32_t)(c - wlo);
        if (o < (uint32_t)wlen) return sw[o];
    }
    return x[c];
}

// Four consecutive stored values starting at the 4-aligned nonzero k0,
// widened to the accumulation type: binary64 (two 16-byte loads), binary32
// (one 16-byte load) or bfloat16 bit patterns (one 8-byte load; a bfloat16
// is the upper half of the binary32 with the same bits).
struct Vals4d { double v[4]; };
struct Vals4f { float v[4]; };

__device__ __forceinline__ Vals4d load4(const double *vals, int32_t k0) {
    const v2d *v2 = reinterpret_cast<const v2d *>(vals);
    const v2d a = __builtin_nontemporal_load(&v2[k0 >> 1]);
    const v2d b = __builtin_nontemporal_load(&v2[(k0 >> 1) + 1]);
    return {{a.x, a.y, b.x, b.y}};
}

__device__ __forceinline__ Vals4f load4(const float *vals, int32_t k0) {
    const v4f a = __builtin_nontemporal_load(&reinterpret_cast<const v4f *>(vals)[k0 >> 2]);
    return {{a.x, a.y, a.z, a.w}};
}

__device__ __forceinline__ Vals4f load4(const uint16_t *vals, int32_t k0) {
    const v2u a = __builtin_nontemporal_load(&reinterpret_cast<const v2u *>(vals)[k0 >> 2]);
    return {{__uint_as_float(a.x << 16), __uint_as_float(a.x & 0xFFFF0000u), __uint_as_float(a.y << 16),
             __uint_as_float(a.y & 0xFFFF0000u)}};
}

}  // namespace

// Sum over aligned groups of g lanes (g a power of two, at most 64); every
// lane of the group receives the total.  Must be reached by the whole wave.
template <class A>
__device__ __forceinline__ A group_sum_unrolled(A v, int g) {
    if (g > 1) v += xor_lanes(v, 1);
    if (g > 2) v += xor_lanes(v, 2);
    if (g > 4) v += xor_lanes(v, 4);
    if (g > 8) v += xor_lanes(v, 8);
    if (g > 16) v += xor_lanes(v, 16);
    if (g > 32) v += xor_lanes(v, 32);
    return v;
}

// Orders the LDS writes of the lanes before the reads that follow.  A
// workgroup block needs a barrier; a wave block (WAVE) only needs the
// compiler to keep its LDS accesses in order, since one wave's LDS
// instructions execute in issue order.
template <bool WAVE>
__device__ __forceinline__ void block_sync() {
    if (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Row sums of a block whose products sit in row order in sprod (offsets
// from the block's aligned start), with the row offsets in sptr: each row
// is summed by 2^floor(log2(WG / rows)) lanes (at most a wave).
template <int WG, bool SPLIT, class V, class A>
__device__ __forceinline__ void sum_rows(const SpmvArgsT<V, A> &a, const v4i d, const A *sprod, const int32_t *sptr,
                                         const int tid) {
    const int32_t nr = d.y - d.x;
    // lanes per row: the largest power of two <= WG / nr, at most 64
    const int q = WG / nr;
    const int lg = q >= 64 ? 6 : 31 - __builtin_clz(q);
    const int g = 1 << lg;
    const int grp = tid >> lg, lane = tid & (g - 1);
    A sum = 0;
    if (grp < nr) {
        const int k1 = sptr[grp + 1];
        for (int k = sptr[grp] + lane; k < k1; k += g) sum += sprod[k];
    }
    sum = group_sum_unrolled(sum, g);
    if (grp < nr && lane == 0) store_row<SPLIT>(a, d.x + grp, sum);
}

// One multi-row block: whole slots [d.x, d.y) with nonzeros [d.z, d.w), run
// by the WG threads of a workgroup (tid = threadIdx.x) or, with WAVE, by the
// 64 lanes of one wave (WG = 64, tid = lane) on the wave's own LDS slices.
template <int WG, int NPT, bool SPLIT, int WMAX, bool WAVE = false, class V, class A>
__device__ __forceinline__ void multi_row_block(const SpmvArgsT<V, A> &a, const v4i d, A *sprod, int32_t *sptr,
                                                const A *swin, int32_t wlo, int32_t wlen,
                                                const int tid = threadIdx.x) {
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.colidx);
    const int32_t zb = d.z & ~3;
    const int32_t nr = d.y - d.x;  // at most WG (schedule)
    const int32_t G = (d.w - zb + 3) >> 2;
    // row pointers first, so that their latency overlaps the data loads;
    // nr + 1 <= WG + 1 of them: one per thread, the last one by thread 0
    // when the block has WG rows
    const int32_t rp0 = a.slot_ptr[d.x + min(tid, nr)];
    const int32_t rp1 = (nr == WG && tid == 0) ? a.slot_ptr[d.x + WG] : 0;
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid + u * WG;
        if (gi < G) {
            const v4i cc = __builtin_nontemporal_load(&c4[(zb >> 2) + gi]);
            const auto vv = load4(a.vals, zb + 4 * gi);
            A *sp = &sprod[4 * gi];
            sp[0] = vv.v[0] * xval<WMAX>(a.x, swin, cc.x, wlo, wlen);
            sp[1] = vv.v[1] * xval<WMAX>(a.x, swin, cc.y, wlo, wlen);
            sp[2] = vv.v[2] * xval<WMAX>(a.x, swin, cc.z, wlo, wlen);
            sp[3] = vv.v[3] * xval<WMAX>(a.x, swin, cc.w, wlo, wlen);
        }
    }
    if (tid <= nr) sptr[tid] = rp0 - zb;
    if (nr == WG && tid == 0) sptr[WG] = rp1 - zb;
    block_sync<WAVE>();
    sum_rows<WG, SPLIT>(a, d, sprod, sptr, tid);
}

// Gather-sorted blocks: the nonzeros of every multi-row block also live in
// a second device copy (scol, sval), sorted by column, at a 64-aligned
// offset sofs[block]; every index carries in its upper bits the nonzero's
// offset in row order from the block's aligned start.  The copy is
// interleaved in chunks of 64 sorted entries: the 16 lanes of a quarter
// wave load one chunk with the usual 16-byte loads, lane l of the quarter
// holding sorted entries 16 j + l (j = 0..3), so the j-th gather
// instruction of a quarter reads 16 consecutive sorted columns and lanes
// that hit one cache line of x share one request.  The last chunk is padded
// with all-ones indices.  The products go back to their row-order slots in
// LDS and the rows are summed as in multi_row_block.
template <int WG, int NPT, bool SPLIT, class V, class A>
__device__ __forceinline__ void sorted_row_block(const SpmvArgsT<V, A> &a, const v4i d, int32_t so, A *sprod,
                                                 int32_t *sptr) {
    constexpr int SH = pack_shift(WG * NPT);
    constexpr int MASK = (1 << SH) - 1;
    const int tid = threadIdx.x;
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.scol);
    const int32_t zb = d.z & ~3;
    const int32_t nr = d.y - d.x;  // at most WG (schedule)
    const int32_t ngroups = ((d.w - d.z + 63) & ~63) >> 2;  // 16-byte groups of the padded chunks
    const int32_t rp0 = a.slot_ptr[d.x + min(tid, nr)];
    const int32_t rp1 = (nr == WG && tid == 0) ? a.slot_ptr[d.x + WG] : 0;
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid + u * WG;
        if (gi < ngroups) {
            const v4i cc = __builtin_nontemporal_load(&c4[(so >> 2) + gi]);
            const auto vv = load4(a.sval, so + 4 * gi);
            const int32_t c[4] = {cc.x, cc.y, cc.z, cc.w};
            A xv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) xv[j] = c[j] != -1 ? a.x[c[j] & MASK] : A(0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c[j] != -1) sprod[(uint32_t)c[j] >> SH] = vv.v[j] * xv[j];
        }
    }
    if (tid <= nr) sptr[tid] = rp0 - zb;
    if (nr == WG && tid == 0) sptr[WG] = rp1 - zb;
    __syncthreads();
    sum_rows<WG, SPLIT>(a, d, sprod, sptr, tid);
}

// A multi-row block read through 16-bit indices: the offsets from the
// block's smallest column cb come four to a thread in one 8-byte load
// (instead of 16 bytes of 32-bit indices); entries of the aligned start
// before d.z and past d.w belong to other blocks, whose offsets are from
// another base, so they gather x[cb] (a column of this block) and their
// products are dropped, which keeps the four gathers unconditional.  Rows
// are summed as in multi_row_block.
template <int WG, int NPT, bool SPLIT, class V, class A>
__device__ __forceinline__ void compact_row_block(const SpmvArgsT<V, A> &a, const v4i d, int32_t cb, A *sprod,
                                                  int32_t *sptr) {
    const int tid = threadIdx.x;
    const v2u *__restrict__ c4 = reinterpret_cast<const v2u *>(a.c16);
    const int32_t zb = d.z & ~3;
    const int32_t nr = d.y - d.x;  // at most WG (schedule)
    const int32_t G = (d.w - zb + 3) >> 2;
    const int32_t rp0 = a.slot_ptr[d.x + min(tid, nr)];
    const int32_t rp1 = (nr == WG && tid == 0) ? a.slot_ptr[d.x + WG] : 0;
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid + u * WG;
        if (gi < G) {
            const v2u cc = __builtin_nontemporal_load(&c4[(zb >> 2) + gi]);
            const auto vv = load4(a.vals, zb + 4 * gi);
            const int32_t k0 = zb + 4 * gi;
            const int32_t c[4] = {(int32_t)(cc.x & 0xFFFFu), (int32_t)(cc.x >> 16), (int32_t)(cc.y & 0xFFFFu),
                                  (int32_t)(cc.y >> 16)};
            A *sp = &sprod[4 * gi];
            bool in[4];
            A xv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                in[j] = k0 + j >= d.z && k0 + j < d.w;
                xv[j] = a.x[cb + (in[j] ? c[j] : 0)];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) sp[j] = in[j] ? vv.v[j] * xv[j] : A(0);
        }
    }
    if (tid <= nr) sptr[tid] = rp0 - zb;
    if (nr == WG && tid == 0) sptr[WG] = rp1 - zb;
    __syncthreads();
    sum_rows<WG, SPLIT>(a, d, sprod, sptr, tid);
}

// Partial sum number `seg` of long (or cut) slot number lr, which is slot
// `slot`: stored directly when the slot has one partial, else combined by
// the one that arrives last.
template <bool SPLIT, class V, class A>
__device__ __forceinline__ void combine_partial(const SpmvArgsT<V, A> &a, int32_t lr, int32_t seg, int32_t slot,
                                                A part) {
    const int32_t base = a.long_seg_ptr[lr];
    const int32_t nseg = a.long_seg_ptr[lr + 1] - base;
    if (nseg == 1) {
        store_row<SPLIT>(a, slot, part);
    } else {
        // The partial goes to the device-coherent level (an agent-scope
        // atomic store writes through the XCD's L2) and must have landed
        // before the counter moves: the wave waits until the store is
        // acknowledged (vmcnt counts stores on gfx9 parts), and the
        // signal fence keeps the compiler from moving the counter update
        // above that wait.  The segment that sees the final count reads
        // the partials with agent-scope loads issued after its update
        // returned.  A release on the update would instead write back
        // the whole L2 of the XCD (buffer_wbl2) for every segment.
        __hip_atomic_store(&a.partials[base + seg], (double)part, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): expcnt and lgkmcnt left unconstrained
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const uint32_t done =
            __hip_atomic_fetch_add(&a.counters[lr], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == (uint32_t)nseg - 1) {
            A sum = 0;
            for (int32_t k = 0; k < nseg; ++k)
                sum += (A)__hip_atomic_load(&a.partials[base + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.counters[lr], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            store_row<SPLIT>(a, slot, sum);
        }
    }
}

// The partial sum `part` of segment [d.z, d.w) (aligned start zb) of long
// slot d.x (number -1 - d.y).  SPAN is the nonzeros a segment spans from its
// aligned start.
template <int SPAN, bool SPLIT, class V, class A>
__device__ __forceinline__ void combine_segment(const SpmvArgsT<V, A> &a, const v4i d, int32_t zb, A part) {
    const int32_t seg = (zb - (a.slot_ptr[d.x] & ~3)) / SPAN;
    combine_partial<SPLIT>(a, -1 - d.y, seg, d.x, part);
}

// One segment [d.z, d.w) of long slot d.x: one load round like a multi-row
// block, summed in registers and across waves.  A slot cut into several
// segments combines them without atomics on y: each segment stores its
// partial sum, and the workgroup that arrives last (counted by an atomic
// counter) adds the partials in segment order, writes the slot and resets
// the counter for the next product.
template <int WG, int NPT, bool SPLIT, int WMAX, bool WAVE = false, class V, class A>
__device__ __forceinline__ void long_row_segment(const SpmvArgsT<V, A> &a, const v4i d, A *swave, const A *swin,
                                                 int32_t wlo, int32_t wlen, const int tid = threadIdx.x) {
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.colidx);
    const int32_t zb = d.z & ~3;
    const int32_t G = (d.w - zb + 3) >> 2;
    A acc = 0;
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid + u * WG;
        if (gi < G) {
            const int32_t k0 = zb + 4 * gi;
            const v4i cc = __builtin_nontemporal_load(&c4[(zb >> 2) + gi]);
            const auto vv = load4(a.vals, k0);
            const A p0 = vv.v[0] * xval<WMAX>(a.x, swin, cc.x, wlo, wlen);
            const A p1 = vv.v[1] * xval<WMAX>(a.x, swin, cc.y, wlo, wlen);
            const A p2 = vv.v[2] * xval<WMAX>(a.x, swin, cc.z, wlo, wlen);
            const A p3 = vv.v[3] * xval<WMAX>(a.x, swin, cc.w, wlo, wlen);
            acc += (k0 >= d.z) ? p0 : A(0);
            acc += (k0 + 1 >= d.z && k0 + 1 < d.w) ? p1 : A(0);
            acc += (k0 + 2 >= d.z && k0 + 2 < d.w) ? p2 : A(0);
            acc += (k0 + 3 >= d.z && k0 + 3 < d.w) ? p3 : A(0);
        }
    }
    acc = group_sum_unrolled(acc, 64);
    if (!WAVE) {
        if ((tid & 63) == 0) swave[tid >> 6] = acc;
        __syncthreads();
    }
    if (tid == 0) {
        A part = 0;
        if (WAVE) {
            part = acc;
        } else {
#pragma unroll
            for (int w = 0; w < WG / 64; ++w) part += swave[w];
        }
        combine_segment<NPT * WG, SPLIT>(a, d, zb, part);
    }
}

// TILED = false: workgroup i runs block remap(i), no window.  TILED = true:
// workgroup i runs the blocks of tile remap(i) with the tile's LDS window.
template <int WG, int NPT, bool SPLIT, int WMAX, bool TILED, class V, class A>
__global__ __launch_bounds__(WG) void spmv_blocks(SpmvArgsT<V, A> a) {
    __shared__ A sprod[NPT * WG];
    __shared__ int32_t sptr[WG + 1];
    __shared__ A swave[WG / 64];
    __shared__ A swin[WMAX > 0 ? WMAX : 1];
    const int tid = threadIdx.x;
    const int id = unit_of(a, blockIdx.x);
    if (id < 0) return;
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

// ---------------------------------------------------------- pipelined tiles
// The stored values of four consecutive nonzeros as loaded (no widening, so
// that holding them does not wait for the load): two 16-byte binary64
// pairs, one 16-byte binary32 quad, or one 8-byte pair of bfloat16 pairs.
template <class V> struct Raw4;
template <> struct Raw4<double> { v2d a, b; };
template <> struct Raw4<float> { v4f a; };
template <> struct Raw4<uint16_t> { v2u a; };

__device__ __forceinline__ Raw4<double> load_raw4(const double *vals, int32_t k0) {
    const v2d *v2 = reinterpret_cast<const v2d *>(vals);
    return {__builtin_nontemporal_load(&v2[k0 >> 1]), __builtin_nontemporal_load(&v2[(k0 >> 1) + 1])};
}
__device__ __forceinline__ Raw4<float> load_raw4(const float *vals, int32_t k0) {
    return {__builtin_nontemporal_load(&reinterpret_cast<const v4f *>(vals)[k0 >> 2])};
}
__device__ __forceinline__ Raw4<uint16_t> load_raw4(const uint16_t *vals, int32_t k0) {
    return {__builtin_nontemporal_load(&reinterpret_cast<const v2u *>(vals)[k0 >> 2])};
}
__device__ __forceinline__ Vals4d widen4(const Raw4<double> &r) { return {{r.a.x, r.a.y, r.b.x, r.b.y}}; }
__device__ __forceinline__ Vals4f widen4(const Raw4<float> &r) { return {{r.a.x, r.a.y, r.a.z, r.a.w}}; }
__device__ __forceinline__ Vals4f widen4(const Raw4<uint16_t> &r) {
    return {{__uint_as_float(r.a.x << 16), __uint_as_float(r.a.x & 0xFFFF0000u), __uint_as_float(r.a.y << 16),
             __uint_as_float(r.a.y & 0xFFFF0000u)}};
}

// Everything one thread loads for one block before the gathers: the
// descriptor, its row pointers and its NPT indices and values.
template <int NPT, class V>
struct Stage {
    v4i d;
    int32_t rp0, rp1;
    v4i cc[NPT / 4];
    Raw4<V> vv[NPT / 4];
};

template <int WG, int NPT, class V, class A>
__device__ __forceinline__ void load_stage(const SpmvArgsT<V, A> &a, int b, Stage<NPT, V> &st) {
    const int tid = threadIdx.x;
    st.d = reinterpret_cast<const v4i *>(a.blk_desc)[b];
    const v4i d = st.d;
    const int32_t zb = d.z & ~3;
    const int32_t G = (d.w - zb + 3) >> 2;
    st.rp0 = st.rp1 = 0;
    if (d.y >= 0) {
        const int32_t nr = d.y - d.x;
        st.rp0 = a.slot_ptr[d.x + min(tid, nr)];
        if (nr == WG && tid == 0) st.rp1 = a.slot_ptr[d.x + WG];
    }
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.colidx);
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid + u * WG;
        if (gi < G) {
            st.cc[u] = __builtin_nontemporal_load(&c4[(zb >> 2) + gi]);
            st.vv[u] = load_raw4(a.vals, zb + 4 * gi);
        }
    }
}

// Pipelined tiles: one workgroup per tile of blocks (tiles per row group for
// a persistent launch); the loads of block b + 1 are issued right after the
// gathers of block b and before block b's products are reduced, so that a
// round of index and value loads is in flight while the workgroup reduces
// and stores.  The reduction is the one of multi_row_block and
// long_row_segment.
template <int WG, int NPT, bool SPLIT, int WMAX, class V, class A>
__global__ __launch_bounds__(WG) void spmv_pipe(SpmvArgsT<V, A> a) {
    __shared__ A sprod[NPT * WG];
    __shared__ int32_t sptr[WG + 1];
    __shared__ A swave[WG / 64];
    __shared__ A swin[WMAX > 0 ? WMAX : 1];
    const int tid = threadIdx.x;
    const int id = unit_of(a, blockIdx.x);
    if (id < 0) return;
    const v4i tl = reinterpret_cast<const v4i *>(a.tiles)[id];
    const int32_t wlo = tl.z;
    const int32_t wlen = WMAX > 0 ? tl.w : 0;
    if (WMAX > 0 && wlen > 0) {
        for (int i = tid; i < wlen; i += WG) swin[i] = a.x[wlo + i];
        __syncthreads();
    }
    if (tl.x >= tl.y) return;
    Stage<NPT, V> cur, nxt;
    load_stage<WG, NPT>(a, tl.x, cur);
    for (int b = tl.x; b < tl.y; ++b) {
        const v4i d = cur.d;
        const int32_t zb = d.z & ~3;
        const int32_t G = (d.w - zb + 3) >> 2;
        // gathers of this block
        A xv[NPT];
#pragma unroll
        for (int u = 0; u < NPT / 4; ++u) {
            const int gi = tid + u * WG;
            if (gi < G) {
                xv[4 * u] = xval<WMAX>(a.x, swin, cur.cc[u].x, wlo, wlen);
                xv[4 * u + 1] = xval<WMAX>(a.x, swin, cur.cc[u].y, wlo, wlen);
                xv[4 * u + 2] = xval<WMAX>(a.x, swin, cur.cc[u].z, wlo, wlen);
                xv[4 * u + 3] = xval<WMAX>(a.x, swin, cur.cc[u].w, wlo, wlen);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // the next block's loads go out before this block is reduced
        if (b + 1 < tl.y) load_stage<WG, NPT>(a, b + 1, nxt);
        __builtin_amdgcn_sched_barrier(0);
        if (d.y >= 0) {
            const int32_t nr = d.y - d.x;
#pragma unroll
            for (int u = 0; u < NPT / 4; ++u) {
                const int gi = tid + u * WG;
                if (gi < G) {
                    const auto vv = widen4(cur.vv[u]);
                    A *sp = &sprod[4 * gi];
                    sp[0] = vv.v[0] * xv[4 * u];
                    sp[1] = vv.v[1] * xv[4 * u + 1];
                    sp[2] = vv.v[2] * xv[4 * u + 2];
                    sp[3] = vv.v[3] * xv[4 * u + 3];
                }
            }
            if (tid <= nr) sptr[tid] = cur.rp0 - zb;
            if (nr == WG && tid == 0) sptr[WG] = cur.rp1 - zb;
            __syncthreads();
            const int q = WG / nr;
            const int lg = q >= 64 ? 6 : 31 - __builtin_clz(q);
            const int g = 1 << lg;
            const int grp = tid >> lg, lane = tid & (g - 1);
            A sum = 0;
            if (grp < nr) {
                const int k1 = sptr[grp + 1];
                for (int k = sptr[grp] + lane; k < k1; k += g) sum += sprod[k];
            }
            sum = group_sum_unrolled(sum, g);
            if (grp < nr && lane == 0) store_row<SPLIT>(a, d.x + grp, sum);
        } else {
            A acc = 0;
#pragma unroll
            for (int u = 0; u < NPT / 4; ++u) {
                const int gi = tid + u * WG;
                if (gi < G) {
                    const int32_t k0 = zb + 4 * gi;
                    const auto vv = widen4(cur.vv[u]);
                    acc += (k0 >= d.z) ? vv.v[0] * xv[4 * u] : A(0);
                    acc += (k0 + 1 >= d.z && k0 + 1 < d.w) ? vv.v[1] * xv[4 * u + 1] : A(0);
                    acc += (k0 + 2 >= d.z && k0 + 2 < d.w) ? vv.v[2] * xv[4 * u + 2] : A(0);
                    acc += (k0 + 3 >= d.z && k0 + 3 < d.w) ? vv.v[3] * xv[4 * u + 3] : A(0);
                }
            }
            acc = group_sum_unrolled(acc, 64);
            if ((tid & 63) == 0) swave[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                A part = 0;
#pragma unroll
                for (int w = 0; w < WG / 64; ++w) part += swave[w];
                combine_segment<NPT * WG, SPLIT>(a, d, zb, part);
            }
        }
        __syncthreads();  // the next block rewrites sprod, sptr and swave
        cur = nxt;
    }
}

// Wave blocks: every workgroup runs one tile (with its LDS window, loaded
// once), and each of its waves takes the tile's blocks in turn -- wave w the
// blocks first + w, first + w + WG/64, ... -- reducing rows on its own LDS
// slices, so no workgroup barrier follows the window load.  A block is a
// run of whole slots sized for one wave (at most 64 slots and 64 NPT
// nonzeros from the aligned start), or one segment of a long slot.
template <int WG, int NPT, bool SPLIT, int WMAX, class V, class A>
__global__ __launch_bounds__(WG) void spmv_waves(SpmvArgsT<V, A> a) {
    constexpr int NW = WG / 64;
    __shared__ A sprod[NW][NPT * 64];
    __shared__ int32_t sptr[NW][65];
    __shared__ A swin[WMAX > 0 ? WMAX : 1];
    const int id = unit_of(a, blockIdx.x);
    if (id < 0) return;
    const v4i tl = reinterpret_cast<const v4i *>(a.tiles)[id];
    const int32_t wlo = tl.z;
    const int32_t wlen = WMAX > 0 ? tl.w : 0;
    if (WMAX > 0 && wlen > 0) {
        for (int i = threadIdx.x; i < wlen; i += WG) swin[i] = a.x[wlo + i];
        __syncthreads();
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int b = tl.x + w; b < tl.y; b += NW) {
        const v4i d = reinterpret_cast<const v4i *>(a.blk_desc)[b];
        if (d.y >= 0) multi_row_block<64, NPT, SPLIT, WMAX, true>(a, d, sprod[w], sptr[w], swin, wlo, wlen, lane);
        else long_row_segment<64, NPT, SPLIT, WMAX, true>(a, d, sprod[w], swin, wlo, wlen, lane);
        block_sync<true>();  // the next block rewrites this wave's slices
    }
}

// One workgroup per gather-sorted block (XCD mapping as in spmv_blocks);
// long-slot segments as in spmv_blocks, from the stored order.
template <int WG, int NPT, bool SPLIT, class V, class A>
__global__ __launch_bounds__(WG) void spmv_sorted(SpmvArgsT<V, A> a) {
    __shared__ A sprod[NPT * WG];
    __shared__ int32_t sptr[WG + 1];
    __shared__ A swave[WG / 64];
    const int id = unit_of(a, blockIdx.x);
    if (id < 0) return;
    const v4i d = reinterpret_cast<const v4i *>(a.blk_desc)[id];
    if (d.y >= 0) sorted_row_block<WG, NPT, SPLIT>(a, d, a.sofs[id], sprod, sptr);
    else long_row_segment<WG, NPT, SPLIT, 0>(a, d, swave, swave, 0, 0);
}

// ------------------------------------------------------------- scan blocks
// Row sums by a segmented scan over the products of a block, in nonzero
// order.  Thread t holds the NPT consecutive products of its chunk in
// registers.  The owner of every non-empty row records the position of the
// row's last nonzero; a chunk is summarised by (holds a row end, sum after
// its last row end), and an exclusive scan of these pairs over the threads
// (the sum restarts after every row end) gives each thread the partial sum
// of the row that is open where its chunk begins.  The thread that holds
// the last nonzero of a row writes it.  The work per thread no longer
// depends on the longest row of the block, so the schedule cuts such blocks
// by nonzeros and rows alone.

// Inclusive scan of the chunk summaries (f, s) over the lanes of a wave in
// lane order, where lanes a < b combine to (f_a | f_b, f_b ? s_b : s_a + s_b):
// lane l ends with the sum of the products that follow the last row end in
// lanes 0..l, and f = 1 when lanes 0..l hold a row end at all.
template <class A>
__device__ __forceinline__ void wave_seg_scan(A &s, int &f, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const A sp = __shfl_up(s, o, 64);
        const int fp = __shfl_up(f, o, 64);
        if (lane >= o) {
            if (!f) s = sp + s;
            f |= fp;
        }
    }
}

// Records the ends of the rows of a block for the scan: send[r] is the
// block-relative position of the last nonzero of row d.x + r (-1 for an
// empty row, which is written as zero here), sowner[k] the row ending at
// position k.  sowner is not cleared between blocks: the scan takes
// sowner[k] = r as a row end only when r is a row of this block whose
// send[r] is k, and a row that ends at k has written exactly that pair, so
// a stale entry is either rejected or right.  rb, re: the row's bounds.
template <bool SPLIT, class V, class A>
__device__ __forceinline__ void mark_row_ends(const SpmvArgsT<V, A> &a, const v4i d, int32_t rb, int32_t re,
                                              int16_t *send, uint16_t *sowner) {
    const int tid = threadIdx.x;
    const int32_t zb = d.z & ~3;
    if (tid < d.y - d.x) {
        // rows of a block lie in [d.z, d.w), which spans at most WG NPT
        // entries from zb
        send[tid] = re > rb ? (int16_t)(re - 1 - zb) : (int16_t)-1;
        if (re > rb) sowner[re - 1 - zb] = (uint16_t)tid;
        else store_row<SPLIT>(a, d.x + tid, A(0));
    }
}

// Row sums of a block by the segmented scan, once the row ends are marked
// (mark_row_ends, then a barrier): p holds the products of this thread's
// NPT consecutive positions (zero outside the block's nonzeros).
template <int WG, int NPT, bool SPLIT, class V, class A>
__device__ __forceinline__ void scan_sum_rows(const SpmvArgsT<V, A> &a, const v4i d, const A *p, const int16_t *send,
                                              const uint16_t *sowner, A *sws, int32_t *swf) {
    constexpr int NW = WG / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t nr = d.y - d.x;
    uint32_t ends = 0;
    int32_t rows[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int k = tid * NPT + j;
        const int r = sowner[k];
        rows[j] = r;
        if (r < nr && send[r] == k) ends |= 1u << j;
    }
    A s = 0;
#pragma unroll
    for (int j = 0; j < NPT; ++j) s = ((ends >> j) & 1u) ? A(0) : s + p[j];
    int f = ends != 0u;
    wave_seg_scan(s, f, lane);
    // exclusive value of this lane, then the carry from the earlier waves
    A carry = __shfl_up(s, 1, 64);
    int fc = __shfl_up(f, 1, 64);
    if (lane == 0) {
        carry = 0;
        fc = 0;
    }
    if (NW > 1) {
        if (lane == 63) {
            sws[w] = s;
            swf[w] = f;
        }
        __syncthreads();
        if (!fc) {
            A c = 0;
            for (int j = w - 1; j >= 0; --j) {
                c = sws[j] + c;
                if (swf[j]) break;
            }
            carry = c + carry;
        }
    }
    A run = carry;
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        run += p[j];
        if ((ends >> j) & 1u) {
            store_row<SPLIT>(a, d.x + rows[j], run);
            run = 0;
        }
    }
}

// One multi-row block summed by the scan, products computed in registers.
template <int WG, int NPT, bool SPLIT, class V, class A>
__device__ __forceinline__ void scan_row_block(const SpmvArgsT<V, A> &a, const v4i d, int16_t *send,
                                               uint16_t *sowner, A *sws, int32_t *swf) {
    static_assert(NPT == 4 || NPT == 8, "4 or 8 nonzeros per thread");
    const int tid = threadIdx.x;
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.colidx);
    const int32_t zb = d.z & ~3;
    const int32_t nr = d.y - d.x;  // at most WG (schedule)
    const int32_t G = (d.w - zb + 3) >> 2;
    // row bounds first, so that their latency overlaps the data loads
    const int32_t rb = tid < nr ? a.slot_ptr[d.x + tid] : 0;
    const int32_t re = tid < nr ? a.slot_ptr[d.x + tid + 1] : 0;
    A p[NPT];
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid * (NPT / 4) + u;
        const int32_t k0 = zb + 4 * gi;
        A q0 = 0, q1 = 0, q2 = 0, q3 = 0;
        if (gi < G) {
            const v4i cc = __builtin_nontemporal_load(&c4[(zb >> 2) + gi]);
            const auto vv = load4(a.vals, k0);
            q0 = vv.v[0] * a.x[cc.x];
            q1 = vv.v[1] * a.x[cc.y];
            q2 = vv.v[2] * a.x[cc.z];
            q3 = vv.v[3] * a.x[cc.w];
        }
        // entries of the aligned start before d.z, and from d.w on, belong
        // to other blocks
        p[4 * u + 0] = (k0 >= d.z && k0 < d.w) ? q0 : A(0);
        p[4 * u + 1] = (k0 + 1 >= d.z && k0 + 1 < d.w) ? q1 : A(0);
        p[4 * u + 2] = (k0 + 2 >= d.z && k0 + 2 < d.w) ? q2 : A(0);
        p[4 * u + 3] = (k0 + 3 >= d.z && k0 + 3 < d.w) ? q3 : A(0);
    }
    mark_row_ends<SPLIT>(a, d, rb, re, send, sowner);
    __syncthreads();  // row ends recorded
    scan_sum_rows<WG, NPT, SPLIT>(a, d, p, send, sowner, sws, swf);
}

// One gather-sorted block summed by the scan: the products of the sorted
// loads go to their row-order slots in LDS (as in sorted_row_block), and
// every thread then takes its NPT consecutive row-order products from there.
template <int WG, int NPT, bool SPLIT, class V, class A>
__device__ __forceinline__ void sorted_scan_block(const SpmvArgsT<V, A> &a, const v4i d, int32_t so, A *sprod,
                                                  int16_t *send, uint16_t *sowner, A *sws, int32_t *swf) {
    constexpr int SH = pack_shift(WG * NPT);
    constexpr int MASK = (1 << SH) - 1;
    const int tid = threadIdx.x;
    const v4i *__restrict__ c4 = reinterpret_cast<const v4i *>(a.scol);
    const int32_t zb = d.z & ~3;
    const int32_t nr = d.y - d.x;  // at most WG (schedule)
    const int32_t ngroups = ((d.w - d.z + 63) & ~63) >> 2;
    const int32_t rb = tid < nr ? a.slot_ptr[d.x + tid] : 0;
    const int32_t re = tid < nr ? a.slot_ptr[d.x + tid + 1] : 0;
#pragma unroll
    for (int u = 0; u < NPT / 4; ++u) {
        const int gi = tid + u * WG;
        if (gi < ngroups) {
            const v4i cc = __builtin_nontemporal_load(&c4[(so >> 2) + gi]);
            const auto vv = load4(a.sval, so + 4 * gi);
            const int32_t c[4] = {cc.x, cc.y, cc.z, cc.w};
            A xv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) xv[j] = c[j] != -1 ? a.x[c[j] & MASK] : A(0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c[j] != -1) sprod[(uint32_t)c[j] >> SH] = vv.v[j] * xv[j];
        }
    }
    mark_row_ends<SPLIT>(a, d, rb, re, send, sowner);
    __syncthreads();  // products in place, row ends recorded
    A p[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int32_t k = zb + NPT * tid + j;
        p[j] = (k >= d.z && k < d.w) ? sprod[NPT * tid + j] : A(0);
    }
    scan_sum_rows<WG, NPT, SPLIT>(a, d, p, send, sowner, sws, swf);
}

// One workgroup per block (XCD mapping as in spmv_blocks); multi-row blocks
// are summed by the segmented scan, long-slot segments as in spmv_blocks.
template <int WG, int NPT, bool SPLIT, class V, class A>
__global__ __launch_bounds__(WG) void spmv_scan(SpmvArgsT<V, A> a) {
    __shared__ int16_t send[WG];
    __shared__ uint16_t sowner[WG * NPT];
    __shared__ A sws[WG / 64];
    __shared__ int32_t swf[WG / 64];
    const int id = unit_of(a, blockIdx.x);
    if (id < 0) return;
    const v4i d = reinterpret_cast<const v4i *>(a.blk_desc)[id];
    if (d.y >= 0) scan_row_block<WG, NPT, SPLIT>(a, d, send, sowner, sws, swf);
    else long_row_segment<WG, NPT, SPLIT, 0>(a, d, sws, sws, 0, 0);
}

// One workgroup per gather-sorted block summed by the scan (XCD mapping as
// in spmv_blocks); long-slot segments from the stored order.
template <int WG, int NPT, bool SPLIT, class V, class A>
__global__ __launch_bounds__(WG) void spmv_sorted_scan(SpmvArgsT<V, A> a) {
    __shared__ A sprod[NPT * WG];
    __shared__ int16_t send[WG];
    __shared__ uint16_t sowner[NPT * WG];
    __shared__ A sws[WG / 64];
    __shared__ int32_t swf[WG / 64];
    const int id = unit_of(a, blockIdx.x);
    if (id < 0) return;
    const v4i d = reinterpret_cast<const v4i *>(a.blk_desc)[id];
    if (d.y >= 0) sorted_scan_block<WG, NPT, SPLIT>(a, d, a.sofs[id], sprod, send, sowner, sws, swf);
    else long_row_segment<WG, NPT, SPLIT, 0>(a, d, sws, sws, 0, 0);
}

// One workgroup per block with 16-bit indices where the block has them
// (XCD mapping as in spmv_blocks); other blocks read the 32-bit indices.
template <int WG, int NPT, bool SPLIT, class V, class A>
__global__ __launch_bounds__(WG) void spmv_compact(SpmvArgsT<V, A> a) {
    __shared__ A sprod[NPT * WG];
    __shared__ int32_t sptr[WG + 1];
    __shared__ A swave[WG / 64];
    const int id = unit_of(a, blockIdx.x);
    if (id < 0) return;
    const v4i d = reinterpret_cast<const v4i *>(a.blk_desc)[id];
    if (d.y < 0) {
        long_row_segment<WG, NPT, SPLIT, 0>(a, d, swave, swave, 0, 0);
        return;
    }
    const int32_t cb = a.cbase[id];
    if (cb >= 0) compact_row_block<WG, NPT, SPLIT>(a, d, cb, sprod, sptr);
    else multi_row_block<WG, NPT, SPLIT, 0>(a, d, sprod, sptr, swave, 0, 0);
}

// ------------------------------------------------------------------ batched
// One persistent launch over the blocks of many matrices.  Each workgroup
// takes the next item from a queue counter (items are sorted by decreasing
// work on the host, so the queue ends with small items) until the queue is
// empty.  An item is one block or long-row segment of one matrix; a matrix
// with one right-hand side and unit strides runs the row-block SpMV code,
// any other matrix the multiple-right-hand-side code below: lanes form
// groups of k (one lane per right-hand side) and each group sums whole rows,
// reading one contiguous row of X per nonzero.

// sum over z = z0, z0 + step, ... < z1 of a_z * X[col_z, j]: eight nonzeros
// per round, so that the eight index/value loads and then the eight gathers
// of X rows are in flight together instead of one dependent chain per
// nonzero
__device__ __forceinline__ double spmm_dot(const BatchMat &M, int32_t z0, int32_t z1, int32_t step, int j) {
    double sum = 0.0;
    int32_t z = z0;
    for (; z + 7 * step < z1; z += 8 * step) {
        int32_t c[8];
        double v[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c[u] = M.colidx[z + u * step];
            v[u] = M.vals[z + u * step];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = M.X[(int64_t)c[u] * M.ldx + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += v[u] * xv[u];
    }
    for (; z < z1; z += step) sum += M.vals[z] * M.X[(int64_t)M.colidx[z] * M.ldx + j];
    return sum;
}

template <int WG>
__device__ __forceinline__ void spmm_block(const BatchMat &M, const int32_t *it, double *red) {
    const int tid = threadIdx.x;
    const int k = M.k;
    const int32_t s_lo = it[1], s_hi = it[2], z_lo = it[3], z_hi = it[4];
    const int ngroups = WG / k;
    const int g = tid / k, j = tid - g * k;
    if (s_hi >= 0) {
        // a group of k lanes per row: lane j sums a_z * X[col_z, j] over the
        // row; the k lanes read one contiguous row of X per nonzero
        if (g < ngroups)
            for (int32_t r = s_lo + g; r < s_hi; r += ngroups)
                M.Y[(int64_t)r * M.ldy + j] = spmm_dot(M, M.slot_ptr[r], M.slot_ptr[r + 1], 1, j);
        return;
    }
    // a segment of a long row: the groups share its nonzeros, their sums meet
    // in LDS, and the segments are combined by the one that arrives last
    // (see long_row_segment)
    __shared__ uint32_t last;
    double sum = 0.0;
    if (g < ngroups) sum = spmm_dot(M, z_lo + g, z_hi, ngroups, j);
    if (g < ngroups) red[g * k + j] = sum;
    __syncthreads();
    if (tid < k) {
        sum = 0.0;
        for (int q = 0; q < ngroups; ++q) sum += red[q * k + tid];
    }
    const int32_t lr = -1 - s_hi;
    const int32_t base = M.long_seg_ptr[lr], nseg = M.long_seg_ptr[lr + 1] - base;
    if (nseg == 1) {
        if (tid < k) M.Y[(int64_t)s_lo * M.ldy + tid] = sum;
        return;
    }
    const int32_t seg = (z_lo - M.slot_ptr[s_lo]) / M.span;
    if (tid < k) {
        __hip_atomic_store(&M.partials[(int64_t)(base + seg) * k + tid], sum, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the partial has landed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    __syncthreads();
    if (tid == 0)
        last = __hip_atomic_fetch_add(&M.counters[lr], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               (uint32_t)nseg - 1;
    __syncthreads();
    if (last) {
        if (tid < k) {
            double tot = 0.0;
            for (int32_t q = 0; q < nseg; ++q)
                tot += __hip_atomic_load(&M.partials[(int64_t)(base + q) * k + tid], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
            M.Y[(int64_t)s_lo * M.ldy + tid] = tot;
        }
        if (tid == 0) __hip_atomic_store(&M.counters[lr], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int WG>
__global__ __launch_bounds__(WG) void batch_kernel(BatchArgs b) {
    __shared__ double lds[4 * WG];
    __shared__ int32_t sptr[WG + 1];
    __shared__ double swave[WG / 64];
    __shared__ int32_t item_sh;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0)
            item_sh = (int32_t)__hip_atomic_fetch_add(b.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int32_t item = item_sh;
        __syncthreads();
        if (item >= b.nitems) break;
        const int32_t *it = &b.items[5 * (int64_t)item];
        const BatchMat &M = b.mats[it[0]];
        if (M.k == 1 && M.ldx == 1 && M.ldy == 1) {
            SpmvArgs a{};
            a.slot_ptr = M.slot_ptr;
            a.colidx = M.colidx;
            a.vals = M.vals;
            a.x = M.X;
            a.y = M.Y;
            a.long_seg_ptr = M.long_seg_ptr;
            a.partials = M.partials;
            a.counters = M.counters;
            const v4i d = {it[1], it[2], it[3], it[4]};
            if (d.y >= 0) multi_row_block<WG, 4, false, 0>(a, d, lds, sptr, lds, 0, 0);
            else long_row_segment<WG, 4, false, 0>(a, d, swave, lds, 0, 0);
        } else {
            spmm_block<WG>(M, it, lds);
        }
        __syncthreads();
    }
}

__global__ void queue_reset_kernel(uint32_t *q) { *q = 0u; }

// ---------------------------------------------------------------- CG vectors
// Conjugate-gradient vector operations of the precision mode.  Dot products
// are summed per workgroup in a fixed order and the workgroup sums by one
// more workgroup in index order, so they are reproducible.

constexpr int kDotWG = 256;
constexpr int kDotMaxGroups = 1024;

template <class T>
__global__ __launch_bounds__(kDotWG) void dot_partial_kernel(const T *__restrict__ a, const T *__restrict__ b,
                                                             int64_t n, T *__restrict__ part) {
    __shared__ T sw[kDotWG / 64];
    T acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kDotWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDotWG)
        acc += a[i] * b[i];
    acc = group_sum_unrolled(acc, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T s = 0;
        for (int w = 0; w < kDotWG / 64; ++w) s += sw[w];
        part[blockIdx.x] = s;
    }
}

template <class T>
__global__ __launch_bounds__(kDotWG) void sum_kernel(const T *__restrict__ part, int n, T *__restrict__ out) {
    __shared__ T sw[kDotWG / 64];
    T acc = 0;
    for (int i = threadIdx.x; i < n; i += kDotWG) acc += part[i];
    acc = group_sum_unrolled(acc, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T s = 0;
        for (int w = 0; w < kDotWG / 64; ++w) s += sw[w];
        *out = s;
    }
}

// r_low = r / scale; p = r_low; d = 0
template <class T>
__global__ void cg_start_kernel(const double *__restrict__ r, double inv_scale, T *__restrict__ rl,
                                T *__restrict__ p, T *__restrict__ d, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        T v = (T)(r[i] * inv_scale);
        rl[i] = v;
        p[i] = v;
        d[i] = 0;
    }
}

// alpha = rr / pq; d += alpha p; r -= alpha q
template <class T>
__global__ void cg_update_kernel(const T *__restrict__ rr, const T *__restrict__ pq, T *__restrict__ d,
                                 T *__restrict__ r, const T *__restrict__ p, const T *__restrict__ q, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const T alpha = *pq != T(0) ? *rr / *pq : T(0);
        d[i] += alpha * p[i];
        r[i] -= alpha * q[i];
    }
}

// beta = rr_new / rr; p = r + beta p
template <class T>
__global__ void cg_direction_kernel(const T *__restrict__ rr, const T *__restrict__ rr_new, T *__restrict__ p,
                                    const T *__restrict__ r, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = r[i] + (*rr != T(0) ? *rr_new / *rr : T(0)) * p[i];
}

// x += scale * d (binary64 update)
template <class T>
__global__ void ir_update_kernel(double *__restrict__ x, const T *__restrict__ d, double scale, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += scale * (double)d[i];
}

// r = b - Ax (binary64 residual)
__global__ void residual_kernel(const double *__restrict__ b, const double *__restrict__ ax, double *__restrict__ r,
                                int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = b[i] - ax[i];
}

__global__ void to_f32_kernel(const double *__restrict__ x, float *__restrict__ out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)x[i];
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
// Workgroups of a launch: one per unit, or with the XCD mapping 8 times the
// largest number of units of a row group.  Groups hold nearly equal
// nonzeros, but a row long enough to fill most of a group puts many
// one-round segments into it; when the largest group has over 1.5 times the
// mean number of units, the launch keeps the hardware order instead, so
// that one XCD does not run most of the work.
template <class V, class A>
unsigned grid_of_units(SpmvArgsT<V, A> &a) {
    if (!a.xcd_remap) return (unsigned)a.ntiles;
    int mx = 0;
    for (int g = 0; g < kXcdGroups; ++g) mx = std::max(mx, a.xcd_ptr[g + 1] - a.xcd_ptr[g]);
    if (2 * kXcdGroups * (int64_t)mx > 3 * (int64_t)a.ntiles) {
        a.xcd_remap = 0;
        return (unsigned)a.ntiles;
    }
    return (unsigned)(kXcdGroups * mx);
}

template <int WG, int NPT, int WMAX, class V, class A>
hipError_t launch_variant(const SpmvArgsT<V, A> &a0, bool split, bool tiled, hipStream_t s) {
    if (a0.ntiles <= 0) return hipSuccess;
    SpmvArgsT<V, A> a = a0;
    const unsigned grid = grid_of_units(a);
    if (WMAX == 0 && !tiled) {
        if (split)
            hipLaunchKernelGGL((spmv_blocks<WG, NPT, true, 0, false, V, A>), dim3(grid), dim3(WG), 0, s, a);
        else
            hipLaunchKernelGGL((spmv_blocks<WG, NPT, false, 0, false, V, A>), dim3(grid), dim3(WG), 0, s, a);
    } else {
        if (split)
            hipLaunchKernelGGL((spmv_blocks<WG, NPT, true, WMAX, true, V, A>), dim3(grid), dim3(WG), 0, s, a);
        else
            hipLaunchKernelGGL((spmv_blocks<WG, NPT, false, WMAX, true, V, A>), dim3(grid), dim3(WG), 0, s, a);
    }
    return hipGetLastError();
}

template <int WG, int NPT, int WMAX, class V, class A>
hipError_t launch_waves(const SpmvArgsT<V, A> &a0, bool split, bool, hipStream_t s) {
    if (a0.ntiles <= 0) return hipSuccess;
    SpmvArgsT<V, A> a = a0;
    const unsigned grid = grid_of_units(a);
    if (split)
        hipLaunchKernelGGL((spmv_waves<WG, NPT, true, WMAX, V, A>), dim3(grid), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((spmv_waves<WG, NPT, false, WMAX, V, A>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

template <int WG, int NPT, int WMAX, class V, class A>
hipError_t launch_pipe(const SpmvArgsT<V, A> &a0, bool split, bool, hipStream_t s) {
    if (a0.ntiles <= 0) return hipSuccess;
    SpmvArgsT<V, A> a = a0;
    const unsigned grid = grid_of_units(a);
    if (split)
        hipLaunchKernelGGL((spmv_pipe<WG, NPT, true, WMAX, V, A>), dim3(grid), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((spmv_pipe<WG, NPT, false, WMAX, V, A>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

template <int WG, int NPT, int WMAX, class V, class A>
hipError_t launch_scan(const SpmvArgsT<V, A> &a0, bool split, bool, hipStream_t s) {
    static_assert(WMAX == 0, "scan blocks take no window");
    if (a0.ntiles <= 0) return hipSuccess;
    SpmvArgsT<V, A> a = a0;
    const unsigned grid = grid_of_units(a);
    if (split)
        hipLaunchKernelGGL((spmv_scan<WG, NPT, true, V, A>), dim3(grid), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((spmv_scan<WG, NPT, false, V, A>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

template <int WG, int NPT, int WMAX, class V, class A>
hipError_t launch_sorted(const SpmvArgsT<V, A> &a0, bool split, bool, hipStream_t s) {
    static_assert(WMAX == 0, "gather-sorted blocks take no window");
    if (a0.ntiles <= 0) return hipSuccess;
    SpmvArgsT<V, A> a = a0;
    const unsigned grid = grid_of_units(a);
    if (split)
        hipLaunchKernelGGL((spmv_sorted<WG, NPT, true, V, A>), dim3(grid), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((spmv_sorted<WG, NPT, false, V, A>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

template <int WG, int NPT, int WMAX, class V, class A>
hipError_t launch_sorted_scan(const SpmvArgsT<V, A> &a0, bool split, bool, hipStream_t s) {
    static_assert(WMAX == 0, "gather-sorted scan blocks take no window");
    if (a0.ntiles <= 0) return hipSuccess;
    SpmvArgsT<V, A> a = a0;
    const unsigned grid = grid_of_units(a);
    if (split)
        hipLaunchKernelGGL((spmv_sorted_scan<WG, NPT, true, V, A>), dim3(grid), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((spmv_sorted_scan<WG, NPT, false, V, A>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

template <int WG, int NPT, int WMAX, class V, class A>
hipError_t launch_compact(const SpmvArgsT<V, A> &a0, bool split, bool, hipStream_t s) {
    static_assert(WMAX == 0, "compact-index blocks take no window");
    if (a0.ntiles <= 0) return hipSuccess;
    SpmvArgsT<V, A> a = a0;
    const unsigned grid = grid_of_units(a);
    if (split)
        hipLaunchKernelGGL((spmv_compact<WG, NPT, true, V, A>), dim3(grid), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((spmv_compact<WG, NPT, false, V, A>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

template <class V, class A>
struct Variant {
    int wg, npt, wmax;
    hipError_t (*fn)(const SpmvArgsT<V, A> &, bool, bool, hipStream_t);
};

// scan-block kernels (no window, 4 nonzeros per thread: with 8, the two
// 16-byte loads of a thread's consecutive chunk leave every load
// instruction of a wave half-used lines, measured 1.5x slower), every
// precision
template <class V, class A>
struct ScanTable {
    static constexpr Variant<V, A> v[] = {
        {128, 4, 0, launch_scan<128, 4, 0, V, A>},
        {256, 4, 0, launch_scan<256, 4, 0, V, A>},
        {512, 4, 0, launch_scan<512, 4, 0, V, A>},
        {1024, 4, 0, launch_scan<1024, 4, 0, V, A>},
    };
};

// gather-sorted kernels (binary64)
struct SortedTable {
    static constexpr Variant<double, double> v[] = {
        {128, 4, 0, launch_sorted<128, 4, 0, double, double>},
        {256, 4, 0, launch_sorted<256, 4, 0, double, double>},
        {512, 4, 0, launch_sorted<512, 4, 0, double, double>},
        {1024, 4, 0, launch_sorted<1024, 4, 0, double, double>},
        {256, 8, 0, launch_sorted<256, 8, 0, double, double>},
        {512, 8, 0, launch_sorted<512, 8, 0, double, double>},
    };
};

// compact-index kernels (binary64)
struct CompactTable {
    static constexpr Variant<double, double> v[] = {
        {128, 4, 0, launch_compact<128, 4, 0, double, double>},
        {256, 4, 0, launch_compact<256, 4, 0, double, double>},
        {512, 4, 0, launch_compact<512, 4, 0, double, double>},
    };
};

// gather-sorted scan kernels (binary64)
struct SortedScanTable {
    static constexpr Variant<double, double> v[] = {
        {256, 4, 0, launch_sorted_scan<256, 4, 0, double, double>},
        {512, 4, 0, launch_sorted_scan<512, 4, 0, double, double>},
        {1024, 4, 0, launch_sorted_scan<1024, 4, 0, double, double>},
        {256, 8, 0, launch_sorted_scan<256, 8, 0, double, double>},
        {512, 8, 0, launch_sorted_scan<512, 8, 0, double, double>},
    };
};

// pipelined-tile kernels (binary64 with optional windows; low precisions
// without)
template <class V, class A>
struct PipeTable;
template <>
struct PipeTable<double, double> {
    static constexpr Variant<double, double> v[] = {
        {256, 4, 0, launch_pipe<256, 4, 0, double, double>},
        {512, 4, 0, launch_pipe<512, 4, 0, double, double>},
        {256, 8, 0, launch_pipe<256, 8, 0, double, double>},
        {1024, 4, 0, launch_pipe<1024, 4, 0, double, double>},
        {256, 4, 8192, launch_pipe<256, 4, 8192, double, double>},
        {512, 4, 16384, launch_pipe<512, 4, 16384, double, double>},
    };
};
template <class V>
struct LowPipeTable {
    static constexpr Variant<V, float> v[] = {
        {256, 4, 0, launch_pipe<256, 4, 0, V, float>},
        {512, 4, 0, launch_pipe<512, 4, 0, V, float>},
    };
};
template <>
struct PipeTable<float, float> : LowPipeTable<float> {};
template <>
struct PipeTable<uint16_t, float> : LowPipeTable<uint16_t> {};

// wave-block kernels: workgroup size, nonzeros per lane, window capacity
// (LDS: WG/64 slices of 64 NPT products and 65 row offsets, plus the window);
// the low precisions take the shapes without a window
template <class V, class A>
struct WaveTable;

template <>
struct WaveTable<double, double> {
    static constexpr Variant<double, double> v[] = {
        {256, 4, 0, launch_waves<256, 4, 0, double, double>},
        {512, 4, 0, launch_waves<512, 4, 0, double, double>},
        {1024, 4, 0, launch_waves<1024, 4, 0, double, double>},
        {256, 8, 0, launch_waves<256, 8, 0, double, double>},
        {512, 8, 0, launch_waves<512, 8, 0, double, double>},
        {256, 4, 8192, launch_waves<256, 4, 8192, double, double>},
        {512, 4, 16384, launch_waves<512, 4, 16384, double, double>},
        {512, 8, 8192, launch_waves<512, 8, 8192, double, double>},
        {1024, 4, 15360, launch_waves<1024, 4, 15360, double, double>},
    };
};

template <class V>
struct LowWaveTable {
    static constexpr Variant<V, float> v[] = {
        {256, 4, 0, launch_waves<256, 4, 0, V, float>},
        {512, 4, 0, launch_waves<512, 4, 0, V, float>},
        {1024, 4, 0, launch_waves<1024, 4, 0, V, float>},
        {256, 8, 0, launch_waves<256, 8, 0, V, float>},
        {512, 8, 0, launch_waves<512, 8, 0, V, float>},
    };
};
template <>
struct WaveTable<float, float> : LowWaveTable<float> {};
template <>
struct WaveTable<uint16_t, float> : LowWaveTable<uint16_t> {};

// binary64: every schedule shape; low precision: the untiled shapes
template <class V, class A>
struct Table;

template <>
struct Table<double, double> {
    static constexpr Variant<double, double> v[] = {
        {64, 8, 0, launch_variant<64, 8, 0, double, double>},
        {128, 4, 0, launch_variant<128, 4, 0, double, double>},
        {128, 8, 0, launch_variant<128, 8, 0, double, double>},
        {256, 4, 0, launch_variant<256, 4, 0, double, double>},
        {256, 8, 0, launch_variant<256, 8, 0, double, double>},
        {512, 4, 0, launch_variant<512, 4, 0, double, double>},
        {128, 4, 4096, launch_variant<128, 4, 4096, double, double>},
        {128, 4, 8192, launch_variant<128, 4, 8192, double, double>},
        {128, 4, 16384, launch_variant<128, 4, 16384, double, double>},
        {256, 4, 4096, launch_variant<256, 4, 4096, double, double>},
        {256, 4, 8192, launch_variant<256, 4, 8192, double, double>},
        {256, 4, 16384, launch_variant<256, 4, 16384, double, double>},
        {512, 4, 16384, launch_variant<512, 4, 16384, double, double>},
        {1024, 4, 15360, launch_variant<1024, 4, 15360, double, double>},
    };
};

template <class V>
struct LowTable {
    static constexpr Variant<V, float> v[] = {
        {64, 8, 0, launch_variant<64, 8, 0, V, float>},
        {128, 4, 0, launch_variant<128, 4, 0, V, float>},
        {128, 8, 0, launch_variant<128, 8, 0, V, float>},
        {256, 4, 0, launch_variant<256, 4, 0, V, float>},
        {256, 8, 0, launch_variant<256, 8, 0, V, float>},
        {512, 4, 0, launch_variant<512, 4, 0, V, float>},
    };
};
template <>
struct Table<float, float> : LowTable<float> {};
template <>
struct Table<uint16_t, float> : LowTable<uint16_t> {};

template <class TableT>
bool find_in(int wg, int npt, int window_entries, int *wmax_out) {
    int best = -1;
    for (const auto &v : TableT::v) {
        if (v.wg != wg || v.npt != npt) continue;
        if (window_entries <= 0 ? v.wmax == 0 : v.wmax >= window_entries) {
            if (best < 0 || v.wmax < best) best = v.wmax;
        }
    }
    if (best < 0) return false;
    if (wmax_out) *wmax_out = best;
    return true;
}

template <class TableT, class V, class A>
hipError_t launch_in(const SpmvArgsT<V, A> &a, int wg, int npt, int window_entries, bool split, hipStream_t s) {
    int wmax = 0;
    if (!find_in<TableT>(wg, npt, window_entries, &wmax)) return hipErrorInvalidValue;
    for (const auto &v : TableT::v)
        if (v.wg == wg && v.npt == npt && v.wmax == wmax) return v.fn(a, split, true, s);
    return hipErrorInvalidValue;
}

template <class V, class A>
bool find_wave_variant(int wg, int npt, int window_entries, int *wmax_out) {
    int best = -1;
    for (const auto &v : WaveTable<V, A>::v) {
        if (v.wg != wg || v.npt != npt) continue;
        if (window_entries <= 0 ? v.wmax == 0 : v.wmax >= window_entries) {
            if (best < 0 || v.wmax < best) best = v.wmax;
        }
    }
    if (best < 0) return false;
    if (wmax_out) *wmax_out = best;
    return true;
}

template <class V, class A>
bool find_variant(int wg, int npt, int window_entries, int *wmax_out) {
    int best = -1;
    for (const auto &v : Table<V, A>::v) {
        if (v.wg != wg || v.npt != npt) continue;
        if (window_entries <= 0 ? v.wmax == 0 : v.wmax >= window_entries) {
            if (best < 0 || v.wmax < best) best = v.wmax;
        }
    }
    if (best < 0) return false;
    if (wmax_out) *wmax_out = best;
    return true;
}

template <class V, class A>
hipError_t launch_wave_any(const SpmvArgsT<V, A> &a, int wg, int npt, int window_entries, bool split,
                           hipStream_t s) {
    int wmax = 0;
    if (!find_wave_variant<V, A>(wg, npt, window_entries, &wmax)) return hipErrorInvalidValue;
    for (const auto &v : WaveTable<V, A>::v)
        if (v.wg == wg && v.npt == npt && v.wmax == wmax) return v.fn(a, split, true, s);
    return hipErrorInvalidValue;
}

template <class V, class A>
hipError_t launch_any(const SpmvArgsT<V, A> &a, int wg, int npt, int window_entries, bool tiled, bool split,
                      hipStream_t s) {
    int wmax = 0;
    if (!find_variant<V, A>(wg, npt, window_entries, &wmax)) return hipErrorInvalidValue;
    for (const auto &v : Table<V, A>::v)
        if (v.wg == wg && v.npt == npt && v.wmax == wmax) return v.fn(a, split, tiled, s);
    return hipErrorInvalidValue;
}
}  // namespace

bool spmv_variant_exists(int wg, int npt, int window_entries, int *wmax_out, Kind k) {
    switch (k) {
        case Kind::Pipe: return find_in<PipeTable<double, double>>(wg, npt, window_entries, wmax_out);
        case Kind::Waves: return find_wave_variant<double, double>(wg, npt, window_entries, wmax_out);
        case Kind::Scan: return find_in<ScanTable<double, double>>(wg, npt, window_entries, wmax_out);
        case Kind::Sorted: return find_in<SortedTable>(wg, npt, window_entries, wmax_out);
        case Kind::SortedScan: return find_in<SortedScanTable>(wg, npt, window_entries, wmax_out);
        case Kind::Compact: return find_in<CompactTable>(wg, npt, window_entries, wmax_out);
        default: return find_variant<double, double>(wg, npt, window_entries, wmax_out);
    }
}

bool spmv_lowp_variant_exists(int wg, int npt, Kind k) {
    switch (k) {
        case Kind::Pipe: return find_in<PipeTable<float, float>>(wg, npt, -1, nullptr);
        case Kind::Waves: return find_wave_variant<float, float>(wg, npt, -1, nullptr);
        case Kind::Scan: return find_in<ScanTable<float, float>>(wg, npt, -1, nullptr);
        case Kind::Sorted:
        case Kind::SortedScan:
        case Kind::Compact: return false;
        default: return find_variant<float, float>(wg, npt, -1, nullptr);
    }
}

hipError_t launch_spmv(const SpmvArgs &a, int wg, int npt, int window_entries, bool tiled, bool split,
                       hipStream_t s, Kind k) {
    switch (k) {
        case Kind::Pipe: return launch_in<PipeTable<double, double>>(a, wg, npt, window_entries, split, s);
        case Kind::Waves: return launch_wave_any(a, wg, npt, window_entries, split, s);
        case Kind::Scan: return launch_in<ScanTable<double, double>>(a, wg, npt, window_entries, split, s);
        case Kind::Sorted: return launch_in<SortedTable>(a, wg, npt, window_entries, split, s);
        case Kind::SortedScan: return launch_in<SortedScanTable>(a, wg, npt, window_entries, split, s);
        case Kind::Compact: return launch_in<CompactTable>(a, wg, npt, window_entries, split, s);
        default: return launch_any(a, wg, npt, window_entries, tiled, split, s);
    }
}

namespace {
template <class V>
hipError_t launch_lowp(const SpmvArgsT<V, float> &a, int wg, int npt, bool split, hipStream_t s, Kind k) {
    switch (k) {
        case Kind::Pipe: return launch_in<PipeTable<V, float>>(a, wg, npt, -1, split, s);
        case Kind::Waves: return launch_wave_any(a, wg, npt, -1, split, s);
        case Kind::Scan: return launch_in<ScanTable<V, float>>(a, wg, npt, -1, split, s);
        case Kind::Sorted:
        case Kind::SortedScan:
        case Kind::Compact: return hipErrorInvalidValue;
        default: return launch_any(a, wg, npt, -1, false, split, s);
    }
}
}  // namespace

hipError_t launch_spmv_f32(const SpmvArgsT<float, float> &a, int wg, int npt, bool split, hipStream_t s, Kind k) {
    return launch_lowp(a, wg, npt, split, s, k);
}

hipError_t launch_spmv_bf16(const SpmvArgsT<uint16_t, float> &a, int wg, int npt, bool split, hipStream_t s,
                            Kind k) {
    return launch_lowp(a, wg, npt, split, s, k);
}

hipError_t launch_batch(const BatchArgs &b, int grid, hipStream_t s) {
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(1), 0, s, b.queue);
    if (b.nitems > 0 && grid > 0)
        hipLaunchKernelGGL(batch_kernel<kBatchWG>, dim3(grid), dim3(kBatchWG), 0, s, b);
    return hipGetLastError();
}

int batch_grid() {
    int dev = 0, cus = 256, per = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<kBatchWG>, kBatchWG, 0) != hipSuccess || per < 1)
        per = 4;
    return cus * per;
}

static inline unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

int dot_groups(int64_t n) { return (int)std::min<int64_t>(kDotMaxGroups, std::max<int64_t>(1, (n + kDotWG - 1) / kDotWG)); }

template <class T>
hipError_t launch_dot(const T *a, const T *b, int64_t n, T *part, T *out, hipStream_t s) {
    const int g = dot_groups(n);
    hipLaunchKernelGGL(dot_partial_kernel<T>, dim3(g), dim3(kDotWG), 0, s, a, b, n, part);
    hipLaunchKernelGGL(sum_kernel<T>, dim3(1), dim3(kDotWG), 0, s, part, g, out);
    return hipGetLastError();
}
template hipError_t launch_dot<float>(const float *, const float *, int64_t, float *, float *, hipStream_t);
template hipError_t launch_dot<double>(const double *, const double *, int64_t, double *, double *, hipStream_t);

template <class T>
hipError_t launch_cg_start(const double *r, double inv_scale, T *rl, T *p, T *d, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cg_start_kernel<T>, dim3(grid_of(n)), dim3(256), 0, s, r, inv_scale, rl, p, d, n);
    return hipGetLastError();
}
template hipError_t launch_cg_start<float>(const double *, double, float *, float *, float *, int64_t, hipStream_t);
template hipError_t launch_cg_start<double>(const double *, double, double *, double *, double *, int64_t, hipStream_t);

template <class T>
hipError_t launch_cg_update(const T *rr, const T *pq, T *d, T *r, const T *p, const T *q, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cg_update_kernel<T>, dim3(grid_of(n)), dim3(256), 0, s, rr, pq, d, r, p, q, n);
    return hipGetLastError();
}
template hipError_t launch_cg_update<float>(const float *, const float *, float *, float *, const float *,
                                            const float *, int64_t, hipStream_t);
template hipError_t launch_cg_update<double>(const double *, const double *, double *, double *, const double *,
                                             const double *, int64_t, hipStream_t);

template <class T>
hipError_t launch_cg_direction(const T *rr, const T *rr_new, T *p, const T *r, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cg_direction_kernel<T>, dim3(grid_of(n)), dim3(256), 0, s, rr, rr_new, p, r, n);
    return hipGetLastError();
}
template hipError_t launch_cg_direction<float>(const float *, const float *, float *, const float *, int64_t,
                                               hipStream_t);
template hipError_t launch_cg_direction<double>(const double *, const double *, double *, const double *, int64_t,
                                                hipStream_t);

template <class T>
hipError_t launch_ir_update(double *x, const T *d, double scale, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(ir_update_kernel<T>, dim3(grid_of(n)), dim3(256), 0, s, x, d, scale, n);
    return hipGetLastError();
}
template hipError_t launch_ir_update<float>(double *, const float *, double, int64_t, hipStream_t);
template hipError_t launch_ir_update<double>(double *, const double *, double, int64_t, hipStream_t);

hipError_t launch_residual(const double *b, const double *ax, double *r, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(residual_kernel, dim3(grid_of(n)), dim3(256), 0, s, b, ax, r, n);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double *x, float *out, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(to_f32_kernel, dim3(grid_of(n)), dim3(256), 0, s, x, out, n);
    return hipGetLastError();
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
