// Precision mode: values stored in binary32 or bfloat16 with binary32
// accumulation, and a conjugate-gradient solve wrapped in binary64 iterative
// refinement (only the residual b - A x and the solution update are
// binary64).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "api_internal.h"
#include "kernels.h"

using namespace spx;

namespace spx {
void check_lowp_plan(const spx_plan_s &P, int32_t prec, bool need_device) {
    if (prec != SPX_PREC_F32 && prec != SPX_PREC_BF16) fail(SPX_EINVAL, "precision must be SPX_PREC_F32 or SPX_PREC_BF16");
    if (P.form == SPX_FORM_SPLIT) fail(SPX_EUNSUPPORTED, "the precision mode takes plain, SB or DB plans");
    const bool have = prec == SPX_PREC_F32 ? (P.vals32.size() == P.vals.size() && !P.vals.empty()) || P.nnz == 0
                                           : (P.vals16.size() == P.vals.size() && !P.vals.empty()) || P.nnz == 0;
    if (!have) fail(SPX_EINVAL, "spx_plan_add_lowp was not called for this precision");
    if (need_device && !P.on_device) fail(SPX_ENODEVICE, "plan has no device copy");
}

template <class V>
SpmvArgsT<V, float> lowp_args(const spx_plan_s &P, const V *vals, const float *x, float *y) {
    SpmvArgsT<V, float> a{};
    a.slot_ptr = (const int32_t *)P.d_slot_ptr->ptr;
    a.slot_row = nullptr;
    a.colidx = (const int32_t *)P.d_colidx->ptr;
    a.vals = vals;
    a.x = x;
    a.y = y;
    a.blk_desc = (const int32_t *)P.d_blk_desc->ptr;
    a.tiles = (const int32_t *)P.d_tiles->ptr;
    // workgroup blocks run untiled; wave blocks and pipelined tiles run the
    // plan's tiles
    const bool wave = P.tune.wave_blocks != 0 || P.tune.pipeline != 0;
    a.ntiles = (int32_t)(wave ? P.tiles.size() / 4 : P.blk_desc.size() / 4);
    a.xcd_remap = P.tune.xcd_remap;
    const auto &gp = wave ? P.xcd_tile_ptr : P.xcd_blk_ptr;
    std::copy(gp.begin(), gp.end(), a.xcd_ptr);
    a.n = P.n;
    a.long_seg_ptr = (const int32_t *)P.d_long_seg_ptr->ptr;
    a.partials = (double *)P.d_partials->ptr;
    a.counters = (uint32_t *)P.d_counters->ptr;
    return a;
}

hipError_t run_lowp(const spx_plan_s &P, int32_t prec, const float *x, float *y, hipStream_t s) {
    const int wg = P.tune.wg, npt = P.tune.nnz_per_block / block_threads(P.tune);
    const Kind k = kind_of(P.tune);
    if (prec == SPX_PREC_F32)
        return launch_spmv_f32(lowp_args(P, (const float *)P.d_vals32->ptr, x, y), wg, npt, false, s, k);
    return launch_spmv_bf16(lowp_args(P, (const uint16_t *)P.d_vals16->ptr, x, y), wg, npt, false, s, k);
}

// Schedules the precision mode runs: any kernel kind without an LDS window,
// row blocks untiled, of a shape that has a low-precision kernel.
bool lowp_schedule_ok(const Tune &t) {
    const Kind k = kind_of(t);
    if (t.window_entries > 0 || (k == Kind::Blocks && tiled(t))) return false;
    return spmv_lowp_variant_exists(t.wg, t.nnz_per_block / block_threads(t), k);
}
}  // namespace spx

namespace {

// bfloat16 keeps the upper 16 bits of a binary32.  Round to nearest, ties to
// even: the dropped half decides, and an exact half rounds to the even kept
// pattern.  NaNs stay NaN (quiet bit set); a carry out of the mantissa
// correctly steps the exponent (up to infinity).
uint16_t bf16_of(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t kept = u >> 16, dropped = u & 0xFFFFu;
    if (std::isnan(f)) return (uint16_t)(kept | 0x0040u);
    const bool up = dropped > 0x8000u || (dropped == 0x8000u && (kept & 1u));
    return (uint16_t)(kept + (up ? 1u : 0u));
}


// Device workspace of one solve.
struct Work {
    DevPtr r, ax, v[4], part, part64, scal;
    double *d(DevPtr &p) { return (double *)p->ptr; }
};

double read_scalar_d(const double *dev, hipStream_t s) {
    double h = 0.0;
    hip_check(hipMemcpyAsync(&h, dev, 8, hipMemcpyDeviceToHost, s), "scalar copy");
    hip_check(hipStreamSynchronize(s), "scalar copy");
    return h;
}

template <class T>
T read_scalar(const T *dev, hipStream_t s) {
    T h = 0;
    hip_check(hipMemcpyAsync(&h, dev, sizeof(T), hipMemcpyDeviceToHost, s), "scalar copy");
    hip_check(hipStreamSynchronize(s), "scalar copy");
    return h;
}

// Iterations between two reads of the residual norm by the host: each read
// waits for the stream, so reading every iteration would leave the GPU idle
// for a launch round trip per iteration.  The solve may therefore run up to
// kCheckEvery - 1 iterations past the first one that meets its tolerance
// (each only lowers the residual further; the update and direction kernels
// take a zero step once the residual or the curvature is exactly zero).
constexpr int32_t kCheckEvery = 8;

// Inner CG on A_low d = rhs with rhs = r / scale, in precision T, to relative
// residual inner_tol; d ends in w.v[3].  Returns the iterations taken.
template <class T>
int32_t inner_cg(spx_plan_s &P, int32_t prec, Work &w, double scale, double inner_tol, int32_t max_inner,
                 hipStream_t s) {
    const int64_t n = P.n;
    T *rl = (T *)w.v[0]->ptr, *p = (T *)w.v[1]->ptr, *q = (T *)w.v[2]->ptr, *d = (T *)w.v[3]->ptr;
    T *part = (T *)w.part->ptr, *sc = (T *)w.scal->ptr;  // sc[0], sc[1]: rr ping-pong; sc[2]: p.q
    hip_check(launch_cg_start<T>((const double *)w.r->ptr, 1.0 / scale, rl, p, d, n, s), "cg start");
    hip_check(launch_dot<T>(rl, rl, n, part, &sc[0], s), "cg dot");
    T rr = read_scalar(&sc[0], s);
    const double bn = std::sqrt((double)rr);
    int cur = 0;
    int32_t it = 0;
    while (it < max_inner && std::sqrt((double)rr) > inner_tol * bn) {
        if (prec == SPX_PREC_F64)
            hip_check(run_product(P, (const double *)p, (double *)q, 0, s), "cg spmv");
        else
            hip_check(run_lowp(P, prec, (const float *)p, (float *)q, s), "cg spmv");
        hip_check(launch_dot<T>(p, q, n, part, &sc[2], s), "cg dot");
        hip_check(launch_cg_update<T>(&sc[cur], &sc[2], d, rl, p, q, n, s), "cg update");
        hip_check(launch_dot<T>(rl, rl, n, part, &sc[1 - cur], s), "cg dot");
        hip_check(launch_cg_direction<T>(&sc[cur], &sc[1 - cur], p, rl, n, s), "cg direction");
        cur = 1 - cur;
        ++it;
        if (it % kCheckEvery == 0 || it == max_inner) {
            rr = read_scalar(&sc[cur], s);
            if (!std::isfinite((double)rr)) break;
        }
    }
    return it;
}

template <class T>
void solve(spx_plan_s &P, int32_t prec, const double *b, double *x, double tol, double inner_tol, int32_t max_outer,
           int32_t max_inner, spx_cg_stats *st, hipStream_t s) {
    const int64_t n = P.n;
    Work w;
    w.r = dev_alloc(n * 8 + 16);
    w.ax = dev_alloc(n * 8 + 16);
    for (auto &v : w.v) v = dev_alloc(n * sizeof(T) + 16);
    w.part = dev_alloc(dot_groups(n) * sizeof(T) + 16);
    w.part64 = dev_alloc(dot_groups(n) * 8 + 16);
    w.scal = dev_alloc(64);
    double *r = w.d(w.r), *ax = w.d(w.ax), *p64 = w.d(w.part64), *s64 = (double *)w.scal->ptr + 4;
    hip_check(launch_fill(x, 0, n, 0.0, s), "x init");
    hip_check(launch_dot<double>(b, b, n, p64, s64, s), "norm b");
    const double bn = std::sqrt(read_scalar_d(s64, s));
    hip_check(hipMemcpyAsync(r, b, n * 8, hipMemcpyDeviceToDevice, s), "r init");
    double rel = bn > 0 ? 1.0 : 0.0, rn = bn;
    int32_t outer = 0;
    int64_t inner = 0;
    while (rel > tol && outer < max_outer) {
        inner += inner_cg<T>(P, prec, w, rn, inner_tol, max_inner, s);
        hip_check(launch_ir_update<T>(x, (const T *)w.v[3]->ptr, rn, n, s), "ir update");
        hip_check(run_product(P, x, ax, 0, s), "residual spmv");
        hip_check(launch_residual(b, ax, r, n, s), "residual");
        hip_check(launch_dot<double>(r, r, n, p64, s64, s), "residual norm");
        rn = std::sqrt(read_scalar_d(s64, s));
        rel = rn / bn;
        ++outer;
        if (!std::isfinite(rel)) break;
    }
    st->outer = outer;
    st->inner = (int32_t)inner;
    st->rel_residual = rel;
}

}  // namespace

extern "C" {

spx_status spx_plan_add_lowp(spx_plan P, int32_t precision) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (precision != SPX_PREC_F32 && precision != SPX_PREC_BF16)
            fail(SPX_EINVAL, "precision must be SPX_PREC_F32 or SPX_PREC_BF16");
        if (P->form == SPX_FORM_SPLIT) fail(SPX_EUNSUPPORTED, "the precision mode takes plain, SB or DB plans");
        const size_t nz = P->vals.size();
        std::vector<float> v32(nz);
        for (size_t i = 0; i < nz; ++i) v32[i] = (float)P->vals[i];  // round to nearest even
        if (precision == SPX_PREC_F32) {
            P->vals32 = std::move(v32);
            if (P->on_device) {
                P->d_vals32 = dev_upload(P->vals32.data(), nz * 4, 16 * 4, nullptr);
                hip_check(hipStreamSynchronize(nullptr), "lowp upload");
            }
        } else {
            P->vals16.resize(nz);
            for (size_t i = 0; i < nz; ++i) P->vals16[i] = bf16_of(v32[i]);
            if (P->on_device) {
                P->d_vals16 = dev_upload(P->vals16.data(), nz * 2, 16 * 2, nullptr);
                hip_check(hipStreamSynchronize(nullptr), "lowp upload");
            }
        }
    });
}

spx_status spx_plan_export_lowp(spx_plan P, int32_t precision, void *vals) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        check_lowp_plan(*P, precision, false);
        if (!vals) return;
        if (precision == SPX_PREC_F32) std::memcpy(vals, P->vals32.data(), P->vals32.size() * 4);
        else std::memcpy(vals, P->vals16.data(), P->vals16.size() * 2);
    });
}

spx_status spx_spmv_lowp(spx_plan P, int32_t precision, const float *x, float *y, void *stream) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        check_lowp_plan(*P, precision, true);
        if (P->m > 0 && !y) fail(SPX_EINVAL, "y is NULL");
        if (P->nnz > 0 && !x) fail(SPX_EINVAL, "x is NULL");
        if (!lowp_schedule_ok(P->tune))
            fail(SPX_EUNSUPPORTED, "the precision mode runs schedules without an LDS window (row blocks untiled)");
        hip_check(run_lowp(*P, precision, x, y, (hipStream_t)stream), "spmv_lowp launch");
    });
}

spx_status spx_cg_ir(spx_plan P, int32_t precision, const double *b, double *x, double tol, double inner_tol,
                     int32_t max_outer, int32_t max_inner, spx_cg_stats *stats, void *stream) {
    spx_cg_stats st{};
    spx_status rc = guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        // CG needs a symmetric operator: SB/DB permute rows and columns
        // differently, so only the plain form keeps A symmetric
        if (P->form != SPX_FORM_PLAIN) fail(SPX_EUNSUPPORTED, "the solve takes a plain plan");
        if (P->m != P->n) fail(SPX_EINVAL, "the matrix must be square");
        if (precision != SPX_PREC_F64) check_lowp_plan(*P, precision, true);
        if (!P->on_device) fail(SPX_ENODEVICE, "plan has no device copy");
        // binary64 CG runs any schedule; the refined solves' inner products
        // need one that the precision mode runs
        if (precision != SPX_PREC_F64 && !lowp_schedule_ok(P->tune))
            fail(SPX_EUNSUPPORTED, "the solve runs schedules without an LDS window (row blocks untiled)");
        if (!(tol > 0) || !(inner_tol > 0) || max_outer < 1 || max_inner < 1)
            fail(SPX_EINVAL, "tol, inner_tol > 0 and max_outer, max_inner >= 1 required");
        if (P->n > 0 && (!b || !x)) fail(SPX_EINVAL, "NULL vector");
        auto t0 = std::chrono::steady_clock::now();
        hipStream_t s = (hipStream_t)stream;
        if (precision == SPX_PREC_F64)
            solve<double>(*P, precision, b, x, tol, inner_tol, max_outer, max_inner, &st, s);
        else
            solve<float>(*P, precision, b, x, tol, inner_tol, max_outer, max_inner, &st, s);
        hip_check(hipStreamSynchronize(s), "solve");
        st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    });
    if (stats) *stats = st;
    if (rc == SPX_OK && !(st.rel_residual <= tol)) {
        set_last_error("iterative refinement did not reach the tolerance");
        return SPX_ENOTCONV;
    }
    return rc;
}

}  // extern "C"
