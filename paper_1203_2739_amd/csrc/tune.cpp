// Schedule autotuning of a plan: the candidate schedules are timed on the
// caller's vectors with HIP events and the fastest is kept, as OSKI tunes
// its kernel to the matrix by measurement (Section 5.2).
#include <hip/hip_runtime.h>

#include <vector>

#include "api_internal.h"

using namespace spx;

namespace spx {

// Candidate schedules in the order they are tried: the one-block-per-
// workgroup kernel at every workgroup size, with lane groups per row, with
// the segmented-scan row sums and with gather-sorted blocks; wave blocks at
// every workgroup
// size; wave blocks in tiles per row group with an LDS x window, sized so
// that the tiles of a group are about the workgroups one XCD (32 CUs) keeps
// resident: one 1024- or 512-thread workgroup per CU with a 120 or 128 KB
// window, two 256-thread workgroups with 64 KB; then pipelined tiles.
const std::vector<spx_tune> &autotune_candidates() {
    static const std::vector<spx_tune> c = [] {
        std::vector<spx_tune> v;
        auto add = [&v](int wg, int npt, int wave = 0, int tiles = 0, int window = 0, int pipe = 0,
                        int scan = 0, int sorted = 0) {
            spx_tune t{};
            t.wg_size = wg;
            t.nnz_per_block = (wave ? 64 : wg) * npt;
            t.wave_blocks = wave;
            t.tiles_per_group = tiles;
            t.window_entries = window;
            t.pipeline = pipe;
            t.scan_reduce = scan;
            t.sort_gathers = sorted;
            v.push_back(t);
        };
        add(128, 4);
        add(64, 8);
        add(256, 4);
        add(512, 4);
        add(128, 8);
        add(256, 8);
        for (int wg : {128, 256, 512, 1024}) add(wg, 4, 0, 0, 0, 0, 1);
        for (int wg : {128, 256, 512, 1024}) add(wg, 4, 0, 0, 0, 0, 0, 1);
        add(256, 8, 0, 0, 0, 0, 0, 1);
        add(512, 8, 0, 0, 0, 0, 0, 1);
        for (int wg : {256, 512, 1024}) add(wg, 4, 0, 0, 0, 0, 1, 1);
        add(256, 8, 0, 0, 0, 0, 1, 1);
        add(512, 8, 0, 0, 0, 0, 1, 1);
        for (int wg : {128, 256, 512}) {
            add(wg, 4);
            v.back().compact_index = 1;
        }
        add(256, 4, 1);
        add(512, 4, 1);
        add(1024, 4, 1);
        add(512, 8, 1);
        add(1024, 4, 1, 32, 15360);
        add(512, 4, 1, 32, 16384);
        add(256, 4, 1, 64, 8192);
        // pipelined tiles, about as many per row group as one XCD keeps
        // resident (4 workgroups of 512 or 8 of 256 threads on each of 32 CUs)
        add(512, 4, 0, 128, 0, 1);
        add(256, 4, 0, 256, 0, 1);
        add(256, 8, 0, 128, 0, 1);
        add(512, 4, 0, 64, 0, 1);
        return v;
    }();
    return c;
}

}  // namespace spx

namespace {

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    Events() {
        hip_check(hipEventCreate(&a), "event");
        hip_check(hipEventCreate(&b), "event");
    }
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

void retune_to(spx_plan_s &P, const spx_tune &t) {
    spx_tune u = t;
    if (u.window_entries == 0) u.window_entries = -1;
    P.tune = resolve_tune(&u, P.form);
    build_schedule(P);
    hip_check(hipDeviceSynchronize(), "autotune");  // no product of the old schedule in flight
    upload_schedule(P, nullptr);
}

}  // namespace

extern "C" {

int32_t spx_autotune_candidate(int32_t i, spx_tune *out) {
    const auto &c = autotune_candidates();
    if (i >= 0 && i < (int32_t)c.size() && out) *out = c[i];
    return (int32_t)c.size();
}

spx_status spx_plan_autotune(spx_plan P, int32_t precision, const void *x, void *y, int32_t reps,
                             spx_tune *chosen, float *ms, float *cand_ms, void *stream) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (!P->on_device) fail(SPX_ENODEVICE, "plan has no device copy (host-only matrix)");
        if (reps < 1) fail(SPX_EINVAL, "reps must be >= 1");
        if (P->m > 0 && !y) fail(SPX_EINVAL, "y is NULL");
        if (P->nnz > 0 && !x) fail(SPX_EINVAL, "x is NULL");
        if (precision != SPX_PREC_F64) check_lowp_plan(*P, precision, true);
        hipStream_t s = (hipStream_t)stream;
        auto product = [&]() {
            hipError_t e = precision == SPX_PREC_F64
                               ? run_product(*P, (const double *)x, (double *)y, 0, s)
                               : run_lowp(*P, precision, (const float *)x, (float *)y, s);
            hip_check(e, "autotune product");
        };
        Events ev;
        const auto &cands = autotune_candidates();
        int best = -1;
        float best_ms = 0.0f;
        for (size_t c = 0; c < cands.size(); ++c) {
            // the precision mode runs no tiles of workgroup blocks and no window
            if (cand_ms) cand_ms[c] = -1.0f;
            if (precision != SPX_PREC_F64) {
                Tune r;
                bool ok = true;
                try {
                    spx_tune u = cands[c];
                    if (u.window_entries == 0) u.window_entries = -1;
                    r = resolve_tune(&u, P->form);
                } catch (const Error &) {
                    ok = false;
                }
                if (!ok || !lowp_schedule_ok(r)) continue;
            }
            // indices cannot carry the offsets
            if (cands[c].sort_gathers && (int64_t)P->n > ((int64_t)1 << pack_shift(cands[c].nnz_per_block))) continue;
            retune_to(*P, cands[c]);
            for (int w = 0; w < 2; ++w) product();
            hip_check(hipEventRecord(ev.a, s), "event record");
            for (int r = 0; r < reps; ++r) product();
            hip_check(hipEventRecord(ev.b, s), "event record");
            hip_check(hipEventSynchronize(ev.b), "event sync");
            float t = 0.0f;
            hip_check(hipEventElapsedTime(&t, ev.a, ev.b), "elapsed");
            t /= (float)reps;
            if (cand_ms) cand_ms[c] = t;
            if (best < 0 || t < best_ms) {
                best = (int)c;
                best_ms = t;
            }
        }
        retune_to(*P, cands[best]);
        if (chosen) {
            *chosen = spx_tune{};
            chosen->wg_size = P->tune.wg;
            chosen->nnz_per_block = P->tune.nnz_per_block;
            chosen->blocks_per_tile = P->tune.blocks_per_tile;
            chosen->window_entries = P->tune.window_entries;
            chosen->xcd_remap = P->tune.xcd_remap ? 1 : -1;
            chosen->reduce_iters = P->tune.reduce_iters;
            chosen->tiles_per_group = P->tune.tiles_per_group;
            chosen->wave_blocks = P->tune.wave_blocks;
            chosen->pipeline = P->tune.pipeline;
            chosen->scan_reduce = P->tune.scan;
            chosen->sort_gathers = P->tune.sort_gathers;
            chosen->compact_index = P->tune.compact_index;
        }
        if (ms) *ms = best_ms;
    });
}

}  // extern "C"
