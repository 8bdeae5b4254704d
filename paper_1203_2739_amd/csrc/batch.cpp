// Batched products: many matrices of uneven size, each with its own number
// of right-hand sides, run by one persistent launch (capturable in a HIP
// graph), with the schedule picked by measurement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <vector>

#include "api_internal.h"
#include "kernels.h"

using namespace spx;

constexpr int32_t kMultiSpan = 4096;

struct BatchTune {
    int32_t order = 0;         // 0: matrices by decreasing work, blocks in order; 1: all items by decreasing work
    int32_t span_div = 1;      // k > 1: item capacity kMultiSpan / span_div nonzeros
    int32_t reduce_iters = kReduceIters;
};

struct spx_batch_s {
    int32_t count = 0;
    std::vector<spx_plan> plans;
    std::vector<int32_t> k;
    std::vector<BatchMat> mats;      // device pointers; X and Y filled by bind
    std::vector<int32_t> items;
    std::vector<int64_t> item_bytes;
    DevPtr d_mats, d_items, d_queue, d_lsp, d_partials, d_counters;
    BatchTune tune;
    bool bound = false;
    int grid = 0;
    int64_t bytes = 0;               // algorithmic bytes of one run
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    ~spx_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

// Blocks of one matrix.  k == 1: the row-block SpMV rules (whole rows, at
// most 4 WG nonzeros from the 4-aligned start, at most WG rows, bounded
// reduction loop; longer rows in 4-aligned one-round segments).  k > 1:
// whole rows of at most `span` nonzeros in all, longer rows cut into
// segments of `span`.  Items are appended as {mat, s_lo, s_hi, z_lo, z_hi}
// with s_hi = -1 - l for a segment of long row l; lsp gets the partial-sum
// offsets of the long rows.
void matrix_items(int32_t mat, const std::vector<int32_t> &rp, int32_t k, int32_t span, int32_t iters,
                  std::vector<int32_t> &items, std::vector<int32_t> &lsp) {
    const int32_t m = (int32_t)rp.size() - 1;
    lsp.assign(1, 0);
    int32_t b0 = 0, nr = 0;
    int64_t lmax = 0;
    auto close = [&](int32_t s) {
        if (nr > 0) items.insert(items.end(), {mat, b0, s, rp[b0], rp[s]});
        b0 = s;
        nr = 0;
        lmax = 0;
    };
    for (int32_t s = 0; s < m; ++s) {
        const int64_t ps = rp[s], pe = rp[s + 1], len = pe - ps;
        const bool longrow = k == 1 ? (len > span - 3 || (len + 63) / 64 > iters) : len > span;
        if (longrow) {
            close(s);
            const int32_t lr = (int32_t)lsp.size() - 1;
            int32_t nseg = 0;
            if (k == 1) {
                for (int64_t z = ps, e = (ps & ~(int64_t)3) + span; z < pe; z = e, e += span, ++nseg)
                    items.insert(items.end(), {mat, s, -1 - lr, (int32_t)z, (int32_t)std::min<int64_t>(e, pe)});
            } else {
                for (int64_t z = ps; z < pe; z += span, ++nseg)
                    items.insert(items.end(), {mat, s, -1 - lr, (int32_t)z, (int32_t)std::min<int64_t>(z + span, pe)});
            }
            lsp.push_back(lsp.back() + nseg);
            b0 = s + 1;
            continue;
        }
        if (k == 1) {
            const int64_t zb = rp[b0] & ~(int64_t)3;
            const int64_t lm = std::max(lmax, len);
            int32_t q = kBatchWG / (nr + 1), g = 1;
            while (g * 2 <= q && g < 64) g *= 2;
            if (nr > 0 && (pe - zb > span || nr + 1 > kBatchWG || (lm + g - 1) / g > iters)) close(s);
        } else if (nr > 0 && pe - rp[b0] > span) {
            close(s);
        }
        ++nr;
        lmax = std::max(lmax, len);
    }
    close(m);
}

void build_items(spx_batch_s &B) {
    const int32_t cnt = B.count;
    std::vector<std::vector<int32_t>> its(cnt), lsps(cnt);
    for (int32_t i = 0; i < cnt; ++i) {
        const spx_plan_s &P = *B.plans[i];
        const int32_t k = B.k[i];
        // k > 1: items of about kMultiSpan nonzeros (rows longer than that are
        // cut into segments of that length)
        const int32_t span = k == 1 ? 4 * kBatchWG : std::max(64, kMultiSpan / B.tune.span_div);
        matrix_items(i, P.slot_ptr, k, span, B.tune.reduce_iters, its[i], lsps[i]);
        B.mats[i].span = span;
    }
    // long-row scratch of all matrices in one allocation each
    std::vector<int32_t> lsp_all;
    std::vector<int64_t> lsp_off(cnt), part_off(cnt), cnt_off(cnt);
    int64_t parts = 0, ctrs = 0;
    for (int32_t i = 0; i < cnt; ++i) {
        lsp_off[i] = (int64_t)lsp_all.size();
        lsp_all.insert(lsp_all.end(), lsps[i].begin(), lsps[i].end());
        part_off[i] = parts;
        cnt_off[i] = ctrs;
        parts += (int64_t)lsps[i].back() * B.k[i];
        ctrs += (int64_t)lsps[i].size() - 1;
    }
    B.d_lsp = dev_upload(lsp_all.data(), lsp_all.size() * 4, 16, nullptr);
    B.d_partials = dev_alloc(parts * 8 + 16);
    B.d_counters = dev_alloc(ctrs * 4 + 16);
    hip_check(hipMemset(B.d_counters->ptr, 0, ctrs * 4 + 16), "batch counters");
    for (int32_t i = 0; i < cnt; ++i) {
        B.mats[i].long_seg_ptr = (const int32_t *)B.d_lsp->ptr + lsp_off[i];
        B.mats[i].partials = (double *)B.d_partials->ptr + part_off[i];
        B.mats[i].counters = (uint32_t *)B.d_counters->ptr + cnt_off[i];
    }
    // work of an item: streamed matrix bytes, gathered x and written y
    auto cost = [&](const int32_t *it) {
        const int64_t nz = it[4] - it[3], k = B.k[it[0]];
        const int64_t rows = it[2] >= 0 ? it[2] - it[1] : 1;
        return nz * (12 + 8 * k) + rows * 8 * k;
    };
    std::vector<const int32_t *> order;
    std::vector<int32_t> mat_order(cnt);
    std::iota(mat_order.begin(), mat_order.end(), 0);
    std::vector<int64_t> mat_work(cnt, 0);
    for (int32_t i = 0; i < cnt; ++i)
        for (size_t t = 0; t < its[i].size(); t += 5) mat_work[i] += cost(&its[i][t]);
    std::stable_sort(mat_order.begin(), mat_order.end(), [&](int32_t a, int32_t b) { return mat_work[a] > mat_work[b]; });
    for (int32_t i : mat_order)
        for (size_t t = 0; t < its[i].size(); t += 5) order.push_back(&its[i][t]);
    if (B.tune.order == 1)
        std::stable_sort(order.begin(), order.end(), [&](const int32_t *a, const int32_t *b) { return cost(a) > cost(b); });
    B.items.clear();
    B.item_bytes.clear();
    for (const int32_t *it : order) {
        B.items.insert(B.items.end(), it, it + 5);
        B.item_bytes.push_back(cost(it));
    }
    B.d_items = dev_upload(B.items.data(), B.items.size() * 4, 16, nullptr);
    if (B.bound) B.d_mats = dev_upload(B.mats.data(), B.mats.size() * sizeof(BatchMat), 0, nullptr);
    hip_check(hipStreamSynchronize(nullptr), "batch upload");
    if (B.exec) {  // a captured graph holds the old item table
        (void)hipGraphExecDestroy(B.exec);
        (void)hipGraphDestroy(B.graph);
        B.exec = nullptr;
        B.graph = nullptr;
    }
}

BatchArgs args_of(spx_batch_s &B) {
    BatchArgs a{};
    a.mats = (const BatchMat *)B.d_mats->ptr;
    a.items = (const int32_t *)B.d_items->ptr;
    a.nitems = (int32_t)(B.items.size() / 5);
    a.queue = (uint32_t *)B.d_queue->ptr;
    return a;
}

void run(spx_batch_s &B, hipStream_t s) {
    if (!B.bound) fail(SPX_EINVAL, "spx_batch_bind was not called");
    hip_check(launch_batch(args_of(B), B.grid, s), "batch launch");
}

}  // namespace

extern "C" {

spx_status spx_batch_create(int32_t count, const spx_plan *plans, const int32_t *nrhs, spx_batch *out) {
    return guarded([&] {
        if (!out) fail(SPX_EINVAL, "out is NULL");
        *out = nullptr;
        if (count < 0 || (count > 0 && (!plans || !nrhs))) fail(SPX_EINVAL, "bad batch description");
        std::unique_ptr<spx_batch_s> B(new spx_batch_s());
        B->count = count;
        for (int32_t i = 0; i < count; ++i) {
            spx_plan P = plans[i];
            if (!P) fail(SPX_EINVAL, "NULL plan in batch");
            if (P->form == SPX_FORM_SPLIT) fail(SPX_EUNSUPPORTED, "batched products take plain, SB or DB plans");
            if (!P->on_device) fail(SPX_ENODEVICE, "plan has no device copy");
            if (nrhs[i] < 1 || nrhs[i] > 64) fail(SPX_EINVAL, "right-hand sides per matrix must be 1..64");
            B->plans.push_back(P);
            B->k.push_back(nrhs[i]);
            BatchMat M{};
            M.slot_ptr = (const int32_t *)P->d_slot_ptr->ptr;
            M.colidx = (const int32_t *)P->d_colidx->ptr;
            M.vals = (const double *)P->d_vals->ptr;
            M.k = nrhs[i];
            B->mats.push_back(M);
            B->bytes += 12 * P->nnz + 4 * ((int64_t)P->m + 1) + 8 * (int64_t)nrhs[i] * ((int64_t)P->n + P->m);
        }
        B->d_queue = dev_alloc(64);
        B->grid = batch_grid();
        build_items(*B);
        *out = B.release();
    });
}

void spx_batch_destroy(spx_batch B) { delete B; }

spx_status spx_batch_bind(spx_batch B, const double *const *X, const int64_t *ldx, double *const *Y,
                          const int64_t *ldy) {
    return guarded([&] {
        if (!B) fail(SPX_EINVAL, "NULL handle");
        if (B->count > 0 && (!X || !ldx || !Y || !ldy)) fail(SPX_EINVAL, "NULL vector table");
        for (int32_t i = 0; i < B->count; ++i) {
            const spx_plan_s &P = *B->plans[i];
            const int32_t k = B->k[i];
            if (ldx[i] < k || ldy[i] < k) fail(SPX_EINVAL, "leading dimensions must be >= the right-hand sides");
            if (k == 1 && (ldx[i] != 1 || ldy[i] != 1)) fail(SPX_EINVAL, "one right-hand side needs unit strides");
            if ((P.n > 0 && P.nnz > 0 && !X[i]) || (P.m > 0 && !Y[i])) fail(SPX_EINVAL, "NULL vector");
            B->mats[i].X = X[i];
            B->mats[i].Y = Y[i];
            B->mats[i].ldx = ldx[i];
            B->mats[i].ldy = ldy[i];
        }
        B->d_mats = dev_upload(B->mats.data(), B->mats.size() * sizeof(BatchMat), 16, nullptr);
        hip_check(hipStreamSynchronize(nullptr), "batch bind");
        B->bound = true;
        if (B->exec) {  // the graph holds the old pointer table
            (void)hipGraphExecDestroy(B->exec);
            (void)hipGraphDestroy(B->graph);
            B->exec = nullptr;
            B->graph = nullptr;
        }
    });
}

spx_status spx_batch_run(spx_batch B, void *stream) {
    return guarded([&] {
        if (!B) fail(SPX_EINVAL, "NULL handle");
        run(*B, (hipStream_t)stream);
    });
}

spx_status spx_batch_capture(spx_batch B) {
    return guarded([&] {
        if (!B) fail(SPX_EINVAL, "NULL handle");
        if (!B->bound) fail(SPX_EINVAL, "spx_batch_bind was not called");
        if (!B->cap_stream) hip_check(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking), "stream");
        if (B->exec) {
            (void)hipGraphExecDestroy(B->exec);
            (void)hipGraphDestroy(B->graph);
            B->exec = nullptr;
            B->graph = nullptr;
        }
        hip_check(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        hipError_t e = launch_batch(args_of(*B), B->grid, B->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(B->cap_stream, &g);
        hip_check(e, "captured launch");
        hip_check(e2, "end capture");
        B->graph = g;
        hip_check(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0), "graph instantiate");
    });
}

spx_status spx_batch_replay(spx_batch B, void *stream) {
    return guarded([&] {
        if (!B) fail(SPX_EINVAL, "NULL handle");
        if (!B->exec) fail(SPX_EINVAL, "spx_batch_capture was not called (or the batch changed since)");
        hip_check(hipGraphLaunch(B->exec, (hipStream_t)stream), "graph launch");
    });
}

spx_status spx_batch_autotune(spx_batch B, int32_t reps, spx_batch_config *best, void *stream) {
    return guarded([&] {
        if (!B) fail(SPX_EINVAL, "NULL handle");
        if (!B->bound) fail(SPX_EINVAL, "spx_batch_bind was not called");
        if (reps < 1) reps = 3;
        hipStream_t s = (hipStream_t)stream;
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        BatchTune bestt = B->tune;
        float bestms = -1.0f;
        for (int32_t order : {0, 1})
            for (int32_t sd : {1, 2})
                for (int32_t it : {16, 64}) {
                    B->tune = BatchTune{order, sd, it};
                    build_items(*B);
                    run(*B, s);  // warm-up
                    hip_check(hipEventRecord(e0, s), "event");
                    for (int32_t r = 0; r < reps; ++r) run(*B, s);
                    hip_check(hipEventRecord(e1, s), "event");
                    hip_check(hipEventSynchronize(e1), "event");
                    float ms = 0.0f;
                    hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
                    ms /= (float)reps;
                    if (bestms < 0 || ms < bestms) {
                        bestms = ms;
                        bestt = B->tune;
                    }
                }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        B->tune = bestt;
        build_items(*B);
        if (best) {
            best->order = bestt.order;
            best->span_div = bestt.span_div;
            best->reduce_iters = bestt.reduce_iters;
            best->ms = bestms;
        }
    });
}

spx_status spx_batch_configure(spx_batch B, const spx_batch_config *cfg) {
    return guarded([&] {
        if (!B || !cfg) fail(SPX_EINVAL, "NULL argument");
        if ((cfg->order != 0 && cfg->order != 1) || cfg->span_div < 1 || cfg->span_div > 64 ||
            cfg->reduce_iters < 1 || cfg->reduce_iters > 64)
            fail(SPX_EINVAL, "bad batch configuration");
        B->tune = BatchTune{cfg->order, cfg->span_div, cfg->reduce_iters};
        build_items(*B);
    });
}

spx_status spx_batch_info(spx_batch B, int32_t *nitems, int64_t *bytes, int32_t *grid) {
    return guarded([&] {
        if (!B) fail(SPX_EINVAL, "NULL handle");
        if (nitems) *nitems = (int32_t)(B->items.size() / 5);
        if (bytes) *bytes = B->bytes;
        if (grid) *grid = B->grid;
    });
}

spx_status spx_spmv_batched(int32_t count, const spx_plan *plans, const int32_t *nrhs, const double *const *X,
                            const int64_t *ldx, double *const *Y, const int64_t *ldy, void *stream) {
    spx_batch B = nullptr;
    spx_status rc = spx_batch_create(count, plans, nrhs, &B);
    if (rc == SPX_OK) rc = spx_batch_bind(B, X, ldx, Y, ldy);
    if (rc == SPX_OK) rc = spx_batch_run(B, stream);
    if (rc == SPX_OK)
        rc = guarded([&] { hip_check(hipStreamSynchronize((hipStream_t)stream), "batched products"); });
    spx_batch_destroy(B);
    return rc;
}

}  // extern "C"
