// C interface of libspx: validation, handles, device residency and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>

#include "api_internal.h"
#include "kernels.h"

namespace spx {

thread_local std::string g_err;

void set_last_error(const std::string &msg) { g_err = msg; }

[[noreturn]] void fail(spx_status code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(SPX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

DevBuf::~DevBuf() {
    if (ptr) (void)hipFree(ptr);
}

DevPtr dev_alloc(size_t bytes) {
    auto b = std::make_shared<DevBuf>();
    b->bytes = bytes;
    if (bytes) {
        hipError_t e = hipMalloc(&b->ptr, bytes);
        if (e != hipSuccess) {
            b->ptr = nullptr;
            (void)hipGetLastError();
            fail(e == hipErrorOutOfMemory ? SPX_ENOMEM : SPX_EHIP,
                 std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    return b;
}

DevPtr dev_upload(const void *host, size_t bytes, size_t pad_bytes, void *stream) {
    DevPtr b = dev_alloc(bytes + pad_bytes);
    hipStream_t s = (hipStream_t)stream;
    if (bytes) hip_check(hipMemcpyAsync(b->ptr, host, bytes, hipMemcpyHostToDevice, s), "upload");
    if (pad_bytes)
        hip_check(hipMemsetAsync((char *)b->ptr + bytes, 0, pad_bytes, s), "upload padding");
    return b;
}

Tune resolve_tune(const spx_tune *t, int form) {
    (void)form;
    Tune r;
    if (t) {
        if (t->wg_size) r.wg = t->wg_size;
        if (t->nnz_per_block) r.nnz_per_block = t->nnz_per_block;
        if (t->blocks_per_tile) r.blocks_per_tile = t->blocks_per_tile;
        if (t->window_entries) r.window_entries = t->window_entries;
        if (t->xcd_remap) r.xcd_remap = t->xcd_remap > 0 ? 1 : 0;
        if (t->reduce_iters) r.reduce_iters = t->reduce_iters;
        if (t->tiles_per_group) r.tiles_per_group = t->tiles_per_group;
        if (t->wave_blocks) r.wave_blocks = t->wave_blocks > 0 ? 1 : 0;
        if (t->pipeline) r.pipeline = t->pipeline > 0 ? 1 : 0;
        if (t->scan_reduce) r.scan = t->scan_reduce > 0 ? 1 : 0;
        if (t->sort_gathers) r.sort_gathers = t->sort_gathers > 0 ? 1 : 0;
        if (t->compact_index) r.compact_index = t->compact_index > 0 ? 1 : 0;
    }
    if (r.wg != 64 && r.wg != 128 && r.wg != 256 && r.wg != 512 && r.wg != 1024)
        fail(SPX_EINVAL, "wg_size must be 64, 128, 256, 512 or 1024");
    if (r.tiles_per_group < 0 || r.tiles_per_group > 4096) fail(SPX_EINVAL, "tiles_per_group must be in 0..4096");
    if (r.wave_blocks && r.wg < 256) fail(SPX_EINVAL, "wave_blocks needs wg_size 256, 512 or 1024");
    if (r.pipeline && r.wave_blocks) fail(SPX_EINVAL, "pipeline and wave_blocks exclude each other");
    if (r.pipeline && r.tiles_per_group == 0 && r.blocks_per_tile <= 1)
        fail(SPX_EINVAL, "pipeline needs tiles (tiles_per_group, or blocks_per_tile > 1)");
    if (r.scan && (r.wave_blocks || r.pipeline || r.tiles_per_group > 0 || r.blocks_per_tile > 1 ||
                   (t && t->window_entries > 0)))
        fail(SPX_EINVAL, "scan_reduce runs one block per workgroup: no tiles, windows, wave blocks or pipeline");
    if (r.sort_gathers && (r.wave_blocks || r.pipeline || r.tiles_per_group > 0 || r.blocks_per_tile > 1 ||
                           (t && t->window_entries > 0)))
        fail(SPX_EINVAL, "sort_gathers runs one block per workgroup: no tiles, windows, wave blocks or pipeline");
    if (r.compact_index && (r.sort_gathers || r.scan || r.wave_blocks || r.pipeline || r.tiles_per_group > 0 ||
                            r.blocks_per_tile > 1 || (t && t->window_entries > 0)))
        fail(SPX_EINVAL, "compact_index runs workgroup row blocks alone: no tiles, windows, wave blocks, pipeline, "
                         "scan_reduce or sort_gathers");
    if (!r.wave_blocks && !r.pipeline && !r.scan && !r.sort_gathers && r.wg == 1024 &&
        (r.tiles_per_group == 0 || (t && t->window_entries <= 0)))
        fail(SPX_EUNSUPPORTED, "wg_size 1024 runs only scan blocks, gather-sorted blocks, wave blocks, pipelined "
                               "tiles or tiles per row group with an LDS window");
    const int32_t bt = block_threads(r);
    if (!t || !t->nnz_per_block) r.nnz_per_block = (bt == 64 && !r.wave_blocks ? 8 : kDefaultNpt) * bt;
    if (r.nnz_per_block != 4 * bt && r.nnz_per_block != 8 * bt)
        fail(SPX_EINVAL, r.wave_blocks ? "nnz_per_block must be 256 or 512 with wave_blocks (4 or 8 per lane)"
                                       : "nnz_per_block must be 4 or 8 times wg_size (nonzeros per thread)");
    if (r.reduce_iters < 1 || r.reduce_iters > 64) fail(SPX_EINVAL, "reduce_iters must be in 1..64");
    if (r.blocks_per_tile < 1) fail(SPX_EINVAL, "blocks_per_tile must be >= 1");
    if (r.window_entries < 0) r.window_entries = -1;
    int wmax = 0;
    if (!spmv_variant_exists(r.wg, r.nnz_per_block / bt, r.window_entries, &wmax, kind_of(r)))
        fail(SPX_EUNSUPPORTED, "no kernel variant for this wg_size / window");
    return r;
}

}  // namespace spx

using namespace spx;

static constexpr size_t kPadEntries = 16;

static void validate_csr(int32_t m, int32_t n, int64_t nnz, const int32_t *rowptr,
                         const int32_t *colidx, const double *vals) {
    if (m < 0 || n < 0) fail(SPX_EINVAL, "negative dimension");
    if (nnz < 0 || nnz > (int64_t)INT32_MAX - 64) fail(SPX_EINVAL, "nnz out of range");
    if (!rowptr) fail(SPX_EINVAL, "rowptr is NULL");
    if (nnz > 0 && (!colidx || !vals)) fail(SPX_EINVAL, "colidx or vals is NULL");
    if (rowptr[0] != 0) fail(SPX_EINVAL, "rowptr[0] != 0");
    if ((int64_t)rowptr[m] != nnz) fail(SPX_EINVAL, "rowptr[m] != nnz");
    for (int32_t i = 0; i < m; ++i) {
        if (rowptr[i + 1] < rowptr[i]) fail(SPX_EINVAL, "rowptr decreases at row " + std::to_string(i));
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t c = colidx[p];
            if (c < 0 || c >= n) fail(SPX_EINVAL, "column index out of range in row " + std::to_string(i));
            if (p > rowptr[i] && colidx[p - 1] >= c)
                fail(SPX_EINVAL, "column indices not strictly increasing in row " + std::to_string(i));
        }
    }
}

static spx_mat_s *make_mat(int32_t m, int32_t n, int64_t nnz, const int32_t *rowptr,
                           const int32_t *colidx, const double *vals) {
    validate_csr(m, n, nnz, rowptr, colidx, vals);
    auto *A = new spx_mat_s();
    A->h.m = m;
    A->h.n = n;
    A->h.nnz = nnz;
    A->h.rowptr.assign(rowptr, rowptr + m + 1);
    if (nnz) {
        A->h.colidx.assign(colidx, colidx + nnz);
        A->h.vals.assign(vals, vals + nnz);
    }
    return A;
}

static void upload_mat(spx_mat_s &A, void *stream) {
    const CsrHost &h = A.h;
    A.d_rowptr = dev_upload(h.rowptr.data(), h.rowptr.size() * 4, 0, stream);
    A.d_colidx = dev_upload(h.colidx.data(), h.colidx.size() * 4, kPadEntries * 4, stream);
    A.d_vals = dev_upload(h.vals.data(), h.vals.size() * 8, kPadEntries * 8, stream);
    hip_check(hipStreamSynchronize((hipStream_t)stream), "upload");
    A.on_device = true;
}

namespace spx {
void upload_plan(spx_plan_s &P, const spx_mat_s &A, void *stream) {
    if (!A.on_device) {
        P.on_device = false;
        return;
    }
    if (P.form == SPX_FORM_PLAIN) {
        P.d_slot_ptr = A.d_rowptr;
        P.d_colidx = A.d_colidx;
        P.d_vals = A.d_vals;
    } else {
        P.d_slot_ptr = dev_upload(P.slot_ptr.data(), P.slot_ptr.size() * 4, 0, stream);
        P.d_colidx = dev_upload(P.colidx.data(), P.colidx.size() * 4, kPadEntries * 4, stream);
        P.d_vals = dev_upload(P.vals.data(), P.vals.size() * 8, kPadEntries * 8, stream);
        if (!P.slot_row.empty())
            P.d_slot_row = dev_upload(P.slot_row.data(), P.slot_row.size() * 4, 0, stream);
        if (!P.row_perm.empty())
            P.d_row_perm = dev_upload(P.row_perm.data(), P.row_perm.size() * 4, 0, stream);
        if (!P.col_perm.empty())
            P.d_col_perm = dev_upload(P.col_perm.data(), P.col_perm.size() * 4, 0, stream);
    }
    upload_schedule(P, stream);
    P.on_device = true;
}

// Device copies of the schedule and of the long-slot scratch (partial sums
// and arrival counters, which start at zero).
void upload_schedule(spx_plan_s &P, void *stream) {
    P.d_blk_desc = dev_upload(P.blk_desc.data(), P.blk_desc.size() * 4, 16, stream);
    if (P.tune.sort_gathers) {
        P.d_colidx_sorted = dev_upload(P.colidx_sorted.data(), P.colidx_sorted.size() * 4, 16, stream);
        P.d_vals_sorted = dev_upload(P.vals_sorted.data(), P.vals_sorted.size() * 8, 16, stream);
        P.d_sorted_ofs = dev_upload(P.sorted_ofs.data(), P.sorted_ofs.size() * 4, 16, stream);
    } else {
        P.d_colidx_sorted.reset();
        P.d_vals_sorted.reset();
        P.d_sorted_ofs.reset();
    }
    if (P.tune.compact_index) {
        P.d_colidx16 = dev_upload(P.colidx16.data(), P.colidx16.size() * 2, kPadEntries * 2, stream);
        P.d_blk_cbase = dev_upload(P.blk_cbase.data(), P.blk_cbase.size() * 4, 16, stream);
    } else {
        P.d_colidx16.reset();
        P.d_blk_cbase.reset();
    }
    P.d_tiles = dev_upload(P.tiles.data(), P.tiles.size() * 4, 16, stream);
    P.d_long_seg_ptr = dev_upload(P.long_seg_ptr.data(), P.long_seg_ptr.size() * 4, 16, stream);
    size_t nlong = P.long_seg_ptr.empty() ? 0 : P.long_seg_ptr.size() - 1;
    size_t nseg = nlong ? (size_t)P.long_seg_ptr.back() : 0;
    P.d_partials = dev_alloc(nseg * 8 + 16);
    P.d_counters = dev_alloc(nlong * 4 + 16);
    hip_check(hipMemsetAsync(P.d_counters->ptr, 0, nlong * 4 + 16, (hipStream_t)stream), "counter init");
    hip_check(hipStreamSynchronize((hipStream_t)stream), "plan upload");
}
}  // namespace spx

// A plan of form SB, DB or split from a given partition (leaves as given
// by r), with the schedule `tune` (NULL: library default), uploaded when A
// has a device copy.
spx_plan_s *spx::plan_from_partition(const spx_mat_s &A, int form, int32_t K, const PartitionResult &r,
                                     const spx_tune *tune) {
    std::unique_ptr<spx_plan_s> P(new spx_plan_s());
    P->K = K;
    if (form == SPX_FORM_SPLIT) plan_from_split(*P, A.h, r);
    else plan_from_rowparts(*P, A.h, r, form == SPX_FORM_DB);
    spx_tune t{};
    if (tune) t = *tune;
    P->tune = resolve_tune(&t, P->form);
    build_schedule(*P);
    upload_plan(*P, A, nullptr);
    return P.release();
}

static void apply_tune(spx_plan_s &P, const spx_tune *tune, int64_t window_bytes) {
    spx_tune t{};
    if (tune) t = *tune;
    (void)window_bytes;  // leaves are sized by the partition; LDS windows only on request
    P.tune = resolve_tune(&t, P.form);
    build_schedule(P);
}

static void write_outputs(const spx_plan_s &P, int32_t *row_perm, int32_t *col_perm) {
    if (row_perm) std::copy(P.row_perm.begin(), P.row_perm.end(), row_perm);
    if (col_perm) std::copy(P.col_perm.begin(), P.col_perm.end(), col_perm);
}

static spx_status build_reordered(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed,
                                  Model model, int32_t *row_perm, int32_t *col_perm,
                                  int32_t *part_out, const spx_tune *tune, spx_plan *out,
                                  int64_t row_net_cost = kSplitRowNetCostDefault) {
    return guarded([&] {
        if (!A || !out) fail(SPX_EINVAL, "NULL handle");
        if (K < 1) fail(SPX_EINVAL, "K must be >= 1");
        if (window_bytes < 0) fail(SPX_EINVAL, "window_bytes must be >= 0");
        *out = nullptr;
        std::unique_ptr<spx_plan_s> P(new spx_plan_s());
        P->K = K;
        const CsrHost &h = A->h;
        PartitionResult r = partition(h, model, K, window_bytes / 8, seed, row_net_cost);
        if (model == Model::ColumnNet) plan_from_rowparts(*P, h, r, false);
        else if (model == Model::ERowColumnNet || model == Model::RowNet) plan_from_rowparts(*P, h, r, true);
        else plan_from_split(*P, h, r);
        apply_tune(*P, tune, window_bytes);
        upload_plan(*P, *A, nullptr);
        write_outputs(*P, row_perm, col_perm);
        if (part_out) {
            if (model == Model::RowColumnNet) std::copy(P->part_a.begin(), P->part_a.end(), part_out);
            else std::copy(P->part_ptr.begin(), P->part_ptr.begin() + (model == Model::ColumnNet ? K + 1 : K + 2), part_out);
        }
        *out = P.release();
    });
}

hipError_t spx::run_product(spx_plan_s &P, const double *x, double *y, int32_t accumulate, hipStream_t s) {
    SpmvArgs a{};
    a.slot_ptr = (const int32_t *)P.d_slot_ptr->ptr;
    a.slot_row = P.d_slot_row ? (const int32_t *)P.d_slot_row->ptr : nullptr;
    a.colidx = (const int32_t *)P.d_colidx->ptr;
    a.vals = (const double *)P.d_vals->ptr;
    if (P.tune.sort_gathers) {
        a.scol = (const int32_t *)P.d_colidx_sorted->ptr;
        a.sval = (const double *)P.d_vals_sorted->ptr;
        a.sofs = (const int32_t *)P.d_sorted_ofs->ptr;
    }
    if (P.tune.compact_index) {
        a.c16 = (const uint16_t *)P.d_colidx16->ptr;
        a.cbase = (const int32_t *)P.d_blk_cbase->ptr;
    }
    a.x = x;
    a.y = y;
    a.blk_desc = (const int32_t *)P.d_blk_desc->ptr;
    a.tiles = (const int32_t *)P.d_tiles->ptr;
    const bool tl = tiled(P.tune);
    a.ntiles = (int32_t)(tl ? P.tiles.size() / 4 : P.blk_desc.size() / 4);
    a.xcd_remap = P.tune.xcd_remap;
    std::copy(tl ? P.xcd_tile_ptr.begin() : P.xcd_blk_ptr.begin(),
              tl ? P.xcd_tile_ptr.end() : P.xcd_blk_ptr.end(), a.xcd_ptr);
    a.n = P.n;
    a.long_seg_ptr = (const int32_t *)P.d_long_seg_ptr->ptr;
    a.partials = (double *)P.d_partials->ptr;
    a.counters = (uint32_t *)P.d_counters->ptr;
    bool split = P.form == SPX_FORM_SPLIT;
    if (split) {
        a.shared_begin = P.row_border_begin;
        a.accumulate = accumulate == 1 ? 1 : 0;
        if (accumulate == 0) {  // shared rows and rows without nonzeros
            hipError_t e = launch_fill(y, P.row_border_begin, P.m, 0.0, s);
            if (e != hipSuccess) return e;
        }
    }

    return launch_spmv(a, P.tune.wg, P.tune.nnz_per_block / block_threads(P.tune), P.tune.window_entries, tl, split,
                       s, kind_of(P.tune));
}

extern "C" {

const char *spx_last_error(void) { return spx::g_err.c_str(); }

const char *spx_version(void) { return "spx 0.1 (gfx950)"; }

spx_status spx_set_num_threads(int32_t nthreads) {
    return guarded([&] {
        if (nthreads < 1) fail(SPX_EINVAL, "nthreads must be >= 1");
        set_num_threads(nthreads);
    });
}

spx_status spx_csr_create_host(int32_t m, int32_t n, int64_t nnz, const int32_t *rowptr,
                               const int32_t *colidx, const double *vals, spx_mat *out) {
    return guarded([&] {
        if (!out) fail(SPX_EINVAL, "out is NULL");
        *out = make_mat(m, n, nnz, rowptr, colidx, vals);
    });
}

spx_status spx_csr_upload(int32_t m, int32_t n, int64_t nnz, const int32_t *rowptr,
                          const int32_t *colidx, const double *vals, void *stream, spx_mat *out) {
    return guarded([&] {
        if (!out) fail(SPX_EINVAL, "out is NULL");
        *out = nullptr;
        std::unique_ptr<spx_mat_s> A(make_mat(m, n, nnz, rowptr, colidx, vals));
        upload_mat(*A, stream);
        *out = A.release();
    });
}

void spx_mat_destroy(spx_mat A) { delete A; }

spx_status spx_plan_plain(spx_mat A, const spx_tune *tune, spx_plan *out) {
    return guarded([&] {
        if (!A || !out) fail(SPX_EINVAL, "NULL handle");
        *out = nullptr;
        std::unique_ptr<spx_plan_s> P(new spx_plan_s());
        plan_plain(*P, A->h);
        apply_tune(*P, tune, 0);
        upload_plan(*P, *A, nullptr);
        *out = P.release();
    });
}

spx_status spx_plan_from_parts(spx_mat A, int32_t form, int32_t K, const int32_t *parts, const spx_tune *tune,
                               int32_t *row_perm, int32_t *col_perm, spx_plan *out) {
    return guarded([&] {
        if (!A || !out || !parts) fail(SPX_EINVAL, "NULL argument");
        if (K < 1) fail(SPX_EINVAL, "K must be >= 1");
        if (form != SPX_FORM_SB && form != SPX_FORM_DB && form != SPX_FORM_SPLIT)
            fail(SPX_EINVAL, "form must be SB, DB or split");
        *out = nullptr;
        const CsrHost &h = A->h;
        const int64_t cnt = form == SPX_FORM_SPLIT ? h.nnz : h.m;
        const int32_t hi = form == SPX_FORM_DB ? K : K - 1;
        PartitionResult r;
        r.part.assign(parts, parts + cnt);
        r.leaf.resize(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            if (parts[i] < 0 || parts[i] > hi) fail(SPX_EINVAL, "part index out of range");
            r.leaf[i] = parts[i] < K ? parts[i] : 0;
        }
        r.nleaves = K;
        std::unique_ptr<spx_plan_s> P(new spx_plan_s());
        P->K = K;
        if (form == SPX_FORM_SPLIT) plan_from_split(*P, h, r);
        else plan_from_rowparts(*P, h, r, form == SPX_FORM_DB);
        apply_tune(*P, tune, 0);
        upload_plan(*P, *A, nullptr);
        write_outputs(*P, row_perm, col_perm);
        *out = P.release();
    });
}

spx_status spx_reorder_sb(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed,
                          int32_t *row_perm, int32_t *col_perm, int32_t *part_ptr,
                          const spx_tune *tune, spx_plan *out) {
    return build_reordered(A, K, window_bytes, seed, Model::ColumnNet, row_perm, col_perm,
                           part_ptr, tune, out);
}

spx_status spx_reorder_db(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed,
                          int32_t *row_perm, int32_t *col_perm, int32_t *part_ptr,
                          const spx_tune *tune, spx_plan *out) {
    return build_reordered(A, K, window_bytes, seed, Model::ERowColumnNet, row_perm, col_perm,
                           part_ptr, tune, out);
}

spx_status spx_split(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed,
                     int32_t *row_perm, int32_t *col_perm, int32_t *nz_part,
                     const spx_tune *tune, spx_plan *out) {
    return build_reordered(A, K, window_bytes, seed, Model::RowColumnNet, row_perm, col_perm,
                           nz_part, tune, out);
}

spx_status spx_reorder_rn(spx_mat A, int32_t K, uint64_t seed, int32_t *row_perm, int32_t *col_perm,
                          int32_t *part_ptr, const spx_tune *tune, spx_plan *out) {
    return build_reordered(A, K, 0, seed, Model::RowNet, row_perm, col_perm, part_ptr, tune, out);
}

spx_status spx_split_ex(spx_mat A, int32_t K, int64_t window_bytes, uint64_t seed, int32_t row_net_cost,
                        int32_t *row_perm, int32_t *col_perm, int32_t *nz_part, const spx_tune *tune,
                        spx_plan *out) {
    if (row_net_cost < 1 || row_net_cost > 1 << 20) {
        spx::set_last_error("row_net_cost must be in 1..2^20");
        return SPX_EINVAL;
    }
    return build_reordered(A, K, window_bytes, seed, Model::RowColumnNet, row_perm, col_perm,
                           nz_part, tune, out, row_net_cost);
}

spx_status spx_plan_retune(spx_plan P, const spx_tune *tune) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        spx_plan_s tmp;  // validate before touching the plan
        tmp.form = P->form;
        spx_tune t{};
        if (tune) t = *tune;
        if (t.window_entries == 0) t.window_entries = -1;
        Tune r = resolve_tune(&t, P->form);
        P->tune = r;
        build_schedule(*P);
        if (P->on_device) {
            hip_check(hipDeviceSynchronize(), "retune");  // no product of the old schedule in flight
            upload_schedule(*P, nullptr);
        }
    });
}

void spx_plan_destroy(spx_plan P) { delete P; }

spx_status spx_plan_info_get(spx_plan P, spx_plan_info *info) {
    return guarded([&] {
        if (!P || !info) fail(SPX_EINVAL, "NULL argument");
        std::memset(info, 0, sizeof(*info));
        info->form = P->form;
        info->K = P->K;
        info->m = P->m;
        info->n = P->n;
        info->nnz = P->nnz;
        info->nleaves = P->nleaves;
        info->nblocks = (int32_t)(P->blk_desc.size() / 4);
        info->ntiles = (int32_t)(P->tiles.size() / 4);
        info->nslots = (int32_t)P->slot_ptr.size() - 1;
        info->row_border_begin = P->row_border_begin;
        info->row_empty_begin = P->row_empty_begin;
        info->col_border_begin = P->col_border_begin;
        info->wg_size = P->tune.wg;
        info->nnz_per_block = P->tune.nnz_per_block;
        info->blocks_per_tile = P->tune.blocks_per_tile;
        info->window_entries = P->tune.window_entries;
        info->sum_lambda_col = P->sum_lambda_col;
        info->sum_lambda_row = P->sum_lambda_row;
        info->border_row_nnz = P->border_row_nnz;
        info->cut_connectivity = P->cut;
        info->nnz_compact = P->nnz_compact;
        info->bytes_matrix = 12 * P->nnz - 2 * P->nnz_compact + 4 * (int64_t)P->slot_ptr.size() +
                             4 * (int64_t)P->slot_row.size() + 4 * (int64_t)P->blk_desc.size() +
                             4 * (int64_t)P->tiles.size();
        info->bytes_window = P->window_bytes_fill;
        info->window_nnz = P->window_nnz;
        info->partition_seconds = P->partition_seconds;
        info->plan_seconds = P->plan_seconds;
        info->reduce_iters = P->tune.reduce_iters;
        info->nlong_rows = P->long_seg_ptr.empty() ? 0 : (int32_t)P->long_seg_ptr.size() - 1;
        info->tiles_per_group = P->tune.tiles_per_group;
        info->wave_blocks = P->tune.wave_blocks;
        info->pipeline = P->tune.pipeline;
        info->scan_reduce = P->tune.scan;
        info->sort_gathers = P->tune.sort_gathers;
        info->compact_index = P->tune.compact_index;
    });
}

spx_status spx_spmv(spx_plan P, const double *x, double *y, void *stream) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (!P->on_device) fail(SPX_ENODEVICE, "plan has no device copy (host-only matrix)");
        if (P->m > 0 && !y) fail(SPX_EINVAL, "y is NULL");
        if (P->nnz > 0 && !x) fail(SPX_EINVAL, "x is NULL");
        hip_check(run_product(*P, x, y, 0, (hipStream_t)stream), "spmv launch");
    });
}

spx_status spx_spmv_split(spx_plan P, const double *x, double *y, int32_t accumulate, void *stream) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (P->form != SPX_FORM_SPLIT) fail(SPX_EUNSUPPORTED, "not a split plan");
        if (!P->on_device) fail(SPX_ENODEVICE, "plan has no device copy (host-only matrix)");
        if (P->m > 0 && !y) fail(SPX_EINVAL, "y is NULL");
        if (P->nnz > 0 && !x) fail(SPX_EINVAL, "x is NULL");
        if (accumulate < 0 || accumulate > 2) fail(SPX_EINVAL, "accumulate must be 0, 1 or 2");
        hip_check(run_product(*P, x, y, accumulate, (hipStream_t)stream), "spmv_split launch");
    });
}

spx_status spx_split_prepare_y(spx_plan P, double *y, void *stream) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (P->form != SPX_FORM_SPLIT) fail(SPX_EUNSUPPORTED, "not a split plan");
        if (!P->on_device) fail(SPX_ENODEVICE, "plan has no device copy");
        if (P->m > 0 && !y) fail(SPX_EINVAL, "y is NULL");
        hip_check(launch_fill(y, P->row_border_begin, P->m, 0.0, (hipStream_t)stream), "prepare_y launch");
    });
}

spx_status spx_permute_x(spx_plan P, const double *x, double *x_hat, void *stream) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (P->form == SPX_FORM_PLAIN) fail(SPX_EUNSUPPORTED, "plain plans are not reordered");
        if (!P->on_device) fail(SPX_ENODEVICE, "plan has no device copy");
        if (P->n > 0 && (!x || !x_hat)) fail(SPX_EINVAL, "NULL vector");
        hip_check(launch_gather(x, (const int32_t *)P->d_col_perm->ptr, x_hat, P->n, (hipStream_t)stream),
                  "permute_x launch");
    });
}

spx_status spx_unpermute_y(spx_plan P, const double *y_hat, double *y, void *stream) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (P->form == SPX_FORM_PLAIN) fail(SPX_EUNSUPPORTED, "plain plans are not reordered");
        if (!P->on_device) fail(SPX_ENODEVICE, "plan has no device copy");
        if (P->m > 0 && (!y || !y_hat)) fail(SPX_EINVAL, "NULL vector");
        hip_check(launch_scatter(y_hat, (const int32_t *)P->d_row_perm->ptr, y, P->m, (hipStream_t)stream),
                  "unpermute_y launch");
    });
}

spx_status spx_plan_export_csr(spx_plan P, int32_t *rowptr, int32_t *colidx, double *vals) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (P->form == SPX_FORM_SPLIT) fail(SPX_EUNSUPPORTED, "split plans store per-leaf GCSR");
        if (rowptr) std::copy(P->slot_ptr.begin(), P->slot_ptr.end(), rowptr);
        if (colidx) std::copy(P->colidx.begin(), P->colidx.end(), colidx);
        if (vals) std::copy(P->vals.begin(), P->vals.end(), vals);
    });
}

spx_status spx_plan_export_split(spx_plan P, int32_t *leaf_slot_ptr, int32_t *slot_row,
                                 int32_t *slot_ptr, int32_t *colidx, double *vals) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (P->form != SPX_FORM_SPLIT) fail(SPX_EUNSUPPORTED, "not a split plan");
        if (leaf_slot_ptr) std::copy(P->leaf_slot_ptr.begin(), P->leaf_slot_ptr.end(), leaf_slot_ptr);
        if (slot_row) std::copy(P->slot_row.begin(), P->slot_row.end(), slot_row);
        if (slot_ptr) std::copy(P->slot_ptr.begin(), P->slot_ptr.end(), slot_ptr);
        if (colidx) std::copy(P->colidx.begin(), P->colidx.end(), colidx);
        if (vals) std::copy(P->vals.begin(), P->vals.end(), vals);
    });
}

spx_status spx_plan_export_parts(spx_plan P, int32_t *a, int32_t *b) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (P->form == SPX_FORM_PLAIN || P->form == SPX_FORM_ORDER)
            fail(SPX_EUNSUPPORTED, "plain and ordered plans have no partition");
        if (a) std::copy(P->part_a.begin(), P->part_a.end(), a);
        if (b) std::copy(P->part_b.begin(), P->part_b.end(), b);
    });
}

spx_status spx_plan_export_perm(spx_plan P, int32_t *row_perm, int32_t *col_perm) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (P->form == SPX_FORM_PLAIN) {
            for (int32_t i = 0; row_perm && i < P->m; ++i) row_perm[i] = i;
            for (int32_t j = 0; col_perm && j < P->n; ++j) col_perm[j] = j;
            return;
        }
        write_outputs(*P, row_perm, col_perm);
    });
}

spx_status spx_plan_export_sched(spx_plan P, int32_t *blk_desc, int32_t *tiles) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (blk_desc) std::copy(P->blk_desc.begin(), P->blk_desc.end(), blk_desc);
        if (tiles) std::copy(P->tiles.begin(), P->tiles.end(), tiles);
    });
}

spx_status spx_plan_export_gather_order(spx_plan P, int64_t *len, int32_t *ofs, uint32_t *colidx, double *vals) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (!P->tune.sort_gathers) fail(SPX_EUNSUPPORTED, "the plan is not tuned with sort_gathers");
        if (len) *len = (int64_t)P->colidx_sorted.size();
        if (ofs) std::copy(P->sorted_ofs.begin(), P->sorted_ofs.end(), ofs);
        if (colidx) std::copy(P->colidx_sorted.begin(), P->colidx_sorted.end(), colidx);
        if (vals) std::copy(P->vals_sorted.begin(), P->vals_sorted.end(), vals);
    });
}

spx_status spx_plan_export_compact(spx_plan P, uint16_t *colidx16, int32_t *cbase) {
    return guarded([&] {
        if (!P) fail(SPX_EINVAL, "NULL handle");
        if (!P->tune.compact_index) fail(SPX_EUNSUPPORTED, "the plan is not tuned with compact_index");
        if (colidx16) std::copy(P->colidx16.begin(), P->colidx16.end(), colidx16);
        if (cbase) std::copy(P->blk_cbase.begin(), P->blk_cbase.end(), cbase);
    });
}

int64_t spx_stream_sink_len(int64_t bytes) { return bytes > 0 ? stream_grid(bytes) : 0; }

spx_status spx_stream_read(const void *src, int64_t bytes, double *sink, void *stream) {
    return guarded([&] {
        if (bytes < 0 || bytes % 16) fail(SPX_EINVAL, "bytes must be a non-negative multiple of 16");
        if (bytes && (!src || !sink)) fail(SPX_EINVAL, "NULL pointer");
        hip_check(launch_stream_read(src, bytes, sink, (hipStream_t)stream), "stream_read launch");
    });
}

spx_status spx_stream_copy(const void *src, void *dst, int64_t bytes, void *stream) {
    return guarded([&] {
        if (bytes < 0 || bytes % 16) fail(SPX_EINVAL, "bytes must be a non-negative multiple of 16");
        if (bytes && (!src || !dst)) fail(SPX_EINVAL, "NULL pointer");
        hip_check(launch_stream_copy(src, dst, bytes, (hipStream_t)stream), "stream_copy launch");
    });
}

}  // extern "C"
