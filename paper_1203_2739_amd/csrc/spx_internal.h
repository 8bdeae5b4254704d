// Internal declarations shared by the host-side translation units of libspx.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/spx.h"
#include "sched_limits.h"

namespace spx {

// ---------------------------------------------------------------- errors
struct Error {
    spx_status code;
    std::string msg;
};
[[noreturn]] void fail(spx_status code, const std::string &msg);
void set_last_error(const std::string &msg);

// ------------------------------------------------------------- hypergraph
// Pins stored both ways: net -> vertices and vertex -> nets.
struct Hypergraph {
    int32_t nv = 0, nn = 0;
    std::vector<int64_t> vw;     // vertex weights
    std::vector<int64_t> nc;     // net costs
    std::vector<uint8_t> nrow;   // 1 = row net removed when cut (DB model)
    std::vector<int64_t> xpins;  // [nn+1]
    std::vector<int32_t> pins;
    std::vector<int64_t> xnets;  // [nv+1]
    std::vector<int32_t> vnets;
    int64_t total_weight() const;
    void build_vertex_side();    // fills xnets/vnets from xpins/pins
};

// One bisection: side[v] in {0, 1}; part 0 gets about frac0 of the weight.
// Returns the cutsize (sum of costs of cut nets).  `threads` bounds the
// threads its contraction may use; the result does not depend on it.
int64_t bisect(const Hypergraph &H, double frac0, double eps, uint64_t seed,
               std::vector<uint8_t> &side, int32_t threads = 1);

// Matrix in CSR (host).
struct CsrHost {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    std::vector<int32_t> rowptr, colidx;
    std::vector<double> vals;
};

// RowNet: the row-net model of sHP_RN (columns are vertices, rows are nets;
// Section 5.1), given as rows: a row whose columns lie in one part joins it,
// a row reaching several parts goes to the row border (part K).
enum class Model { ColumnNet, ERowColumnNet, RowColumnNet, RowNet };

// Recursive bisection into K parts, optionally refined into leaves whose
// window (distinct columns, plus distinct rows for the split) fits
// window_entries.  For ColumnNet: out_part/out_leaf have m entries (rows).
// For ERowColumnNet: m entries, part K marks a row of R_B.  For
// RowColumnNet: nnz entries (nonzeros in CSR order).  Leaves are numbered
// part-major.  Returns the top-level connectivity cutsize.
struct PartitionResult {
    std::vector<int32_t> part, leaf;
    int32_t nleaves = 0;
    int64_t cut = 0;
    double seconds = 0.0;
};
// Cost of a row net of the split's row-column-net model relative to a
// column net (1 each in Corollary 4).
constexpr int64_t kSplitRowNetCostDefault = 32;
PartitionResult partition(const CsrHost &A, Model model, int32_t K, int64_t window_entries,
                          uint64_t seed, int64_t row_net_cost = kSplitRowNetCostDefault);

int32_t num_threads();
void set_num_threads(int32_t t);

// Device buffer owned through shared_ptr so that plans outlive matrices.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    ~DevBuf();
};
using DevPtr = std::shared_ptr<DevBuf>;
DevPtr dev_alloc(size_t bytes);
DevPtr dev_upload(const void *host, size_t bytes, size_t pad_bytes, void *stream);

struct Tune {
    int32_t wg = kDefaultWG, nnz_per_block = kDefaultNpt * kDefaultWG, blocks_per_tile = 1, window_entries = -1;
    int32_t xcd_remap = 1, reduce_iters = kReduceIters, tiles_per_group = 0, wave_blocks = 0, pipeline = 0;
    int32_t scan = 0, sort_gathers = 0, compact_index = 0;
};
Tune resolve_tune(const spx_tune *t, int form);
inline bool tiled(const Tune &t) {
    return t.window_entries > 0 || t.blocks_per_tile > 1 || t.tiles_per_group > 0 || t.wave_blocks;
}
// Threads that run one row block: a wave in wave-block schedules.
inline int32_t block_threads(const Tune &t) { return t.wave_blocks ? 64 : t.wg; }
inline Kind kind_of(const Tune &t) {
    return t.pipeline      ? Kind::Pipe
           : t.wave_blocks ? Kind::Waves
           : t.scan && t.sort_gathers ? Kind::SortedScan
           : t.scan        ? Kind::Scan
           : t.sort_gathers ? Kind::Sorted
           : t.compact_index ? Kind::Compact
                            : Kind::Blocks;
}

}  // namespace spx

// Handles.
struct spx_mat_s {
    spx::CsrHost h;
    bool on_device = false;
    spx::DevPtr d_rowptr, d_colidx, d_vals;
};

struct spx_plan_s {
    int form = SPX_FORM_PLAIN;
    int32_t K = 1, m = 0, n = 0;
    int64_t nnz = 0;
    bool on_device = false;
    // stored matrix: slots are rows (plain/SB/DB) or (leaf, row) pairs (split)
    std::vector<int32_t> slot_ptr, slot_row, colidx;
    std::vector<double> vals;
    std::vector<int32_t> row_perm, col_perm;
    std::vector<int32_t> part_a, part_b;        // r2p/r2leaf or nz_part/nz_leaf
    std::vector<int32_t> part_ptr;              // rows per part (+ border)
    std::vector<int32_t> leaf_slot_ptr;         // slots per leaf
    std::vector<int32_t> leaf_col_lo, leaf_col_hi;  // exclusive column range per leaf
    int32_t nleaves = 0;
    int32_t row_border_begin = 0, row_empty_begin = 0, col_border_begin = 0;
    // schedule
    spx::Tune tune;
    std::vector<int32_t> blk_slot;              // [nblocks+1]
    std::vector<int32_t> blk_desc;              // 4 per block: slot range, nonzero range
    std::vector<int32_t> tiles;                 // 4 per tile
    std::vector<int32_t> long_seg_ptr;          // [nlong+1] first partial-sum entry of each long slot
    std::vector<int32_t> xcd_blk_ptr, xcd_tile_ptr;  // [kXcdGroups+1] first block / tile of each row group
    // sort_gathers: the nonzeros of every multi-row block sorted by column,
    // indices carrying the row-order offset in their upper bits, in
    // interleaved 64-entry chunks at the block's offset sorted_ofs[b]
    std::vector<uint32_t> colidx_sorted;
    std::vector<double> vals_sorted;
    std::vector<int32_t> sorted_ofs;
    // compact_index: 16-bit column offsets from blk_cbase[b] (the smallest
    // column of block b, or -1 when its columns span 65,536 or more, or for
    // a long-slot segment), at the stored positions
    std::vector<uint16_t> colidx16;
    std::vector<int32_t> blk_cbase;
    int64_t nnz_compact = 0;
    std::vector<float> vals32;                  // precision mode: values rounded to binary32
    std::vector<uint16_t> vals16;               // precision mode: binary32 values rounded to bfloat16
    int64_t window_nnz = 0, window_bytes_fill = 0;
    // device copies
    spx::DevPtr d_slot_ptr, d_slot_row, d_colidx, d_vals, d_row_perm, d_col_perm;
    spx::DevPtr d_blk_desc, d_tiles, d_long_seg_ptr, d_partials, d_counters;
    spx::DevPtr d_colidx_sorted, d_vals_sorted, d_sorted_ofs, d_colidx16, d_blk_cbase;
    spx::DevPtr d_vals32, d_vals16;
    // statistics
    int64_t sum_lambda_col = 0, sum_lambda_row = 0, border_row_nnz = 0, cut = 0;
    double partition_seconds = 0.0, plan_seconds = 0.0;
};

namespace spx {
// plan.cpp
void build_schedule(spx_plan_s &P);
void upload_plan(spx_plan_s &P, const spx_mat_s &A, void *stream);
void upload_schedule(spx_plan_s &P, void *stream);
void plan_from_rowparts(spx_plan_s &P, const CsrHost &A, const PartitionResult &r, bool db);
void plan_from_split(spx_plan_s &P, const CsrHost &A, const PartitionResult &r);
void plan_plain(spx_plan_s &P, const CsrHost &A);
void plan_from_perm(spx_plan_s &P, const CsrHost &A, const int32_t *row_perm, const int32_t *col_perm);
// orderings.cpp: row and column orders (new -> old) of the comparison
// orderings on the bipartite graph of A
void order_bfs(const CsrHost &A, int32_t *row_perm, int32_t *col_perm);
void order_rcm(const CsrHost &A, int32_t *row_perm, int32_t *col_perm);
}  // namespace spx
