// Limits shared by the schedule builder and the kernels.
#pragma once

namespace spx {
// Every thread of a workgroup stages 4 or 8 consecutive nonzeros of a row
// block (npt); loads start at a 4-aligned nonzero, so a block of a workgroup
// of WG threads spans at most npt * WG nonzeros counted from its aligned
// start.
constexpr int kDefaultWG = 128;
constexpr int kDefaultNpt = 4;
// Default bound on the strided reduction loop of a row inside a block:
// ceil(row length / lanes given to the row).
constexpr int kReduceIters = 64;
// Row groups: the stored rows (slots) are cut into this many runs of nearly
// equal nonzeros (a slot starting at storage offset s is in group
// floor(kXcdGroups * s / nnz)); the kernels run the blocks of group g on XCD
// g of the MI355X, and the plans order columns by the groups that read them.
constexpr int kXcdGroups = 8;
// Kernel that runs a schedule: row blocks, wave blocks, pipelined tiles, row
// blocks summed by a segmented scan, row blocks stored sorted by column,
// both of the last two, or row blocks with 16-bit block-local indices.
enum class Kind : int { Blocks = 0, Waves = 1, Pipe = 2, Scan = 3, Sorted = 4, SortedScan = 5, Compact = 6 };
// Gather-sorted storage: a column index keeps the nonzero's offset in row
// order from its block's aligned start (below nt, the block's capacity) in
// its upper bits; the column takes the low pack_shift(nt) bits, so columns
// must be below 2^pack_shift(nt).
constexpr int pack_shift(int nt) {
    int b = 0;
    while ((1 << b) < nt) ++b;
    return 32 - b;
}
}  // namespace spx
