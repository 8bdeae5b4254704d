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
}  // namespace spx
