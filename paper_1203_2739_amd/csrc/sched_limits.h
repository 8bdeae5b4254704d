// Limits shared by the schedule builder and the kernels.
#pragma once

namespace spx {
// A chunk is what one wave stages at a time: 4 nonzeros per lane.  Loads
// start at a 4-aligned nonzero, so a chunk holds at most kChunkSpan - 3.
constexpr int kChunkSpan = 256;
// Rows starting in one chunk, at most.
constexpr int kChunkRows = 256;
}  // namespace spx
