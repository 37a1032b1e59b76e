// Host finish (Section 2.1.3): Melkman's hull of the simple polygon.
#pragma once
#include <cstdint>

namespace chainhull {

// xy: m interleaved (x, y) vertices of a simple polygon; idx: their point
// indices.  Writes the hull (CCW from the smallest (y, x), collinear points
// excluded) to out and its size to *out_count.  Returns 0, or -1 when a
// coordinate is out of range or the deque runs empty (input not simple).
int melkman_finish(const int32_t* xy, const int32_t* idx, int64_t m, int32_t* out, int64_t* out_count);

}  // namespace chainhull
