// Size limits of the library's 32-bit indexed work arrays, as plain host
// arithmetic (no HIP types), so that they can be compiled and checked on
// their own.
#pragma once

#include <stdint.h>

namespace start {

// The upstream chain indexes its (particle, list entry) pairs with 32-bit
// offsets, a prefix sum of the list lengths.  The lengths are summed in 64
// bits first; a total above 2^31 - 1 is refused before anything is narrowed
// (a 32-bit sum of ~2^32 entries would wrap to a small, wrong size).
constexpr uint64_t kMaxUpstreamPairs = ((uint64_t)1 << 31) - 1;
inline bool upstream_pairs_fit(uint64_t total) { return total <= kMaxUpstreamPairs; }

// The neighbour pairs (particle, neighbour within 2h) are indexed the same
// way: their counts are summed in 64 bits and more than 2^31 - 1 refused.
constexpr uint64_t kMaxNeighbourPairs = ((uint64_t)1 << 31) - 1;
inline bool neighbour_pairs_fit(uint64_t total) { return total <= kMaxNeighbourPairs; }

}  // namespace start
