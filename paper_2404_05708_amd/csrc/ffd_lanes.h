// Arguments and launcher of the one-pair-per-lane kernel (ffd_lanes.hip):
// batches whose pairs are all short, 64 pairs per wavefront.
#ifndef FFD_LANES_H
#define FFD_LANES_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffd {

struct LaneArgs {
  const void *X[2];       // coordinate arrays of the two curve sets (float32, or int32 for the exact path)
  const int32_t *off[2];  // their curve offsets in points (device; each set below 2^31 points)
  const int32_t *order;   // lane k -> pair index; the top bit set: the second set's curve holds the rows
  void *out;              // float32 or int64 results, indexed by pair
  int32_t col_count;      // 0: pair p is curve p of both sets; > 0: curve p / col_count of the first set
                          // against curve p % col_count of the second (query set x database)
  int32_t metric;         // squared cells: 0 Euclidean (the root taken once per pair), 1 squared Euclidean
  int32_t cell;           // ground distance: 0 squared Euclidean, 1 Euclidean (DTW), 2 Manhattan, 3 Chebyshev,
                          // 4 Levenshtein (int32 symbols, float32 values, int64 results)
  int32_t dtw;            // 1: dynamic time warping (Appendix B), 0: the Frechet distance
  int32_t classes;        // classes of column count, 1 ... kLaneClasses, most columns first
  int32_t cols[8];        // columns a lane of class c holds (a multiple of 8, at most 64)
  int64_t first[9];       // class c: lanes [first[c], first[c + 1]) of order
  int64_t block_first[9]; // class c: workgroups [block_first[c], block_first[c + 1]) of the launch
};

// Classes of column count: a lane holds its column curve padded to the next
// multiple of kLaneColStep columns.
constexpr int kLaneClasses = 8;
constexpr int kLaneColStep = 8;

// The largest column curve a lane holds in registers for D coordinates (16,
// 32 or 64), by value type.  (A lane holds M x D coordinates and M table
// values: at most about 192 registers' worth.)
constexpr int lane_cols_max(bool exact, int D) {
  return exact ? (D <= 2 ? 32 : 16) : (D <= 2 ? 64 : 32);
}

// Workgroups (of 256 lanes) of a launch.
constexpr int kLaneBlock = 256;

// One launch for every class (their workgroups in a.block_first), D
// coordinates (1 ... 4); every class's column count at most lane_cols_max.
hipError_t launch_lanes(bool exact, int D, const LaneArgs &a, hipStream_t st);

}  // namespace ffd

#endif  // FFD_LANES_H
