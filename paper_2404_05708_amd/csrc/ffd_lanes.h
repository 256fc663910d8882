// Arguments and launcher of the one-pair-per-lane kernel (ffd_lanes.hip):
// batches whose pairs are all short, 64 pairs per wavefront.
#ifndef FFD_LANES_H
#define FFD_LANES_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffd {

struct LaneArgs {
  const void *X[2];       // coordinate arrays of the two curve sets (float32, or int32 for the exact path)
  const int64_t *off[2];  // their curve offsets in points (device)
  const int32_t *order;   // lane k -> pair index; the top bit set: the second set's curve holds the rows
  void *out;              // float32 or int64 results, indexed by pair
  int64_t npairs;         // lanes of this launch
  int32_t metric;         // 0 Euclidean (the root taken once per pair), 1 squared Euclidean
};

// The largest column curve a lane holds in registers for D coordinates (16,
// 32 or 64), by value type.
constexpr int lane_cols_max(bool exact, int D) {
  return exact ? (D <= 2 ? 32 : 16) : (D <= 2 ? 64 : 32);
}

// One launch of a shape: M columns (16, 32 or 64, at most lane_cols_max),
// D coordinates (1 ... 4).
hipError_t launch_lanes(bool exact, int M, int D, const LaneArgs &a, hipStream_t st);

}  // namespace ffd

#endif  // FFD_LANES_H
