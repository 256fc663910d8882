// The discrete Frechet kernel with LDS rings between the waves of a
// workgroup (single long pairs pipelined over consecutive waves), compiled
// in its own unit so that the variant without rings carries none of its
// code.
#include "ffd_launch.h"

namespace ffd {

namespace {
struct RingsSel {
  static constexpr bool kExact = true;
  static constexpr bool kFloat = true;
  static constexpr int kOnlyD = 0;
  template <int R, int D, typename V>
  static auto kernel() { return &stream_kernel<R, D, V, true>; }
};
}  // namespace

hipError_t launch_stream_rings(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
  return Launcher<RingsSel>::launch(exact, R, D, a, wpb, coop, st);
}

hipError_t occupancy_stream_rings(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu) {
  return Launcher<RingsSel>::occupancy(exact, R, D, wpb, lds, blocks_per_cu);
}

}  // namespace ffd
