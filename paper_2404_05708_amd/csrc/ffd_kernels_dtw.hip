// Dynamic time warping kernels with squared Euclidean cells (Appendix B):
// float32 coordinates, and int32 coordinates summed exactly in FP64.
#include "ffd_launch.h"

namespace ffd {

namespace {
struct DtwSqSel {
  static constexpr bool kExact = true;
  template <int R, int D, typename V>
  static auto kernel() { return &dtw_kernel<R, D, V, 1>; }
};
}  // namespace

hipError_t launch_dtw_sq(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
  return Launcher<DtwSqSel>::launch(exact, R, D, a, wpb, coop, st);
}

hipError_t occupancy_dtw_sq(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu) {
  return Launcher<DtwSqSel>::occupancy(exact, R, D, wpb, lds, blocks_per_cu);
}

}  // namespace ffd
