// Dynamic time warping kernels with Euclidean cells (a correctly rounded
// float32 square root per cell; float32 coordinates only).
#include "ffd_launch.h"

namespace ffd {

namespace {
struct DtwEucSel {
  static constexpr bool kExact = false;
  template <int R, int D, typename V>
  static auto kernel() { return &dtw_kernel<R, D, V, 2>; }
};
}  // namespace

hipError_t launch_dtw_euc(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
  return Launcher<DtwEucSel>::launch(exact, R, D, a, wpb, coop, st);
}

hipError_t occupancy_dtw_euc(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu) {
  return Launcher<DtwEucSel>::occupancy(exact, R, D, wpb, lds, blocks_per_cu);
}

}  // namespace ffd
