// Kernels of one measure / ground distance (OP = measure + 2 * cell, see
// ffd_stream.h) other than the Frechet distance on squared Euclidean cells.
// This unit is compiled once per OP (-DFFD_OP=...), in parallel: 1 DTW of
// squared Euclidean cells, 3 DTW of Euclidean cells (float32 only), 4
// Frechet on Manhattan cells, 5 DTW on Manhattan cells, 6 Frechet on
// Chebyshev cells, 7 DTW on Chebyshev cells, 8 Levenshtein (int32 symbols,
// float32 values), 10 Frechet and 11 DTW on great-circle distances (float32
// (latitude, longitude) input, FP64 unit vectors: the value type double,
// D = 3).
#include "ffd_launch.h"

#ifndef FFD_OP
#error "compile with -DFFD_OP=<op>"
#endif

#define FFD_CAT2(a, b) a##b
#define FFD_CAT(a, b) FFD_CAT2(a, b)

namespace ffd {

namespace {
struct OpSel {
  // int32 coordinates (exact FP64 values) for every op but Euclidean cells
  // and Levenshtein; float32 coordinates for every op but the great-circle
  // ones, which compute in FP64 (their `exact` shape) on float32 input;
  // Levenshtein runs on float32 values with int32 symbols as bit patterns
  static constexpr bool kExact = FFD_OP != 3 && FFD_OP != 8;
  static constexpr bool kFloat = FFD_OP != 10 && FFD_OP != 11;
  static constexpr int kOnlyD = FFD_OP == 10 || FFD_OP == 11 ? 3 : 0;
  template <int R, int D, typename V>
  static auto kernel() { return &op_kernel<R, D, V, FFD_OP>; }
};
}  // namespace

hipError_t FFD_CAT(launch_op_, FFD_OP)(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop,
                                       hipStream_t st) {
  return Launcher<OpSel>::launch(exact, R, D, a, wpb, coop, st);
}

hipError_t FFD_CAT(occupancy_op_, FFD_OP)(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu) {
  return Launcher<OpSel>::occupancy(exact, R, D, wpb, lds, blocks_per_cu);
}

}  // namespace ffd
