// The discrete Frechet kernel without LDS rings between waves (batched,
// cross and serving launches, and single pairs that are not pipelined),
// and the small kernel that clears progress flags for graph replays.
#include "ffd_launch.h"

namespace ffd {

namespace {
struct PlainSel {
  static constexpr bool kExact = true;
  static constexpr bool kFloat = true;
  static constexpr int kOnlyD = 0;
  template <int R, int D, typename V>
  static auto kernel() { return &stream_kernel<R, D, V, false>; }
};
}  // namespace

hipError_t launch_stream_plain(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
  return Launcher<PlainSel>::launch(exact, R, D, a, wpb, coop, st);
}

hipError_t occupancy_stream_plain(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu) {
  return Launcher<PlainSel>::occupancy(exact, R, D, wpb, lds, blocks_per_cu);
}

// Zero n 64-bit words (progress flags and the error word of a launch that
// is recorded into a graph: its replays share one epoch, so each replay
// starts from cleared flags).  A kernel, not a memset node.
__global__ void clear_words_kernel(uint64_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t clear_words(uint64_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(clear_words_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace ffd
