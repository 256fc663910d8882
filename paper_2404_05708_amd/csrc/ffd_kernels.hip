// The stream kernel without LDS rings between waves (batched, cross and
// serving launches, and single pairs that are not pipelined).
#define FFD_RINGS false
#define FFD_LAUNCH_NAME launch_stream_plain
#define FFD_OCC_NAME occupancy_stream_plain
// Launchers of the stream kernel, one translation unit per ring setting
// (RINGS selects the variant that can hand rows between the waves of a
// workgroup through LDS; the two are compiled in parallel).
#include "ffd_stream.h"

namespace ffd {

namespace {

// A launch whose waves wait on each other (boundary rows over links) is
// cooperative: the runtime then either makes every workgroup resident at
// once or refuses the launch, so a waiting wave never waits for a wave that
// cannot start.
template <int R, int D, typename V>
hipError_t launch_t(const KernelArgs &a, int waves_per_block, bool coop, hipStream_t st) {
  int blocks = (a.nwaves + waves_per_block - 1) / waves_per_block;
  size_t lds = (size_t)a.lds_per_wave * waves_per_block;
  if (coop) {
    KernelArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&stream_kernel<R, D, V, FFD_RINGS>),
                                      dim3(blocks), dim3(waves_per_block * kWave), args, (unsigned)lds, st);
  }
  hipLaunchKernelGGL((stream_kernel<R, D, V, FFD_RINGS>), dim3(blocks), dim3(waves_per_block * kWave), lds, st, a);
  return hipGetLastError();
}

template <int R, typename V>
hipError_t launch_d(int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
  switch (D) {
    case 1: return launch_t<R, 1, V>(a, wpb, coop, st);
    case 2: return launch_t<R, 2, V>(a, wpb, coop, st);
    case 3: return launch_t<R, 3, V>(a, wpb, coop, st);
    case 4: return launch_t<R, 4, V>(a, wpb, coop, st);
  }
  return hipErrorInvalidValue;
}

template <typename V>
hipError_t launch_r(int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
  switch (R) {
    case 1: return launch_d<1, V>(D, a, wpb, coop, st);
    case 2: return launch_d<2, V>(D, a, wpb, coop, st);
    case 4: return launch_d<4, V>(D, a, wpb, coop, st);
    case 8: return launch_d<8, V>(D, a, wpb, coop, st);
  }
  return hipErrorInvalidValue;
}

template <int R, int D, typename V>
hipError_t occ_t(int wpb, size_t lds, int *blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, stream_kernel<R, D, V, FFD_RINGS>, wpb * kWave, lds);
}

template <int R, typename V>
hipError_t occ_d(int D, int wpb, size_t lds, int *blocks) {
  switch (D) {
    case 1: return occ_t<R, 1, V>(wpb, lds, blocks);
    case 2: return occ_t<R, 2, V>(wpb, lds, blocks);
    case 3: return occ_t<R, 3, V>(wpb, lds, blocks);
    case 4: return occ_t<R, 4, V>(wpb, lds, blocks);
  }
  return hipErrorInvalidValue;
}

template <typename V>
hipError_t occ_r(int R, int D, int wpb, size_t lds, int *blocks) {
  switch (R) {
    case 1: return occ_d<1, V>(D, wpb, lds, blocks);
    case 2: return occ_d<2, V>(D, wpb, lds, blocks);
    case 4: return occ_d<4, V>(D, wpb, lds, blocks);
    case 8: return occ_d<8, V>(D, wpb, lds, blocks);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t FFD_LAUNCH_NAME(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
  return exact ? launch_r<double>(R, D, a, wpb, coop, st) : launch_r<float>(R, D, a, wpb, coop, st);
}

// Workgroups of `wpb` waves using `lds` bytes that one CU holds at once.
hipError_t FFD_OCC_NAME(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu) {
  return exact ? occ_r<double>(R, D, wpb, lds, blocks_per_cu) : occ_r<float>(R, D, wpb, lds, blocks_per_cu);
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
