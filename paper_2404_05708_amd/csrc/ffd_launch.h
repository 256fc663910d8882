// Launch and occupancy helpers shared by the kernel translation units.  Each
// unit instantiates one kernel family (a selector `Sel` whose
// `Sel::kernel<R, D, V>()` names the kernel for a launch shape) for every
// shape R in {1, 2, 4, 8}, D in {1, ..., 4}, and the wide shapes (R, D) =
// (2, 8) and (1, 16) (curves of 5 to 16 coordinates; see kernel_dim), only D =
// Sel::kOnlyD when that is not 0, and the value types it supports.
#ifndef FFD_LAUNCH_H
#define FFD_LAUNCH_H

#include "ffd_stream.h"

namespace ffd {

// Every (R, D) shape: R rows per lane, D coordinates per point in the kernel.
#define FFD_SHAPES(X) \
  X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(2, 1) X(2, 2) X(2, 3) X(2, 4) \
  X(4, 1) X(4, 2) X(4, 3) X(4, 4) X(8, 1) X(8, 2) X(8, 3) X(8, 4) \
  X(2, 8) X(1, 16)

template <class Sel>
struct Launcher {
  // A launch whose waves wait on each other (boundary rows over links) is
  // cooperative: the runtime then either makes every workgroup resident at
  // once or refuses the launch, so a waiting wave never waits for a wave
  // that cannot start.
  template <int R, int D, typename V>
  static hipError_t one(const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
    if constexpr (Sel::kOnlyD != 0 && D != Sel::kOnlyD) {
      return hipErrorInvalidValue;
    } else {
      const void *k = reinterpret_cast<const void *>(Sel::template kernel<R, D, V>());
      unsigned blocks = (unsigned)((a.nwaves + wpb - 1) / wpb);
      unsigned lds = (unsigned)((size_t)a.lds_per_wave * wpb);
      KernelArgs copy = a;
      void *args[] = {&copy};
      if (coop) return hipLaunchCooperativeKernel(k, dim3(blocks), dim3(wpb * kWave), args, lds, st);
      return hipLaunchKernel(k, dim3(blocks), dim3(wpb * kWave), args, lds, st);
    }
  }

  template <int R, int D, typename V>
  static hipError_t occ(int wpb, size_t lds, int *blocks) {
    if constexpr (Sel::kOnlyD != 0 && D != Sel::kOnlyD) {
      return hipErrorInvalidValue;
    } else {
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, Sel::template kernel<R, D, V>(), wpb * kWave,
                                                          lds);
    }
  }

  template <typename V>
  static hipError_t launch_v(int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
    switch (R * 32 + D) {
#define FFD_CASE(r, d) \
  case r * 32 + d: return one<r, d, V>(a, wpb, coop, st);
      FFD_SHAPES(FFD_CASE)
#undef FFD_CASE
    }
    return hipErrorInvalidValue;
  }

  template <typename V>
  static hipError_t occ_v(int R, int D, int wpb, size_t lds, int *blocks) {
    switch (R * 32 + D) {
#define FFD_CASE(r, d) \
  case r * 32 + d: return occ<r, d, V>(wpb, lds, blocks);
      FFD_SHAPES(FFD_CASE)
#undef FFD_CASE
    }
    return hipErrorInvalidValue;
  }

  static hipError_t launch(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st) {
    if constexpr (Sel::kExact) {
      if (exact) return launch_v<double>(R, D, a, wpb, coop, st);
    } else {
      if (exact) return hipErrorInvalidValue;
    }
    if constexpr (Sel::kFloat) return launch_v<float>(R, D, a, wpb, coop, st);
    return hipErrorInvalidValue;
  }

  // Workgroups of `wpb` waves using `lds` bytes that one CU holds at once.
  static hipError_t occupancy(bool exact, int R, int D, int wpb, size_t lds, int *blocks) {
    if constexpr (Sel::kExact) {
      if (exact) return occ_v<double>(R, D, wpb, lds, blocks);
    } else {
      if (exact) return hipErrorInvalidValue;
    }
    if constexpr (Sel::kFloat) return occ_v<float>(R, D, wpb, lds, blocks);
    return hipErrorInvalidValue;
  }
};

}  // namespace ffd

#endif  // FFD_LAUNCH_H
