// The Frechet kernel on squared cells with 3, 5, 6 or 7 rows per lane
// (float coordinates, no LDS rings).  Serving launches use these shapes
// when a band of 64 R rows fits their queries more closely than a
// power-of-two R: the rows of a band past a query's end are computed and
// dropped, so a 300-point query wastes 41 % of a 512-row band and 6 % of a
// 320-row one.  Kept in a unit of its own so the other launches carry none
// of this code.
#include "ffd_launch.h"

namespace ffd {

namespace {
struct ServeSel {
  static constexpr bool kExact = false;
  static constexpr bool kFloat = true;
  static constexpr int kOnlyD = 0;
  template <int R, int D, typename V>
  static auto kernel() { return &stream_kernel<R, D, V, false>; }
};
}  // namespace

#define FFD_SERVE_SHAPES(X) \
  X(3, 1) X(3, 2) X(3, 3) X(3, 4) X(5, 1) X(5, 2) X(5, 3) X(5, 4) \
  X(6, 1) X(6, 2) X(6, 3) X(6, 4) X(7, 1) X(7, 2) X(7, 3) X(7, 4)

hipError_t launch_stream_serve(int R, int D, const KernelArgs &a, int wpb, hipStream_t st) {
  switch (R * 8 + D) {
#define FFD_CASE(r, d) \
  case r * 8 + d: return Launcher<ServeSel>::one<r, d, float>(a, wpb, false, st);
    FFD_SERVE_SHAPES(FFD_CASE)
#undef FFD_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace ffd
