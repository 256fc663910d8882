// Short pairs, one pair per lane: the batching of the paper's Sec. 4, where
// each lane of a vector unit runs the whole linear-memory recurrence
// (Theorem 1, Algorithm 2) for its own pair.  The anti-diagonal sweep of
// the streaming kernels gives a pair at least a 64-row band and 16
// separator steps, most of which a pair of a few dozen points leaves idle;
// here a wavefront holds 64 pairs.
//
// Lane k takes pair order[k].  Its shorter curve (at most M points, the
// column curve) stays in registers, its last point repeated up to M
// columns: repeating a point leaves the distance unchanged (Sec. 4,
// footnote), and the selections of Eq. (1) return one of the table's own
// values, so the result at column M - 1 has the bits of the result at the
// curve's own last column.  The lane sweeps the rows of the other curve
// one by one, keeping one table row of M values in registers: the value
// above a cell is the row's old value, the diagonal the old value one
// column to the left, the left neighbour the value just computed.  The
// first row starts from the corner M_{-1,-1} = -inf with +inf elsewhere
// around the table (the boundary reading of the streaming kernels), so Eq.
// (1) itself produces the first row and column.  Each cell is evaluated as
// everywhere else in the library (d2 = dx*dx, then fma(dk, dk, d2), FP64 for
// int32 coordinates) and the Euclidean root is taken once per pair, so the
// results equal the streaming kernels' bit for bit.
//
// The host sorts the pairs of a launch by row count, so that the lanes of a
// wavefront sweep about as many rows each.
#include "ffd_lanes.h"

#include "ffd_stream.h"

namespace ffd {

namespace {

template <int M, int D, typename V>
__global__ __launch_bounds__(256) void lane_kernel(LaneArgs a) {
  using N = Num<V>;
  using C = typename N::Coord;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.npairs) return;
  const int32_t raw = a.order[k];
  const bool swap = raw < 0;
  const int32_t idx = raw & 0x7fffffff;
  const C *Xr = static_cast<const C *>(swap ? a.X[1] : a.X[0]);
  const C *Xc = static_cast<const C *>(swap ? a.X[0] : a.X[1]);
  const int64_t *offr = swap ? a.off[1] : a.off[0];
  const int64_t *offc = swap ? a.off[0] : a.off[1];
  const int64_t ro = offr[idx], n = offr[idx + 1] - ro;
  const int64_t co = offc[idx], m = offc[idx + 1] - co;

  V q[M][D];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int64_t jj = j < m ? j : m - 1;
#pragma unroll
    for (int c = 0; c < D; ++c) q[j][c] = N::cvt(Xc[(co + jj) * D + c]);
  }
  V row[M];
#pragma unroll
  for (int j = 0; j < M; ++j) row[j] = N::inf();

  // the points of the rows, loaded kAhead rows before they are swept (a
  // lane's loads are gathers from its own curve; a row of 16 columns is
  // shorter than their latency)
  constexpr int kAhead = 8;
  C nxt[kAhead][D];
#pragma unroll
  for (int r = 0; r < kAhead; ++r) {
    const int64_t ir = r < n ? r : n - 1;
#pragma unroll
    for (int c = 0; c < D; ++c) nxt[r][c] = Xr[(ro + ir) * D + c];
  }
  for (int64_t i0 = 0; i0 < n; i0 += kAhead) {
#pragma unroll
    for (int r = 0; r < kAhead; ++r) {
      const int64_t i = i0 + r;
      if (i < n) {
        V p[D];
#pragma unroll
        for (int c = 0; c < D; ++c) p[c] = N::cvt(nxt[r][c]);
        const int64_t in = i + kAhead < n ? i + kAhead : n - 1;
#pragma unroll
        for (int c = 0; c < D; ++c) nxt[r][c] = Xr[(ro + in) * D + c];
        V diag = i == 0 ? -N::inf() : N::inf();  // M_{i-1,-1}: the corner above the first row
        V left = N::inf();                       // M_{i,-1}
#pragma unroll
        for (int j = 0; j < M; ++j) {
          V t = p[0] - q[j][0];
          V d = t * t;
#pragma unroll
          for (int c = 1; c < D; ++c) {
            V w = p[c] - q[j][c];
            d = N::fma(w, w, d);
          }
          const V v = N::mx(N::mn(N::mn(row[j], diag), left), d);
          diag = row[j];
          row[j] = v;
          left = v;
        }
      }
    }
  }
  N::store(a.out, idx, row[M - 1], a.metric);
}

template <int M, typename V>
hipError_t launch_m(int D, const LaneArgs &a, hipStream_t st) {
  const unsigned blocks = (unsigned)((a.npairs + 255) / 256);
  switch (D) {
    case 1: hipLaunchKernelGGL((lane_kernel<M, 1, V>), dim3(blocks), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((lane_kernel<M, 2, V>), dim3(blocks), dim3(256), 0, st, a); break;
    case 3:
      if constexpr (M <= lane_cols_max(sizeof(V) == 8, 3)) {
        hipLaunchKernelGGL((lane_kernel<M, 3, V>), dim3(blocks), dim3(256), 0, st, a);
        break;
      }
      return hipErrorInvalidValue;
    case 4:
      if constexpr (M <= lane_cols_max(sizeof(V) == 8, 4)) {
        hipLaunchKernelGGL((lane_kernel<M, 4, V>), dim3(blocks), dim3(256), 0, st, a);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename V>
hipError_t launch_v(int M, int D, const LaneArgs &a, hipStream_t st) {
  if (M > lane_cols_max(sizeof(V) == 8, D)) return hipErrorInvalidValue;
  switch (M) {
    case 16: return launch_m<16, V>(D, a, st);
    case 32: return launch_m<32, V>(D, a, st);
    case 64:
      if constexpr (sizeof(V) == 4) return launch_m<64, V>(D, a, st);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_lanes(bool exact, int M, int D, const LaneArgs &a, hipStream_t st) {
  if (a.npairs <= 0) return hipSuccess;
  return exact ? launch_v<double>(M, D, a, st) : launch_v<float>(M, D, a, st);
}

}  // namespace ffd
