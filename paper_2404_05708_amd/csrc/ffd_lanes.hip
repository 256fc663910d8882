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
// everywhere else in the library (d2 = dx*dx, then fma(dk, dk, d2); for
// Manhattan and Chebyshev cells |d0|, then the sum or maximum with |dk|;
// FP64 for int32 coordinates) and the Euclidean root is taken once per
// pair, so the results equal the streaming kernels' bit for bit.
//
// A lane sweeps its rows two at a time, both rows' cells of a column
// together: the second row's cell takes the first row's as its value above,
// so the two chains of selections (one per row, through the left
// neighbours) overlap in the instruction stream.  A curve of odd length has
// its last point repeated once more (exact, as above).
//
// Dynamic time warping (Appendix B, Algorithm B.1: the outer max becomes a
// sum, the corner 0) runs on the same sweep; sums are not selections, so
// there the padding is not exact: the result is read at the column curve's
// own last column (columns to its right never feed it), and the second row
// of a pair is dropped when the row curve has no row left.  The Levenshtein
// distance (Appendix B, Algorithm B.2; CELL 4) likewise: int32 symbol
// vectors compared as bit patterns, integer table values in float32 (exact
// below 2^24), M_ij = min(min(M_{i-1,j}, M_{i,j-1}) + 1, M_{i-1,j-1} + d_ij)
// with the ramps M_{-1,j} = j + 1, M_{i,-1} = i + 1 and a 0 corner, as the
// streaming kernel evaluates it.
//
// One launch covers every class of column count (multiples of 8 up to 64
// columns; the registers are those of the widest class), its workgroups of
// the widest class first; the host sorts the pairs of a class by row count, so that the
// lanes of a wavefront sweep about as many rows each and the longest
// wavefronts start first.
#include "ffd_lanes.h"

#include "ffd_stream.h"

namespace ffd {

namespace {

// The ground distance of a cell (CELL 0 squared Euclidean, 2 Manhattan, 3
// Chebyshev, 4 the Levenshtein symbol mismatch), in the streaming kernels'
// order of operations.
template <int D, typename V, int CELL>
__device__ __forceinline__ V cell_value(const V (&p)[D], const V (&q)[D]) {
  using N = Num<V>;
  if constexpr (CELL == 4) {
    bool ne = false;
#pragma unroll
    for (int c = 0; c < D; ++c) ne = ne || __builtin_bit_cast(uint32_t, p[c]) != __builtin_bit_cast(uint32_t, q[c]);
    return ne ? V(1) : V(0);
  } else if constexpr (CELL == 1) {
    return N::sqrt_cell(cell_value<D, V, 0>(p, q));  // DTW of Euclidean cells: a root per cell
  } else if constexpr (CELL >= 2) {
    V s = N::abs(p[0] - q[0]);
#pragma unroll
    for (int c = 1; c < D; ++c) {
      V w = N::abs(p[c] - q[c]);
      s = CELL == 2 ? s + w : N::mx(s, w);
    }
    return s;
  } else {
    V t = p[0] - q[0];
    V s = t * t;
#pragma unroll
    for (int c = 1; c < D; ++c) {
      V w = p[c] - q[c];
      s = N::fma(w, w, s);
    }
    return s;
  }
}

template <int M, int D, typename V, int CELL, bool DTW>
__device__ __forceinline__ void lane_pair(const LaneArgs &a, int64_t k) {
  using N = Num<V>;
  using C = typename N::Coord;  // float for Levenshtein: the int32 symbols travel as bit patterns
  constexpr bool LEV = CELL == 4;
  constexpr bool SUM = DTW || LEV;  // not a selection: no exact padding
  const int32_t raw = a.order[k];
  const bool swap = raw < 0;
  const int32_t idx = raw & 0x7fffffff;
  // the pair's curve in each set: the same index, or (query, database curve)
  const int32_t i0 = a.col_count > 0 ? idx / a.col_count : idx;
  const int32_t i1 = a.col_count > 0 ? idx - i0 * a.col_count : idx;
  const C *Xr = static_cast<const C *>(swap ? a.X[1] : a.X[0]);
  const C *Xc = static_cast<const C *>(swap ? a.X[0] : a.X[1]);
  const int32_t *offr = swap ? a.off[1] : a.off[0];
  const int32_t *offc = swap ? a.off[0] : a.off[1];
  const int32_t ir = swap ? i1 : i0, ic = swap ? i0 : i1;
  const int64_t ro = offr[ir], n = offr[ir + 1] - ro;
  const int64_t co = offc[ic], m = offc[ic + 1] - co;

  V q[M][D];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int64_t jj = j < m ? j : m - 1;
#pragma unroll
    for (int c = 0; c < D; ++c) q[j][c] = N::cvt(Xc[(co + jj) * D + c]);
  }
  V row[M];  // M_{-1,j}: +inf (Frechet, DTW), j + 1 (Levenshtein)
#pragma unroll
  for (int j = 0; j < M; ++j) row[j] = LEV ? V(j + 1) : N::inf();

  // the points of the rows, loaded kAhead row pairs before they are swept
  // (a lane's loads are gathers from its own curve)
  constexpr int kAhead = 4;
  // where a slot's next points are loaded: after the row step's branch for
  // the float kernels (measured 2-3 % faster on 262,144 short pairs), inside
  // it for Levenshtein (3 % faster there: one int32 coordinate per point)
  constexpr bool kLoadAfter = !LEV;
  C nxt[kAhead][2][D];
  auto load_pair = [&](int64_t i, C (&dst)[2][D]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t ir = i + h < n ? i + h : n - 1;
#pragma unroll
      for (int c = 0; c < D; ++c) dst[h][c] = Xr[(ro + ir) * D + c];
    }
  };
#pragma unroll
  for (int r = 0; r < kAhead; ++r) load_pair(2 * r, nxt[r]);
  for (int64_t i0 = 0; i0 < n; i0 += 2 * kAhead) {
#pragma unroll
    for (int r = 0; r < kAhead; ++r) {
      const int64_t i = i0 + 2 * r;
      if (i < n) {
        V pa[D], pb[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          pa[c] = N::cvt(nxt[r][0][c]);
          pb[c] = N::cvt(nxt[r][1][c]);  // row i + 1, or row n - 1 again
        }
        if constexpr (!kLoadAfter) load_pair(i + 2 * kAhead, nxt[r]);
        // M_{i-1,-1}: the corner above the first row (-inf for the Frechet
        // distance, 0 for DTW), +inf below it; Levenshtein: the ramp i
        V diag_a = LEV ? V(i) : (i == 0 ? (DTW ? V(0) : -N::inf()) : N::inf());
        V left_a = LEV ? V(i + 1) : N::inf();      // M_{i,-1}
        V diag_b = LEV ? V(i + 1) : N::inf();      // M_{i,-1}
        V left_b = LEV ? V(i + 2) : N::inf();      // M_{i+1,-1}
        const bool two = !SUM || i + 1 < n;        // sums: no repeated row
#pragma unroll
        for (int j = 0; j < M; ++j) {
          V va, vb;
          if constexpr (LEV) {
            // neighbouring values of the table differ by at most one: on a
            // match the diagonal is the least candidate, otherwise the
            // three candidates share the + 1 (the streaming kernel's form)
            va = cell_value<D, V, CELL>(pa, q[j]) == V(0) ? diag_a : N::mn(N::mn(row[j], left_a), diag_a) + V(1);
            vb = cell_value<D, V, CELL>(pb, q[j]) == V(0) ? diag_b : N::mn(N::mn(va, left_b), diag_b) + V(1);
          } else {
            const V da = cell_value<D, V, CELL>(pa, q[j]);
            const V db = cell_value<D, V, CELL>(pb, q[j]);
            if constexpr (DTW) {
              va = N::mn(N::mn(row[j], diag_a), left_a) + da;
              vb = N::mn(N::mn(va, diag_b), left_b) + db;
            } else {
              va = N::mx(N::mn(N::mn(row[j], diag_a), left_a), da);
              vb = N::mx(N::mn(N::mn(va, diag_b), left_b), db);
            }
          }
          diag_a = row[j];
          left_a = va;
          diag_b = va;
          left_b = vb;
          row[j] = SUM ? (two ? vb : va) : vb;
        }
      }
      // the next points into this slot, on every lane (the index is clamped
      // to the curve): a load inside the branch above has to land before
      // the branch ends, where its registers merge with the lanes that
      // skipped it
      if constexpr (kLoadAfter) load_pair(i + 2 * kAhead, nxt[r]);
    }
  }
  if constexpr (SUM) {
    // the value at the column curve's own last column
    V res = row[0];
#pragma unroll
    for (int j = 1; j < M; ++j) res = j == m - 1 ? row[j] : res;
    if constexpr (LEV) static_cast<int64_t *>(a.out)[idx] = (int64_t)res;
    else N::store_value(a.out, idx, res);
  } else if constexpr (CELL == 0) {
    N::store(a.out, idx, row[M - 1], a.metric);
  } else {
    N::store_value(a.out, idx, row[M - 1]);
  }
}

template <int M, int D, typename V, int CELL, bool DTW>
__device__ __forceinline__ void lane_class(const LaneArgs &a, int64_t k) {
  if constexpr (M <= lane_cols_max(sizeof(V) == 8, D)) lane_pair<M, D, V, CELL, DTW>(a, k);
}

template <int D, typename V, int CELL, bool DTW>
__global__ __launch_bounds__(kLaneBlock) void lane_kernel(LaneArgs a) {
  const int64_t b = blockIdx.x;
  int c = 0;
  while (c + 1 < a.classes && b >= a.block_first[c + 1]) ++c;
  const int64_t k = a.first[c] + (b - a.block_first[c]) * kLaneBlock + threadIdx.x;
  if (k >= a.first[c + 1]) return;
  switch (a.cols[c]) {
    case 64: lane_class<64, D, V, CELL, DTW>(a, k); break;
    case 56: lane_class<56, D, V, CELL, DTW>(a, k); break;
    case 48: lane_class<48, D, V, CELL, DTW>(a, k); break;
    case 40: lane_class<40, D, V, CELL, DTW>(a, k); break;
    case 32: lane_class<32, D, V, CELL, DTW>(a, k); break;
    case 24: lane_class<24, D, V, CELL, DTW>(a, k); break;
    case 16: lane_class<16, D, V, CELL, DTW>(a, k); break;
    default: lane_class<8, D, V, CELL, DTW>(a, k); break;
  }
}

template <typename V, int CELL, bool DTW>
hipError_t launch_c(int D, const LaneArgs &a, hipStream_t st) {
  const unsigned blocks = (unsigned)a.block_first[a.classes];
  switch (D) {
    case 1: hipLaunchKernelGGL((lane_kernel<1, V, CELL, DTW>), dim3(blocks), dim3(kLaneBlock), 0, st, a); break;
    case 2: hipLaunchKernelGGL((lane_kernel<2, V, CELL, DTW>), dim3(blocks), dim3(kLaneBlock), 0, st, a); break;
    case 3: hipLaunchKernelGGL((lane_kernel<3, V, CELL, DTW>), dim3(blocks), dim3(kLaneBlock), 0, st, a); break;
    case 4: hipLaunchKernelGGL((lane_kernel<4, V, CELL, DTW>), dim3(blocks), dim3(kLaneBlock), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename V>
hipError_t launch_v(int D, const LaneArgs &a, hipStream_t st) {
  for (int c = 0; c < a.classes; ++c)
    if (a.cols[c] > lane_cols_max(sizeof(V) == 8, D)) return hipErrorInvalidValue;
  if (a.dtw) {
    switch (a.cell) {
      case 0: return launch_c<V, 0, true>(D, a, st);
      case 1:
        if constexpr (sizeof(V) == 4) return launch_c<V, 1, true>(D, a, st);  // float32 coordinates only
        return hipErrorInvalidValue;
      case 2: return launch_c<V, 2, true>(D, a, st);
      case 3: return launch_c<V, 3, true>(D, a, st);
    }
    return hipErrorInvalidValue;
  }
  switch (a.cell) {
    case 0: return launch_c<V, 0, false>(D, a, st);
    case 2: return launch_c<V, 2, false>(D, a, st);
    case 3: return launch_c<V, 3, false>(D, a, st);
    case 4:
      if constexpr (sizeof(V) == 4) return launch_c<V, 4, false>(D, a, st);  // Levenshtein: float32 values
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_lanes(bool exact, int D, const LaneArgs &a, hipStream_t st) {
  if (a.classes < 1 || a.classes > kLaneClasses || a.block_first[a.classes] <= 0) return hipSuccess;
  return exact ? launch_v<double>(D, a, st) : launch_v<float>(D, a, st);
}

}  // namespace ffd
