// Early-abandoning discrete Frechet sweep: the decider "is delta <= eps?"
// and the exact evaluations of the k-nearest-neighbour search.
//
// The recurrence is Eq. (1) of arXiv 2404.05708 on squared Euclidean cells
// in float32, with the same cell expression as the streaming kernels
// (d2 = dx*dx, then d2 = fma(dk, dk, d2)), so every value that is not
// abandoned has the same bits as theirs.
//
// Mapping: one wave takes one pair at a time from a work counter; lane l
// holds R consecutive rows of a band of 64 R rows and computes column t - l
// at step t (the row above comes from lane l - 1 through a DPP shift).  A
// band starts with an empty pipeline (64 steps of ramp); the bottom row of
// a band goes to the wave's scratch row in global memory for the next band
// of the same pair.
//
// Early abandoning.  M_ij is the smallest, over monotone paths from (0, 0)
// to (i, j), of the largest cell on the path, so delta = M_PQ is at least
// M of every cell of a set that each full path must cross.  After each
// group of 16 steps the wave checks such a set: every lane's current cells
// (rows i at column c_l = t - l), the value each lane last received from the
// lane above (row i - 1 at column c_l: a path can step diagonally past the
// staircase there), in bands after the first the smallest value of the band
// above's bottom row to the right of lane 0's column (kept as suffix
// minima), and in bands before the last the smallest value of this band's
// bottom row so far (a path can leave the band downwards left of the
// staircase).  Rows not yet reached hold +inf.  If every one of them exceeds the
// threshold, so does delta, and the wave drops the pair (+inf) and takes the
// next one.  The check stops once lane 0 passes the last column: cells
// beyond the column curve's end are not cells of the table.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ffd_bounded.h"
#include "ffd_plan.h"

namespace ffd {

namespace {

constexpr int kWaveB = 64;
constexpr int kGroupB = 16;

__device__ __forceinline__ float shift_in(float old, float src) {
  int r = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, src),
                                      0x138 /* wave_shr:1 */, 0xf, 0xf, false);
  return __builtin_bit_cast(float, r);
}

__device__ __forceinline__ float load_l2(const float *p) {
  // rows written by this wave earlier: read past the vector L1
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// D = 8 and 16 are the kernels of curves with 5 to 16 coordinates (GEN): a
// point has a.dim coordinates in memory and zeros past them in registers,
// which leaves every cell's bits unchanged (a zero difference adds an exact
// zero); they read each column point at its step rather than a group ahead,
// since a group would take 8 or 16 registers per point and step.
template <int R, int D>
struct Bounded {
  static constexpr bool GEN = D > 4;
  static constexpr int QG = GEN ? 1 : kGroupB;  // column points held a group ahead
  const BoundedArgs &a;
  int lane;
  float *hand0;  // two bottom rows (this band, the band above) and suffix minima
  float *smin;

  __device__ Bounded(const BoundedArgs &args, int lane_, int wave) : a(args), lane(lane_) {
    hand0 = a.rows + (int64_t)wave * 3 * a.row_cap;
    smin = hand0 + 2 * a.row_cap;
  }

  // values per point in the input arrays, and value k of the point at pt
  __device__ int32_t in_dim() const {
    if constexpr (GEN) return a.dim;
    else return D;
  }
  __device__ float coord(const float *pt, int k) const {
    if constexpr (GEN) return k < a.dim ? pt[k] : 0.0f;
    else return pt[k];
  }

  // The column point of step t for this lane (column t - lane, clamped to
  // the last; columns before the first are +inf points).
  __device__ __forceinline__ void load_point(int32_t t, const float *qb, int32_t m, float (&q)[D]) const {
    int32_t j = t - lane;
    const bool sep = j < 0;
    j = sep ? 0 : (j > m - 1 ? m - 1 : j);
    const float *pt = qb + (int64_t)j * in_dim();
#pragma unroll
    for (int k2 = 0; k2 < D; ++k2) q[k2] = sep ? __builtin_huge_valf() : coord(pt, k2);
  }

  // Column points of the group starting at t0 for this lane (columns
  // t0 + u - lane, clamped to the last; columns before the first are +inf
  // points, so their cells are +inf) and lane 0's row-above values.
  // (The host keeps m * D below 2^31, so 32-bit offsets from the curve's
  // first point address every column.)
  __device__ __forceinline__ void load_group(int32_t t0, const float *qb, int32_t m, bool above,
                                             const float *hin, float (&q)[QG][D], float (&h)[kGroupB]) {
    if constexpr (GEN) {
      // the points are read at their steps (load_point)
#pragma unroll
      for (int u = 0; u < kGroupB; ++u) {
        int32_t c = t0 + u;
        h[u] = above && c < m ? load_l2(hin + c) : __builtin_huge_valf();
      }
    } else if (t0 >= kWaveB - 1 && t0 + kGroupB <= m) {
      // every lane's 16 columns lie inside the curve: no separators and no
      // clamping, one base address and immediate offsets
      const float *qc = qb + (t0 - lane) * D;
#pragma unroll
      for (int u = 0; u < kGroupB; ++u)
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) q[u][k2] = qc[u * D + k2];
      if (above) {
#pragma unroll
        for (int u = 0; u < kGroupB; ++u) h[u] = load_l2(hin + t0 + u);
      } else {
#pragma unroll
        for (int u = 0; u < kGroupB; ++u) h[u] = __builtin_huge_valf();
      }
    } else {
#pragma unroll
      for (int u = 0; u < kGroupB; ++u) {
        int32_t j = t0 + u - lane;
        const bool sep = j < 0;
        j = sep ? 0 : (j > m - 1 ? m - 1 : j);
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) q[u][k2] = sep ? __builtin_huge_valf() : qb[j * D + k2];
        int32_t c = t0 + u;
        h[u] = above && c < m ? load_l2(hin + c) : __builtin_huge_valf();
      }
    }
  }

  // Suffix minima of the bottom row just written (m values): smin[j] =
  // min(row[j .. m - 1]), smin[m] = +inf.
  __device__ void suffix_minima(const float *row, int32_t m) {
    const float inf = __builtin_huge_valf();
    int32_t chunk = (m + kWaveB - 1) / kWaveB;
    int32_t lo = lane * chunk, hi = lo + chunk < m ? lo + chunk : m;
    float cm = inf;
    for (int32_t j = lo; j < hi; ++j) cm = __builtin_fminf(cm, load_l2(row + j));
    float s = cm;
    for (int d = 1; d < kWaveB; d <<= 1) {
      float o = __shfl_down(s, d, kWaveB);
      if (lane + d < kWaveB) s = __builtin_fminf(s, o);
    }
    float run = __shfl_down(s, 1, kWaveB);
    if (lane == kWaveB - 1) run = inf;
    for (int32_t j = hi - 1; j >= lo; --j) {
      run = __builtin_fminf(run, load_l2(row + j));
      smin[j] = run;
    }
    if (lane == 0) smin[m] = inf;
  }

  // One pair; returns the value lane `ln` holds for M_{n-1,m-1} (squared),
  // or +inf on every lane when the pair was abandoned.
  // (swap: the pair's curves exchange roles, row curve ci of the second set
  // against column curve ri of the first; the distance is symmetric)
  __device__ float pair(int32_t ri, int32_t ci, bool swap, float eps2, int &ln_out) {
    const float inf = __builtin_huge_valf();
    const float *Xr = swap ? a.X1 : a.X0, *Xc = swap ? a.X0 : a.X1;
    const int64_t *offr = swap ? a.off1 : a.off0, *offc = swap ? a.off0 : a.off1;
    if (swap) {
      const int32_t t = ri;
      ri = ci;
      ci = t;
    }
    const int64_t ro = offr[ri], n = offr[ri + 1] - ro;
    const int64_t co = offc[ci];
    const int32_t m = (int32_t)(offc[ci + 1] - co);
    const float *qb = Xc + co * in_dim();
    const int64_t band_rows = (int64_t)kWaveB * R;
    const int nb = (int)((n + band_rows - 1) / band_rows);
    const int64_t last = (n - 1) - (int64_t)(nb - 1) * band_rows;
    const int ln = (int)(last / R), rn = (int)(last % R);
    const int32_t T = (int32_t)((m + kWaveB - 1 + kGroupB - 1) / kGroupB * kGroupB);
    ln_out = ln;
    float res = inf;
    for (int b = 0; b < nb; ++b) {
      const float *hin = hand0 + ((b + 1) & 1) * a.row_cap;
      float *hout = hand0 + (b & 1) * a.row_cap;
      const bool above = b > 0, store = b < nb - 1, last_band = b == nb - 1;
      float p[R][D];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int64_t i = (int64_t)b * band_rows + (int64_t)lane * R + r;
        if (i > n - 1) i = n - 1;
        const float *pt = Xr + (ro + i) * in_dim();
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) p[r][k2] = coord(pt, k2);
      }
      float Mp[R];
#pragma unroll
      for (int r = 0; r < R; ++r) Mp[r] = inf;
      // lane 0's diagonal at column 0: the corner (-inf) in the first band,
      // M_{i-1,-1} = +inf below it
      float upPrev = above ? inf : -inf;
      float bmin = inf;  // lane 63: smallest bottom-row value so far
      float qn[QG][D], hn[kGroupB];
      load_group(0, qb, m, above, hin, qn, hn);
      bool dead = false;
      for (int32_t t0 = 0; t0 < T; t0 += kGroupB) {
        float q[QG][D], h[kGroupB];
#pragma unroll
        for (int u = 0; u < kGroupB; ++u) h[u] = hn[u];
#pragma unroll
        for (int u = 0; u < QG; ++u)
#pragma unroll
          for (int k2 = 0; k2 < D; ++k2) q[u][k2] = qn[u][k2];
        if (t0 + kGroupB < T) load_group(t0 + kGroupB, qb, m, above, hin, qn, hn);
        float hb[kGroupB];
#pragma unroll
        for (int u = 0; u < kGroupB; ++u) {
          const int32_t t = t0 + u;
          float qv[D];
          if constexpr (GEN) {
            load_point(t, qb, m, qv);
          } else {
#pragma unroll
            for (int k2 = 0; k2 < D; ++k2) qv[k2] = q[GEN ? 0 : u][k2];
          }
          float up = shift_in(h[u], Mp[R - 1]);
          float above_v = up, diag = upPrev;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            float dx = p[r][0] - qv[0];
            float s = dx * dx;
#pragma unroll
            for (int k2 = 1; k2 < D; ++k2) {
              float w = p[r][k2] - qv[k2];
              s = __builtin_fmaf(w, w, s);
            }
            float v = __builtin_fmaxf(__builtin_fminf(__builtin_fminf(above_v, diag), Mp[r]), s);
            diag = Mp[r];
            above_v = v;
            Mp[r] = v;
          }
          upPrev = up;
          hb[u] = Mp[R - 1];
          if (last_band && t == m - 1 + ln) {
            float sel = Mp[0];
#pragma unroll
            for (int r = 1; r < R; ++r) sel = rn == r ? Mp[r] : sel;
            res = lane == ln ? sel : res;
          }
        }
        if (store) {
          // this band's bottom row so far (lane 63's value is the one used;
          // columns before the first are not cells)
          if (t0 >= kWaveB - 1) {
#pragma unroll
            for (int u = 0; u < kGroupB; u += 2) bmin = __builtin_fminf(bmin, __builtin_fminf(hb[u], hb[u + 1]));
          } else {
#pragma unroll
            for (int u = 0; u < kGroupB; ++u) bmin = __builtin_fminf(bmin, t0 + u - lane < 0 ? inf : hb[u]);
          }
        }
        if (store && lane == kWaveB - 1) {
#pragma unroll
          for (int u = 0; u < kGroupB; ++u) {
            int32_t c = t0 + u - (kWaveB - 1);
            if (c >= 0 && c < m) hout[c] = hb[u];
          }
        }
        if (t0 + kGroupB - 1 <= m - 1) {
          float f = upPrev;
#pragma unroll
          for (int r = 0; r < R; ++r) f = __builtin_fminf(f, Mp[r]);
          if (above && lane == 0) f = __builtin_fminf(f, load_l2(smin + t0 + kGroupB));
          if (store && lane == kWaveB - 1) f = __builtin_fminf(f, bmin);
          if (__ballot(!(f > eps2)) == 0) {
            dead = true;
            break;
          }
        }
      }
      if (dead) return inf;
      if (store) {
        __threadfence();
        suffix_minima(hout, m);
        __threadfence();
      }
    }
    return res;
  }
};

template <int R, int D>
__global__ __launch_bounds__(256, 2) void bounded_kernel(BoundedArgs a) {
  const int lane = threadIdx.x & (kWaveB - 1);
  const int wave = (int)(blockIdx.x * (blockDim.x / kWaveB) + threadIdx.x / kWaveB);
  Bounded<R, D> s(a, lane, wave);
  for (;;) {
    uint32_t k = 0;
    if (lane == 0) k = atomicAdd(a.counter, 1u);
    k = __builtin_amdgcn_readfirstlane(k);
    if ((int64_t)k >= a.npairs) break;
    // the top bit of a work item marks a pair swept with its curves' roles
    // exchanged (decider only: no fixed row, no (row, column) mapping)
    const int32_t raw = a.order[k];
    const bool swap = raw < 0;
    const int32_t idx = raw & 0x7fffffff;
    int32_t ri = a.fixed_row >= 0 ? a.fixed_row : idx, ci = idx;
    if (a.col_count > 0) {
      const int32_t row = idx / (int32_t)a.col_count;
      ci = idx - row * (int32_t)a.col_count;
      if (a.fixed_row < 0) ri = row;
    }
    const float eps2 = a.row_eps2 ? a.row_eps2[ri] : a.eps2;
    int ln = 0;
    float v = s.pair(ri, ci, swap, eps2, ln);
    if (lane == ln) {
      float o = __builtin_huge_valf();
      if (v <= eps2) o = a.metric == 0 ? (float)__builtin_sqrt((double)v) : v;
      a.out[idx] = o;
    }
  }
}

// Squared distances of the first points and of the last points of a query
// and every database curve, in the cells' float32 expression: every
// coupling contains both corner cells, so delta^2 is at least the larger.
template <int D>
__global__ void endpoint_bound_kernel(const float *q, int64_t n, const float *X, const int64_t *off, int64_t count,
                                      float *lb) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const float *a0 = X + off[c] * D, *a1 = X + (off[c + 1] - 1) * D;
  const float *q1 = q + (n - 1) * D;
  float dx = q[0] - a0[0], s0 = dx * dx;
  float ex = q1[0] - a1[0], s1 = ex * ex;
#pragma unroll
  for (int k2 = 1; k2 < D; ++k2) {
    float w = q[k2] - a0[k2];
    s0 = __builtin_fmaf(w, w, s0);
    float z = q1[k2] - a1[k2];
    s1 = __builtin_fmaf(z, z, s1);
  }
  lb[c] = __builtin_fmaxf(s0, s1);
}

// The same bound for nq queries (CSR offsets q_off) against every curve:
// lb[i * count + c].
template <int D>
__global__ void endpoint_bound_batch_kernel(const float *Q, const int64_t *q_off, int64_t nq, const float *X,
                                            const int64_t *off, int64_t count, float *lb) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nq * count) return;
  const int64_t i = g / count, c = g - i * count;
  const float *q0 = Q + q_off[i] * D, *q1 = Q + (q_off[i + 1] - 1) * D;
  const float *a0 = X + off[c] * D, *a1 = X + (off[c + 1] - 1) * D;
  float dx = q0[0] - a0[0], s0 = dx * dx;
  float ex = q1[0] - a1[0], s1 = ex * ex;
#pragma unroll
  for (int k2 = 1; k2 < D; ++k2) {
    float w = q0[k2] - a0[k2];
    s0 = __builtin_fmaf(w, w, s0);
    float z = q1[k2] - a1[k2];
    s1 = __builtin_fmaf(z, z, s1);
  }
  lb[g] = __builtin_fmaxf(s0, s1);
}

// The bounds for curves of 5 to 16 coordinates (dim at run time).
__device__ __forceinline__ float corner_cell(const float *x, const float *y, int dim) {
  float dx = x[0] - y[0], s = dx * dx;
  for (int k2 = 1; k2 < dim; ++k2) {
    float w = x[k2] - y[k2];
    s = __builtin_fmaf(w, w, s);
  }
  return s;
}

__global__ void endpoint_bound_wide_kernel(const float *q, int64_t n, const float *X, const int64_t *off,
                                           int64_t count, int dim, float *lb) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const float *a0 = X + off[c] * dim, *a1 = X + (off[c + 1] - 1) * dim;
  lb[c] = __builtin_fmaxf(corner_cell(q, a0, dim), corner_cell(q + (n - 1) * dim, a1, dim));
}

__global__ void endpoint_bound_batch_wide_kernel(const float *Q, const int64_t *q_off, int64_t nq, const float *X,
                                                 const int64_t *off, int64_t count, int dim, float *lb) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nq * count) return;
  const int64_t i = g / count, c = g - i * count;
  const float *q0 = Q + q_off[i] * dim, *q1 = Q + (q_off[i + 1] - 1) * dim;
  const float *a0 = X + off[c] * dim, *a1 = X + (off[c + 1] - 1) * dim;
  lb[g] = __builtin_fmaxf(corner_cell(q0, a0, dim), corner_cell(q1, a1, dim));
}

template <int R>
hipError_t launch_r(int D, const BoundedArgs &a, int blocks, hipStream_t st) {
  switch (D) {
    case 1: hipLaunchKernelGGL((bounded_kernel<R, 1>), dim3(blocks), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((bounded_kernel<R, 2>), dim3(blocks), dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL((bounded_kernel<R, 3>), dim3(blocks), dim3(256), 0, st, a); break;
    case 4: hipLaunchKernelGGL((bounded_kernel<R, 4>), dim3(blocks), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bounded(int R, int D, const BoundedArgs &a, int nwaves, hipStream_t st) {
  int blocks = (nwaves + 3) / 4;
  if (D > 4) {
    // curves of 5 to 16 coordinates: the kernels of 8 (R = 2) and 16 (R = 1)
    if (R != wide_rows(D) || a.dim != D || D > 16) return hipErrorInvalidValue;
    if (D <= 8) hipLaunchKernelGGL((bounded_kernel<2, 8>), dim3(blocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((bounded_kernel<1, 16>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
  }
  switch (R) {
    case 1: return launch_r<1>(D, a, blocks, st);
    case 2: return launch_r<2>(D, a, blocks, st);
    case 4: return launch_r<4>(D, a, blocks, st);
    case 8: return launch_r<8>(D, a, blocks, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_endpoint_bound(int D, const float *q, int64_t n, const float *X, const int64_t *off, int64_t count,
                                 float *lb, hipStream_t st) {
  unsigned blocks = (unsigned)((count + 255) / 256);
  if (D > 4) {
    hipLaunchKernelGGL(endpoint_bound_wide_kernel, dim3(blocks), dim3(256), 0, st, q, n, X, off, count, D, lb);
    return hipGetLastError();
  }
  switch (D) {
    case 1: hipLaunchKernelGGL(endpoint_bound_kernel<1>, dim3(blocks), dim3(256), 0, st, q, n, X, off, count, lb); break;
    case 2: hipLaunchKernelGGL(endpoint_bound_kernel<2>, dim3(blocks), dim3(256), 0, st, q, n, X, off, count, lb); break;
    case 3: hipLaunchKernelGGL(endpoint_bound_kernel<3>, dim3(blocks), dim3(256), 0, st, q, n, X, off, count, lb); break;
    case 4: hipLaunchKernelGGL(endpoint_bound_kernel<4>, dim3(blocks), dim3(256), 0, st, q, n, X, off, count, lb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_endpoint_bound_batch(int D, const float *Q, const int64_t *q_off, int64_t nq, const float *X,
                                       const int64_t *off, int64_t count, float *lb, hipStream_t st) {
  unsigned blocks = (unsigned)((nq * count + 255) / 256);
  if (D > 4) {
    hipLaunchKernelGGL(endpoint_bound_batch_wide_kernel, dim3(blocks), dim3(256), 0, st, Q, q_off, nq, X, off, count,
                       D, lb);
    return hipGetLastError();
  }
  switch (D) {
#define FFD_EPB_CASE(d)                                                                                           \
  case d:                                                                                                         \
    hipLaunchKernelGGL(endpoint_bound_batch_kernel<d>, dim3(blocks), dim3(256), 0, st, Q, q_off, nq, X, off, count, \
                       lb);                                                                                       \
    break;
    FFD_EPB_CASE(1) FFD_EPB_CASE(2) FFD_EPB_CASE(3) FFD_EPB_CASE(4)
#undef FFD_EPB_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ffd
