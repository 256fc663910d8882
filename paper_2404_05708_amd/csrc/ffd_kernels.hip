// Discrete Frechet distance kernels for gfx950 (CDNA4, wave64).
//
// The recurrence is Eq. (1) of Meinert, arXiv 2404.05708:
//   M_ij = max{ min{M_{i-1,j}, M_{i-1,j-1}, M_{i,j-1}}, d_ij },  delta = M_PQ,
// evaluated branch-free with O(Q) state (Theorem 1; Algorithms 2 and 5) and
// with d_ij computed lazily per cell.  The paper parallelises across curves
// (Sec. 4); because the max-min step is not associative (Sec. 4) the only
// parallelism inside one pair is the anti-diagonal, which is what a wave
// sweeps here:
//
//  * lane l of a wave holds R consecutive rows of the row curve and, at step
//    t, computes column t - l; the value of the row above its top row comes
//    from lane l-1 through a full-wave DPP shift (wave_shr:1), the previous
//    step's copy of it is the diagonal, and the lane's own previous values
//    are the left neighbours -- two live anti-diagonals in registers;
//  * lane 0 takes the row above from LDS: the bottom row of the band above
//    (written by lane 63 earlier in the same stream) or the top boundary;
//  * column points stream through a 256-entry LDS ring that the wave refills
//    every 64 steps, one entry per lane, from global memory;
//  * every task starts with a separator column whose point is +inf in every
//    coordinate, so d = +inf in that column for every row: this resets the
//    left neighbours to +inf (the boundary M_{i,0} = +inf) without a branch,
//    and a -inf entry of the top boundary at the separator gives the corner
//    M_{0,0} = -inf, which makes Eq. (1) produce the first row and column
//    (running maxima, Algorithms 3-5) by itself;
//  * rows past the end of a curve repeat its last point and columns past the
//    end repeat its last column point: repeating points does not change the
//    distance (Sec. 4, footnote), so padding is exact.
//
// The squared distance is evaluated as d2 = dx*dx, then d2 = fma(dk, dk, d2)
// for k >= 1, in the value type; the recurrence runs on d2 and the Euclidean
// result is the correctly rounded square root of the selected d2 (min and
// max commute with the monotone square root).  The exact path widens int32
// coordinates to FP64, where every operation on these integers is exact.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ffd_plan.h"

namespace ffd {

template <typename V>
struct Num;

template <>
struct Num<float> {
  using Coord = float;
  __device__ static __forceinline__ float inf() { return __builtin_huge_valf(); }
  __device__ static __forceinline__ float cvt(float x) { return x; }
  __device__ static __forceinline__ float mn(float a, float b) { return __builtin_fminf(a, b); }
  __device__ static __forceinline__ float mx(float a, float b) { return __builtin_fmaxf(a, b); }
  __device__ static __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
  // Lane l receives src of lane l-1; lane 0 keeps `old`.
  __device__ static __forceinline__ float shift_in(float old, float src) {
    int r = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, src),
                                        0x138 /* wave_shr:1 */, 0xf, 0xf, false);
    return __builtin_bit_cast(float, r);
  }
  __device__ static __forceinline__ void store(void *out, int64_t idx, float v, int metric) {
    float r = metric == 0 ? (float)__builtin_sqrt((double)v) : v;
    static_cast<float *>(out)[idx] = r;
  }
};

template <>
struct Num<double> {
  using Coord = int32_t;
  __device__ static __forceinline__ double inf() { return __builtin_huge_val(); }
  __device__ static __forceinline__ double cvt(int32_t x) { return (double)x; }
  __device__ static __forceinline__ double mn(double a, double b) { return __builtin_fmin(a, b); }
  __device__ static __forceinline__ double mx(double a, double b) { return __builtin_fmax(a, b); }
  __device__ static __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
  __device__ static __forceinline__ double shift_in(double old, double src) {
    uint64_t o = __builtin_bit_cast(uint64_t, old), s = __builtin_bit_cast(uint64_t, src);
    int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)s, 0x138, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(s >> 32), 0x138,
                                         0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  }
  __device__ static __forceinline__ void store(void *out, int64_t idx, double v, int) {
    static_cast<int64_t *>(out)[idx] = (int64_t)v;
  }
};

// Task descriptor kept in LDS (32 bytes).
struct Desc {
  int32_t S;          // stream position of the separator
  int32_t L;          // stream length
  int32_t ghost;      // 1: lane 0 reads the top boundary, 0: the hand-off row
  int32_t hand_out;   // 1: lane 63 writes the hand-off row for the next task
  int32_t out_lo, out_hi;  // result index, -1 = none
  int32_t drain;      // 1: padding task after the last job
  int32_t pad;
};

__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int R, int D, typename V>
struct Stream {
  using N = Num<V>;
  using C = typename N::Coord;
  static constexpr int DP = D == 3 ? 4 : D;
  struct alignas(sizeof(V) * DP) Pt {
    V c[DP];
  };

  const KernelArgs &a;
  int lane;
  LdsLayout lay;
  unsigned char *base;  // this wave's LDS region

  // ---- fill cursor: enumerates tasks (job, column curve, band) --------------
  int32_t j, jend;          // job range of this wave
  int32_t c, b, nb;         // column curve within the job, band, bands of the row curve
  int32_t row_sel, col_sel, col_first, col_count, out_stride;
  int64_t row_off, n, out_base;
  bool exhausted;
  int32_t next_id;          // id of the next task to create
  // task covering the current fill chunk start, and the one after it
  int32_t cS, cL, cdrain, ccol_sel; int64_t ccol_off, cm;
  int32_t xS, xL, xdrain, xcol_sel; int64_t xcol_off, xm;
  bool has_next;
  // per-lane prefetch registers
  C qbuf[D];
  bool qsep;
  C ptmp[R][D];
  bool ptmp_pending;
  int32_t ptmp_slot;

  __device__ Stream(const KernelArgs &args, int lane_, unsigned char *b_) : a(args), lane(lane_), base(b_) {}

  __device__ Pt *ring() const { return reinterpret_cast<Pt *>(base + lay.ring); }
  __device__ V *ghost() const { return reinterpret_cast<V *>(base + lay.ghost); }
  __device__ V *sink() const { return reinterpret_cast<V *>(base + lay.sink); }
  __device__ V *hand() const { return reinterpret_cast<V *>(base + lay.hand); }
  __device__ V *pst(int slot) const { return reinterpret_cast<V *>(base + lay.pst) + slot * (kWave * R * D); }
  __device__ Desc *desc(int id) const { return reinterpret_cast<Desc *>(base + lay.desc) + (id & (kDescSlots - 1)); }

  // Kernel-argument arrays are only indexed with selects: a dynamic index
  // would make the compiler copy the arguments to scratch memory.
  __device__ const C *coords(int sel) const {
    return static_cast<const C *>(sel ? a.X[1] : a.X[0]);
  }
  __device__ int64_t curve_off(int sel, int64_t idx) const {
    if (a.jobs == nullptr) {
      int64_t lo = sel ? a.inl_off[1][0] : a.inl_off[0][0];
      int64_t hi = sel ? a.inl_off[1][1] : a.inl_off[0][1];
      return idx == 0 ? lo : hi;
    }
    return (sel ? a.off[1] : a.off[0])[idx];
  }

  __device__ void load_job(int32_t jj) {
    int32_t ri;
    if (a.jobs) {
      const Job *jb = a.jobs + jj;
      row_sel = uni(jb->row_sel);
      ri = uni(jb->row_idx);
      col_sel = uni(jb->col_sel);
      col_first = uni(jb->col_first);
      col_count = uni(jb->col_count);
      out_stride = uni(jb->out_stride);
      out_base = uni64(jb->out_base);
    } else {
      row_sel = a.inl_job.row_sel;
      ri = a.inl_job.row_idx;
      col_sel = a.inl_job.col_sel;
      col_first = a.inl_job.col_first;
      col_count = a.inl_job.col_count;
      out_stride = a.inl_job.out_stride;
      out_base = a.inl_job.out_base;
    }
    row_off = uni64(curve_off(row_sel, ri));
    n = uni64(curve_off(row_sel, ri + 1)) - row_off;
    nb = (int32_t)bands_for(n, R);
    c = 0;
    b = 0;
  }

  // Create the next task in stream order starting at position S.  Writes its
  // descriptor, issues the loads of its band rows into ptmp, and returns its
  // stream parameters through the output references.
  __device__ void make_task(int32_t S, int32_t &L, int32_t &drain, int32_t &csel, int64_t &coff,
                            int64_t &m) {
    int32_t id = next_id++;
    Desc d;
    d.S = S;
    d.pad = 0;
    if (exhausted) {
      L = kMinTask;
      drain = 1;
      csel = 0;
      coff = 0;
      m = 1;
      d.L = L; d.ghost = 1; d.hand_out = 0; d.out_lo = -1; d.out_hi = -1; d.drain = 1;
    } else {
      int32_t k = col_first + c;
      coff = uni64(curve_off(col_sel, k));
      m = uni64(curve_off(col_sel, k + 1)) - coff;
      csel = col_sel;
      bool chained = nb > 1;
      L = (int32_t)task_len(m, chained);
      drain = 0;
      int64_t oi = (b == nb - 1) ? out_base + (int64_t)c * out_stride : -1;
      d.L = L; d.ghost = b == 0; d.hand_out = b + 1 < nb; d.drain = 0;
      d.out_lo = (int32_t)(uint32_t)(uint64_t)oi;
      d.out_hi = (int32_t)(uint32_t)((uint64_t)oi >> 32);
      // band rows of this lane, clamped to the last point (repetition is exact)
      const C *X = coords(row_sel);
      int64_t r0 = (int64_t)b * kWave * R + (int64_t)lane * R;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int64_t ri = r0 + r < n ? r0 + r : n - 1;
        const C *pt = X + (row_off + ri) * D;
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) ptmp[r][k2] = pt[k2];
      }
      ptmp_pending = true;
      ptmp_slot = id & 1;
      // advance: next band, next column curve, next job
      if (++b == nb) {
        b = 0;
        if (++c == col_count) {
          if (++j == jend) exhausted = true;
          else load_job(j);
        }
      }
    }
    if (lane == 0) *desc(id) = d;
  }

  // Issue the global loads of ring entries [t, t + 64): one per lane.
  __device__ void fill_load(int32_t t) {
    while (cS + cL <= t) {
      if (!has_next) {
        make_task(cS + cL, xL, xdrain, xcol_sel, xcol_off, xm);
        xS = cS + cL;
      }
      cS = xS; cL = xL; cdrain = xdrain; ccol_sel = xcol_sel; ccol_off = xcol_off; cm = xm;
      has_next = false;
    }
    if (cS + cL < t + kFill && !has_next) {
      xS = cS + cL;
      make_task(xS, xL, xdrain, xcol_sel, xcol_off, xm);
      has_next = true;
    }
    int32_t tau = t + lane;
    bool nxt = tau >= cS + cL;
    int32_t x = tau - (nxt ? xS : cS);
    int64_t m = nxt ? xm : cm;
    int64_t co = nxt ? xcol_off : ccol_off;
    int32_t sel = nxt ? xcol_sel : ccol_sel;
    bool drain = nxt ? xdrain : cdrain;
    qsep = drain || x == 0;
    int64_t idx = x - 1;
    if (idx > m - 1) idx = m - 1;
    if (idx < 0) idx = 0;
    if (drain) { co = 0; idx = 0; sel = 0; }
    const C *X = coords(sel);
    const C *pt = X + (co + idx) * D;
#pragma unroll
    for (int k2 = 0; k2 < D; ++k2) qbuf[k2] = pt[k2];
  }

  // Write the entries loaded by the previous fill_load (for positions
  // [t, t + 64)) and any pending band rows.
  __device__ void fill_write(int32_t t) {
    Pt e;
#pragma unroll
    for (int k2 = 0; k2 < DP; ++k2) e.c[k2] = k2 < D ? (qsep ? N::inf() : N::cvt(qbuf[k2])) : V(0);
    int slot = (t + lane) & (kRing - 1);
    ring()[slot] = e;
    if (slot < kGroup) ring()[slot + kRing] = e;
    if (ptmp_pending) {
      V *dst = pst(ptmp_slot) + lane * (R * D);
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) dst[r * D + k2] = N::cvt(ptmp[r][k2]);
      ptmp_pending = false;
    }
  }

  template <bool WINDOW>
  __device__ __forceinline__ void group(int32_t t0, int32_t win0, const V *hin, V *hout,
                                        V (&p)[R][D], const V (&pn)[R][D], V (&Mp)[R], V &upPrev,
                                        V &res) {
    const Pt *qr = ring() + ((t0 - lane) & (kRing - 1));
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      Pt q = qr[u];
      V h = hin[u];
      V bottom = Mp[R - 1];
      if (lane == kWave - 1) hout[u] = bottom;
      if (u == kGroup - 1) res = bottom;
      if (WINDOW) {
        bool sw = lane == t0 + u - win0;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k2 = 0; k2 < D; ++k2) p[r][k2] = sw ? pn[r][k2] : p[r][k2];
      }
      V up = N::shift_in(h, bottom);
      V dd[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        V t = p[r][0] - q.c[0];
        V s = t * t;
#pragma unroll
        for (int k2 = 1; k2 < D; ++k2) {
          V w = p[r][k2] - q.c[k2];
          s = N::fma(w, w, s);
        }
        dd[r] = s;
      }
      V above = up, diag = upPrev;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        V v = N::mx(N::mn(N::mn(above, diag), Mp[r]), dd[r]);
        diag = Mp[r];
        above = v;
        Mp[r] = v;
      }
      upPrev = up;
    }
  }

  __device__ void run(int32_t wave) {
    lay = lds_layout(R, D, (int)sizeof(V), a.hcap);
    if (a.jobs) {
      j = uni(a.wave_jobs[wave]);
      jend = uni(a.wave_jobs[wave + 1]);
    } else {
      j = 0;
      jend = wave == 0 ? 1 : 0;
    }
    if (j >= jend) return;
    exhausted = false;
    next_id = 0;
    has_next = false;
    ptmp_pending = false;
    load_job(j);

    // constant LDS: top boundary and ring entries before the stream start;
    // row staging starts as zeros so that no lane ever reads uninitialised LDS
    for (int i = lane; i <= kGroup; i += kWave) ghost()[i] = i == 0 ? -N::inf() : N::inf();
    for (int i = lane; i < 2 * kWave * R * D; i += kWave) pst(0)[i] = V(0);
    {
      Pt e;
#pragma unroll
      for (int k2 = 0; k2 < DP; ++k2) e.c[k2] = N::inf();
      ring()[kRing - kWave + lane] = e;  // positions -64 .. -1
    }
    // first task and the first two ring chunks
    cS = 0;
    make_task(0, cL, cdrain, ccol_sel, ccol_off, cm);
    fill_load(0);
    fill_write(0);
    fill_load(kFill);

    V p[R][D], pn[R][D], Mp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Mp[r] = N::inf();
#pragma unroll
      for (int k2 = 0; k2 < D; ++k2) p[r][k2] = V(0);
    }
    V upPrev = N::inf();

    // lane-0 cursor: task containing the group's first step
    int32_t id0 = -1, S0 = 0, L0 = 0, g0 = 1, win0 = 0;
    // lane-63 cursor: task containing column t0 - 64 (starts in a pseudo-task)
    int32_t id63 = -1, S63 = -kWave, L63 = kWave, hand63 = 0;
    int64_t out63 = -1;

    for (int32_t t0 = 0;; t0 += kGroup) {
      if (t0 > a.max_steps) break;  // guard: the plan bounds every stream's length
      if ((t0 & (kFill - 1)) == 0) {
        fill_write(t0 + kFill);
        fill_load(t0 + 2 * kFill);
      }
      if (t0 - kWave == S63 + L63) {
        ++id63;
        Desc d = *desc(id63);
        if (uni(d.drain)) break;
        S63 = uni(d.S);
        L63 = uni(d.L);
        hand63 = uni(d.hand_out);
        out63 = (int64_t)(((uint64_t)(uint32_t)uni(d.out_hi) << 32) | (uint32_t)uni(d.out_lo));
      }
      bool window = false;
      if (t0 == S0 + L0) {
        ++id0;
        Desc d = *desc(id0);
        S0 = uni(d.S);
        L0 = uni(d.L);
        g0 = uni(d.ghost);
        win0 = t0;
        const V *src = pst(id0 & 1) + lane * (R * D);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k2 = 0; k2 < D; ++k2) pn[r][k2] = src[r * D + k2];
      }
      window = t0 < win0 + kWave;
      const V *hin = g0 ? ghost() + (t0 == S0 ? 0 : 1) : hand() + (t0 - S0);
      V *hout = hand63 ? hand() + (t0 - kWave - S63) : sink();
      V res;
      if (window)
        group<true>(t0, win0, hin, hout, p, pn, Mp, upPrev, res);
      else
        group<false>(t0, win0, hin, hout, p, pn, Mp, upPrev, res);
      if (t0 + kGroup - kWave == S63 + L63 && out63 >= 0 && lane == kWave - 1)
        N::store(a.out, out63, res, a.metric);
    }
  }
};

template <int R, int D, typename V>
__global__ __launch_bounds__(256) void stream_kernel(KernelArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  int lane = threadIdx.x & (kWave - 1);
  int wib = threadIdx.x / kWave;
  int wave = blockIdx.x * (blockDim.x / kWave) + wib;
  if (wave >= a.nwaves) return;
  Stream<R, D, V> s(a, lane, smem + wib * a.lds_per_wave);
  s.run(wave);
}

// ------------------------------------------------------------------ launcher

template <int R, int D, typename V>
static hipError_t launch_t(const KernelArgs &a, int waves_per_block, hipStream_t st) {
  int blocks = (a.nwaves + waves_per_block - 1) / waves_per_block;
  size_t lds = (size_t)a.lds_per_wave * waves_per_block;
  hipLaunchKernelGGL((stream_kernel<R, D, V>), dim3(blocks), dim3(waves_per_block * kWave), lds, st, a);
  return hipGetLastError();
}

template <int R, typename V>
static hipError_t launch_d(int D, const KernelArgs &a, int wpb, hipStream_t st) {
  switch (D) {
    case 1: return launch_t<R, 1, V>(a, wpb, st);
    case 2: return launch_t<R, 2, V>(a, wpb, st);
    case 3: return launch_t<R, 3, V>(a, wpb, st);
    case 4: return launch_t<R, 4, V>(a, wpb, st);
  }
  return hipErrorInvalidValue;
}

template <typename V>
static hipError_t launch_r(int R, int D, const KernelArgs &a, int wpb, hipStream_t st) {
  switch (R) {
    case 1: return launch_d<1, V>(D, a, wpb, st);
    case 2: return launch_d<2, V>(D, a, wpb, st);
    case 4: return launch_d<4, V>(D, a, wpb, st);
    case 8: return launch_d<8, V>(D, a, wpb, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stream(bool exact, int R, int D, const KernelArgs &a, int wpb, hipStream_t st) {
  return exact ? launch_r<double>(R, D, a, wpb, st) : launch_r<float>(R, D, a, wpb, st);
}

}  // namespace ffd
