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
//  * every task starts with at least 16 separator columns whose point is
//    +inf in every coordinate, so d = +inf there for every row: this resets
//    the left neighbours to +inf (the boundary M_{i,0} = +inf) without a
//    branch, and a -inf entry of the top boundary at the last separator
//    gives the corner M_{0,0} = -inf, which makes Eq. (1) produce the first
//    row and column (running maxima, Algorithms 3-5) by itself; the task's
//    m columns follow and end the task;
//  * a lane must use the new task's rows from its first real column on;
//    while its columns are separators the rows do not matter, so the lanes
//    take them in 16-lane blocks at group boundaries (block k at the start
//    of the (k+1)-th group of the task), with no per-step select;
//  * rows past the end of a curve repeat its last point: repeating points
//    does not change the distance (Sec. 4, footnote), so padding is exact.
//
// Other ground distances (Sec. 3: the method assumes nothing about it) and
// dynamic time warping (Appendix B, Algorithm B.1: the outer max replaced by
// a sum, M_ij = min{...} + d_ij) run on the same sweep; the template
// argument OP = measure + 2 * cell selects them: measure 0 Frechet, 1 DTW;
// cell 0 squared Euclidean, 1 Euclidean (the hardware square root per cell,
// DTW only: the Frechet kernel takes one root per pair), 2 Manhattan
// (sum of |dk|), 3 Chebyshev (max of |dk|); OP 8 is the Levenshtein
// distance of int32 symbol sequences (Appendix B, Algorithm B.2); OP 10
// and 11 are the Frechet distance and DTW of curves on the sphere under the
// great-circle distance (see Stream::HAV).  Sums are
// not selections, so row padding is no longer exact: the DTW corner is 0,
// and the result M_{n-1,m-1} is taken from the lane holding row n-1 at the
// moment it enters the next task, when its registers still hold the last
// column of the old one.  Levenshtein also sets the new task's first
// (separator) column to its boundary M_{i,-1} = i + 1 at that moment; the
// recurrence keeps it through the other separators, and lane 0's top
// boundary is the ramp M_{-1,j} = j + 1 after a 0 corner.  The separators of
// a Levenshtein task carry a flag in an extra slot of the ring entry, since
// every int32 value is a possible symbol.
//
// The squared distance is evaluated as d2 = dx*dx, then d2 = fma(dk, dk, d2)
// for k >= 1, in the value type; the recurrence runs on d2 and the Euclidean
// result is the correctly rounded square root of the selected d2 (min and
// max commute with the monotone square root).  The exact path widens int32
// coordinates to FP64, where every operation on these integers is exact.
#ifndef FFD_STREAM_H
#define FFD_STREAM_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
  __device__ static __forceinline__ float abs(float a) { return __builtin_fabsf(a); }
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
  // the hardware square root (v_sqrt_f32, within 1 ulp); the correctly
  // rounded library form costs about 16 more instructions per cell
  __device__ static __forceinline__ float sqrt_cell(float x) { return __builtin_amdgcn_sqrtf(x); }
  __device__ static __forceinline__ void store_value(void *out, int64_t idx, float v) {
    static_cast<float *>(out)[idx] = v;
  }
  // the result of a pair whose wave abandoned a wait: NaN
  __device__ static __forceinline__ float poison() { return __builtin_nanf(""); }
};

template <>
struct Num<double> {
  using Coord = int32_t;
  __device__ static __forceinline__ double inf() { return __builtin_huge_val(); }
  __device__ static __forceinline__ double cvt(int32_t x) { return (double)x; }
  __device__ static __forceinline__ double mn(double a, double b) { return __builtin_fmin(a, b); }
  __device__ static __forceinline__ double mx(double a, double b) { return __builtin_fmax(a, b); }
  __device__ static __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
  __device__ static __forceinline__ double abs(double a) { return __builtin_fabs(a); }
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
  __device__ static __forceinline__ double sqrt_cell(double x) { return __builtin_sqrt(x); }
  __device__ static __forceinline__ void store_value(void *out, int64_t idx, double v) {
    static_cast<int64_t *>(out)[idx] = (int64_t)v;
  }
  // the result of a pair whose wave abandoned a wait: -1 (no distance is negative)
  __device__ static __forceinline__ double poison() { return -1.0; }
};

// Task descriptor kept in LDS (64 bytes).
// where lane 0's row above comes from
enum : int32_t { kHinGhost = 0, kHinHand = 1, kHinLink = 2, kHinRing = 3 };
// where lane 63's bottom row goes
enum : int32_t { kHoutSink = 0, kHoutHand = 1, kHoutLink = 2, kHoutRing = 3 };
struct Desc {
  int32_t S;           // stream position of the separator
  int32_t L;           // stream length
  int32_t hin, hout;   // boundary modes
  int32_t out_lo, out_hi;  // result index, -1 = none
  int32_t drain;       // bit 0: padding task after the last job; bits 1-3 and 4-9: the
                       // register and lane of the curve's last row in this band;
                       // bits 10-16: the separator count; bits 17+: the band
                       // (Levenshtein only)
  int32_t flag_in, flag_out;
  int32_t rel_in;      // entries of the incoming link before this task's row
  int32_t rel_out;     // entries of the outgoing link before this task's row
  int32_t src;         // kHinRing: the workgroup wave whose ring holds the row above
  int64_t link_in;     // element of this task's incoming boundary row (x = 0)
  int64_t link_out;    // element of this task's outgoing boundary row
};
static_assert(sizeof(Desc) == 64, "descriptor size");

__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Bound of a link wait: s_sleep 2 is about 128 clocks, so about 2^29 clocks
// (a quarter of a second) before the wait is abandoned and reported.
constexpr int kSpinLimit = 1 << 22;

// s_waitcnt operand (gfx9 encoding) that waits for vmcnt = 0 only.
constexpr int kWaitVmcnt0 = 0x0F70;

// OP = measure + 2 * cell (measure 0 Frechet, 1 DTW; cell 0 squared
// Euclidean, 1 Euclidean, 2 Manhattan, 3 Chebyshev).
template <int R, int D, typename V, bool RINGS, int OP = 0>
struct Stream {
  static constexpr bool DTW = (OP & 1) != 0;
  static constexpr int CELL = OP >> 1;
  // OP 8: Levenshtein distance of int32 symbol sequences (cell 4:
  // [p_i != q_j]; M_ij = min{M_{i-1,j} + 1, M_{i,j-1} + 1, M_{i-1,j-1} + d_ij}),
  // instantiated with V = float: the symbols travel as their bit patterns
  // (compared, never computed with) and the values are integers below 2^24,
  // exact in float32 (the host limits n + m)
  static constexpr bool LEV = OP == 8;
  // the result is taken from the lane of the curve's last row at its switch
  static constexpr bool CAP = DTW || LEV;
  // OP 10 and 11 (cell 5): points are (latitude, longitude) in radians,
  // float32, and the ground distance is the central angle between them.
  // Each point becomes its FP64 unit vector u = (cos lat cos lon, cos lat
  // sin lon, sin lat) when it is staged in LDS (once per band row and once
  // per ring entry), and the cell is the squared chord |u - v|^2 with D = 3.
  // The angle 2 asin(|u - v| / 2) is an increasing function of it, so the
  // Frechet sweep (OP 10) selects on chords and takes the angle once per
  // pair; DTW (OP 11) sums angles and takes one per cell.
  static constexpr bool HAV = CELL == 5;
  static constexpr int DI = HAV ? 2 : D;  // values per point in registers
  // D = 8 and 16: the kernels of curves with 5 to 16 coordinates; a point
  // has a.dim coordinates in memory and zeros past them in registers
  static constexpr bool GEN = D > 4;
  using N = Num<V>;
  using C = std::conditional_t<HAV, float, typename N::Coord>;
  static_assert(!HAV || (D == 3 && sizeof(V) == 8), "great-circle sweeps run on FP64 unit vectors");
  // values per ring entry; Levenshtein keeps a separator flag in slot D
  static constexpr int DP = LEV ? lev_dim(D) : pad_dim(D);
  struct alignas(sizeof(V) * DP) Pt {
    V c[DP];
  };

  const KernelArgs &a;
  int lane;
  int wib;              // wave index within the workgroup
  LdsLayout lay;
  unsigned char *base;  // this wave's LDS region

  // ---- fill cursor: enumerates tasks (job, column curve, band) --------------
  // Task covering a fill chunk start, or the one after it.
  struct FillTask {
    int32_t S, L, drain, col_sel, hin, flag_in, rel, pad;
    int64_t col_off, m, link_in;
  };
  // Everything the refill needs; it lives in LDS between refills (every
  // kFill steps) so that it occupies no registers in the hot loop.
  struct FillState {
    int32_t j, jend;          // job range of this wave
    int32_t c, b, nb;         // column curve within the job, band, bands of the row curve
    int32_t b_first, b_end;   // band range of the job
    int32_t row_sel, col_sel, col_first, col_count, out_stride, flag_in, flag_out;
    int32_t exhausted, next_id, has_next, ptmp_pending, ptmp_slot, idle;
    int32_t pub_flag[2];      // link counts stored by the last flush, published at the next one
    uint32_t pub_count[2];
    int64_t row_off, n, out_base, link_in, link_out, link_rel;
    FillTask cur, nxt;
  };
  // per-lane prefetch registers
  C qbuf[DI];
  bool qsep;
  V hbuf;
  int32_t hslot;            // stream position of an incoming link value (-1: none)
  C ptmp[R][DI];
  int32_t err;

  __device__ Stream(const KernelArgs &args, int lane_, int wib_, unsigned char *b_)
      : a(args), lane(lane_), wib(wib_), base(b_) {}

  __device__ Pt *ring() const { return reinterpret_cast<Pt *>(base + lay.ring); }
  __device__ V *ghost() const { return reinterpret_cast<V *>(base + lay.ghost); }
  __device__ V *sink() const { return reinterpret_cast<V *>(base + lay.sink); }
  __device__ V *hand() const { return reinterpret_cast<V *>(base + lay.hand); }
  __device__ V *lring() const { return reinterpret_cast<V *>(base + lay.lring); }
  __device__ V *pst(int slot) const { return reinterpret_cast<V *>(base + lay.pst) + slot * (kWave * R * D); }
  __device__ Desc *desc(int id) const { return reinterpret_cast<Desc *>(base + lay.desc) + (id & (kDescSlots - 1)); }
  __device__ FillState *fstate() const { return reinterpret_cast<FillState *>(base + lay.fill); }
  __device__ V *links() const { return static_cast<V *>(a.links); }

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

  // values per point in the input arrays
  __device__ int32_t in_dim() const {
    if constexpr (GEN) return a.dim;
    else return DI;
  }
  // value k of the point at pt (k < DI); zero past the curves' coordinates
  __device__ C coord(const C *pt, int k) const {
    if constexpr (GEN) return k < a.dim ? pt[k] : C(0);
    else return pt[k];
  }

  __device__ static void uni_task(FillTask &t) {
    t.S = uni(t.S); t.L = uni(t.L); t.drain = uni(t.drain); t.col_sel = uni(t.col_sel);
    t.hin = uni(t.hin); t.flag_in = uni(t.flag_in); t.rel = uni(t.rel);
    t.col_off = uni64(t.col_off); t.m = uni64(t.m); t.link_in = uni64(t.link_in);
  }

  // Read the refill state from LDS (the same values in every lane).
  // Read the refill state from LDS.  Every lane reads the same values;
  // only the fields that steer control flow are made scalar (the rest stay
  // in vector registers, which keeps the scalar register file from spilling).
  __device__ __forceinline__ void load_state(FillState &f) const {
    f = *fstate();
    f.exhausted = uni(f.exhausted); f.has_next = uni(f.has_next); f.idle = uni(f.idle);
    f.ptmp_pending = uni(f.ptmp_pending);
    f.pub_flag[0] = uni(f.pub_flag[0]); f.pub_flag[1] = uni(f.pub_flag[1]);
    f.cur.S = uni(f.cur.S); f.cur.L = uni(f.cur.L); f.cur.hin = uni(f.cur.hin);
    f.nxt.S = uni(f.nxt.S); f.nxt.L = uni(f.nxt.L); f.nxt.hin = uni(f.nxt.hin);
  }

  __device__ __forceinline__ void store_state(const FillState &f) const {
    if (lane == 0) *fstate() = f;
  }

  __device__ __forceinline__ void load_job(FillState &f, int32_t jj) const {
    int32_t ri, bf, bc;
    if (a.jobs) {
      const Job *jb = a.jobs + jj;
      f.row_sel = uni(jb->row_sel);
      ri = uni(jb->row_idx);
      f.col_sel = uni(jb->col_sel);
      f.col_first = uni(jb->col_first);
      f.col_count = uni(jb->col_count);
      f.out_stride = uni(jb->out_stride);
      f.out_base = uni64(jb->out_base);
      f.link_in = uni64(jb->link_in);
      f.link_out = uni64(jb->link_out);
      bf = uni(jb->band_first);
      bc = uni(jb->band_count);
      f.flag_in = uni(jb->flag_in);
      f.flag_out = uni(jb->flag_out);
    } else {
      f.row_sel = a.inl_job.row_sel;
      ri = a.inl_job.row_idx;
      f.col_sel = a.inl_job.col_sel;
      f.col_first = a.inl_job.col_first;
      f.col_count = a.inl_job.col_count;
      f.out_stride = a.inl_job.out_stride;
      f.out_base = a.inl_job.out_base;
      f.link_in = a.inl_job.link_in;
      f.link_out = a.inl_job.link_out;
      bf = a.inl_job.band_first;
      bc = a.inl_job.band_count;
      f.flag_in = a.inl_job.flag_in;
      f.flag_out = a.inl_job.flag_out;
    }
    f.c = 0;
    f.link_rel = 0;
    if (f.row_sel == kRowIdle) {  // padding: col_count steps of separators
      f.idle = f.col_count;
      f.nb = 1;
      f.b_first = f.b = 0;
      f.b_end = 1;
      f.col_count = 1;
      return;
    }
    f.idle = 0;
    f.row_off = uni64(curve_off(f.row_sel, ri));
    f.n = uni64(curve_off(f.row_sel, ri + 1)) - f.row_off;
    f.nb = (int32_t)bands_for(f.n, R);
    f.b_first = bf;
    f.b_end = bc > 0 && bf + bc < f.nb ? bf + bc : f.nb;
    f.b = f.b_first;
  }

  // Create the next task in stream order starting at position S: write its
  // descriptor, issue the loads of its band rows into ptmp, return its
  // stream parameters.
  __device__ __forceinline__ void make_task(FillState &f, int32_t S, FillTask &t) {
    int32_t id = f.next_id++;
    Desc d;
    d.S = S;
    d.src = 0;
    d.rel_in = d.rel_out = 0;
    t.S = S;
    t.rel = 0;
    t.pad = 0;
    if (f.exhausted || f.idle) {
      // separators only: after the last job (drain: the stream ends), or an
      // idle job (the stream goes on)
      t.L = f.exhausted ? kMinTask : f.idle; t.drain = 1; t.col_sel = 0; t.col_off = 0; t.m = 1;
      t.hin = kHinGhost; t.flag_in = -1; t.link_in = 0;
      d.L = t.L; d.hin = kHinGhost; d.hout = kHoutSink; d.out_lo = -1; d.out_hi = -1; d.drain = f.exhausted;
      d.flag_in = -1; d.flag_out = -1; d.link_in = 0; d.link_out = 0;
      if (!f.exhausted) {
        if (++f.j == f.jend) f.exhausted = 1;
        else load_job(f, f.j);
      }
    } else {
      int32_t k = f.col_first + f.c;
      t.col_off = uni64(curve_off(f.col_sel, k));
      t.m = uni64(curve_off(f.col_sel, k + 1)) - t.col_off;
      t.col_sel = f.col_sel;
      t.L = (int32_t)task_len(t.m, f.nb > 1);
      t.drain = 0;
      int32_t b = f.b, nb = f.nb;
      int64_t oi = (b == nb - 1) ? f.out_base + (int64_t)f.c * f.out_stride : -1;
      int32_t hin = b == 0 ? kHinGhost : (b == f.b_first ? kHinLink : kHinHand);
      int32_t hout = b == nb - 1 ? kHoutSink : (b + 1 == f.b_end ? kHoutLink : kHoutHand);
      if (hin == kHinLink && f.flag_in <= -2) {
        hin = kHinRing;
        d.src = -2 - f.flag_in;
      }
      if (hout == kHoutLink && f.flag_out == -2) hout = kHoutRing;
      t.hin = hin;
      t.flag_in = f.flag_in;
      t.link_in = f.link_in + f.link_rel;
      t.rel = (int32_t)f.link_rel;
      d.rel_in = d.rel_out = (int32_t)f.link_rel;
      d.L = t.L; d.hin = hin; d.hout = hout;
      {
        // separator count; the register and lane of the curve's last row
        // (DTW, Levenshtein); the band (Levenshtein)
        int64_t last = f.n - 1 - (int64_t)b * kWave * R;
        int32_t lr = last < kWave * R ? (int32_t)last : kWave * R - 1;
        d.drain = ((lr % R) << 1) | ((lr / R) << 4) | ((int32_t)(t.L - t.m) << 10) | (LEV ? b << 17 : 0);
      }
      d.out_lo = (int32_t)(uint32_t)(uint64_t)oi;
      d.out_hi = (int32_t)(uint32_t)((uint64_t)oi >> 32);
      d.flag_in = f.flag_in;
      d.flag_out = f.flag_out;
      d.link_in = f.link_in + f.link_rel;
      d.link_out = f.link_out + f.link_rel;
      // band rows of this lane, clamped to the last point (repetition is exact)
      const C *X = coords(f.row_sel);
      int64_t r0 = (int64_t)b * kWave * R + (int64_t)lane * R;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int64_t ri = r0 + r < f.n ? r0 + r : f.n - 1;
        const C *pt = X + (f.row_off + ri) * in_dim();
#pragma unroll
        for (int k2 = 0; k2 < DI; ++k2) ptmp[r][k2] = coord(pt, k2);
      }
      f.ptmp_pending = 1;
      f.ptmp_slot = id & 1;
      // advance: next band, next column curve, next job
      if (++f.b == f.b_end) {
        f.b = f.b_first;
        f.link_rel += t.L;
        if (++f.c == f.col_count) {
          if (++f.j == f.jend) f.exhausted = 1;
          else load_job(f, f.j);
        }
      }
    }
    if (lane == 0) *desc(id) = d;
  }

  // Wait until the link flag reports at least `need` entries of this launch.
  // Agent-scope polling of the count; the row itself is then read with
  // agent-scope loads (see flush_links).
  __device__ void wait_link(int32_t flag, uint32_t need) {
    if (err) return;  // after an abandoned wait the wave waits no more (its results are poisoned)
    uint64_t want = flag_word(a.epoch, need);
    uint64_t *fl = a.flags + flag;
    for (int it = 0;; ++it) {
      uint64_t v = __hip_atomic_load(fl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((uint32_t)(v >> 32) == a.epoch && v >= want) break;
      if (it == kSpinLimit) {
        err |= 2;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    // the row is read with agent-scope loads issued after this point (the
    // exit depends on the loaded count); keep the compiler from moving them
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }

  // Make f.cur the task containing stream position t, and f.nxt the one
  // after it if f.cur ends before t + kFill.
  __device__ __forceinline__ void advance(FillState &f, int32_t t) {
    while (f.cur.S + f.cur.L <= t) {
      if (!f.has_next) make_task(f, f.cur.S + f.cur.L, f.nxt);
      f.cur = f.nxt;
      f.has_next = 0;
    }
    if (f.cur.S + f.cur.L < t + kFill && !f.has_next) {
      make_task(f, f.cur.S + f.cur.L, f.nxt);
      f.has_next = 1;
    }
  }

  // Issue the global loads of ring entries [t, t + 64), one per lane; f
  // describes that chunk (advance(f, t)).
  __device__ __forceinline__ void ring_load(const FillState &f, int32_t t) {
    const FillTask &cur = f.cur, &nxt = f.nxt;
    int32_t tau = t + lane;
    bool in_next = tau >= cur.S + cur.L;
    int32_t x = tau - (in_next ? nxt.S : cur.S);
    int64_t m = in_next ? nxt.m : cur.m;
    int64_t co = in_next ? nxt.col_off : cur.col_off;
    int32_t sel = in_next ? nxt.col_sel : cur.col_sel;
    bool drain = in_next ? nxt.drain : cur.drain;
    int64_t npre = (in_next ? nxt.L : cur.L) - m;
    qsep = drain || x < npre;
    int64_t idx = x - npre;
    if (idx > m - 1) idx = m - 1;
    if (idx < 0) idx = 0;
    if (drain) { co = 0; idx = 0; sel = 0; }
    const C *X = coords(sel);
    const C *pt = X + (co + idx) * in_dim();
#pragma unroll
    for (int k2 = 0; k2 < DI; ++k2) qbuf[k2] = coord(pt, k2);
  }

  // Issue the loads of the incoming boundary values of positions
  // [t, t + 64) for tasks whose band above ran on another wave, after
  // waiting for them to be published; f describes that chunk.  They are
  // written to LDS at the refill of step t, just before their first use.
  __device__ __forceinline__ void link_load(const FillState &f, int32_t t) {
    const FillTask &cur = f.cur, &nxt = f.nxt;
    if (cur.hin == kHinLink) {
      int32_t hi = t + kFill - cur.S;
      wait_link(cur.flag_in, (uint32_t)(cur.rel + (hi < cur.L ? hi : cur.L)));
    }
    if (f.has_next && nxt.hin == kHinLink) {
      int32_t hi = t + kFill - nxt.S;
      if (hi > 0) wait_link(nxt.flag_in, (uint32_t)(nxt.rel + (hi < nxt.L ? hi : nxt.L)));
    }
    int32_t tau = t + lane;
    bool in_next = tau >= cur.S + cur.L;
    int32_t x = tau - (in_next ? nxt.S : cur.S);
    bool glink = (in_next ? nxt.hin : cur.hin) == kHinLink;
    int64_t lk = in_next ? nxt.link_in : cur.link_in;
    hslot = glink ? tau : -1;  // the link ring is indexed by stream position
    if (glink) hbuf = __hip_atomic_load(links() + lk + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  __device__ void link_write() {
    if (hslot >= 0) {
      int ls = hslot & (kLinkRing - 1);
      lring()[ls] = hbuf;  // read a group at a time from a group-aligned position: no wrap
    }
  }

  // Write the ring entries loaded by the previous ring_load (for positions
  // [t, t + 64)) and any pending band rows.
  // HAV: the unit vector of a (latitude, longitude) point, in FP64.
  __device__ static __forceinline__ void stage(const C *in, V *out) {
    double sf, cf, sl, cl;
    sincos((double)in[0], &sf, &cf);
    sincos((double)in[1], &sl, &cl);
    out[0] = cf * cl;
    out[1] = cf * sl;
    out[2] = sf;
  }

  __device__ __forceinline__ void fill_write(FillState &f, int32_t t) {
    Pt e;
    if constexpr (HAV) {
      V u[D];
      stage(qbuf, u);
#pragma unroll
      for (int k2 = 0; k2 < DP; ++k2) e.c[k2] = k2 < D ? (qsep ? N::inf() : u[k2]) : V(0);
    } else if constexpr (LEV) {
      // symbols as they are (int32 bit patterns), the flag set on separators
#pragma unroll
      for (int k2 = 0; k2 < DP; ++k2) e.c[k2] = k2 < D ? N::cvt(qbuf[k2]) : (k2 == D && qsep ? V(1) : V(0));
    } else {
#pragma unroll
      for (int k2 = 0; k2 < DP; ++k2) e.c[k2] = k2 < D ? (qsep ? N::inf() : N::cvt(qbuf[k2])) : V(0);
    }
    int slot = (t + lane) & (kRing - 1);
    ring()[slot] = e;
    if (slot < kGroup) ring()[slot + kRing] = e;
    if (f.ptmp_pending) {
      V *dst = pst(f.ptmp_slot) + lane * (R * D);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (HAV) {
          stage(ptmp[r], dst + r * D);
        } else {
#pragma unroll
          for (int k2 = 0; k2 < D; ++k2) dst[r * D + k2] = N::cvt(ptmp[r][k2]);
        }
      }
      f.ptmp_pending = 0;
    }
  }

  static_assert(sizeof(FillState) <= kFillStateBytes, "refill state does not fit its LDS slot");

  // One refill, at step t0: store the outgoing boundary entries staged
  // during the last kWave steps; write the incoming boundary values of
  // [t0, t0 + 64) and the ring chunk [t0 + 64, t0 + 128) loaded last time;
  // load the incoming boundary values of [t0 + 64, t0 + 128) and the ring
  // chunk [t0 + 128, t0 + 192).
  __device__ __forceinline__ void refill(int32_t t0) {
    FillState f;
    load_state(f);
    if (a.flags) flush_links(f, t0 - 2 * kWave, false);  // launches without links skip it
    link_write();
    fill_write(f, t0 + kFill);
    link_load(f, t0 + kFill);
    advance(f, t0 + 2 * kFill);
    ring_load(f, t0 + 2 * kFill);
    store_state(f);
  }

  // Column points and top-boundary values of one group of kGroup steps,
  // read from LDS one group ahead of their use.  The wide kernels (GEN)
  // would need 8 or 16 registers per point and step: they keep the group's
  // ring address and read each point at its step (the ring chunk of a group
  // is only rewritten at a later refill).
  struct GroupIn {
    Pt q[GEN ? 1 : kGroup];
    const Pt *qp;
    V h[kGroup];
  };

  __device__ __forceinline__ void load_group(int32_t t, const V *hin, GroupIn &g) const {
    const Pt *qr = ring() + ((t - lane) & (kRing - 1));
    g.qp = qr;
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      if constexpr (!GEN) g.q[u] = qr[u];
      g.h[u] = hin[u];
    }
  }

  __device__ __forceinline__ static const Pt &entry(const GroupIn &g, int u) {
    if constexpr (GEN) return g.qp[u];
    else return g.q[u];
  }

  // Row state of the lane: the R rows it holds, the rows of the next task,
  // the left neighbours (previous column) and the previous top value.
  V p[R][D], pn[R][D], Mp[R];
  V upPrev;
  // lane-0 cursor (task containing the group being loaded) and window start
  int32_t id0, S0, L0, g0, src0, win0, win_cur;
  int32_t pre0;  // separator columns of lane 0's task
  V bnd0;        // Levenshtein: boundary value M_{i,-1} = i + 1 of this lane's first row in lane 0's task
  int32_t rc63, ls63;  // DTW: register and lane of the last row of lane 63's task
  V cap;         // DTW: this lane's value of the last column, taken at its task switch
  // lane-63 cursor: task containing column t0 - 64
  int32_t id63, S63, L63, hout63, flag63, rel63;
  int64_t out63, link63;

  // One code path for every group: the row switch of a task window and the
  // link store are uniform branches, so the hot registers stay where they
  // are (code variants of the group made the compiler shuffle them at every
  // merge).
  template <bool PLAIN>
  __device__ __forceinline__ void group(int32_t t0, int32_t win, bool window, const GroupIn &g, V *hout,
                                        V &res, int32_t rc) {
    if (PLAIN) window = false;
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      V bottom = Mp[R - 1];
      // every lane stores (no exec-mask change in the hot loop); only lane
      // 63's address can be the hand-off row or the link staging ring, the
      // others land in the sink
      hout[u] = bottom;
      if (u == kGroup - 1) res = bottom;
      bool sw = false;
      if (CAP && window) {
        // the lane enters the new task: its registers hold the old task's
        // last column (the result of DTW or Levenshtein is taken here), and
        // it takes the new task's rows
        sw = lane == t0 + u - win;
        V sel = Mp[0];
#pragma unroll
        for (int r = 1; r < R; ++r) sel = rc == r ? Mp[r] : sel;
        cap = sw ? sel : cap;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k2 = 0; k2 < D; ++k2) p[r][k2] = sw ? pn[r][k2] : p[r][k2];
      }
      V up = N::shift_in(g.h[u], bottom);
      const Pt &qe = entry(g, u);
      V dd[R];
      bool same[R];  // Levenshtein: p_i = q_j (a separator matches nothing)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        V t = p[r][0] - qe.c[0];
        V s;
        if constexpr (CELL >= 2 && !HAV) {
          // Manhattan: s = |d0| + |d1| + ...; Chebyshev: max of |dk|
          s = N::abs(t);
#pragma unroll
          for (int k2 = 1; k2 < D; ++k2) {
            V w = N::abs(p[r][k2] - qe.c[k2]);
            s = CELL == 2 ? s + w : N::mx(s, w);
          }
        } else {
          s = t * t;
#pragma unroll
          for (int k2 = 1; k2 < D; ++k2) {
            V w = p[r][k2] - qe.c[k2];
            s = N::fma(w, w, s);
          }
          if constexpr (CELL == 1) s = N::sqrt_cell(s);
          if constexpr (HAV && DTW) {
            // the angle per cell, from the FP64 chord through float32 (the
            // hardware square root and the float arcsine: a few float ulps
            // per cell, summed in FP64); separators (+inf) stay +inf, a
            // chord rounded past the diameter is the antipode
            float c = 0.5f * __builtin_amdgcn_sqrtf((float)s);
            s = c <= 1.0f ? 2.0 * (double)asinf(c) : (s < N::inf() ? 3.141592653589793 : s);
          }
        }
        if constexpr (LEV) {
          // symbols compared as bit patterns; a separator (flag slot set)
          // differs from every symbol
          bool ne = __builtin_bit_cast(uint32_t, qe.c[D]) != 0u;
#pragma unroll
          for (int k2 = 0; k2 < D; ++k2)
            ne = ne || __builtin_bit_cast(uint32_t, p[r][k2]) != __builtin_bit_cast(uint32_t, qe.c[k2]);
          same[r] = !ne;
        }
        dd[r] = s;
      }
      V above = up, diag = upPrev;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        V v;
        // Levenshtein: M_{i,j} = min(M_{i-1,j} + 1, M_{i,j-1} + 1,
        // M_{i-1,j-1} + [p_i != q_j]).  Neighbouring values of the table
        // differ by at most one, so on a match the diagonal is the least of
        // the three, and otherwise the three candidates share the + 1; the
        // separator columns take the second form, as before
        if constexpr (LEV) v = same[r] ? diag : N::mn(N::mn(above, Mp[r]), diag) + V(1);
        else if constexpr (DTW) v = N::mn(N::mn(above, diag), Mp[r]) + dd[r];
        else v = N::mx(N::mn(N::mn(above, diag), Mp[r]), dd[r]);
        diag = Mp[r];
        above = v;
        Mp[r] = v;
      }
      if (LEV && window) {
        // the new task's first (separator) column holds the boundary
        // M_{i,-1} = i + 1; the recurrence keeps it through the other
        // separators (above = i, diagonal = i, d = 1)
#pragma unroll
        for (int r = 0; r < R; ++r) Mp[r] = sw ? bnd0 + V(r) : Mp[r];
      }
      upPrev = up;
    }
  }

  // Address of lane 0's top-boundary values for the group starting at t.
  // The byte offset is formed with integer selects: a chain of pointer
  // returns here was compiled (ROCm 7.2) into code that read the address
  // from an undefined register on the link path.
  __device__ __forceinline__ const V *hin_at(int32_t t) const {
    // ghost = [+inf x kGroup, corner, +inf x kGroup]; the corner sits at
    // the task's last separator column c
    int32_t c = S0 + pre0 - 1;
    int32_t og = lay.ghost + (c >= t && c < t + kGroup ? kGroup - (c - t) : 0) * (int32_t)sizeof(V);
    if constexpr (LEV) og = lay.ghost;  // the ramp written for this group
    int32_t oh = lay.hand + (t - S0) * (int32_t)sizeof(V);
    int32_t ol = lay.lring + (t & (kLinkRing - 1)) * (int32_t)sizeof(V);
    int32_t off = g0 == kHinGhost ? og : (g0 == kHinHand ? oh : ol);
    if (RINGS && g0 == kHinRing)
      off = (src0 - wib) * a.lds_per_wave + lay.xring + ((t - S0) & (kXRing - 1)) * (int32_t)sizeof(V);
    return reinterpret_cast<const V *>(base + off);
  }

  // Advance lane 0's cursor to the group starting at t; at a task start,
  // read the task's rows (pn) for the switch window.
  __device__ __forceinline__ void lane0_to(int32_t t) {
    if (t == S0 + L0) {
      ++id0;
      Desc d = *desc(id0);
      S0 = uni(d.S);
      L0 = uni(d.L);
      g0 = uni(d.hin);
      src0 = uni(d.src);
      pre0 = LEV ? (uni(d.drain) >> 10) & 127 : uni(d.drain) >> 10;  // the band bits are Levenshtein's only
      if constexpr (LEV) bnd0 = V((int64_t)(uni(d.drain) >> 17) * (kWave * R) + lane * R + 1);
      win0 = t;
      const V *src = pst(id0 & 1) + lane * (R * D);
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) pn[r][k2] = src[r * D + k2];
    }
  }

  __device__ V *lstage() const { return reinterpret_cast<V *>(base + lay.lstage); }

  // Counters of a wave's LDS ring (entries written by its lane 63, entries
  // read by the consumer's lane 0), for the wave `w` of this workgroup.
  __device__ int32_t *xctr(int32_t w) const {
    return reinterpret_cast<int32_t *>(base + (w - wib) * a.lds_per_wave + lay.xctr);
  }

  // Spin (bounded) until *c >= need; workgroup-scope acquire.
  __device__ void wait_ctr(int32_t *c, int32_t need) {
    if (err) return;
    for (int it = 0;; ++it) {
      if (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= need) break;
      if (it == kSpinLimit) {
        err |= 2;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }

  // Store the outgoing boundary-row entries of stream positions
  // [lo, lo + kWave) from the LDS staging ring to their link buffers -- one
  // coalesced store per lane every kFill steps instead of a store per step
  // -- and publish how many entries of each link row are in memory.  The
  // positions must belong to lane 63's current task (id63), the one before
  // it, or later tasks whose entries are not staged yet (skipped).
  //
  // The row's stores are agent-scope stores, which go through to the
  // device's coherence point; once the wave's stores have completed
  // (vmcnt 0) an agent-scope store of the count is ordered after them for
  // any reader that loads the count and then the row at agent scope.  No
  // L2 write-back is needed: nothing a reader depends on is dirty in this
  // XCD's L2.  To avoid waiting for the stores just issued, the counts of a
  // flush are published at the next one (kFill steps later, when every
  // older memory operation of the wave has long completed), or at once at
  // the end of the stream (`last`).
#ifdef FFD_DEBUG_JITTER
  // Debug builds only: a pause of 0 to 7 short sleeps before a progress
  // publication, varying with the wave and a stream quantity, so that tests
  // see the waits on it resolve in many orders.
  __device__ __forceinline__ void jitter(uint32_t x) const {
    uint32_t h = ((uint32_t)blockIdx.x * 0x9E3779B1u) ^ ((uint32_t)wib * 0x85EBCA77u) ^ (x * 0xC2B2AE3Du);
    h ^= h >> 15;
    for (uint32_t i = 0; i < (h & 7u); ++i) __builtin_amdgcn_s_sleep(2);
  }
#else
  __device__ __forceinline__ void jitter(uint32_t) const {}
#endif

  __device__ void publish_pending(FillState &f) {
    if (f.pub_flag[0] >= 0 || f.pub_flag[1] >= 0) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      jitter(f.pub_count[0] + f.pub_count[1]);
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
          if (f.pub_flag[k] >= 0)
            __hip_atomic_store(a.flags + f.pub_flag[k], flag_word(a.epoch, f.pub_count[k]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
      f.pub_flag[0] = f.pub_flag[1] = -1;
    }
  }

  __device__ void flush_links(FillState &f, int32_t lo, bool last) {
    publish_pending(f);
    int32_t p = lo + lane;
    bool have_prev = id63 > 0;
    int32_t pS = 0, pL = 0, phout = kHoutSink, pflag = -1, prel = 0;
    int64_t plink = 0;
    if (have_prev) {
      const Desc *d = desc(id63 - 1);
      pS = uni(d->S);
      pL = uni(d->L);
      phout = uni(d->hout);
      pflag = uni(d->flag_out);
      prel = uni(d->rel_out);
      plink = uni64(d->link_out);
    }
    bool in_cur = p >= S63;
    int32_t x = p - (in_cur ? S63 : pS);
    bool stage = in_cur ? (hout63 == kHoutLink && x < L63) : (have_prev && phout == kHoutLink && p >= pS);
    int64_t lk = in_cur ? link63 : plink;
    if (stage) {
      V v = lstage()[p & (kLinkRing - 1)];
      __hip_atomic_store(links() + lk + x, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (have_prev && phout == kHoutLink && pS + pL > lo) {
      f.pub_flag[0] = pflag;
      f.pub_count[0] = (uint32_t)(prel + pL);
    }
    if (hout63 == kHoutLink && lo + kWave > S63) {
      int32_t done = lo + kWave - S63;
      f.pub_flag[1] = flag63;
      f.pub_count[1] = (uint32_t)(rel63 + (done < L63 ? done : L63));
    }
    if (last) publish_pending(f);
  }

  // One group: refill the ring, move the lane-63 cursor, prefetch the next
  // group into `nxt`, compute this group from `cur`.  Returns false when the
  // stream has ended.
  __device__ __forceinline__ bool step(int32_t t0) {
    if (t0 > a.max_steps) {  // guard: the plan bounds every stream's length
      err |= 1;
      return false;
    }
    if ((t0 & (kFill - 1)) == 0) refill(t0);
    if (t0 - kWave == S63 + L63) {
      Desc d = *desc(id63 + 1);
      if (uni(d.drain) & 1) {
        // end of the stream: store what is still staged (positions from
        // the last flush to the end of lane 63's last task) and publish
        if (a.flags) {
          FillState f;
          load_state(f);
          flush_links(f, (t0 & ~(kFill - 1)) - kWave, true);
        }
        return false;
      }
      ++id63;
      S63 = uni(d.S);
      L63 = uni(d.L);
      hout63 = uni(d.hout);
      flag63 = uni(d.flag_out);
      rel63 = uni(d.rel_out);
      link63 = uni64(d.link_out);
      out63 = (int64_t)(((uint64_t)(uint32_t)uni(d.out_hi) << 32) | (uint32_t)uni(d.out_lo));
      if constexpr (CAP) {
        rc63 = (uni(d.drain) >> 1) & 7;
        ls63 = (uni(d.drain) >> 4) & 63;
      }
    }
    int32_t x63 = t0 - kWave - S63;
    // lane 63's bottom row: the hand-off row, the link staging ring (by
    // stream position; a group never wraps it), this wave's ring for a
    // consumer in the workgroup (by column), or the sink
    int32_t hoff = lay.sink + lane * (int32_t)sizeof(V);
    if (lane == kWave - 1 && hout63 == kHoutHand) hoff = lay.hand + x63 * (int32_t)sizeof(V);
    if (lane == kWave - 1 && hout63 == kHoutLink)
      hoff = lay.lstage + ((t0 - kWave) & (kLinkRing - 1)) * (int32_t)sizeof(V);
    if (RINGS && lane == kWave - 1 && hout63 == kHoutRing)
      hoff = lay.xring + (x63 & (kXRing - 1)) * (int32_t)sizeof(V);
    // the ring entries this group overwrites must have been read
    if (RINGS && hout63 == kHoutRing) wait_ctr(xctr(wib) + 1, x63 + kGroup - kXRing);
    V *hout = reinterpret_cast<V *>(base + hoff);
    lane0_to(t0);
    if (LEV && g0 == kHinGhost && lane < kGroup) {
      // Levenshtein top boundary: 0 over the separators, then M_{-1,j} = j + 1
      int32_t j1 = t0 + lane - S0 - pre0 + 1;
      ghost()[lane] = V(j1 > 0 ? j1 : 0);
    }
    GroupIn g;
    if (RINGS && g0 == kHinRing) {
      // the producing wave must have written this group's entries; once
      // they are read, tell it how far it may overwrite
      int32_t x0 = t0 - S0;
      wait_ctr(xctr(src0), x0 + kGroup < L0 ? x0 + kGroup : L0);
      load_group(t0, hin_at(t0), g);
      jitter((uint32_t)t0);
      if (lane == 0) __hip_atomic_store(xctr(src0) + 1, x0 + kGroup, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      load_group(t0, hin_at(t0), g);
    }
    V res;
    // Frechet: 16-lane block k takes the task's rows at the start of group
    // k + 1 of the task: its lanes are then on separator columns 1 .. 16 (a
    // task has at least 16), so no real column of either task sees the
    // wrong rows.  (DTW and Levenshtein switch per lane in the window
    // groups, where they also take their result.)
    if (!CAP && t0 > win0 && t0 <= win0 + kWave) {
      bool take = (lane >> 4) == ((t0 - win0) >> 4) - 1;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) p[r][k2] = take ? pn[r][k2] : p[r][k2];
    }
    bool window = CAP && t0 < win0 + kWave;
    if (!window) group<true>(t0, win0, false, g, hout, res, rc63);
    else group<false>(t0, win0, window, g, hout, res, rc63);
    if (RINGS && hout63 == kHoutRing) jitter((uint32_t)x63);
    if (RINGS && hout63 == kHoutRing && lane == 0)
      __hip_atomic_store(xctr(wib), x63 + kGroup < L63 ? x63 + kGroup : L63, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
    if constexpr (LEV) {
      if (t0 + kGroup - kWave == S63 + L63 && out63 >= 0 && lane == ls63)
        static_cast<int64_t *>(a.out)[out63] = err ? (int64_t)-1 : (int64_t)cap;
    } else if constexpr (CAP && HAV) {
      if (t0 + kGroup - kWave == S63 + L63 && out63 >= 0 && lane == ls63)
        static_cast<float *>(a.out)[out63] = err ? __builtin_nanf("") : (float)cap;
    } else if constexpr (CAP) {
      if (t0 + kGroup - kWave == S63 + L63 && out63 >= 0 && lane == ls63)
        N::store_value(a.out, out63, err ? N::poison() : cap);
    } else if constexpr (HAV) {
      // the central angle of the selected squared chord, in FP64, rounded
      // once to FP32 (the chord is clamped at the diameter)
      if (t0 + kGroup - kWave == S63 + L63 && out63 >= 0 && lane == kWave - 1) {
        double h = 0.5 * __builtin_sqrt((double)res);
        static_cast<float *>(a.out)[out63] = err ? __builtin_nanf("") : (float)(2.0 * asin(h < 1.0 ? h : 1.0));
      }
    } else if constexpr (CELL != 0) {
      if (t0 + kGroup - kWave == S63 + L63 && out63 >= 0 && lane == kWave - 1)
        N::store_value(a.out, out63, err ? N::poison() : res);
    } else {
      if (t0 + kGroup - kWave == S63 + L63 && out63 >= 0 && lane == kWave - 1)
        N::store(a.out, out63, err ? N::poison() : res, a.metric);
    }
    return true;
  }

  __device__ __forceinline__ void run(int32_t wave) {
    lay = lds_layout(R, D, (int)sizeof(V), a.hcap, RINGS, DP);
    int32_t j0, j1;
    if (a.jobs) {
      j0 = uni(a.wave_jobs[wave]);
      j1 = uni(a.wave_jobs[wave + 1]);
    } else {
      j0 = 0;
      j1 = wave == 0 ? 1 : 0;
    }
    if (j0 >= j1) return;
    err = 0;
    hslot = -1;

    // constant LDS: top boundary and ring entries before the stream start;
    // row staging starts as zeros so that no lane ever reads uninitialised LDS
    for (int i = lane; i <= 2 * kGroup; i += kWave) ghost()[i] = i == kGroup ? (DTW ? V(0) : -N::inf()) : N::inf();
    for (int i = lane; i < 2 * kWave * R * D; i += kWave) pst(0)[i] = V(0);
    {
      Pt e;
#pragma unroll
      for (int k2 = 0; k2 < DP; ++k2) e.c[k2] = N::inf();
      ring()[kRing - kWave + lane] = e;  // positions -64 .. -1
    }
    // first task and the first two ring chunks
    {
      FillState f;
      f.j = j0;
      f.jend = j1;
      f.exhausted = 0;
      f.next_id = 0;
      f.has_next = 0;
      f.ptmp_pending = 0;
      f.ptmp_slot = 0;
      f.pub_flag[0] = f.pub_flag[1] = -1;
      f.pub_count[0] = f.pub_count[1] = 0;
      load_job(f, j0);
      make_task(f, 0, f.cur);
      advance(f, 0);
      ring_load(f, 0);
      link_load(f, 0);
      fill_write(f, 0);
      advance(f, kFill);
      ring_load(f, kFill);
      store_state(f);
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
      Mp[r] = N::inf();
#pragma unroll
      for (int k2 = 0; k2 < D; ++k2) p[r][k2] = V(0);
    }
    upPrev = N::inf();
    id0 = -1; S0 = 0; L0 = 0; g0 = kHinGhost; src0 = 0; win0 = 0;
    id63 = -1; S63 = -kWave; L63 = kWave; hout63 = kHoutSink; flag63 = -1; rel63 = 0; out63 = -1;
    link63 = 0;
    pre0 = 1; rc63 = 0; ls63 = kWave - 1; cap = V(0); bnd0 = V(1);

    for (int32_t t0 = 0;; t0 += kGroup)
      if (!step(t0)) break;
    if (err && lane == 0 && a.err)
      atomicMax(reinterpret_cast<unsigned long long *>(a.err),
                (unsigned long long)flag_word(a.epoch, (uint32_t)err));
  }
};

template <int R, int D, typename V, bool RINGS>
__global__ __launch_bounds__(256) void stream_kernel(KernelArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  int lane = threadIdx.x & (kWave - 1);
  int wib = threadIdx.x / kWave;
  int wave = blockIdx.x * (blockDim.x / kWave) + wib;
  if (RINGS) {
    // zero this wave's ring counters before any wave of the workgroup reads them
    if (lane < 2) {
      LdsLayout L = lds_layout(R, D, (int)sizeof(V), a.hcap, true);
      reinterpret_cast<int32_t *>(smem + wib * a.lds_per_wave + L.xctr)[lane] = 0;
    }
    __syncthreads();
  }
  if (wave >= a.nwaves) return;
  Stream<R, D, V, RINGS> s(a, lane, wib, smem + wib * a.lds_per_wave);
  s.run(wave);
}

// The other measures and ground distances (OP as for Stream, OP != 0) on the
// same sweep; their plans never use LDS rings between waves.
template <int R, int D, typename V, int OP>
__global__ __launch_bounds__(256) void op_kernel(KernelArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  int lane = threadIdx.x & (kWave - 1);
  int wib = threadIdx.x / kWave;
  int wave = blockIdx.x * (blockDim.x / kWave) + wib;
  if (wave >= a.nwaves) return;
  Stream<R, D, V, false, OP> s(a, lane, wib, smem + wib * a.lds_per_wave);
  s.run(wave);
}

}  // namespace ffd

#endif  // FFD_STREAM_H
