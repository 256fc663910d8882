// Pipelined sweep of one long pair (the discrete Frechet distance of
// Eq. (1) on squared cells, Theorem 1's O(Q) state per band).
//
// The row curve is cut into bands of 64 R rows.  Band b runs on one
// wavefront: lane l holds rows [64 R b + R l, 64 R b + R l + R) and at step t
// updates column t - l, taking the value above its top row from lane l - 1
// (DPP wave_shr:1) and its left neighbours from its own registers -- the
// anti-diagonal sweep of the streaming kernels, without task switching: a
// wave sweeps its band once, from the first column to the last.
//
// Bands follow each other down the rows.  Band b + 1 needs band b's bottom
// row; lane 63 of band b produces column j at step j + 63 and writes it, in
// batches of four columns, to a ring in LDS by step j + 66.  Four computing
// waves of a workgroup (one per SIMD of the compute unit) hold four
// consecutive bands and run in lockstep, one 16-step group per barrier
// phase, each wave kPipeLag groups behind the one above it: the 16 values
// above a group are then all written in an earlier phase, and the wave reads
// them at the start of the group.
//
// A fifth wave of the workgroup computes nothing: it keeps the computing
// waves supplied, so that they issue no global memory instruction and carry
// no work but their band's (with one wave per SIMD, every instruction a
// computing wave issues lengthens the phase of the whole workgroup).  It
// loads the column points 16 per phase into a ring of the workgroup (a
// group's points two phases before the first wave reads them), polls the
// incoming link values (two groups ahead) into the first wave's ring, and
// stores the last wave's bottom row from its ring to the outgoing link.
// Link rows live in global memory, one value per column, initialised to the
// all-ones pattern, a NaN that no table value takes (every value of the
// table is a squared distance or +inf); the next workgroup polls the values
// themselves, so neither side needs a flag or a fence.  Workgroups form one
// chain in an order that keeps consecutive workgroups on the same XCD (the
// hardware deals workgroups to the eight XCDs in turn), so a link stays
// inside one L2 except at the seven XCD boundaries.  A pair with more bands
// than computing waves runs in passes: the wave of chain position c takes
// bands c, c + W, c + 2 W, ...; the band after a pass's last one reads its
// link like any other.
//
// Boundaries (reading c11 of the paper's recurrence): columns before the
// first hold +inf points, so every lane's left neighbour starts at +inf
// (M_{i,-1} = +inf); the first band's top is +inf (M_{-1,j} = +inf) with
// a -inf diagonal at the first column (the corner), which makes Eq. (1)
// produce the first row and column; rows past the curve's end repeat its
// last point, which leaves the distance unchanged (Sec. 4, footnote).
#ifndef FFD_PIPE_H
#define FFD_PIPE_H

#include "ffd_pipe_args.h"
#include "ffd_stream.h"

namespace ffd {

// LDS of a workgroup, byte offsets: the column ring, then per wave the
// hand-off ring (its bottom row, read by the next wave), the sink of the
// other lanes' batched writes (four values per lane at a 16-byte stride, so
// that a batch touches every bank once) and the ring of incoming link values.
template <int D, typename V>
struct PipeLds {
  static constexpr int DP = pad_dim(D);
  static constexpr int kQRing = 2 * kPipeRing;                                       // column ring entries
  static constexpr int kQ = 0;                                                       // (kQRing + 16) points
  static constexpr int kWave0 = kQ + (kQRing + kPipeGroup) * DP * (int)sizeof(V);
  static constexpr int kH = 0;                                                       // hand-off ring
  static constexpr int kSink = kH + kPipeRing * (int)sizeof(V);                      // 4 per lane + 16
  static constexpr int kIn = kSink + (4 * kWave + kPipeGroup) * (int)sizeof(V);      // incoming link values
  static constexpr int kWaveBytes = kIn + kPipeRing * (int)sizeof(V);
  static constexpr int kTotal = kWave0 + kPipeWaves * kWaveBytes;                    // per workgroup
};

template <int R, int D, typename V>
__global__ __launch_bounds__(kPipeThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void pipe_kernel(PipeArgs a) {
  using N = Num<V>;
  using C = typename N::Coord;
  using L = PipeLds<D, V>;
  constexpr int DP = L::DP;
  constexpr int QR = L::kQRing;
  struct alignas(sizeof(V) * DP) Pt {
    V c[DP];
  };
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = threadIdx.x / kWave;  // kPipeWaves: the helper wave
  const bool helper = wib == kPipeWaves;
  Pt *qring = reinterpret_cast<Pt *>(smem + L::kQ);
  auto wave_base = [&](int w) { return smem + L::kWave0 + w * L::kWaveBytes; };
  V *hring = reinterpret_cast<V *>(wave_base(helper ? 0 : wib) + L::kH);
  // the top row of this wave's band: the ring of the wave above, or (first
  // wave of the workgroup) the incoming link values
  const V *hin = wib > 0 && !helper ? reinterpret_cast<const V *>(wave_base(wib - 1) + L::kH)
                                    : reinterpret_cast<const V *>(wave_base(0) + L::kIn);
  V *inring = reinterpret_cast<V *>(wave_base(0) + L::kIn);                   // written by the helper
  const V *lastring = reinterpret_cast<const V *>(wave_base(kPipeWaves - 1) + L::kH);  // read by the helper

  // chain position of this workgroup
  const int32_t blk = blockIdx.x;
  const int32_t chain = a.xcd_span > 0 ? (blk % 8) * a.xcd_span + blk / 8 : blk;
  const int32_t W = a.nwg * kPipeWaves;
  const C *X = static_cast<const C *>(a.X);
  const C *Y = static_cast<const C *>(a.Y);
  V *links = static_cast<V *>(a.links);
  const V inf = N::inf();
  using Bits = std::conditional_t<sizeof(V) == 8, uint64_t, uint32_t>;
  const Bits kUnset = ~(Bits)0;
  int32_t err = 0;

  // groups a wave computes per pass: lane 63 reaches the last column at
  // step m + 62 and has written it to its ring by step m + 65; the helper
  // stores column j of the last wave's row to the link at that wave's group
  // j / 16 + 5
  const int32_t gwork = (int32_t)((a.m - 1) / kPipeGroup) + 6;
  const int32_t phases = gwork + (kPipeWaves - 1) * kPipeLag;
  const int32_t passes = (a.nb + W - 1) / W;

  for (int32_t pass = 0; pass < passes; ++pass) {
    const int32_t b0 = pass * W + chain * kPipeWaves;  // the workgroup's first band
    const int32_t b = helper ? a.nb : b0 + wib;        // this wave's band (>= nb: none)
    const bool active = b < a.nb;
    const bool fill = helper && b0 < a.nb;             // the helper has work in this pass
    const bool link_in = fill && b0 > 0;               // the first band reads a link
    const bool link_out = fill && b0 + kPipeWaves < a.nb;  // the last band writes one
    const int64_t lrow_in = (int64_t)(b0 - 1) / kPipeWaves, lrow_out = (int64_t)b0 / kPipeWaves;

    // rows of this lane, the last point repeated past the curve's end
    V p[R][D], Mp[R];
    {
      const int64_t r0 = (int64_t)b * kWave * R + (int64_t)lane * R;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int64_t ri = r0 + r < a.n ? r0 + r : a.n - 1;
        if (!active) ri = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) p[r][k] = N::cvt(X[ri * D + k]);
        Mp[r] = inf;
      }
    }
    // diagonal of lane 0 at the first column: the corner for the first band
    V upPrev = (b == 0 && lane == 0) ? -inf : inf;
    V bprev = inf;  // lane 63's bottom value of the previous step

    // The helper's global loads are issued at least one phase before they
    // are waited for: the 16 column points of group h (lanes 0 .. 15 own one
    // each; every lane loads a valid address, so the loaded registers are
    // never merged with other values and nothing waits for them early), put
    // in the ring at phase h - 2 (the first wave reads a group one phase
    // ahead), and the 16 link values of group h, loaded at phase h - 3 and
    // put in the first wave's ring at phase h - 1, polled again while any is
    // still unset.
    C qload[D];
    bool qmine = false;
    auto col_issue = [&](int64_t h) {
      int64_t col = h * kPipeGroup + (lane & (kPipeGroup - 1));
      qmine = lane < kPipeGroup && col < a.m;
      int64_t cc = col < a.m ? col : a.m - 1;
#pragma unroll
      for (int k = 0; k < D; ++k) qload[k] = Y[cc * D + k];
    };
    auto col_put = [&](int64_t col, bool in, const C *v) {
      Pt e;
#pragma unroll
      for (int k = 0; k < DP; ++k) e.c[k] = k < D ? (in ? N::cvt(v[k]) : inf) : V(0);
      int slot = (int)(col & (QR - 1));
      qring[slot] = e;
      if (slot < kPipeGroup) qring[slot + QR] = e;
    };
    auto col_take = [&](int64_t h) {
      if (lane < kPipeGroup) col_put(h * kPipeGroup + lane, qmine, qload);
    };
    // two link loads in flight (groups h and h + 1), in two register sets
    V lval0 = inf, lval1 = inf;
    bool lmine0 = false, lmine1 = false;
    auto link_issue = [&](int64_t h, V &lval, bool &lmine) {
      int64_t col = h * kPipeGroup + (lane & (kPipeGroup - 1));
      lmine = lane < kPipeGroup && col < a.m;
      int64_t cc = col < a.m ? col : a.m - 1;
      lval = __hip_atomic_load(links + lrow_in * a.link_stride + cc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // a wait lasts at most a.patience ticks of the real-time counter (the
    // host sizes it far above the modelled run time); once one wait has
    // been abandoned the wave waits no more, so a launch always ends
    auto link_take = [&](int64_t h, V &lval, bool &lmine) {
      uint64_t t_begin = 0;
      for (int it = 0;; ++it) {
        bool ok = !lmine || __builtin_bit_cast(Bits, lval) != kUnset;
        if (__builtin_amdgcn_ballot_w64(!ok) == 0) break;
        if (err) break;
        uint64_t now = __builtin_amdgcn_s_memrealtime();
        if (it == 0) t_begin = now;
        else if (now - t_begin > a.patience) {
          err |= 2;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        link_issue(h, lval, lmine);
      }
      if (lane < kPipeGroup) inring[(int)((h * kPipeGroup + lane) & (kPipeRing - 1))] = lmine ? lval : inf;
    };
    if (fill) {
      // columns -64 .. -1 are +inf points; groups 0 and 1 go in now, group 2 is loaded
      {
        C none[D];
#pragma unroll
        for (int k = 0; k < D; ++k) none[k] = C(0);
        col_put(lane - kWave, false, none);
      }
      for (int h = 0; h < 2; ++h) {
        col_issue(h);
        col_take(h);
      }
      col_issue(2);
      if (link_in) {
        link_issue(0, lval0, lmine0);
        link_issue(1, lval1, lmine1);
        link_take(0, lval0, lmine0);
        link_issue(2, lval0, lmine0);
      } else {
        // the first band: +inf above every column
        for (int i = lane; i < kPipeRing; i += kWave) inring[i] = inf;
      }
    }
    // every global load so far has returned (the rows, the first columns
    // and link values): the waits in the loop then only ever concern the
    // helper's loads of the phases before
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();

    // a group's column points, read one group ahead from two buffers used in
    // turn (FP64 values: read at the start of the group into one buffer, so
    // that a wave's registers fit two waves on one SIMD)
    constexpr bool kAhead = sizeof(V) == 4;
    Pt qa[kPipeGroup], qb[kPipeGroup];
    auto load_q = [&](int64_t g, Pt *q) {
      const Pt *qr = qring + (int)((g * kPipeGroup - lane) & (QR - 1));
#pragma unroll
      for (int u = 0; u < kPipeGroup; ++u) q[u] = qr[u];
    };
    const int32_t start = wib * kPipeLag;
    // one barrier phase: the helper's ring and link work, or this wave's
    // group g (if any) from qc, with the next group's points read into qn;
    // (lv, lm) is the link register set of group ph + 1
    auto phase = [&](int32_t ph, Pt *qc, Pt *qn, V &lv, bool &lm) {
      if (fill) {
        if (ph < gwork) {
          col_take(ph + 2);
          col_issue(ph + 3);
          if (link_in) {
            link_take(ph + 1, lv, lm);
            link_issue(ph + 3, lv, lm);
          }
        }
        // link out: columns [t0 - 80, t0 - 64) of the last wave's row at
        // its group t0 / 16 = ph - 3 kPipeLag, all in its ring since its
        // group before; lanes 0 .. 15 store one each
        if (link_out) {
          int64_t col = (int64_t)(ph - (kPipeWaves - 1) * kPipeLag) * kPipeGroup - kWave - kPipeGroup + lane;
          if (lane < kPipeGroup && col >= 0 && col < a.m)
            __hip_atomic_store(links + lrow_out * a.link_stride + col, lastring[(int)(col & (kPipeRing - 1))],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      const int32_t g = ph - start;
      if (active && g >= 0 && g < gwork) {
        const int64_t t0 = (int64_t)g * kPipeGroup;
        if (kAhead) {
          if (g == 0) load_q(0, qc);
          load_q(g + 1, qn);
        } else {
          load_q(g, qc);
        }
        // the values above this group's columns (written in earlier phases)
        V hc[kPipeGroup];
        {
          const V *hr = hin + (int)(t0 & (kPipeRing - 1));
#pragma unroll
          for (int u = 0; u < kPipeGroup; ++u) hc[u] = hr[u];
        }
        // lane 63 writes its bottom values of columns [t0 - 64, t0 - 48) in
        // four batches of four; the other lanes write to their own sink
        int32_t hidx = lane == kWave - 1 ? (int32_t)((t0 - kWave) & (kPipeRing - 1)) : kPipeRing + 4 * lane;
        V *hout = hring + hidx;
        V bots[4];
        bots[0] = bprev;
#pragma unroll
        for (int u = 0; u < kPipeGroup; ++u) {
          V bottom = Mp[R - 1];
          V up = N::shift_in(hc[u], bottom);
          V above = up, diag = upPrev;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            V t = p[r][0] - qc[u].c[0];
            V s = t * t;
#pragma unroll
            for (int k = 1; k < D; ++k) {
              V w = p[r][k] - qc[u].c[k];
              s = N::fma(w, w, s);
            }
            V v = N::mx(N::mn(N::mn(above, diag), Mp[r]), s);
            diag = Mp[r];
            above = v;
            Mp[r] = v;
          }
          upPrev = up;
          // Mp[R - 1] is now column t0 + u - 63 of the bottom row (lane 63)
          if ((u & 3) == 2) {
            bots[3] = Mp[R - 1];
#pragma unroll
            for (int k = 0; k < 4; ++k) hout[u - 2 + k] = bots[k];
          } else {
            bots[(u + 1) & 3] = Mp[R - 1];
          }
        }
        bprev = Mp[R - 1];
      }
      // (the helper's last phases have written every column group the
      // waves read: column group h is read at the earliest by the first
      // wave's group h - 1, and the 512-entry ring keeps 32 groups)
      __syncthreads();
    };
    for (int32_t ph = 0; ph < phases; ph += 2) {
      phase(ph, qa, kAhead ? qb : qa, lval1, lmine1);
      if (ph + 1 < phases) phase(ph + 1, kAhead ? qb : qa, qa, lval0, lmine0);
    }
    // the result: the last band's bottom value at the last column, which
    // lane 63 wrote to this wave's ring (the ring is not overwritten before
    // 256 further columns); a launch that abandoned a wait stores NaN (-1
    // for int64 results)
    if (active && b == a.nb - 1 && lane == 0) {
      V v = hring[(int)((a.m - 1) & (kPipeRing - 1))];
      if (err) v = __builtin_bit_cast(V, kUnset);
      if constexpr (sizeof(V) == 8) {
        static_cast<int64_t *>(a.out)[0] = err ? (int64_t)-1 : (int64_t)v;
      } else {
        N::store(a.out, 0, v, a.metric);
      }
    }
  }
  if (err && lane == 0 && a.err)
    atomicMax(reinterpret_cast<unsigned long long *>(a.err), (unsigned long long)flag_word(a.epoch, (uint32_t)err));
}

}  // namespace ffd

#endif  // FFD_PIPE_H
