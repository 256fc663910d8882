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
// batches of four columns, to a ring in LDS by step j + 66.  Four waves of a
// workgroup (one per SIMD of the compute unit) hold four consecutive bands
// and run in lockstep, one 16-step group per barrier phase, each wave
// kPipeLag groups behind the one above it: the 16 values above a group are
// then all written in an earlier phase, and the wave reads them at the start
// of the group.  The column points go through one ring of the workgroup,
// filled by the second wave 16 columns per group, ahead of the first wave
// (the one furthest ahead), so that the computing waves issue no global
// loads of their own and every global load is waited for a whole group after
// it was issued; the first wave takes the incoming link values instead, so
// that the extra work is split between two waves.  The bottom row of a
// workgroup's last band goes to global memory ("link" rows, one value per
// column, initialised to the all-ones pattern, a NaN that no table value
// takes: every value of the table is a squared distance or +inf), stored by
// lane 63 straight from its registers with each LDS batch; the first wave of
// the next workgroup polls the values themselves, so neither side needs a
// flag or a fence.  Workgroups form one chain in an order that keeps
// consecutive workgroups on the same XCD (the hardware deals workgroups to
// the eight XCDs in turn), so a link stays inside one L2 except at the seven
// XCD boundaries.  A pair with more bands than waves runs in passes: the wave
// of chain position c takes bands c, c + W, c + 2 W, ...; the band after a
// pass's last one reads its link like any other.
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
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void pipe_kernel(PipeArgs a) {
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
  const int wib = threadIdx.x / kWave;
  Pt *qring = reinterpret_cast<Pt *>(smem + L::kQ);
  unsigned char *base = smem + L::kWave0 + wib * L::kWaveBytes;
  V *hring = reinterpret_cast<V *>(base + L::kH);
  V *inring = reinterpret_cast<V *>(base + L::kIn);
  // the top row of this wave's band: the ring of the wave above, or (first
  // wave of the workgroup) the values it copies in from its link
  const V *hin = wib > 0 ? reinterpret_cast<const V *>(smem + L::kWave0 + (wib - 1) * L::kWaveBytes + L::kH)
                         : inring;

  // chain position of this workgroup
  const int32_t blk = blockIdx.x;
  const int32_t chain = a.xcd_span > 0 ? (blk % 8) * a.xcd_span + blk / 8 : blk;
  const int32_t W = a.nwg * kPipeWaves;
  const int32_t cpos = chain * kPipeWaves + wib;
  const C *X = static_cast<const C *>(a.X);
  const C *Y = static_cast<const C *>(a.Y);
  V *links = static_cast<V *>(a.links);
  const V inf = N::inf();
  using Bits = std::conditional_t<sizeof(V) == 8, uint64_t, uint32_t>;
  const Bits kUnset = ~(Bits)0;
  int32_t err = 0;

  // groups a wave computes per pass: lane 63 reaches the last column at
  // step m + 62 and has written it (to its ring and its link row) by step
  // m + 65
  const int32_t gwork = (int32_t)((a.m + 66 + kPipeGroup - 1) / kPipeGroup);
  const int32_t phases = gwork + (kPipeWaves - 1) * kPipeLag;
  const int32_t passes = (a.nb + W - 1) / W;

  for (int32_t pass = 0; pass < passes; ++pass) {
    const int32_t b0 = pass * W + chain * kPipeWaves;  // the workgroup's first band
    const int32_t b = b0 + wib;                        // this wave's band (>= nb: none)
    const bool active = b < a.nb;
    const bool filler = wib == 1 && b0 < a.nb;         // fills the column ring for the workgroup
    const bool link_in = active && b > 0 && wib == 0;
    const bool link_out = active && b + 1 < a.nb && wib == kPipeWaves - 1;
    const int64_t lrow_in = (int64_t)(b - 1) / kPipeWaves, lrow_out = (int64_t)b / kPipeWaves;

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

    // Global loads are issued in one group and waited for in the next.  The
    // filler wave loads the 16 column points of group h (lanes 0 .. 15 own
    // one each; every lane loads a valid address, so the loaded registers
    // are never merged with other values and nothing waits for them early)
    // and puts them in the ring at phase h - 2: the first wave reads a group
    // one phase ahead.  The first wave loads the 16 link values of group h
    // and puts them in its incoming ring at its group h - 1.
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
    V lval = inf;
    bool lmine = false;
    auto link_issue = [&](int64_t h) {
      int64_t col = h * kPipeGroup + (lane & (kPipeGroup - 1));
      lmine = lane < kPipeGroup && col < a.m;
      int64_t cc = col < a.m ? col : a.m - 1;
      lval = __hip_atomic_load(links + lrow_in * a.link_stride + cc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // a wait lasts at most a.patience ticks of the real-time counter (the
    // host sizes it far above the modelled run time); once one wait has
    // been abandoned the wave waits no more, so a launch always ends
    auto link_take = [&](int64_t h) {
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
        link_issue(h);
      }
      if (lane < kPipeGroup) inring[(int)((h * kPipeGroup + lane) & (kPipeRing - 1))] = lmine ? lval : inf;
    };
    if (filler) {
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
    }
    if (link_in) {
      link_issue(0);
      link_take(0);
      link_issue(1);
    } else if (wib == 0) {
      // the first band: +inf above every column
      for (int i = lane; i < kPipeRing; i += kWave) inring[i] = inf;
    }
    // every global load so far has returned (the rows, the first columns
    // and link values): the waits in the loop then only ever concern the
    // loads of the group before
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();

    // a group's column points, read one group ahead; two buffers used in turn
    Pt qa[kPipeGroup], qb[kPipeGroup];
    auto load_q = [&](int64_t g, Pt *q) {
      const Pt *qr = qring + (int)((g * kPipeGroup - lane) & (QR - 1));
#pragma unroll
      for (int u = 0; u < kPipeGroup; ++u) q[u] = qr[u];
    };
    const int32_t start = wib * kPipeLag;
    // one barrier phase: the filler's ring work, then this wave's group g
    // (if any) from qc, with the next group's points read into qn
    auto phase = [&](int32_t ph, Pt *qc, Pt *qn) {
      if (filler && ph < gwork) {
        col_take(ph + 2);
        col_issue(ph + 3);
      }
      const int32_t g = ph - start;
      if (active && g >= 0 && g < gwork) {
        const int64_t t0 = (int64_t)g * kPipeGroup;
        if (link_in) {
          link_take(g + 1);
          link_issue(g + 2);
        }
        if (g == 0) load_q(0, qc);
        load_q(g + 1, qn);
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
        V *lout = links + lrow_out * a.link_stride;
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
            // the same four columns, t0 + u - 66 .. t0 + u - 63, to the link
            // row (a multiple of 4 below m: the row's stride, a multiple of
            // 64 not below m, holds all four)
            const int64_t col = t0 + u - 66;
            if (link_out && lane == kWave - 1 && col >= 0 && col < a.m) {
#pragma unroll
              for (int k = 0; k < 4; ++k)
                __hip_atomic_store(lout + col + k, bots[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          } else {
            bots[(u + 1) & 3] = Mp[R - 1];
          }
        }
        bprev = Mp[R - 1];
      }
      // (the filler's last phases have written every column group the
      // waves read: column group h is read at the earliest by the first
      // wave's group h - 1, and the 512-entry ring keeps 32 groups)
      __syncthreads();
    };
    for (int32_t ph = 0; ph < phases; ph += 2) {
      phase(ph, qa, qb);
      if (ph + 1 < phases) phase(ph + 1, qb, qa);
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
