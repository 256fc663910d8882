// Work description shared by the host planner (ffd_host.cpp) and the
// kernels (ffd_kernels.hip).  Internal to the library.
//
// Execution model.  One wavefront (64 lanes) runs one "stream".  Lane l
// holds R consecutive points (rows) of a row curve and, at step t, updates
// column t - l of the recurrence of Eq. (1), so the 64 lanes sweep an
// anti-diagonal wavefront.  Columns arrive as a stream: every task (one
// band of 64*R rows against one column curve) contributes a separator
// column followed by the column curve's points, so the lanes move from one
// task to the next without draining.  A wave runs the tasks of its jobs back
// to back; a job is one row curve against a contiguous range of column
// curves, every column curve in turn, a range of bands of the row curve in
// turn.  Consecutive bands on one wave hand the bottom row of one band to
// the next through LDS; when the bands of a row curve are split over
// several waves, the last band of one wave's range writes its bottom row to
// a link buffer in global memory and publishes its progress with a release
// store, and the wave holding the next band reads it after an acquire load
// (a "link").
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#define FFD_HD inline
#else
#define FFD_HD __host__ __device__ inline
#endif

namespace ffd {

constexpr int kWave = 64;            // lanes per wavefront
constexpr int kGroup = 16;           // steps per unrolled group; task lengths are multiples
constexpr int kRing = 256;           // column ring entries per wave (power of two)
constexpr int kFill = 64;            // steps between ring refills (= one entry per lane)
constexpr int kMinTask = 80;         // shortest task stream: >= kWave + kGroup, so the next band reads a
                                     // hand-off entry a group after lane 63 wrote it
constexpr int kMinTaskChained = 80;  // shortest stream when a band hands its bottom row on
constexpr int kDescSlots = 16;       // task descriptors in flight per wave
constexpr int kLinkRing = 256;       // LDS ring for boundary rows arriving over a link
constexpr int kXRing = 512;          // LDS ring for a bottom row handed to a wave of the same workgroup
constexpr int kFillStateBytes = 256; // per-wave refill state kept in LDS

// A job whose row_sel is kRowIdle computes nothing for col_count stream
// steps (padding that keeps a consumer band far enough behind its producer).
constexpr int32_t kRowIdle = 2;

struct Job {           // 64 bytes, device-resident plan entry
  int64_t out_base;    // output index of the first column curve of the job
  int64_t link_in;     // first element of the incoming link buffer (-1: none)
  int64_t link_out;    // first element of the outgoing link buffer (-1: none)
  int32_t row_sel;     // which coordinate array holds the row curve (0 or 1), or kRowIdle
  int32_t row_idx;     // index of the row curve in that array's offsets
  int32_t col_sel;     // which array holds the column curves
  int32_t col_first;   // first column curve
  int32_t col_count;   // number of column curves
  int32_t out_stride;  // output index step between consecutive column curves
  int32_t band_first;  // bands [band_first, band_first + band_count) of the row curve
  int32_t band_count;  // (band_count <= 0: all bands from band_first on)
  int32_t flag_in;     // progress flag of the incoming link (-1: none; <= -2: the row above comes
                       // through the LDS ring of wave -2 - flag_in of the same workgroup)
  int32_t flag_out;    // progress flag of the outgoing link (-1: none; -2: the bottom row goes to
                       // this wave's LDS ring, read by another wave of the workgroup)
};

// Progress flags hold (epoch << 32) | entries published; the epoch changes
// with every launch, so flags never need clearing.
FFD_HD uint64_t flag_word(uint32_t epoch, uint32_t count) { return ((uint64_t)epoch << 32) | count; }

// Bands of 64*R rows needed for a row curve of n points.
FFD_HD int64_t bands_for(int64_t n, int R) { return (n + (int64_t)kWave * R - 1) / ((int64_t)kWave * R); }

// Stream length of one task: at least kGroup separator columns, then the m
// columns, rounded up to a multiple of kGroup and to the minimum length (the
// separators come first so that a 16-lane block of the wave can take the
// task's rows at a group boundary, while its columns are still separators).
FFD_HD int64_t task_len(int64_t m, bool chained) {
  int64_t L = (m + kGroup + kGroup - 1) / kGroup * kGroup;
  int64_t lo = chained ? kMinTaskChained : kMinTask;
  return L < lo ? lo : L;
}

// LDS carve-up of one wave's region (byte offsets).  vsize is the byte size
// of the value type (4: float32 path, 8: exact path with FP64 values).
struct LdsLayout {
  int ring;   // (kRing + kGroup) column points; the last kGroup mirror the first
  int ghost;  // top boundary of a first band: 2 kGroup + 1 values, +inf except the
              // corner in the middle (-inf for the Frechet distance, 0 for DTW)
  int sink;   // kWave + kGroup values: bottom-row stores that hand nothing on
  int hand;   // hcap values: bottom row of the band above (same wave)
  int lring;  // kLinkRing values: boundary row arriving over a link
  int lstage; // kLinkRing values: outgoing boundary row, by stream position, until it is stored
  int xring;  // kXRing values: bottom row read by another wave of the workgroup
  int xctr;   // two int32 counters of that ring: entries written, entries read
  int pst;    // two slots of 64 * R * D row coordinates (next task's rows)
  int desc;   // kDescSlots task descriptors of 64 bytes
  int fill;   // refill state of the wave (kFillStateBytes)
  int total;
};

FFD_HD int align16(int x) { return (x + 15) & ~15; }
FFD_HD constexpr int pad_dim(int D) { return D == 3 ? 4 : D; }
// Levenshtein ring entries: the D symbol values and a separator flag, padded
// to a power of two.
FFD_HD constexpr int lev_dim(int D) { return D == 1 ? 2 : (D <= 3 ? 4 : (D <= 7 ? 8 : (D <= 15 ? 16 : 32))); }
// Coordinates per point of the kernel that runs curves of D coordinates:
// up to four, a kernel of their own; five to eight, the kernel of eight;
// nine to sixteen, the kernel of sixteen.  The wider kernels read the
// curves' own D coordinates per point and hold zeros in the others: a zero
// difference adds nothing to a sum of squares or of absolute values,
// changes no maximum of absolute values and no symbol comparison, so the
// results are those of D coordinates, bit for bit.
FFD_HD constexpr int kernel_dim(int D) { return D <= 4 ? D : (D <= 8 ? 8 : 16); }
// The wider kernels exist for one R each (a lane's registers hold its R
// rows twice): 2 rows per lane for the kernel of 8, 1 for the kernel of 16.
FFD_HD constexpr int wide_rows(int D) { return D <= 8 ? 2 : 1; }

// rings: the wave also owns a ring that hands its bottom row to another
// wave of its workgroup.  dtw: the layout of the DTW kernels.
// dp: values per ring entry (0: pad_dim(D)).
FFD_HD LdsLayout lds_layout(int R, int D, int vsize, int hcap, bool rings, int dp = 0) {
  LdsLayout L;
  int o = 0;
  L.ring = o;  o += (kRing + kGroup) * (dp ? dp : pad_dim(D)) * vsize;
  L.ghost = o; o += (2 * kGroup + 1) * vsize;
  L.sink = o;  o += (kWave + kGroup) * vsize;
  o = align16(o); L.hand = o; o += hcap * vsize;
  o = align16(o); L.lring = o; o += kLinkRing * vsize;
  o = align16(o); L.lstage = o; o += kLinkRing * vsize;
  o = align16(o); L.xring = o; o += rings ? kXRing * vsize : 0;
  o = align16(o); L.xctr = o; o += rings ? 16 : 0;
  o = align16(o); L.pst = o;  o += 2 * kWave * R * D * vsize;
  o = align16(o); L.desc = o; o += kDescSlots * 64;
  o = align16(o); L.fill = o; o += kFillStateBytes;
  L.total = align16(o);
  return L;
}

struct KernelArgs {
  const void *X[2];          // coordinate arrays, device (float32 or int32)
  const int64_t *off[2];     // curve offsets in points, device; unused in single-pair mode
  const Job *jobs;           // device plan; nullptr = single-pair mode (inline below)
  const int32_t *wave_jobs;  // [nwaves + 1]: jobs of wave w are [wave_jobs[w], wave_jobs[w+1])
  void *out;                 // float32 or int64 results, device
  int64_t inl_off[2][2];     // single-pair mode: curve 0 of each array is [off[s][0], off[s][1])
  Job inl_job;               // single-pair mode job
  int32_t nwaves;
  int32_t metric;            // 0 Euclidean, 1 squared
  int32_t hcap;              // hand-off row entries per wave (max chained task length)
  int32_t lds_per_wave;      // bytes of LDS per wave
  int32_t max_steps;         // upper bound of any wave's stream length (loop guard)
  uint32_t epoch;            // launch number, tags progress flags
  void *links;               // link buffers (value type of the path), device
  uint64_t *flags;           // progress flags, device
  uint64_t *err;             // error word (epoch << 32 | bits): bit 0 loop guard hit,
                             // bit 1 link wait abandoned; the largest word of a launch wins
  int32_t rings;             // nonzero: some jobs hand rows between waves through LDS rings
  int32_t dim;               // coordinates per point of the curves (at most the kernel's D)
};

// A link buffer holds the boundary rows of a job's column curves back to
// back; the row of column curve c starts at the sum of task_len(m, true) over
// the job's earlier column curves.

}  // namespace ffd
