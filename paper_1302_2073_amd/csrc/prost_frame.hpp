// Persistent per-frame kernel of pROST (Sec. 3.3, Steps 1-3, plus the 3x3
// median of Sec. 3.4) for one video stream.
//
// One launch processes one frame (or, in the sequence form, several frames
// with the tile kept in registers between them and U stored after the last
// one).  The m x k subspace U is split into workgroup tiles of `tpw` pixels
// (all colour entries of a pixel stay in one tile); each thread keeps NR rows
// of U in registers for the whole frame (K floats per row, or K bfloat16
// pairs per two rows with bfloat16 storage), so U is read from HBM once and
// written once per frame (per launch in the sequence form).
// The frame's sequence of dependent reductions runs as gang-wide reductions
// between all workgroups of the launch (cooperative launch, so all of them
// are resident):
//   for each CG step j:  A: g = -U^T(w phi'(r)), f = sum w phi(r)
//                        B: d^T H d = sum w c(r) (u.d)^2
//   eta pass:            a = U^T eta, ||eta||^2, f at the final y
// The 3x3 median of a frame's labels runs at the start of the next launch
// (or in median_kernel when the mask is asked for first), which saves the
// exchange that would otherwise separate the label writes from the median.
// Every workgroup reduces the published partials in the same fixed order, so
// all of them hold bit-identical k-vectors without a broadcast step.  Waiting
// workgroups spin on epoch-tagged float64 slots (each thread on its own
// values, no barrier inside the wait, bounded by a wall-clock time-out).
#pragma once

#include <utility>

#include "prost_device.hpp"
#include "../../include/prost.h"

namespace prost {
inline namespace PROST_BLOCK_NS {

struct FrameArgs {
  void* U;               // K planes of ldU entries (storage type)
  const void* x;         // frame, m entries (storage type); used when xtab is NULL
  const void* const* xtab;  // ring of `ring` frame pointers, frame n at xtab[n % ring]
  int ring;
  uint8_t* lab;          // raw labels, P bytes (read: previous frame, write: this frame)
  uint8_t* mask;         // median-filtered mask, P bytes
  double* y;             // k coefficients (float64 state)
  long long* nframe;     // frame counter
  pros_stats* stats;     // statistics of the frame
  double* part;          // (2 * G + kExtraSlots) * kSlot doubles of workgroup partials
  unsigned* sync;        // [0] arrival counter, [1] counter base, [2] error bits, [3] epoch base
  long long ldU;
  int m, P, C, W, H, k;
  int G, tpw;
  CostParams cp;
  float delta, omega;
  double t_init, t_min, tau;
  int J;
  int labels_after_update;
  int weights_from_filtered;
  long long timeout;     // wall-clock ticks a barrier may wait
  long long* trace;      // optional per-tile timestamps (diagnostics), 64 per tile
  int pair_aligned;      // bfloat16: row pairs are aligned 32-bit words (U planes and frame)
  float* pre_mean;       // pre-processing (Sec. 3.4): running average (m), NULL when off
  float* pre_m2;         // per-entry sum of squared deviations (m)
  double* pre_stat;      // [0] entry sum of pre_m2, [1] initialization frames accumulated
  int i_init;            // length of the initialization phase
  float* score;          // optional: |r'| of every entry after Step 3 (m floats), or NULL
  int ysolve;            // 0: CG with the PR+ direction, 1: gradient descent
  int sync_mode;         // 0: counter barrier + all-read, 1: tagged gather/broadcast,
                         // 2: two-level tagged gather (groups of tiles with equal t % 8),
                         // 3: every workgroup reads all tagged partials
  int curv;              // curvature schedule of a CG step: 0 = d^T H d in a second pass
                         // and exchange, 1 = H reduced with the gradient (one wide exchange)
  const void* const* seq;  // frames 1 .. nseq - 1 of a sequence launch (frame 0 is x), device array;
                           // with xtab (batched form) the ring is read instead
  int nseq;                // frames processed by this launch (1: one frame)
};

constexpr int kReplicas = 8;      // copies of a gathered result (spread the pollers)
constexpr int kExtraSlots = 32;   // slots beyond 2 G: replicas / XCD-level slots

// Shared k-space state of one workgroup (all float64 unless noted).
constexpr int kMaxNR = 32;   // register rows per thread (bfloat16 pairs at small k)
template <int K>
struct KSpace {
  double y[K];
  double d[K];
  double gp[K];     // previous gradient
  double dp[K];     // previous direction
  double a[K];      // U^T eta
  double red[kSlot];
  double gd;        // g . d of the current step
  float df[K];      // direction (float) for the row passes
  float vf[K];      // v = y/||y||
  float af[K];      // a (float)
  float yf[K];
  float scal[8];    // row-pass scalars
  int flag[4];      // [0] stop CG, [1] bad frame, [2] do update
  double pre_sum;   // pre-processing: entry sum of the deviation sums after this frame
  float pre_inv_s;  // 1 / scale applied to this frame
  float pre_inv_n;  // 1 / (frames accumulated including this one)
  int pre_upd;      // this frame joins the running average
};

// Workgroup-shared scratch of one frame tile (sized for the largest k / NR).
// Wide exchange (IRLS step, one-exchange curvature schedule): g, f and the upper triangle of H
// (K + 1 + K (K + 1) / 2 <= 153 values) in vectors of kWideMax float64.
constexpr int kWideChunks = 5;
constexpr int kWideMax = kWideChunks * kSlot;
constexpr int kWideIn = kWideMax + kSlot;   // room for the last zero-padded chunk

struct FrameSmem {
  KSpace<kMaxK> ks;
  double red[kWaves][kSlot];
  double wg[kSlot];
  double big[kBlock];          // one float64 per thread (gathers)
  int ctl[4];
  uint8_t flag[kBlock * kMaxNR];
  double wide_in[kWideIn];     // wide exchange: this workgroup's partials
  double wide_out[kWideMax];   // wide exchange: gang totals
  double hs[kMaxK][kMaxK + 1]; // IRLS: augmented [H | -g] for the k-space solve
};


// Diagnostics: wall-clock timestamp `idx` (< 64) of a tile, by thread 0.
__device__ __forceinline__ void trace_point(const FrameArgs& a, int tile, int idx) {
  if (a.trace && thread_index() == 0 && idx < 64) a.trace[(size_t)tile * 64 + idx] = wall_clock64();
}

// Waits for component `comp` of the tagged slots q = row0, row0 + rs, ...
// (q < n, slot q at base + q * qstride) to carry epoch ep and returns their
// sum in slot order.  Each thread spins on its own values with no barrier
// inside the wait (a barrier per poll round made every round cost a memory
// round trip plus two workgroup barriers); `bad` is set on time-out or when
// another workgroup has raised the time-out bit.
__device__ __forceinline__ double spin_sum(const double* base, int n, int rs, size_t qstride, int comp, int row0,
                                           unsigned ep, const FrameArgs& a, int& bad) {
  double v = 0.0;
  const long long t0 = now_ticks();
  for (int q = row0; q < n; q += rs) {
    const double* p = base + (size_t)q * qstride + comp;
    double x = ld_tagged(p);
    unsigned spins = 0;
    while (tag_of(x) != ep) {
      x = ld_tagged(p);
      if ((++spins & 63u) == 0 &&
          (now_ticks() - t0 > a.timeout ||
           (__hip_atomic_load(&a.sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout))) {
        bad = 1;
        return v;
      }
    }
    v += untag(x);
  }
  return v;
}

// Uniform end of a spin wait: false in every thread (and the gang's
// time-out bit raised) if any thread gave up.  The barrier also publishes
// the threads' s_big entries.
__device__ __forceinline__ bool spin_end(int bad, const FrameArgs& a) {
  if (__syncthreads_or(bad)) {
    if (thread_index() == 0) __hip_atomic_fetch_or(&a.sync[2], kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
  return true;
}

// Workgroup + gang reduction of L float partials held by every thread.
// Result (float64, identical in every workgroup) lands in s_out[0..L).
// Tagged gather/broadcast: every workgroup publishes its tagged partial
// vector; the gang's tile 0 polls all of them, sums them in tile order and
// publishes the tagged totals in kReplicas copies that the other workgroups
// poll.  No shared counter, so no serialised atomics on one address.
// `fenced` adds release/acquire fences around the exchange so that plain
// global writes made before it (labels) are visible after it.
template <int L>
__device__ __forceinline__ bool gang_reduce_tagged(const double* wg_sum, const FrameArgs& a, const int tile,
                                                   int& nbar, unsigned ebase, double* s_big,
                                                   double* s_out, int* s_ctl, bool fenced) {
  const int tid = thread_index();
  const int lane = tid & 63;
  const int wv = tid >> 6;
  ++nbar;
  const unsigned ep = (ebase + (unsigned)nbar) & 0xFFu;
  double* slots = a.part;                                 // G slots
  double* rep = a.part + (size_t)2 * a.G * kSlot;         // kReplicas slots
  if (fenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (tid < L) st_tagged(&slots[(size_t)tile * kSlot + tid], tag_value(wg_sum[tid], ep));
  if (tile == 0) {
    constexpr int kRows = kBlock / 32;
    const int comp = tid & 31, row0 = tid >> 5;
    int bad = 0;
    const double v = (comp < L) ? spin_sum(slots, a.G, kRows, kSlot, comp, row0, ep, a, bad) : 0.0;
    s_big[tid] = v;
    if (!spin_end(bad, a)) return false;
    if (tid < L) {
      double tot = 0.0;
#pragma unroll
      for (int r = 0; r < kRows; ++r) tot += s_big[r * 32 + tid];
      s_out[tid] = untag(tag_value(tot, ep));   // what every other workgroup will read
    }
    if (fenced) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    __syncthreads();
    for (int q = tid; q < kReplicas * L; q += kBlock) {
      const int r = q / L, i = q - r * L;
      st_tagged(&rep[(size_t)r * kSlot + i], tag_value(s_out[i], ep));
    }
    __syncthreads();
    return true;
  }
  // other workgroups: poll their replica
  if (tid == 0) s_ctl[1] = 0;
  __syncthreads();
  if (tid < L) {
    const double* src = &rep[(size_t)(tile % kReplicas) * kSlot + tid];
    const long long t0 = now_ticks();
    unsigned spins = 0;
    while (true) {
      const double x = ld_tagged(src);
      if (tag_of(x) == ep) {
        s_out[tid] = untag(x);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 63u) == 0) {
        if ((__hip_atomic_load(&a.sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout) ||
            now_ticks() - t0 > a.timeout) {
          __hip_atomic_fetch_or(&a.sync[2], kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_ctl[1] = 1;
          break;
        }
      }
    }
  }
  if (fenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  return s_ctl[1] == 0;
}

// Tagged all-read helper: waits for n tagged slots (stride kSlot) to carry
// the epoch, summing component c in slot order.  Thread layout: component
// tid % 32, slots tid / 32, tid / 32 + kRows, ...; the kRows partial sums are
// then added in order.  Uniform exit; false on time-out.
template <int L>
__device__ __forceinline__ bool poll_sum_slots(const double* slots, int nslots, unsigned ep, const FrameArgs& a,
                                               double* s_big, double* out) {
  const int tid = thread_index();
  constexpr int kRows = kBlock / 32;
  const int comp = tid & 31, row0 = tid >> 5;
  int bad = 0;
  const double v = (comp < L) ? spin_sum(slots, nslots, kRows, kSlot, comp, row0, ep, a, bad) : 0.0;
  s_big[tid] = v;
  if (!spin_end(bad, a)) return false;
  if (tid < L) {
    double tot = 0.0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) tot += s_big[r * 32 + tid];
    out[tid] = tot;
  }
  __syncthreads();
  return true;
}

// Two-level tagged exchange: the tiles t = x, x + 8, x + 16, ... form group x
// (x < 8); group x's first tile gathers their tagged partials and publishes
// the group sum; every workgroup then reads the (at most 8) group sums and
// adds them in group order.  Two hops; every workgroup ends with
// bit-identical totals.
template <int L>
__device__ __forceinline__ bool gang_reduce_2level(const double* wg_sum, const FrameArgs& a, const int tile,
                                                   int& nbar, unsigned ebase, double* s_big,
                                                   double* s_out, int* s_ctl, bool fenced) {
  const int tid = thread_index();
  ++nbar;
  const unsigned ep = (ebase + (unsigned)nbar) & 0xFFu;
  const int x = tile & 7;
  const int ngrp = min(8, a.G);
  double* slots = a.part;                                            // G level-1 slots
  double* gs = a.part + (size_t)a.G * kSlot + (size_t)(nbar & 1) * 8 * kSlot;   // 2 x 8 group sums
  if (fenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (tid < L) st_tagged(&slots[(size_t)tile * kSlot + tid], tag_value(wg_sum[tid], ep));
  if (tile < 8) {   // group leader: members x, x + 8, ... (slot stride 8)
    const int n = (a.G - x + 7) >> 3;
    const int comp = tid & 31, row0 = tid >> 5;
    constexpr int kRows = kBlock / 32;
    int bad = 0;
    const double v = (comp < L) ? spin_sum(slots + (size_t)x * kSlot, n, kRows, (size_t)8 * kSlot, comp, row0, ep, a, bad)
                                : 0.0;
    s_big[tid] = v;
    if (!spin_end(bad, a)) return false;
    if (tid < L) {
      double g = 0.0;
      for (int r = 0; r < kRows; ++r) g += s_big[r * 32 + tid];
      st_tagged(&gs[(size_t)x * kSlot + tid], tag_value(g, ep));
    }
    trace_point(a, tile, 25 + 3 * (nbar - 1));
    __syncthreads();
  }
  if (!poll_sum_slots<L>(gs, ngrp, ep, a, s_big, s_out)) return false;
  if (fenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// One-hop tagged exchange: every workgroup publishes its tagged partial and
// reads all G of them directly (G^2 small reads, one round trip).
template <int L>
__device__ __forceinline__ bool gang_reduce_allread(const double* wg_sum, const FrameArgs& a, const int tile,
                                                    int& nbar, unsigned ebase, double* s_big,
                                                    double* s_out, bool fenced) {
  const int tid = thread_index();
  ++nbar;
  const unsigned ep = (ebase + (unsigned)nbar) & 0xFFu;
  double* slots = a.part + (size_t)(nbar & 1) * a.G * kSlot;      // double-buffered
  if (fenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (tid < L) st_tagged(&slots[(size_t)tile * kSlot + tid], tag_value(wg_sum[tid], ep));
  if (!poll_sum_slots<L>(slots, a.G, ep, a, s_big, s_out)) return false;
  if (fenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Poll n tagged vectors of LT values (vector q at base + q * qstride) until
// every value carries epoch ep; out[v] = sum over q in order.  Threads:
// value tid % kWideMax, vectors tid / kWideMax + 3 i.  Uniform exit.
__device__ __forceinline__ bool poll_sum_wide(const double* base, int n, int qstride, int LT, unsigned ep,
                                              const FrameArgs& a, double* s_big, double* out) {
  const int tid = thread_index();
  constexpr int kRowsW = kBlock / kWideMax;
  const int v = tid % kWideMax, row = tid / kWideMax;
  const bool act = row < kRowsW && v < LT;
  int bad = 0;
  const double acc = act ? spin_sum(base, n, kRowsW, (size_t)qstride, v, row, ep, a, bad) : 0.0;
  s_big[tid] = acc;
  if (!spin_end(bad, a)) return false;
  if (tid < LT) {
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < kRowsW; ++r) t += s_big[r * kWideMax + tid];
    out[tid] = t;
  }
  __syncthreads();
  return true;
}

// Gang sum of LT (<= kWideMax) float64 values per workgroup, in the
// two-hop form of sync mode 2 (groups of tiles t = x mod 8), in its own
// region of the exchange buffer after the regular slots.  Every workgroup
// ends with bit-identical totals in out.
__device__ __forceinline__ bool gang_reduce_wide(const double* in, int LT, const FrameArgs& a, const int tile,
                                                 int& nbar, unsigned ebase, double* s_big, double* out) {
  const int tid = thread_index();
  ++nbar;
  if (a.G == 1) {   // a gang of one workgroup: its sums are the totals
    for (int q = tid; q < LT; q += kBlock) out[q] = in[q];
    __syncthreads();
    return true;
  }
  const unsigned ep = (ebase + (unsigned)nbar) & 0xFFu;
  const int x = tile & 7;
  const int ngrp = min(8, a.G);
  double* slots = a.part + (size_t)(2 * a.G + kExtraSlots) * kSlot;           // G vectors
  double* gs = slots + (size_t)a.G * kWideMax + (size_t)(nbar & 1) * 8 * kWideMax;   // 2 x 8 group sums
  for (int q = tid; q < LT; q += kBlock) st_tagged(&slots[(size_t)tile * kWideMax + q], tag_value(in[q], ep));
  if (tile < 8) {   // group leader: members x, x + 8, ...
    const int n = (a.G - x + 7) >> 3;
    if (!poll_sum_wide(slots + (size_t)x * kWideMax, n, 8 * kWideMax, LT, ep, a, s_big, out)) return false;
    for (int q = tid; q < LT; q += kBlock) st_tagged(&gs[(size_t)x * kWideMax + q], tag_value(out[q], ep));
  }
  return poll_sum_wide(gs, ngrp, kWideMax, LT, ep, a, s_big, out);
}

// Workgroup sum of L float partials (one value per thread each), float64
// result in wg_sum[0..L) (shared).
template <int L>
__device__ __forceinline__ void wg_reduce(float (&acc)[L], double (*s_red)[kSlot], double* wg_sum) {
  const int lane = thread_index() & 63;
  const int wv = thread_index() >> 6;
  int comp;
  const float v = wave_reduce_scatter<L>(acc, comp);
  if (wave_rs_owner<L>(lane) && comp < L) s_red[wv][comp] = (double)v;
  __syncthreads();
  if (thread_index() < L) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) v += s_red[q][thread_index()];
    wg_sum[thread_index()] = v;
  }
  __syncthreads();
}

template <int L>
__device__ __forceinline__ bool gang_reduce_counter(float (&acc)[L], const FrameArgs& a, const int tile, int& nbar,
                                                    unsigned base, double (*s_red)[kSlot], double* s_big,
                                                    double* s_out, int* s_ctl) {
  const int lane = thread_index() & 63;
  const int wv = thread_index() >> 6;
  // 1. per wave
  {
    int comp;
    const float v = wave_reduce_scatter<L>(acc, comp);
    if (wave_rs_owner<L>(lane) && comp < L) s_red[wv][comp] = (double)v;
  }
  __syncthreads();
  double* slot = a.part + ((size_t)(nbar & 1) * a.G + tile) * kSlot;
  if (thread_index() < L) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) v += s_red[q][thread_index()];
    __hip_atomic_store(&slot[thread_index()], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // 2. gang barrier
  ++nbar;
  if (!gang_barrier(a.sync, base + (unsigned)a.G * (unsigned)nbar, a.timeout, s_ctl)) return false;
  // 3. every workgroup sums all partials in the same order: thread t adds
  // component t % 32 of slots t / 32, t / 32 + kRows, ... (contiguous loads),
  // then the kRows partial sums of each component are added in order.
  // Plain (cached) loads: the barrier's acquire fence invalidated stale lines,
  // so the first workgroup of each XCD pulls the partials into its L2.
  const double* buf = a.part + (size_t)((nbar - 1) & 1) * a.G * kSlot;
  constexpr int kRows = kBlock / 32;
  const int comp = thread_index() & 31, row0 = thread_index() >> 5;
  double v = 0.0;
  if (comp < L)
    for (int w = row0; w < a.G; w += kRows) v += buf[(size_t)w * kSlot + comp];
  s_big[thread_index()] = v;
  __syncthreads();
  if (thread_index() < L) {
    double tot = 0.0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) tot += s_big[r * 32 + thread_index()];
    s_out[thread_index()] = tot;
  }
  __syncthreads();
  return true;
}

// Gang-wide sum of L float partials: every workgroup of the gang ends with
// the same float64 totals in s_out[0..L).
template <int L>
__device__ __forceinline__ bool gang_reduce_impl(float (&acc)[L], const FrameArgs& a, const int tile, int& nbar,
                                                 unsigned base, unsigned ebase, FrameSmem& sm, double* s_out,
                                                 bool fenced) {
  if (a.G == 1) {   // a gang of one workgroup: its sums are the totals, no memory exchange
    ++nbar;
    wg_reduce<L>(acc, sm.red, s_out);
    return true;
  }
  if (a.sync_mode == 1) {
    wg_reduce<L>(acc, sm.red, sm.wg);
    return gang_reduce_tagged<L>(sm.wg, a, tile, nbar, ebase, sm.big, s_out, sm.ctl, fenced);
  }
  if (a.sync_mode == 2) {
    wg_reduce<L>(acc, sm.red, sm.wg);
    trace_point(a, tile, 24 + 3 * nbar);
    return gang_reduce_2level<L>(sm.wg, a, tile, nbar, ebase, sm.big, s_out, sm.ctl, fenced);
  }
  if (a.sync_mode == 3) {
    wg_reduce<L>(acc, sm.red, sm.wg);
    return gang_reduce_allread<L>(sm.wg, a, tile, nbar, ebase, sm.big, s_out, fenced);
  }
  return gang_reduce_counter<L>(acc, a, tile, nbar, base, sm.red, sm.big, s_out, sm.ctl);
}


template <int L>
__device__ __forceinline__ bool gang_reduce(float (&acc)[L], const FrameArgs& a, const int tile, int& nbar,
                                            unsigned base, unsigned ebase, FrameSmem& sm, double* s_out,
                                            bool fenced = false) {
  trace_point(a, tile, 2 + 2 * nbar);
  const bool ok = gang_reduce_impl<L>(acc, a, tile, nbar, base, ebase, sm, s_out, fenced);
  trace_point(a, tile, 1 + 2 * nbar);
  return ok;
}


// 3x3 median of binary labels (>= 5 of the 9 neighbours, edges replicated,
// Sec. 3.4) for pixels [p0, p0 + npx) of a W x H image.
// COH: the labels were written in this launch by other workgroups, with
// device-coherent stores; read them with device-coherent loads.
template <bool COH = false>
__device__ __forceinline__ void median3x3_range(const uint8_t* __restrict__ lab, uint8_t* __restrict__ mask, int W,
                                                int H, int p0, int npx) {
  // kMedBatch pixels per thread at a time: their 9 kMedBatch loads are all
  // issued before the first is used (an entry past the tile loads the
  // tile's last pixel again and is not stored), so a tile costs one memory
  // latency per batch instead of one per pixel
  constexpr int kMedBatch = 3;
  for (int pl0 = thread_index(); pl0 < npx; pl0 += kMedBatch * blockDim.x) {
    int rb[kMedBatch][3], cb[kMedBatch][3];   // clamped neighbour rows (times W) and columns
#pragma unroll
    for (int b = 0; b < kMedBatch; ++b) {
      const int pix = p0 + min(pl0 + b * (int)blockDim.x, npx - 1);
      const int row = pix / W, col = pix - row * W;
      rb[b][0] = max(row - 1, 0) * W;
      rb[b][1] = row * W;
      rb[b][2] = min(row + 1, H - 1) * W;
      cb[b][0] = max(col - 1, 0);
      cb[b][1] = col;
      cb[b][2] = min(col + 1, W - 1);
    }
    uint8_t v[kMedBatch][9];
#pragma unroll
    for (int b = 0; b < kMedBatch; ++b)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const uint8_t* p = lab + rb[b][i] + cb[b][j];
          v[b][3 * i + j] = COH ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
        }
#pragma unroll
    for (int b = 0; b < kMedBatch; ++b) {
      int cnt = 0;
#pragma unroll
      for (int t = 0; t < 9; ++t) cnt += v[b][t];
      const int pl = pl0 + b * (int)blockDim.x;
      if (pl < npx) mask[p0 + pl] = (cnt >= 5) ? 1 : 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Pieces shared by the two register layouts of a tile
// ---------------------------------------------------------------------------

// Per-tile constants.
struct TileCtx {
  int p0, npx, nq;        // first pixel, pixels, register rows (npx * C)
  unsigned base, ebase;   // exchange counter / epoch bases of this launch
  long long n;            // frame index
  bool lead;              // tile 0 writes the stream's statistics and y
};

// Reads y and the frame index, then filters the previous frame's labels of
// this tile into the mask (the labels were written by the previous launch; no
// workgroup rewrites labels before the last exchange of this frame, which
// every workgroup reaches only after this point).
template <int K>
__device__ __forceinline__ TileCtx tile_begin(const FrameArgs& a, const int tile, KSpace<kMaxK>& ks) {
  TileCtx t;
  const int tid = thread_index();
  t.p0 = tile * a.tpw;
  t.npx = min(a.tpw, a.P - t.p0);
  t.nq = t.npx * a.C;
  t.base = __hip_atomic_load(&a.sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  t.ebase = __hip_atomic_load(&a.sync[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  t.n = *a.nframe;
  t.lead = (tile == 0);
  if (tid < K) {
    const double yv = (tid < a.k) ? a.y[tid] : 0.0;
    ks.y[tid] = yv;
    ks.yf[tid] = (float)yv;
  }
  if (tid < 4) ks.flag[tid] = 0;
  if (tid == 0) {
    float inv_s = 1.f, inv_n = 1.f;
    int upd = 0;
    if (a.pre_mean) {
      const double cnt = a.pre_stat[1];
      const double var = cnt >= 2.0 ? a.pre_stat[0] / ((double)a.m * (cnt - 1.0)) : 0.0;
      inv_s = var > 0.0 ? (float)(1.0 / sqrt(var)) : 1.f;
      upd = (t.n < (long long)a.i_init) ? 1 : 0;
      inv_n = (float)(1.0 / (cnt + 1.0));
    }
    ks.pre_inv_s = inv_s;
    ks.pre_inv_n = inv_n;
    ks.pre_upd = upd;
    ks.pre_sum = 0.0;
  }
  __syncthreads();
  trace_point(a, tile, 0);
  median3x3_range(a.lab, a.mask, a.W, a.H, t.p0, t.npx);
  __syncthreads();
  trace_point(a, tile, 1);
  return t;
}

// Pre-processing of one frame entry (Sec. 3.4): with upd the entry joins the
// running average (Welford update of mean and deviation sum; the new
// deviation sum is added to m2_sum), then the frame value minus the average
// is scaled by inv_s.  Returns the pre-processed value.
__device__ __forceinline__ float pre_entry(const FrameArgs& a, long long e, float x, bool upd, float inv_n,
                                           float inv_s, float& m2_sum) {
  float mean = a.pre_mean[e];
  if (upd) {
    const float d = x - mean;
    mean = fmaf(d, inv_n, mean);
    m2_sum += fmaf(d, x - mean, a.pre_m2[e]);
  }
  return (x - mean) * inv_s;
}

// Store the running average and deviation sum of one entry after an
// accepted initialization frame (same arithmetic as pre_entry).
__device__ __forceinline__ void pre_store(const FrameArgs& a, long long e, float x, float inv_n) {
  const float mean = a.pre_mean[e];
  const float d = x - mean;
  const float mn = fmaf(d, inv_n, mean);
  a.pre_m2[e] = fmaf(d, x - mn, a.pre_m2[e]);
  a.pre_mean[e] = mn;
}

// PR+ conjugate direction from the reduced gradient and cost in ks.red
// (Sec. 3.3, Step 1): wave 0, lane j owns component j.  Sets ks.d / df / gp,
// ks.gd and the stop flag ks.flag[0]; a non-finite first cost marks the frame
// bad (ks.flag[1]).
template <int K>
__device__ __forceinline__ void cg_direction(const FrameArgs& a, KSpace<kMaxK>& ks, int it, bool lead,
                                             int& restarts) {
  const int tid = thread_index(), lane = tid & 63;
  if (tid < 64) {
    const double g = (lane < K) ? -ks.red[lane] : 0.0;
    const double f = ks.red[K];
    const double gg = row16_sum(g * g);
    int stop = 0;
    if (it == 0 && !(isfinite(f) && isfinite(gg))) {
      stop = 1;
      if (lane == 0) ks.flag[1] = 1;
    }
    if (gg == 0.0) stop = 1;
    if (lead && lane == 0) a.stats->f[it] = f;
    double beta = 0.0, dj = -g;
    if (!stop && it > 0 && a.ysolve == 0) {
      const double gp = (lane < K) ? ks.gp[lane] : 0.0;
      const double num = row16_sum(g * (g - gp));
      const double den = row16_sum(gp * gp);
      beta = fmax(0.0, num / den);
      const double dpv = (lane < K) ? ks.dp[lane] : 0.0;
      dj = -g + beta * dpv;
      const double gdv = row16_sum(g * dj);
      if (gdv >= 0.0) {
        dj = -g;
        if (lane == 0) ++restarts;
      }
    }
    const double gd = row16_sum(g * dj);
    if (lane < K) {
      ks.d[lane] = dj;
      ks.df[lane] = (float)dj;
      ks.gp[lane] = g;
    }
    if (lane == 0) {
      ks.gd = gd;
      ks.flag[0] = stop;
      if (lead) a.stats->beta[it] = beta;
    }
  }
  __syncthreads();
}

// ---- steps with H reduced alongside the gradient (one wide exchange per step) ----

// Upper-triangle pair p -> (row, column) of a K x K matrix, row-major.
__host__ __device__ constexpr int tri_row(int p, int K) {
  int i = 0;
  while (p >= K - i) { p -= K - i; ++i; }
  return i;
}
__host__ __device__ constexpr int tri_col(int p, int K) {
  int i = 0;
  while (p >= K - i) { p -= K - i; ++i; }
  return i + p;
}

template <int K, int P>
struct TriPair {   // compile-time (row, column) of upper-triangle pair P
  static constexpr int i = tri_row(P, K);
  static constexpr int j = tri_col(P, K);
};

// One register row's contribution to chunk C (pairs C*32 .. C*32+31) of H.
template <int K, int C, typename UF, int... Q>
__device__ __forceinline__ void irls_h_row(float (&h)[kSlot], float wci, int row, UF uval,
                                           std::integer_sequence<int, Q...>) {
  constexpr int NP = K * (K + 1) / 2;
  ((C * kSlot + Q < NP
        ? (void)(h[Q] = fmaf(wci * uval(row, TriPair<K, (C * kSlot + Q < NP ? C * kSlot + Q : 0)>::i),
                             uval(row, TriPair<K, (C * kSlot + Q < NP ? C * kSlot + Q : 0)>::j), h[Q]))
        : (void)0),
   ...);
}

template <int K, int ROWS, int C, typename UF, typename PF>
__device__ __forceinline__ void irls_h_chunk(const float (&wc)[ROWS], UF uval, PF pin, FrameSmem& sm) {
  float h[kSlot];
#pragma unroll
  for (int q = 0; q < kSlot; ++q) h[q] = 0.f;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    pin();
    irls_h_row<K, C>(h, wc[i], i, uval, std::make_integer_sequence<int, kSlot>{});
  }
  wg_reduce<kSlot>(h, sm.red, sm.wide_in + K + 1 + C * kSlot);
}

template <int K, int ROWS, typename UF, typename PF, int... C>
__device__ __forceinline__ void irls_h_chunks(const float (&wc)[ROWS], UF uval, PF pin, FrameSmem& sm,
                                              std::integer_sequence<int, C...>) {
  (irls_h_chunk<K, ROWS, C>(wc, uval, pin, sm), ...);
}

// This workgroup's partial sums of H = U^T diag(w c) U (upper triangle),
// 32 entries at a time, into sm.wide_in[K + 1 ...].  uval(i, j): entry j of
// the thread's register row i (j a compile-time constant); wc[i] = w c(r)
// of that row; pin() is called before each row (keeps widened copies of a
// packed tile from being held across rows).
template <int K, int ROWS, typename UF, typename PF>
__device__ __forceinline__ void irls_h_partials(const float (&wc)[ROWS], UF uval, PF pin, FrameSmem& sm) {
  constexpr int NP = K * (K + 1) / 2;
  irls_h_chunks<K, ROWS>(wc, uval, pin, sm, std::make_integer_sequence<int, (NP + kSlot - 1) / kSlot>{});
}

// Solve H d = -g from the gang totals (g, f, H in sm.wide_out) by Gaussian
// elimination without pivoting (H is symmetric positive definite for a
// non-degenerate frame) on the augmented matrix in LDS, all threads, fixed
// order.  Sets ks.d / df, ks.gd, the stop flag (zero gradient or H not
// positive definite) and, in the first step, the bad-frame flag.
template <int K>
__device__ __forceinline__ void irls_direction(const FrameArgs& a, FrameSmem& sm, int it, bool lead) {
  KSpace<kMaxK>& ks = sm.ks;
  const double* tot = sm.wide_out;
  const int tid = thread_index(), lane = tid & 63;
  for (int q = tid; q < K * (K + 1); q += kBlock) {
    const int i = q / (K + 1), j = q - i * (K + 1);
    double v;
    if (j == K) {
      v = tot[i];                     // -g = U^T (w phi'(r))
    } else {
      const int lo = min(i, j), hi = max(i, j);
      v = tot[K + 1 + lo * K - lo * (lo - 1) / 2 + (hi - lo)];
    }
    sm.hs[i][j] = v;
  }
  if (tid == 0) ks.flag[3] = 0;
  __syncthreads();
  if (tid < 64) {
    const double g = (lane < K) ? -tot[lane] : 0.0;
    const double gg = row16_sum(g * g);
    const double f = tot[K];
    int stop = (gg == 0.0) ? 1 : 0;
    if (it == 0 && !(isfinite(f) && isfinite(gg))) {
      stop = 1;
      if (lane == 0) ks.flag[1] = 1;
    }
    if (lead && lane == 0) {
      a.stats->f[it] = f;
      a.stats->beta[it] = 0.0;
    }
    if (lane == 0) ks.flag[3] = stop;
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {          // elimination, rows below k
    const double piv = sm.hs[k][k];
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (tid == 0) ks.flag[3] = 1;      // not positive definite: no step
      break;                             // uniform: every thread reads the same pivot
    }
    const double inv = 1.0 / piv;
    const int w = K - k - 1;
    for (int q = tid; q < w * (w + 1); q += kBlock) {
      const int i = k + 1 + q / (w + 1), j = k + 1 + q % (w + 1);
      sm.hs[i][j] -= sm.hs[i][k] * inv * sm.hs[k][j];
    }
    __syncthreads();
  }
  __syncthreads();
  const bool ok = ks.flag[3] == 0;
  if (ok)
    for (int k = K - 1; k >= 0; --k) {   // back substitution, d_k in place of the right-hand side
      if (tid == 0) sm.hs[k][K] = sm.hs[k][K] / sm.hs[k][k];
      __syncthreads();
      const double dk = sm.hs[k][K];
      for (int i = tid; i < k; i += kBlock) sm.hs[i][K] -= sm.hs[i][k] * dk;
      __syncthreads();
    }
  if (tid < 64) {
    const double g = (lane < K) ? -tot[lane] : 0.0;
    const double dj = (ok && lane < K) ? sm.hs[lane][K] : 0.0;
    const double gd = row16_sum(g * dj);
    if (lane < K) {
      ks.d[lane] = dj;
      ks.df[lane] = (float)dj;
    }
    if (lane == 0) {
      ks.gd = gd;
      ks.flag[0] = ok ? 0 : 1;
    }
  }
  __syncthreads();
}

// y += d (unit step of the IRLS iteration).
template <int K>
__device__ __forceinline__ void irls_advance(const FrameArgs& a, KSpace<kMaxK>& ks, int it, bool lead) {
  const int tid = thread_index();
  if (tid < K) {
    ks.y[tid] += ks.d[tid];
    ks.dp[tid] = ks.d[tid];
  }
  if (lead && tid == 0) a.stats->alpha[it] = 1.0;
}

// CG step of the one-exchange curvature schedule: g and f come from the wide
// totals in sm.wide_out (with the upper triangle of H = U^T diag(w c) U);
// the direction is the one cg_direction forms, and d^T H d is summed from
// the reduced H in a fixed order (lane i: row i of H times d, then the
// 16-lane sum), into ks.red[K + 1].  Same value, up to rounding, as the
// second pass sum_e w c (u_e . d)^2.
template <int K>
__device__ __forceinline__ void wide_cg_direction(const FrameArgs& a, FrameSmem& sm, int it, bool lead,
                                                  int& restarts) {
  KSpace<kMaxK>& ks = sm.ks;
  const double* tot = sm.wide_out;
  const int tid = thread_index(), lane = tid & 63;
  if (tid <= K) ks.red[tid] = tot[tid];
  __syncthreads();
  cg_direction<K>(a, ks, it, lead, restarts);
  if (tid < 64) {
    double t = 0.0;
    if (lane < K) {
      for (int j = 0; j < K; ++j) {
        const int lo = min(lane, j), hi = max(lane, j);
        t = fma(tot[K + 1 + lo * K - lo * (lo - 1) / 2 + (hi - lo)], ks.d[j], t);
      }
      t *= ks.d[lane];
    }
    const double dhd = row16_sum(t);
    if (lane == 0) ks.red[K + 1] = dhd;
  }
  __syncthreads();
}

// Majoriser step along d: alpha = -g.d / d^T H d, y += alpha d.  Returns
// alpha as float for the residual update.
template <int K>
__device__ __forceinline__ float cg_advance(const FrameArgs& a, KSpace<kMaxK>& ks, double dHd, int it, bool lead) {
  const int tid = thread_index();
  const double alpha = -ks.gd / dHd;
  __syncthreads();
  if (tid < K) {
    ks.y[tid] += alpha * ks.d[tid];
    ks.dp[tid] = ks.d[tid];
  }
  if (lead && tid == 0) a.stats->alpha[it] = alpha;
  return (float)alpha;
}

// Step size and angle of the geodesic step and the trigonometric scalars of
// the row pass: t = max(exp(-tau n) t_init, t_min) (Sec. 3.4),
// theta = sigma t, cos(theta) - 1 = -2 sin^2(theta / 2),
// sin(theta) / zeta = 2 sin(theta / 2) cos(theta / 2) / zeta.
// Out of line on purpose: inlined into the persistent kernels, the float64
// polynomial constants of exp and sin were hoisted out of the tile loop and
// held in registers (and spilled) for the whole launch.
struct GeoScalars {
  double t, theta, cm1, sz;
};
__device__ __attribute__((noinline)) GeoScalars geodesic_scalars(double tau_n, double t_init, double t_min,
                                                                 double sigma, double zeta) {
  GeoScalars g;
  g.t = fmax(exp(-tau_n) * t_init, t_min);
  g.theta = sigma * g.t;
  double sh, ch;   // sin and cos of theta / 2 from one range reduction; sin(theta) = 2 sh ch
  sincos(0.5 * g.theta, &sh, &ch);
  g.cm1 = -2.0 * sh * sh;
  g.sz = zeta > 0.0 ? 2.0 * sh * ch / zeta : 0.0;
  return g;
}

// Scalars of the rank-one geodesic step (Sec. 3.3, Step 2) from the reduced
// a = U^T eta, ||eta||^2 and the final cost in ks.red: zeta = ||pi(eta)||,
// nu = ||y||, sigma = zeta nu, theta = sigma t_n; row-pass coefficients in
// ks.scal / vf / af.
template <int K>
__device__ __forceinline__ void geodesic_setup(const FrameArgs& a, KSpace<kMaxK>& ks, long long n, int steps,
                                               bool lead) {
  const int tid = thread_index(), lane = tid & 63;
  if (tid < 64) {
    const double av = (lane < K) ? ks.red[lane] : 0.0;
    const double yv = (lane < K) ? ks.y[lane] : 0.0;
    const double aa = row16_sum(av * av);
    const double yy = row16_sum(yv * yv);
    const double ee = ks.red[K];
    const double zeta = sqrt(fmax(ee - aa, 0.0));
    const double nu = sqrt(yy);
    const double sigma = zeta * nu;
    const int upd = (zeta > 0.0 && nu > 0.0) ? 1 : 0;
    if (lane < K) {
      ks.af[lane] = (float)av;
      ks.vf[lane] = upd ? (float)(yv / nu) : 0.f;
      ks.yf[lane] = (float)yv;
    }
    if (lane == 0) {
      const GeoScalars g = geodesic_scalars(a.tau * (double)n, a.t_init, a.t_min, sigma, zeta);
      ks.scal[0] = upd ? (float)g.cm1 : 0.f;   // cos(theta) - 1
      ks.scal[1] = upd ? (float)g.sz : 0.f;    // sin(theta) / zeta
      ks.scal[2] = (float)nu;
      ks.flag[2] = upd;
      if (lead) {
        a.stats->f[steps] = ks.red[K + 1];
        a.stats->t = g.t;
        a.stats->sigma = sigma;
        a.stats->theta = g.theta;
        a.stats->zeta = zeta;
        a.stats->nu = nu;
        a.stats->updated = upd;
      }
    }
  }
  __syncthreads();
}

// Start of frame i > 0 of a sequence launch: y and the frame index carry
// over in the workgroup (identical in every workgroup of the gang).  The
// finished frame's labels went out with device-coherent stores; every thread
// waits for its stores to complete before any partial of the next frame is
// published, so that the mask of the finished frame (its 3x3 median reads
// neighbouring tiles' labels) can be formed after the next frame's first
// exchange (sequence_median), which no workgroup completes before all have
// published.  (A device-scope release / acquire fence pair would also
// write back and invalidate the L2: measured 3x slower.)
__device__ __forceinline__ void next_frame_begin(KSpace<kMaxK>& ks, TileCtx& t, bool bad) {
  if (!bad) ++t.n;
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this thread's stores have completed
  __syncthreads();   // everyone is past the previous frame's use of ks.flag and s_flag
  if (thread_index() < 4) ks.flag[thread_index()] = 0;
  __syncthreads();
}

// The deferred median of a sequence frame: the previous frame's labels of
// the whole gang are complete once this frame's first exchange is, and no
// workgroup writes this frame's labels before the last exchange.
__device__ __forceinline__ void sequence_median(const FrameArgs& a, const TileCtx& t) {
  median3x3_range<true>(a.lab, a.mask, a.W, a.H, t.p0, t.npx);
}

// Label of tile pixel pl from the per-entry flags of the last labelled frame.
__device__ __forceinline__ bool pixel_label(const uint8_t* s_flag, int C, int npx, int pl) {
  uint8_t f = 0;
  for (int c = 0; c < C; ++c) f |= s_flag[c * npx + pl];
  return f != 0;
}

// Pixel labels (Sec. 3.3, Step 3): foreground when any colour entry was
// flagged in s_flag (entry q = c * npx + pixel).  COH: device-coherent
// stores (read by other workgroups in the same launch).
template <bool COH = false>
__device__ __forceinline__ void write_labels(const FrameArgs& a, const uint8_t* s_flag, int p0, int npx) {
  __syncthreads();
  for (int pl = thread_index(); pl < npx; pl += kBlock) {
    uint8_t f = 0;
    for (int c = 0; c < a.C; ++c) f |= s_flag[c * npx + pl];
    if (COH)
      __hip_atomic_store(&a.lab[p0 + pl], f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      a.lab[p0 + pl] = f;
  }
}

// Statistics, frame counter, y and the exchange bases for the next launch.
__device__ __forceinline__ void tile_end(const FrameArgs& a, const int tile, KSpace<kMaxK>& ks, const TileCtx& t,
                                         int steps, int restarts, bool bad, int nbar) {
  const int tid = thread_index();
  trace_point(a, tile, 63);
  if (t.lead && tid == 0) {
    a.stats->frame = t.n;
    a.stats->cg_steps = steps;
    a.stats->restarts = restarts;
    a.stats->bad_frame = bad ? 1 : 0;
    if (bad) {
      __hip_atomic_fetch_or(&a.sync[2], kErrBadFrame, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      *a.nframe = t.n + 1;
      if (ks.pre_upd) {
        a.pre_stat[0] = ks.pre_sum;
        a.pre_stat[1] = a.pre_stat[1] + 1.0;
      }
    }
    if (a.G == 1) {
      // a one-workgroup gang used no slots or counters: the bases stay
    } else if (a.sync_mode != 0)
      __hip_atomic_store(&a.sync[3], t.ebase + (unsigned)nbar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_store(&a.sync[1], t.base + (unsigned)a.G * (unsigned)nbar, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  if (t.lead && !bad && tid < a.k) a.y[tid] = ks.y[tid];
  __syncthreads();   // shared scratch may be reused by the next tile
}

// ---------------------------------------------------------------------------
// float32 storage: row q = tid + s * kBlock of the tile, K floats per row
// ---------------------------------------------------------------------------
template <int K, int NR, bool EXT, bool WIDE, bool SEQ>
__device__ __forceinline__ bool frame_tile(const FrameArgs& a, const int tile, FrameSmem& sm) {
  KSpace<kMaxK>& ks = sm.ks;
  uint8_t* s_flag = sm.flag;
  int tid = thread_index();
  TileCtx ctx = tile_begin<K>(a, tile, ks);
  int nbar = 0;

  // ---- load the register tile: U rows, residual r = x - U y, weights ----
  const float* __restrict__ Ug = (const float*)a.U;
  const float* __restrict__ xg = (const float*)(a.xtab ? a.xtab[ctx.n % a.ring] : a.x);
  const uint8_t* __restrict__ wsrc = a.weights_from_filtered ? a.mask : a.lab;
  float u[NR][K];
  float r[NR], wt[NR], cw[NR];
  int eix[NR];
  bool u_pending = false;   // sequence: the registers hold an update not yet stored
  auto store_tile = [&]() {  // sequence: the register tile to the U planes
    float* __restrict__ Uw = (float*)a.U;
#pragma unroll
    for (int s = 0; s < NR; ++s)
      if (eix[s] >= 0) {
#pragma unroll
        for (int j = 0; j < K; ++j)
          if (j < a.k) Uw[(long long)j * a.ldU + eix[s]] = u[s][j];
      }
  };
  const bool pre = EXT && a.pre_mean != nullptr;   // compiled out without EXT
  const bool pupd = EXT && ks.pre_upd != 0;
  const float pinv_n = ks.pre_inv_n, pinv_s = ks.pre_inv_s;
  float m2sum = 0.f;
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int q = tid + s * kBlock;
    eix[s] = -1;
    wt[s] = 0.f;
    r[s] = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j) u[s][j] = 0.f;
    if (q < ctx.nq) {
      const int c = q / ctx.npx;
      const int pl = q - c * ctx.npx;
      const int e = c * a.P + ctx.p0 + pl;
      eix[s] = e;
      wt[s] = wsrc[ctx.p0 + pl] ? a.omega : 1.0f;
      float acc = xg[e];
      if (pre) acc = pre_entry(a, e, acc, pupd, pinv_n, pinv_s, m2sum);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j < a.k) u[s][j] = Ug[(long long)j * a.ldU + e];   // columns >= k stay 0
        acc = fmaf(-u[s][j], ks.yf[j], acc);
      }
      r[s] = acc;
    }
  }

  for (int fi = 0;;) {   // frames of this launch; U stays in the registers between them
  if constexpr (SEQ) {
    // Per-row indices re-enter opaquely each frame: otherwise every address
    // derived from them is hoisted out of the frame loop and held in registers.
    tid = thread_index();
#pragma unroll
    for (int s = 0; s < NR; ++s) asm volatile("" : "+v"(eix[s]));
  }
  // ---- Step 1: CG on y ----
  int steps = 0, restarts = 0;
  for (int it = 0; it < a.J; ++it) {
    // phase A: gradient and cost at the current y
    float acc[K + 1];   // g, f
#pragma unroll
    for (int j = 0; j <= K; ++j) acc[j] = 0.f;
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      float phi, c;
      cost_eval(r[s], a.cp, phi, c);
      const float wc = wt[s] * c;
      cw[s] = wc;
      const float wd = wc * r[s];          // w phi'(r)
      acc[K] = fmaf(wt[s], phi, acc[K]);
#pragma unroll
      for (int j = 0; j < K; ++j) acc[j] = fmaf(wd, u[s][j], acc[j]);
    }
    if (WIDE && (a.ysolve == 2 || a.curv == 1)) {   // g, f and H in one (wide) exchange
      wg_reduce<K + 1>(acc, sm.red, sm.wide_in);
      irls_h_partials<K, NR>(cw, [&](int i, int j) { return u[i][j]; }, [] {}, sm);
      if (!gang_reduce_wide(sm.wide_in, K + 1 + K * (K + 1) / 2, a, tile, nbar, ctx.ebase, sm.big, sm.wide_out))
        return false;
      float af = 1.0f;
      if (a.ysolve == 2) {   // IRLS: unit step along -H^{-1} g
        irls_direction<K>(a, sm, it, ctx.lead);
        if (ks.flag[0]) break;
        irls_advance<K>(a, ks, it, ctx.lead);
      } else {               // CG / gradient descent with d^T H d from the reduced H
        wide_cg_direction<K>(a, sm, it, ctx.lead, restarts);
        if (ks.flag[0]) break;
        const double dHd = ks.red[K + 1];
        if (!(dHd > 0.0)) break;
        af = cg_advance<K>(a, ks, dHd, it, ctx.lead);
      }
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) t = fmaf(u[s][j], ks.df[j], t);
        r[s] = fmaf(-af, t, r[s]);
      }
      ++steps;
      __syncthreads();
      continue;
    }
    if (!gang_reduce<K + 1>(acc, a, tile, nbar, ctx.base, ctx.ebase, sm, ks.red)) return false;
    if (SEQ && fi > 0 && it == 0) sequence_median(a, ctx);
    cg_direction<K>(a, ks, it, ctx.lead, restarts);
    if (ks.flag[0]) break;
    // phase B: curvature of the majoriser along d; cw then holds u.d
    float accb[1] = {0.f};
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      float t = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j) t = fmaf(u[s][j], ks.df[j], t);
      accb[0] = fmaf(cw[s] * t, t, accb[0]);
      cw[s] = t;
    }
    if (!gang_reduce<1>(accb, a, tile, nbar, ctx.base, ctx.ebase, sm, ks.red)) return false;
    const double dHd = ks.red[0];
    if (!(dHd > 0.0)) break;   // same decision in every workgroup
    const float af = cg_advance<K>(a, ks, dHd, it, ctx.lead);
#pragma unroll
    for (int s = 0; s < NR; ++s) r[s] = fmaf(-af, cw[s], r[s]);
    ++steps;
    __syncthreads();
  }
  const bool bad = ks.flag[1] != 0;

  if (!bad) {
    // ---- Step 2: eta pass (a = U^T eta, ||eta||^2, final cost) ----
    constexpr int LE = K + 2 + (EXT ? 1 : 0);   // a, ||eta||^2, f (+ pre-processing deviation sum)
    float acce[LE];
#pragma unroll
    for (int j = 0; j < LE; ++j) acce[j] = 0.f;
    if constexpr (EXT) acce[LE - 1] = pupd ? m2sum : 0.f;
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      float phi, c;
      cost_eval(r[s], a.cp, phi, c);
      const float eta = -wt[s] * c * r[s];
      cw[s] = eta;
      acce[K] = fmaf(eta, eta, acce[K]);
      acce[K + 1] = fmaf(wt[s], phi, acce[K + 1]);
#pragma unroll
      for (int j = 0; j < K; ++j) acce[j] = fmaf(eta, u[s][j], acce[j]);
    }
    if (!gang_reduce<LE>(acce, a, tile, nbar, ctx.base, ctx.ebase, sm, ks.red)) return false;
    if (EXT && tid == 0 && pupd) ks.pre_sum = ks.red[K + 2];
    geodesic_setup<K>(a, ks, ctx.n, steps, ctx.lead);
    trace_point(a, tile, 60);

    // ---- Step 2 update + Step 3 labels, one pass over the register tile ----
    float* __restrict__ Uw = (float*)a.U;
    const float cm1 = ks.scal[0], sz = ks.scal[1], nu_f = ks.scal[2];
    const bool upd = ks.flag[2] != 0;
    // a sequence keeps U in the registers (the next frame starts from them)
    // and stores it after its last frame only, in a loop of its own, so the
    // update of the other frames carries no per-entry store decisions
    const bool store_u = !SEQ || fi + 1 >= a.nseq;
    if (SEQ && upd) u_pending = !store_u;
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      const int q = tid + s * kBlock;
      if (eix[s] >= 0) {
        float rl = r[s];
        if (upd) {
          float uv = 0.f, ua = 0.f;
#pragma unroll
          for (int j = 0; j < K; ++j) {
            uv = fmaf(u[s][j], ks.vf[j], uv);
            ua = fmaf(u[s][j], ks.af[j], ua);
          }
          const float coef = fmaf(cm1, uv, -sz * (cw[s] - ua));
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const float nv = fmaf(coef, ks.vf[j], u[s][j]);   // columns >= k stay 0 (v_j = 0)
            if constexpr (SEQ) u[s][j] = nv;
            else if (j < a.k) Uw[(long long)j * a.ldU + eix[s]] = nv;
          }
          if (a.labels_after_update) rl = fmaf(-coef, nu_f, rl);
        }
        if (pre && pupd) pre_store(a, eix[s], xg[eix[s]], pinv_n);
        if (EXT && a.score) a.score[eix[s]] = fabsf(rl);
        s_flag[q] = (fabsf(rl) >= a.delta) ? 1 : 0;
      }
    }
    if (SEQ && upd && store_u) store_tile();
    trace_point(a, tile, 61);
    write_labels<SEQ>(a, s_flag, ctx.p0, ctx.npx);
    trace_point(a, tile, 62);
  }
  tile_end(a, tile, ks, ctx, steps, restarts, bad, nbar);
  if (!SEQ || ++fi >= a.nseq) break;

  // ---- next frame of a sequence: weights from this frame's labels (still in
  // s_flag; unchanged after a rejected frame), residuals of the next frame ----
  next_frame_begin(ks, ctx, bad);
  xg = (const float*)(a.xtab ? a.xtab[ctx.n % a.ring] : a.seq[fi]);
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    if (eix[s] < 0) continue;
    const int q = tid + s * kBlock;
    const int pl = q - (q / ctx.npx) * ctx.npx;
    if (!bad) wt[s] = pixel_label(s_flag, a.C, ctx.npx, pl) ? a.omega : 1.0f;
    float acc = xg[eix[s]];
#pragma unroll
    for (int j = 0; j < K; ++j) acc = fmaf(-u[s][j], ks.yf[j], acc);
    r[s] = acc;
  }
  }
  // the last frame stored nothing (rejected, or no step): store the updated tile
  if (SEQ && u_pending) store_tile();
  return true;
}

// ---------------------------------------------------------------------------
// bfloat16 storage: the register tile keeps U in bfloat16, two rows per
// 32-bit register (row 2i in the low half, row 2i + 1 in the high half), so a
// tile holds twice the rows of the float32 layout in the same registers.
// Values are widened to float32 (exact) where they are used; the update is
// computed in float32 and rounded to nearest-even once, as it is stored.
// Row pair s of thread tid covers rows q0 = 2 (tid + s kBlock) and q0 + 1.
// When a.pair_aligned is set (even P, even tpw, 4-byte aligned frame) a pair
// is one aligned 32-bit word in the U planes and in the frame; otherwise the
// two halves are accessed separately and may lie in two colour planes.
// NL > 0 (batched form): pairs NP .. NP + NL - 1 of every thread are held in
// LDS instead (lt[((s - NP) K + j) kBlock + tid], their residuals after the
// NL K kBlock words, each thread its own words: no barriers), processed by a
// loop that is not unrolled; results are identical.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
__device__ __forceinline__ float bf_half(uint32_t w, int h) { return h ? bf_hi(w) : bf_lo(w); }

// Two float32 values rounded to nearest-even bfloat16 and packed (lo, hi):
// one v_cvt_pk_bf16_f32 on gfx950.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16_rne(float lo, float hi) {
  const f32x2_t v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// Marks the packed tile as redefined at the start of every row pass, so the
// compiler cannot hoist widened float32 copies of U out of the CG loop
// (which would double the registers the tile needs).  No instructions.
template <int NP, int K>
__device__ __forceinline__ void pin_tile(uint32_t (&u)[NP][K]) {
#pragma unroll
  for (int s = 0; s < NP; ++s)
#pragma unroll
    for (int j = 0; j < K; ++j) asm volatile("" : "+v"(u[s][j]));
}

// 32- and 16-bit accesses at a byte offset (32-bit) from a base pointer.
__device__ __forceinline__ uint32_t ld_u32(const uint16_t* base, unsigned boff) {
  return *(const uint32_t*)((const char*)base + boff);
}
__device__ __forceinline__ uint32_t ld_u16(const uint16_t* base, unsigned boff) {
  return *(const uint16_t*)((const char*)base + boff);
}
__device__ __forceinline__ void st_u32(uint16_t* base, unsigned boff, uint32_t v) {
  *(uint32_t*)((char*)base + boff) = v;
}
__device__ __forceinline__ void st_u16(uint16_t* base, unsigned boff, uint16_t v) {
  *(uint16_t*)((char*)base + boff) = v;
}

template <int K, int NP, bool EXT, int NL = 0, bool SEQ = false>
__device__ __forceinline__ bool frame_tile_packed(const FrameArgs& a, const int tile, FrameSmem& sm,
                                                  uint32_t* __restrict__ lt = nullptr) {
  constexpr int NT = NP + NL;   // row pairs per thread: NP in registers, NL in LDS
  static_assert(2 * NT <= kMaxNR && NT <= 16, "row bit masks hold 32 rows");
  static_assert(NL == 0 || !EXT, "the LDS pairs serve the default features only");
  KSpace<kMaxK>& ks = sm.ks;
  uint8_t* s_flag = sm.flag;
  int tid = thread_index();
  TileCtx ctx = tile_begin<K>(a, tile, ks);
  int nbar = 0;
  const bool al = a.pair_aligned != 0;

  // ---- load the register tile ----
  const uint16_t* __restrict__ Ug = (const uint16_t*)a.U;
  const uint16_t* __restrict__ xg = (const uint16_t*)(a.xtab ? a.xtab[ctx.n % a.ring] : a.x);
  const uint8_t* __restrict__ wsrc = a.weights_from_filtered ? a.mask : a.lab;
  uint32_t u[NP][K];
  // cw: w c in phase A, u.d in phase B, eta in the update (register rows);
  // the LDS rows keep r in LDS and recompute these where needed (the same
  // operations on the same values, so the same results)
  float r[2 * NP], cw[2 * NP];
  float* __restrict__ lr = NL > 0 ? (float*)(lt + NL * K * kBlock) : nullptr;   // r of the LDS rows
  uint32_t vbits = 0;         // bit i: row i exists
  uint32_t fbits = 0;         // bit i: row i's pixel was foreground (weight omega)
  uint32_t sbits = 0;         // bit s: pair s continues in the next colour plane
  const bool pre = EXT && a.pre_mean != nullptr;   // compiled out without EXT
  const bool pupd = EXT && ks.pre_upd != 0;
  const float pinv_n = ks.pre_inv_n, pinv_s = ks.pre_inv_s;
  float m2sum = 0.f;
#pragma unroll
  for (int s = 0; s < NP; ++s) {
    const int q0 = 2 * (tid + s * kBlock);
    r[2 * s] = r[2 * s + 1] = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j) u[s][j] = 0u;
    if (q0 < ctx.nq) {
      const int c = q0 / ctx.npx;
      const int pl = q0 - c * ctx.npx;
      const int e = c * a.P + ctx.p0 + pl;
      const bool has1 = q0 + 1 < ctx.nq;
      const bool split = (pl + 1 == ctx.npx);
      const int e1 = split ? e + 1 + (a.P - ctx.npx) : e + 1;
      vbits |= (has1 ? 3u : 1u) << (2 * s);
      if (split) sbits |= 1u << s;
      if (wsrc[ctx.p0 + pl]) fbits |= 1u << (2 * s);
      if (has1 && wsrc[ctx.p0 + (split ? 0 : pl + 1)]) fbits |= 2u << (2 * s);
      // byte offsets in 32 bits from uniform plane bases: the addresses are a
      // scalar base plus one vector offset, not 64-bit vector arithmetic
      const unsigned b0 = 2u * (unsigned)e, b1 = 2u * (unsigned)e1;
      uint32_t xw;
      if (al) xw = ld_u32(xg, b0);
      else xw = ld_u16(xg, b0) | (has1 ? (ld_u16(xg, b1) << 16) : 0u);
      float acc0 = bf_lo(xw), acc1 = bf_hi(xw);
      if (pre) {
        acc0 = pre_entry(a, e, acc0, pupd, pinv_n, pinv_s, m2sum);
        if (has1) acc1 = pre_entry(a, e1, acc1, pupd, pinv_n, pinv_s, m2sum);
      }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j < a.k) {
          const uint16_t* col = Ug + (long long)j * a.ldU;
          u[s][j] = al ? ld_u32(col, b0) : (ld_u16(col, b0) | (has1 ? (ld_u16(col, b1) << 16) : 0u));
        }
        acc0 = fmaf(-bf_lo(u[s][j]), ks.yf[j], acc0);
        acc1 = fmaf(-bf_hi(u[s][j]), ks.yf[j], acc1);
      }
      r[2 * s] = acc0;
      r[2 * s + 1] = has1 ? acc1 : 0.f;
    }
  }
#pragma unroll 1
  for (int s = NP; s < NT; ++s) {   // pairs held in LDS: the same load
    const int q0 = 2 * (tid + s * kBlock);
    uint32_t* lts = lt + (s - NP) * K * kBlock + tid;
    float* rls = lr + (s - NP) * 2 * kBlock + tid;
    rls[0] = rls[kBlock] = 0.f;
    if (q0 < ctx.nq) {
      const int c = q0 / ctx.npx;
      const int pl = q0 - c * ctx.npx;
      const int e = c * a.P + ctx.p0 + pl;
      const bool has1 = q0 + 1 < ctx.nq;
      const bool split = (pl + 1 == ctx.npx);
      const int e1 = split ? e + 1 + (a.P - ctx.npx) : e + 1;
      vbits |= (has1 ? 3u : 1u) << (2 * s);
      if (split) sbits |= 1u << s;
      if (wsrc[ctx.p0 + pl]) fbits |= 1u << (2 * s);
      if (has1 && wsrc[ctx.p0 + (split ? 0 : pl + 1)]) fbits |= 2u << (2 * s);
      const unsigned b0 = 2u * (unsigned)e, b1 = 2u * (unsigned)e1;
      uint32_t xw;
      if (al) xw = ld_u32(xg, b0);
      else xw = ld_u16(xg, b0) | (has1 ? (ld_u16(xg, b1) << 16) : 0u);
      float acc0 = bf_lo(xw), acc1 = bf_hi(xw);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        uint32_t v = 0u;
        if (j < a.k) {
          const uint16_t* col = Ug + (long long)j * a.ldU;
          v = al ? ld_u32(col, b0) : (ld_u16(col, b0) | (has1 ? (ld_u16(col, b1) << 16) : 0u));
        }
        lts[j * kBlock] = v;
        acc0 = fmaf(-bf_lo(v), ks.yf[j], acc0);
        acc1 = fmaf(-bf_hi(v), ks.yf[j], acc1);
      }
      rls[0] = acc0;
      rls[kBlock] = has1 ? acc1 : 0.f;
    } else {
#pragma unroll
      for (int j = 0; j < K; ++j) lts[j * kBlock] = 0u;
    }
  }
  const float om = a.omega;
  auto weight = [&](int i) -> float {
    return ((vbits >> i) & 1u) ? (((fbits >> i) & 1u) ? om : 1.0f) : 0.f;
  };
  static_assert(!(SEQ && NL > 0), "sequences keep register tiles only");
  bool u_pending = false;   // sequence: the registers hold an update not yet stored
  auto store_tile = [&]() {  // sequence: the register tile to the U planes
    uint16_t* __restrict__ Uw = (uint16_t*)a.U;
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int q0 = 2 * (tid + s * kBlock);
      if (q0 >= ctx.nq) continue;
      const bool has1 = (vbits >> (2 * s + 1)) & 1u;
      const int c = q0 / ctx.npx;
      const int e = c * a.P + ctx.p0 + (q0 - c * ctx.npx);
      const int e1 = ((sbits >> s) & 1u) ? e + 1 + (a.P - ctx.npx) : e + 1;
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (j < a.k) {
          uint16_t* col = Uw + (long long)j * a.ldU;
          if (al) {
            st_u32(col, 2u * (unsigned)e, u[s][j]);
          } else {
            st_u16(col, 2u * (unsigned)e, (uint16_t)(u[s][j] & 0xFFFFu));
            if (has1) st_u16(col, 2u * (unsigned)e1, (uint16_t)(u[s][j] >> 16));
          }
        }
    }
  };

  for (int fi = 0;;) {   // frames of this launch; U stays in the registers between them
  if constexpr (SEQ) tid = thread_index();   // re-enters opaquely each frame (see the float32 tile)
  // ---- Step 1: CG on y ----
  int steps = 0, restarts = 0;
  for (int it = 0; it < a.J; ++it) {
    float acc[K + 1];   // g, f
#pragma unroll
    for (int j = 0; j <= K; ++j) acc[j] = 0.f;
    pin_tile(u);
#pragma unroll
    for (int s = 0; s < NP; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 2 * s + h;
        const float wt = weight(i);
        float phi, c;
        cost_eval(r[i], a.cp, phi, c);
        const float wc = wt * c;
        cw[i] = wc;
        const float wd = wc * r[i];
        acc[K] = fmaf(wt, phi, acc[K]);
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] = fmaf(wd, bf_half(u[s][j], h), acc[j]);
      }
#pragma unroll 1
    for (int s = NP; s < NT; ++s) {   // LDS pairs: each word read once for both rows
      const uint32_t* lts = lt + (s - NP) * K * kBlock + tid;
      float* rls = lr + (s - NP) * 2 * kBlock + tid;
      float wd[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float ri = rls[h * kBlock];
        const float wt = weight(2 * s + h);
        float phi, c;
        cost_eval(ri, a.cp, phi, c);
        wd[h] = wt * c * ri;
        acc[K] = fmaf(wt, phi, acc[K]);
      }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t v = lts[j * kBlock];
        acc[j] = fmaf(wd[0], bf_lo(v), acc[j]);
        acc[j] = fmaf(wd[1], bf_hi(v), acc[j]);
      }
    }
    if (!gang_reduce<K + 1>(acc, a, tile, nbar, ctx.base, ctx.ebase, sm, ks.red)) return false;
    if (SEQ && fi > 0 && it == 0) sequence_median(a, ctx);
    cg_direction<K>(a, ks, it, ctx.lead, restarts);
    if (ks.flag[0]) break;
    float accb[1] = {0.f};
    pin_tile(u);
#pragma unroll
    for (int s = 0; s < NP; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 2 * s + h;
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) t = fmaf(bf_half(u[s][j], h), ks.df[j], t);
        accb[0] = fmaf(cw[i] * t, t, accb[0]);
        cw[i] = t;
      }
#pragma unroll 1
    for (int s = NP; s < NT; ++s) {
      const uint32_t* lts = lt + (s - NP) * K * kBlock + tid;
      float* rls = lr + (s - NP) * 2 * kBlock + tid;
      float t0 = 0.f, t1 = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t v = lts[j * kBlock];
        t0 = fmaf(bf_lo(v), ks.df[j], t0);
        t1 = fmaf(bf_hi(v), ks.df[j], t1);
      }
      float wc[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float phi, c;
        cost_eval(rls[h * kBlock], a.cp, phi, c);
        wc[h] = weight(2 * s + h) * c;
      }
      accb[0] = fmaf(wc[0] * t0, t0, accb[0]);
      accb[0] = fmaf(wc[1] * t1, t1, accb[0]);
    }
    if (!gang_reduce<1>(accb, a, tile, nbar, ctx.base, ctx.ebase, sm, ks.red)) return false;
    const double dHd = ks.red[0];
    if (!(dHd > 0.0)) break;
    const float af = cg_advance<K>(a, ks, dHd, it, ctx.lead);
#pragma unroll
    for (int i = 0; i < 2 * NP; ++i) r[i] = fmaf(-af, cw[i], r[i]);
#pragma unroll 1
    for (int s = NP; s < NT; ++s) {   // u.d of the LDS rows again, as in phase B
      const uint32_t* lts = lt + (s - NP) * K * kBlock + tid;
      float* rls = lr + (s - NP) * 2 * kBlock + tid;
      float t0 = 0.f, t1 = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t v = lts[j * kBlock];
        t0 = fmaf(bf_lo(v), ks.df[j], t0);
        t1 = fmaf(bf_hi(v), ks.df[j], t1);
      }
      rls[0] = fmaf(-af, t0, rls[0]);
      rls[kBlock] = fmaf(-af, t1, rls[kBlock]);
    }
    ++steps;
    __syncthreads();
  }
  const bool bad = ks.flag[1] != 0;

  if (!bad) {
    constexpr int LE = K + 2 + (EXT ? 1 : 0);   // a, ||eta||^2, f (+ pre-processing deviation sum)
    float acce[LE];
#pragma unroll
    for (int j = 0; j < LE; ++j) acce[j] = 0.f;
    if constexpr (EXT) acce[LE - 1] = pupd ? m2sum : 0.f;
    pin_tile(u);
#pragma unroll
    for (int s = 0; s < NP; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 2 * s + h;
        const float wt = weight(i);
        float phi, c;
        cost_eval(r[i], a.cp, phi, c);
        const float eta = -wt * c * r[i];
        cw[i] = eta;
        acce[K] = fmaf(eta, eta, acce[K]);
        acce[K + 1] = fmaf(wt, phi, acce[K + 1]);
#pragma unroll
        for (int j = 0; j < K; ++j) acce[j] = fmaf(eta, bf_half(u[s][j], h), acce[j]);
      }
#pragma unroll 1
    for (int s = NP; s < NT; ++s) {
      const uint32_t* lts = lt + (s - NP) * K * kBlock + tid;
      float* rls = lr + (s - NP) * 2 * kBlock + tid;
      float et[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float ri = rls[h * kBlock];
        const float wt = weight(2 * s + h);
        float phi, c;
        cost_eval(ri, a.cp, phi, c);
        const float eta = -wt * c * ri;
        et[h] = eta;
        acce[K] = fmaf(eta, eta, acce[K]);
        acce[K + 1] = fmaf(wt, phi, acce[K + 1]);
      }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t v = lts[j * kBlock];
        acce[j] = fmaf(et[0], bf_lo(v), acce[j]);
        acce[j] = fmaf(et[1], bf_hi(v), acce[j]);
      }
    }
    if (!gang_reduce<LE>(acce, a, tile, nbar, ctx.base, ctx.ebase, sm, ks.red)) return false;
    if (EXT && tid == 0 && pupd) ks.pre_sum = ks.red[K + 2];
    geodesic_setup<K>(a, ks, ctx.n, steps, ctx.lead);
    trace_point(a, tile, 60);

    uint16_t* __restrict__ Uw = (uint16_t*)a.U;
    const float cm1 = ks.scal[0], sz = ks.scal[1], nu_f = ks.scal[2];
    const bool upd = ks.flag[2] != 0;
    // a sequence keeps U in the registers (the next frame starts from them)
    // and stores it after its last frame only, in a loop of its own, so the
    // update of the other frames carries no per-entry store decisions
    const bool store_u = !SEQ || fi + 1 >= a.nseq;
    if (SEQ && upd) u_pending = !store_u;
    pin_tile(u);
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int q0 = 2 * (tid + s * kBlock);
      if (q0 >= ctx.nq) continue;
      const bool has1 = (vbits >> (2 * s + 1)) & 1u;
      const int c = q0 / ctx.npx;
      const int e = c * a.P + ctx.p0 + (q0 - c * ctx.npx);
      const int e1 = ((sbits >> s) & 1u) ? e + 1 + (a.P - ctx.npx) : e + 1;
      float rl0 = r[2 * s], rl1 = r[2 * s + 1];
      if (upd) {
        float uv0 = 0.f, ua0 = 0.f, uv1 = 0.f, ua1 = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const float a0 = bf_lo(u[s][j]), a1 = bf_hi(u[s][j]);
          uv0 = fmaf(a0, ks.vf[j], uv0);
          ua0 = fmaf(a0, ks.af[j], ua0);
          uv1 = fmaf(a1, ks.vf[j], uv1);
          ua1 = fmaf(a1, ks.af[j], ua1);
        }
        const float coef0 = fmaf(cm1, uv0, -sz * (cw[2 * s] - ua0));
        const float coef1 = fmaf(cm1, uv1, -sz * (cw[2 * s + 1] - ua1));
#pragma unroll
        for (int j = 0; j < K; ++j) {
          if constexpr (SEQ) {   // columns >= k stay 0 (v_j = 0)
            u[s][j] = pack_bf16_rne(fmaf(coef0, ks.vf[j], bf_lo(u[s][j])), fmaf(coef1, ks.vf[j], bf_hi(u[s][j])));
          } else if (j < a.k) {
            const uint32_t nw = pack_bf16_rne(fmaf(coef0, ks.vf[j], bf_lo(u[s][j])),
                                              fmaf(coef1, ks.vf[j], bf_hi(u[s][j])));
            uint16_t* col = Uw + (long long)j * a.ldU;
            if (al) {
              st_u32(col, 2u * (unsigned)e, nw);
            } else {
              st_u16(col, 2u * (unsigned)e, (uint16_t)(nw & 0xFFFFu));
              if (has1) st_u16(col, 2u * (unsigned)e1, (uint16_t)(nw >> 16));
            }
          }
        }
        if (a.labels_after_update) {
          rl0 = fmaf(-coef0, nu_f, rl0);
          rl1 = fmaf(-coef1, nu_f, rl1);
        }
      }
      if (pre && pupd) {   // the frame joined the running average: store it
        pre_store(a, e, bf_lo(ld_u16(xg, 2u * (unsigned)e)), pinv_n);
        if (has1) pre_store(a, e1, bf_lo(ld_u16(xg, 2u * (unsigned)e1)), pinv_n);
      }
      if (EXT && a.score) {
        a.score[e] = fabsf(rl0);
        if (has1) a.score[e1] = fabsf(rl1);
      }
      s_flag[q0] = (fabsf(rl0) >= a.delta) ? 1 : 0;
      if (has1) s_flag[q0 + 1] = (fabsf(rl1) >= a.delta) ? 1 : 0;
    }
    if (SEQ && upd && store_u) store_tile();
#pragma unroll 1
    for (int s = NP; s < NT; ++s) {   // LDS pairs (no optional features)
      const int q0 = 2 * (tid + s * kBlock);
      if (q0 >= ctx.nq) continue;
      const uint32_t* lts = lt + (s - NP) * K * kBlock + tid;
      float* rls = lr + (s - NP) * 2 * kBlock + tid;
      const bool has1 = (vbits >> (2 * s + 1)) & 1u;
      const int c = q0 / ctx.npx;
      const int e = c * a.P + ctx.p0 + (q0 - c * ctx.npx);
      const int e1 = ((sbits >> s) & 1u) ? e + 1 + (a.P - ctx.npx) : e + 1;
      float rl0 = rls[0], rl1 = rls[kBlock];
      if (upd) {
        float uv0 = 0.f, ua0 = 0.f, uv1 = 0.f, ua1 = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const uint32_t v = lts[j * kBlock];
          const float a0 = bf_lo(v), a1 = bf_hi(v);
          uv0 = fmaf(a0, ks.vf[j], uv0);
          ua0 = fmaf(a0, ks.af[j], ua0);
          uv1 = fmaf(a1, ks.vf[j], uv1);
          ua1 = fmaf(a1, ks.af[j], ua1);
        }
        float et[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float phi, c;
          const float ri = rls[h * kBlock];
          cost_eval(ri, a.cp, phi, c);
          et[h] = -weight(2 * s + h) * c * ri;
        }
        const float coef0 = fmaf(cm1, uv0, -sz * (et[0] - ua0));
        const float coef1 = fmaf(cm1, uv1, -sz * (et[1] - ua1));
#pragma unroll
        for (int j = 0; j < K; ++j)
          if (j < a.k) {
            const uint32_t v = lts[j * kBlock];
            const uint32_t nw = pack_bf16_rne(fmaf(coef0, ks.vf[j], bf_lo(v)), fmaf(coef1, ks.vf[j], bf_hi(v)));
            uint16_t* col = Uw + (long long)j * a.ldU;
            if (al) {
              st_u32(col, 2u * (unsigned)e, nw);
            } else {
              st_u16(col, 2u * (unsigned)e, (uint16_t)(nw & 0xFFFFu));
              if (has1) st_u16(col, 2u * (unsigned)e1, (uint16_t)(nw >> 16));
            }
          }
        if (a.labels_after_update) {
          rl0 = fmaf(-coef0, nu_f, rl0);
          rl1 = fmaf(-coef1, nu_f, rl1);
        }
      }
      s_flag[q0] = (fabsf(rl0) >= a.delta) ? 1 : 0;
      if (has1) s_flag[q0 + 1] = (fabsf(rl1) >= a.delta) ? 1 : 0;
    }
    trace_point(a, tile, 61);
    write_labels<SEQ>(a, s_flag, ctx.p0, ctx.npx);
    trace_point(a, tile, 62);
  }
  tile_end(a, tile, ks, ctx, steps, restarts, bad, nbar);
  if (!SEQ || NL > 0 || ++fi >= a.nseq) break;   // sequences: register tiles only

  // ---- next frame of a sequence (as in the float32 tile) ----
  next_frame_begin(ks, ctx, bad);
  xg = (const uint16_t*)(a.xtab ? a.xtab[ctx.n % a.ring] : a.seq[fi]);
#pragma unroll
  for (int s = 0; s < NP; ++s) {
    const int q0 = 2 * (tid + s * kBlock);
    if (q0 >= ctx.nq) continue;
    const bool has1 = (vbits >> (2 * s + 1)) & 1u;
    const bool split = (sbits >> s) & 1u;
    const int c = q0 / ctx.npx;
    const int pl = q0 - c * ctx.npx;
    const int e = c * a.P + ctx.p0 + pl;
    const int e1 = split ? e + 1 + (a.P - ctx.npx) : e + 1;
    if (!bad) {
      fbits &= ~(3u << (2 * s));
      if (pixel_label(s_flag, a.C, ctx.npx, pl)) fbits |= 1u << (2 * s);
      if (has1 && pixel_label(s_flag, a.C, ctx.npx, split ? 0 : pl + 1)) fbits |= 2u << (2 * s);
    }
    const unsigned b0 = 2u * (unsigned)e, b1 = 2u * (unsigned)e1;
    uint32_t xw;
    if (al) xw = ld_u32(xg, b0);
    else xw = ld_u16(xg, b0) | (has1 ? (ld_u16(xg, b1) << 16) : 0u);
    float acc0 = bf_lo(xw), acc1 = bf_hi(xw);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      acc0 = fmaf(-bf_lo(u[s][j]), ks.yf[j], acc0);
      acc1 = fmaf(-bf_hi(u[s][j]), ks.yf[j], acc1);
    }
    r[2 * s] = acc0;
    r[2 * s + 1] = has1 ? acc1 : 0.f;
  }
  }
  // the last frame stored nothing (rejected, or no step): store the updated tile
  if (SEQ && u_pending) store_tile();
  return true;
}

// One workgroup's share of one frame in the storage type's register layout.
// Returns false when the gang aborted.
// EXT: the optional features are compiled in (pre-processing when the
// stream has its statistics, per-entry label scores when a score buffer is
// given); without it the hot path carries none of their code.  WIDE: the
// steps that reduce H with the gradient in one wide exchange (the IRLS
// variant and the one-exchange curvature schedule of CG) are compiled in as
// well: float32 tiles of the single-stream kernel only, as the H partials
// would spill the packed tile and the batch kernel's registers.
// SEQ: the sequence form (a.nseq frames per launch, the tile kept in
// registers between frames), a separate instantiation so that the one-frame
// kernels carry none of its loop.
template <int K, int NR, typename TS, bool EXT, bool WIDE = false, int NL = 0, bool SEQ = false>
__device__ __forceinline__ bool run_tile(const FrameArgs& a, const int tile, FrameSmem& sm,
                                         uint32_t* __restrict__ lt = nullptr) {
  if constexpr (sizeof(TS) == 2) {
    static_assert(NR % 2 == 0, "bfloat16 tiles hold row pairs");
    return frame_tile_packed<K, NR / 2, EXT, NL, SEQ>(a, tile, sm, lt);
  } else {
    static_assert(NL == 0, "LDS row pairs: bfloat16 tiles only");
    return frame_tile<K, NR, EXT, WIDE, SEQ>(a, tile, sm);
  }
}

template <int K, int NR, typename TS, bool EXT, bool SEQ = false>
__global__ __launch_bounds__(kBlock, 2) void frame_kernel(FrameArgs a) {
  __shared__ FrameSmem sm;
  run_tile<K, NR, TS, EXT, EXT, 0, SEQ>(a, blockIdx.x, sm);
}

}  // inline namespace PROST_BLOCK_NS
}  // namespace prost
