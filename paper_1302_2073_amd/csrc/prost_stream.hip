// Frames too large for a resident gang of register tiles (Sec. 3.3, Steps
// 1-3, with the step-size rule of Sec. 3.4): the same per-frame arithmetic as
// the frame kernel, but every dependent pass streams U and the frame from
// HBM, one launch per pass, with the k-space work between passes in one
// small workgroup.  Per frame and CG step (Step 1):
//   grad pass:   r = x - U y, phi, c; w c stored per entry; partials of
//                U^T (w phi'(r)) and sum w phi(r)
//   direction:   fixed-order sum of the partials, PR+ direction d
//   curvature:   partials of sum w c (u . d)^2 (the majoriser's d^T H d)
//   advance:     alpha = -g.d / d^T H d, y += alpha d
// (curvature schedule 1 instead: one pass reduces g, f and the upper
// triangle of H = U^T diag(w c) U, and one kernel forms d, d^T H d and the
// step), then (Step 2) the eta pass (eta = -w phi'(r) stored per entry,
// partials of U^T eta, ||eta||^2 and the final cost), the geodesic scalars,
// and one pass that updates U and labels every pixel (Step 3).  A thread
// takes one pixel (all channels), or two adjacent ones in bfloat16 storage
// with even P and aligned planes (32-bit accesses).  Reductions: float32 per
// thread, float64 per workgroup and across workgroups in a fixed order, so
// results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/prost.h"
#include "prost_frame.hpp"
#include "prost_host.hpp"

namespace prost {

constexpr int kStBlock = 256;           // threads per workgroup of a pass (one pixel or pixel pair each)
constexpr int kStWaves = kStBlock / 64;
constexpr int kStRed = 1024;            // threads of the reducing (k-space) kernels
constexpr int kStL = kMaxK + 2;         // partials per workgroup: up to K values and two scalars
constexpr int kStWide = 160;            // schedule 1: g (K), f and H's upper triangle (<= 153 values)
template <int KC>
constexpr int st_nh() { return KC + 1 + KC * (KC + 1) / 2; }
static_assert(st_nh<kMaxK>() <= kStWide, "wide partial vector");

// k-space state of the frame being streamed (device memory, one per handle).
struct StreamKS {
  double y[kMaxK], gp[kMaxK], d[kMaxK], dp[kMaxK];   // y, previous gradient, direction, previous direction
  double gd;
  float yf[kMaxK], yl[kMaxK];   // y as float32 plus its float32 remainder: r = x - U yf - U yl
  float df[kMaxK], vf[kMaxK], af[kMaxK];
  float cm1, sz, nu;
  int stop, bad, upd, steps, restarts;
  double htot[kStWide];   // curvature schedule 1: reduced g, f and upper triangle of H
};

// Workgroup sum of L float partials per thread into part[blk * kStL + q]
// (float64; fixed order: wavefront reduce-scatter, then wavefronts in order).
template <int L>
__device__ __forceinline__ void st_block_partials(float (&acc)[L], double (*red)[kStL], double* __restrict__ part) {
  const int tid = thread_index(), lane = tid & 63, wv = tid >> 6;
  int comp;
  const float v = wave_reduce_scatter<L>(acc, comp);
  if (wave_rs_owner<L>(lane) && comp < L) red[wv][comp] = (double)v;
  __syncthreads();
  if (tid < L) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kStWaves; ++w) s += red[w][tid];
    part[(size_t)blockIdx.x * kStL + tid] = s;
  }
}

// Sum over the nblk workgroups' partials of the first L values, into out[]
// (shared).  Each value is summed by NG = kStRed / Lp threads (Lp: L rounded
// up to a power of two): thread (q, g) takes workgroups g, g + NG, g + 2 NG,
// ... in order (kStUnroll loads in flight), then the NG group sums are
// folded in a fixed tree (the upper half onto the lower, down to 32) and
// those are added in order.  Every step is fixed, so the result is
// deterministic.
constexpr int kStUnroll = 16;
template <int L>
__device__ __forceinline__ void st_sum_partials(const double* __restrict__ part, int nblk, double* grp,
                                                double* out) {
  constexpr int Lp = pow2_at_least(L);
  constexpr int NG = kStRed / Lp;
  static_assert(NG >= 32, "at least 32 threads per value");
  const int t = threadIdx.x, q = t % Lp, g = t / Lp;
  double s = 0.0;
  if (q < L) {
    int b = g;
    for (; b + (kStUnroll - 1) * NG < nblk; b += kStUnroll * NG) {
      double v[kStUnroll];
#pragma unroll
      for (int i = 0; i < kStUnroll; ++i) v[i] = part[(size_t)(b + i * NG) * kStL + q];
#pragma unroll
      for (int i = 0; i < kStUnroll; ++i) s += v[i];
    }
    for (; b < nblk; b += NG) s += part[(size_t)b * kStL + q];
  }
  grp[g * Lp + q] = s;
  __syncthreads();
#pragma unroll
  for (int h = NG / 2; h >= 32; h >>= 1) {
    if (g < h) grp[g * Lp + q] += grp[(g + h) * Lp + q];
    __syncthreads();
  }
  if (t < L) {
    double v = 0.0;
    for (int r = 0; r < 32; ++r) v += grp[r * Lp + t];
    out[t] = v;
  }
  __syncthreads();
}

__device__ __forceinline__ float st_weight(const FrameArgs& a, int p) {
  const uint8_t* src = a.weights_from_filtered ? a.mask : a.lab;
  return src[p] ? a.omega : 1.0f;
}

// Pixels per thread of a pass: one, or (PAIR, bfloat16 with even P and
// 4-byte aligned planes) two adjacent pixels whose entries are one aligned
// 32-bit word in every plane of U and of the frame: half the load and store
// instructions for the same bytes.
template <typename TS, bool PAIR>
struct StPix {
  static_assert(!PAIR || sizeof(TS) == 2, "pairs of bfloat16 entries");
  static constexpr int N = PAIR ? 2 : 1;
};

// The entries of channel c of this thread's pixels p0 (.. p0 + 1): U rows
// (columns >= k are 0) and frame values.
template <int KC, typename TS, bool PAIR>
__device__ __forceinline__ void st_load(const FrameArgs& a, int c, int p0, float (&u)[StPix<TS, PAIR>::N][KC],
                                        float (&x)[StPix<TS, PAIR>::N]) {
  const long long e = (long long)c * a.P + p0;
  if constexpr (PAIR) {
    const uint32_t* __restrict__ U = (const uint32_t*)a.U;
    const uint32_t xw = ((const uint32_t*)a.x)[e >> 1];
    x[0] = bf_lo(xw);
    x[1] = bf_hi(xw);
#pragma unroll
    for (int j = 0; j < KC; ++j) {
      const uint32_t w = (j < a.k) ? U[((long long)j * a.ldU + e) >> 1] : 0u;
      u[0][j] = bf_lo(w);
      u[1][j] = bf_hi(w);
    }
  } else {
    const TS* __restrict__ U = (const TS*)a.U;
    x[0] = ld_elem((const TS*)a.x, e);
#pragma unroll
    for (int j = 0; j < KC; ++j) u[0][j] = (j < a.k) ? ld_elem(U, (long long)j * a.ldU + e) : 0.f;
  }
}

// r = x - U y with y as the float32 pair (value, remainder).
template <int KC>
__device__ __forceinline__ float st_residual(float x, const float (&u)[KC], const float* ys, const float* yl) {
  float r = x, rl = 0.f;
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    r = fmaf(-u[j], ys[j], r);
    rl = fmaf(-u[j], yl[j], rl);
  }
  return r + rl;
}

// y (float64) as the float32 pair the passes use: every pass recomputes
// r = x - U y from the frame, and the remainder keeps that residual as
// accurate as the float64 y (near a fit the gradient is small and a
// float32-rounded y would dominate its error).
__device__ __forceinline__ void st_set_y(StreamKS* ks, int j, double yv) {
  ks->y[j] = yv;
  const float hi = (float)yv;
  ks->yf[j] = hi;
  ks->yl[j] = (float)(yv - (double)hi);
}

// Frame start: y from the handle, flags cleared.
__global__ void st_begin(FrameArgs a, StreamKS* ks) {
  const int t = threadIdx.x;
  if (t < kMaxK) st_set_y(ks, t, (t < a.k) ? a.y[t] : 0.0);
  if (t == 0) {
    ks->stop = ks->bad = ks->upd = ks->steps = ks->restarts = 0;
    a.stats->frame = *a.nframe;
  }
}

// Step 1 gradient pass at the current y (float32 per thread, as the frame kernel).
template <int KC, typename TS, bool PAIR>
__global__ __launch_bounds__(kStBlock) void st_grad(FrameArgs a, const StreamKS* __restrict__ ks, float* __restrict__ wc,
                                                    double* __restrict__ part) {
  constexpr int N = StPix<TS, PAIR>::N;
  if (ks->stop || ks->bad) return;
  __shared__ float ys[KC], yl[KC];
  __shared__ double red[kStWaves][kStL];
  const int tid = thread_index();
  if (tid < KC) {
    ys[tid] = ks->yf[tid];
    yl[tid] = ks->yl[tid];
  }
  __syncthreads();
  const int p0 = (blockIdx.x * kStBlock + tid) * N;
  const bool valid = p0 < a.P;   // with pairs P is even, so both pixels are
  float wt[N];
#pragma unroll
  for (int i = 0; i < N; ++i) wt[i] = valid ? st_weight(a, p0 + i) : 0.f;
  float acc[KC + 1];
#pragma unroll
  for (int j = 0; j <= KC; ++j) acc[j] = 0.f;
  if (valid)
    for (int c = 0; c < a.C; ++c) {
      float u[N][KC], x[N];
      st_load<KC, TS, PAIR>(a, c, p0, u, x);
      const long long e = (long long)c * a.P + p0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float r = st_residual<KC>(x[i], u[i], ys, yl);
        float phi, cc;
        cost_eval(r, a.cp, phi, cc);
        const float w_c = wt[i] * cc;
        wc[e + i] = w_c;
        const float wd = w_c * r;                 // w phi'(r)
        acc[KC] = fmaf(wt[i], phi, acc[KC]);
#pragma unroll
        for (int j = 0; j < KC; ++j) acc[j] = fmaf(wd, u[i][j], acc[j]);
      }
    }
  st_block_partials<KC + 1>(acc, red, part);
}

// PR+ direction from the reduced gradient and cost tot[0..KC] (the frame
// kernel's k-space step), by the first wavefront; d, its float32 copy, the
// previous gradient, g.d and the stop / bad flags land in ks.
template <int KC>
__device__ __forceinline__ void st_dir_core(const FrameArgs& a, StreamKS* ks, const double* tot, int it) {
  const int lane = threadIdx.x;
  const double g = (lane < a.k) ? -tot[lane] : 0.0;
  const double f = tot[KC];
  const double gg = row16_sum(g * g);
  int stop = 0, bad = 0;
  if (it == 0 && !(isfinite(f) && isfinite(gg))) stop = bad = 1;
  if (gg == 0.0) stop = 1;
  double beta = 0.0, dj = -g;
  if (!stop && it > 0 && a.ysolve == 0) {
    const double gpv = (lane < a.k) ? ks->gp[lane] : 0.0;
    const double num = row16_sum(g * (g - gpv));
    const double den = row16_sum(gpv * gpv);
    beta = fmax(0.0, num / den);
    const double dpv = (lane < a.k) ? ks->dp[lane] : 0.0;
    dj = -g + beta * dpv;
    if (row16_sum(g * dj) >= 0.0) {
      dj = -g;
      if (lane == 0) ++ks->restarts;
    }
  }
  const double gd = row16_sum(g * dj);
  if (lane < kMaxK) {
    ks->d[lane] = (lane < a.k) ? dj : 0.0;
    ks->df[lane] = (lane < a.k) ? (float)dj : 0.f;
    ks->gp[lane] = (lane < a.k) ? g : 0.0;
  }
  if (lane == 0) {
    a.stats->f[it] = f;
    a.stats->beta[it] = beta;
    ks->gd = gd;
    ks->stop = stop;
    if (bad) {
      ks->bad = 1;
      __hip_atomic_fetch_or(&a.sync[2], kErrBadFrame, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Majoriser step alpha = -g.d / d^T H d, y += alpha d (stop if d^T H d <= 0).
__device__ __forceinline__ void st_adv_core(const FrameArgs& a, StreamKS* ks, double dHd, int it) {
  const int t = threadIdx.x;
  if (!(dHd > 0.0)) {
    if (t == 0) ks->stop = 1;
    return;
  }
  const double alpha = -ks->gd / dHd;
  if (t < kMaxK) {
    st_set_y(ks, t, ks->y[t] + alpha * ks->d[t]);
    ks->dp[t] = ks->d[t];
  }
  if (t == 0) {
    a.stats->alpha[it] = alpha;
    ks->steps = it + 1;
  }
}

// Reduced gradient and cost -> PR+ direction (curvature schedule 0).
template <int KC>
__global__ __launch_bounds__(kStRed) void st_direction(FrameArgs a, StreamKS* ks, const double* __restrict__ part,
                                                       int nblk, int it) {
  if (ks->stop || ks->bad) return;
  __shared__ double grp[kStRed];
  __shared__ double tot[32];
  st_sum_partials<KC + 1>(part, nblk, grp, tot);
  if (threadIdx.x < 64) st_dir_core<KC>(a, ks, tot, it);
}

// Curvature of the majoriser along d: sum w c (u . d)^2.
template <int KC, typename TS, bool PAIR>
__global__ __launch_bounds__(kStBlock) void st_curv(FrameArgs a, const StreamKS* __restrict__ ks,
                                                    const float* __restrict__ wc, double* __restrict__ part) {
  constexpr int N = StPix<TS, PAIR>::N;
  if (ks->stop || ks->bad) return;
  __shared__ float ds[KC];
  __shared__ double red[kStWaves][kStL];
  const int tid = thread_index();
  if (tid < KC) ds[tid] = ks->df[tid];
  __syncthreads();
  const int p0 = (blockIdx.x * kStBlock + tid) * N;
  float acc[1] = {0.f};
  if (p0 < a.P)
    for (int c = 0; c < a.C; ++c) {
      float u[N][KC], x[N];
      st_load<KC, TS, PAIR>(a, c, p0, u, x);   // x unused: the compiler drops its load
      const long long e = (long long)c * a.P + p0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < KC; ++j) t = fmaf(u[i][j], ds[j], t);
        acc[0] = fmaf(wc[e + i] * t, t, acc[0]);
      }
    }
  st_block_partials<1>(acc, red, part);
}

// Majoriser step: alpha = -g.d / d^T H d, y += alpha d.
__global__ __launch_bounds__(kStRed) void st_advance(FrameArgs a, StreamKS* ks, const double* __restrict__ part,
                                                     int nblk, int it) {
  if (ks->stop || ks->bad) return;
  __shared__ double grp[kStRed];
  __shared__ double tot[32];
  st_sum_partials<1>(part, nblk, grp, tot);
  st_adv_core(a, ks, tot[0], it);
}

// Curvature schedule 1 (d^T H d from the reduced matrix H): one pass per CG
// step reduces g, f and the upper triangle of H = U^T diag(w c) U together
// (k (k + 1) / 2 more products per entry), so the curvature pass and its
// launches drop out.  Partials value-major: part[v * nblk + workgroup].
template <int KC, typename TS, bool PAIR>
__global__ __launch_bounds__(kStBlock) void st_gradh(FrameArgs a, const StreamKS* __restrict__ ks,
                                                     double* __restrict__ part, int nblk) {
  constexpr int N = StPix<TS, PAIR>::N;
  constexpr int NV = st_nh<KC>();
  if (ks->stop || ks->bad) return;
  __shared__ float ys[KC], yl[KC];
  __shared__ double red[kStWaves][NV];
  const int tid = thread_index(), lane = tid & 63, wv = tid >> 6;
  if (tid < KC) {
    ys[tid] = ks->yf[tid];
    yl[tid] = ks->yl[tid];
  }
  __syncthreads();
  const int p0 = (blockIdx.x * kStBlock + tid) * N;
  const bool valid = p0 < a.P;
  float wt[N];
#pragma unroll
  for (int i = 0; i < N; ++i) wt[i] = valid ? st_weight(a, p0 + i) : 0.f;
  float acc[NV];   // g (KC), f, H upper triangle row by row
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.f;
  if (valid)
    for (int c = 0; c < a.C; ++c) {
      float u[N][KC], x[N];
      st_load<KC, TS, PAIR>(a, c, p0, u, x);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float r = st_residual<KC>(x[i], u[i], ys, yl);
        float phi, cc;
        cost_eval(r, a.cp, phi, cc);
        const float w_c = wt[i] * cc;
        const float wd = w_c * r;                 // w phi'(r)
        acc[KC] = fmaf(wt[i], phi, acc[KC]);
#pragma unroll
        for (int j = 0; j < KC; ++j) acc[j] = fmaf(wd, u[i][j], acc[j]);
        int q = KC + 1;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          const float tj = w_c * u[i][j];
#pragma unroll
          for (int l = j; l < KC; ++l) {
            acc[q] = fmaf(tj, u[i][l], acc[q]);
            ++q;
          }
        }
      }
    }
  // workgroup sums in chunks of 32 values (fixed order, float64 across wavefronts)
#pragma unroll
  for (int c0 = 0; c0 < NV; c0 += 32) {
    float ch[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) ch[q] = (c0 + q < NV) ? acc[(c0 + q < NV) ? c0 + q : 0] : 0.f;
    int comp;
    const float v = wave_reduce_scatter<32>(ch, comp);
    if (wave_rs_owner<32>(lane) && c0 + comp < NV) red[wv][c0 + comp] = (double)v;
  }
  __syncthreads();
  for (int q = tid; q < NV; q += kStBlock) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kStWaves; ++w) sum += red[w][q];
    part[(size_t)q * nblk + blockIdx.x] = sum;
  }
}

// Sum of value v's partials over the nblk workgroups (one workgroup per
// value, fixed order) into ks->htot[v].
__global__ __launch_bounds__(256) void st_hsum(StreamKS* ks, const double* __restrict__ part, int nblk) {
  if (ks->stop || ks->bad) return;
  __shared__ double red[4];
  const int v = blockIdx.x, t = threadIdx.x;
  const double* row = part + (size_t)v * nblk;
  double s = 0.0;
  for (int b = t; b < nblk; b += 256) s += row[b];
  s = wave_sum(s);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  if (t == 0) ks->htot[v] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Direction and majoriser step of schedule 1: d^T H d from the reduced H.
template <int KC>
__global__ __launch_bounds__(64) void st_step(FrameArgs a, StreamKS* ks, int it) {
  if (ks->stop || ks->bad) return;
  __shared__ double tot[st_nh<KC>()];
  __shared__ double dsh[KC];
  for (int q = threadIdx.x; q < st_nh<KC>(); q += 64) tot[q] = ks->htot[q];
  __syncthreads();
  st_dir_core<KC>(a, ks, tot, it);
  __syncthreads();
  if (ks->stop || ks->bad) return;
  if (threadIdx.x < KC) dsh[threadIdx.x] = ks->d[threadIdx.x];
  __syncthreads();
  // row i of the triangle by lane i, rows added in order
  __shared__ double rowsum[KC];
  const int i = threadIdx.x;
  if (i < KC) {
    int q = KC + 1 + i * KC - i * (i - 1) / 2;   // H[i][i]
    double sacc = tot[q] * dsh[i] * dsh[i];
    for (int l = i + 1; l < KC; ++l) sacc += 2.0 * tot[++q] * dsh[i] * dsh[l];
    rowsum[i] = sacc;
  }
  __syncthreads();
  double dHd = 0.0;
  for (int r = 0; r < KC; ++r) dHd += rowsum[r];
  st_adv_core(a, ks, dHd, it);
}

// Step 2 eta pass at the final y: eta = -w phi'(r) stored per entry;
// partials of U^T eta, ||eta||^2 and the final cost.
template <int KC, typename TS, bool PAIR>
__global__ __launch_bounds__(kStBlock) void st_eta(FrameArgs a, const StreamKS* __restrict__ ks, float* __restrict__ eta,
                                                   double* __restrict__ part) {
  constexpr int N = StPix<TS, PAIR>::N;
  if (ks->bad) return;
  __shared__ float ys[KC], yl[KC];
  __shared__ double red[kStWaves][kStL];
  const int tid = thread_index();
  if (tid < KC) {
    ys[tid] = ks->yf[tid];
    yl[tid] = ks->yl[tid];
  }
  __syncthreads();
  const int p0 = (blockIdx.x * kStBlock + tid) * N;
  const bool valid = p0 < a.P;
  float wt[N];
#pragma unroll
  for (int i = 0; i < N; ++i) wt[i] = valid ? st_weight(a, p0 + i) : 0.f;
  float acc[KC + 2];
#pragma unroll
  for (int j = 0; j < KC + 2; ++j) acc[j] = 0.f;
  if (valid)
    for (int c = 0; c < a.C; ++c) {
      float u[N][KC], x[N];
      st_load<KC, TS, PAIR>(a, c, p0, u, x);
      const long long e = (long long)c * a.P + p0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float r = st_residual<KC>(x[i], u[i], ys, yl);
        float phi, cc;
        cost_eval(r, a.cp, phi, cc);
        const float et = -wt[i] * cc * r;
        eta[e + i] = et;
        acc[KC] = fmaf(et, et, acc[KC]);
        acc[KC + 1] = fmaf(wt[i], phi, acc[KC + 1]);
#pragma unroll
        for (int j = 0; j < KC; ++j) acc[j] = fmaf(et, u[i][j], acc[j]);
      }
    }
  st_block_partials<KC + 2>(acc, red, part);
}

// Geodesic scalars (Sec. 3.3 Step 2, Sec. 3.4 step size) from the reduced
// a = U^T eta, ||eta||^2 and the final cost, as geodesic_setup does.
template <int KC>
__global__ __launch_bounds__(kStRed) void st_geodesic(FrameArgs a, StreamKS* ks, const double* __restrict__ part,
                                                      int nblk) {
  if (ks->bad) return;
  __shared__ double grp[kStRed];
  __shared__ double tot[32];
  st_sum_partials<KC + 2>(part, nblk, grp, tot);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const double av = (lane < a.k) ? tot[lane] : 0.0;
    const double yv = (lane < a.k) ? ks->y[lane] : 0.0;
    const double aa = row16_sum(av * av);
    const double yy = row16_sum(yv * yv);
    const double ee = tot[KC];
    const double zeta = sqrt(fmax(ee - aa, 0.0));
    const double nu = sqrt(yy);
    const double sigma = zeta * nu;
    const int upd = (zeta > 0.0 && nu > 0.0) ? 1 : 0;
    if (lane < kMaxK) {
      ks->af[lane] = (float)av;
      ks->vf[lane] = upd ? (float)(yv / nu) : 0.f;
    }
    if (lane == 0) {
      const long long n = *a.nframe;
      const GeoScalars g = geodesic_scalars(a.tau * (double)n, a.t_init, a.t_min, sigma, zeta);
      ks->cm1 = upd ? (float)g.cm1 : 0.f;
      ks->sz = upd ? (float)g.sz : 0.f;
      ks->nu = (float)nu;
      ks->upd = upd;
      const int steps = ks->steps;
      a.stats->f[steps] = tot[KC + 1];
      a.stats->cg_steps = steps;
      a.stats->restarts = ks->restarts;
      a.stats->t = g.t;
      a.stats->sigma = sigma;
      a.stats->theta = g.theta;
      a.stats->zeta = zeta;
      a.stats->nu = nu;
      a.stats->updated = upd;
    }
  }
}

// Rank-one geodesic update of every row and the pixel labels (Step 3), one
// pass: u <- u + coef v with coef = (cos theta - 1)(u.v) - (sin theta / zeta)
// (eta - u.a); r' = r - coef nu (r' = x - U' y); label = any channel with
// |r'| >= delta.
template <int KC, typename TS, bool PAIR>
__global__ __launch_bounds__(kStBlock) void st_update(FrameArgs a, const StreamKS* __restrict__ ks,
                                                      const float* __restrict__ eta) {
  constexpr int N = StPix<TS, PAIR>::N;
  if (ks->bad) return;
  __shared__ float ys[KC], yl[KC], vs[KC], as[KC];
  const int tid = thread_index();
  if (tid < KC) {
    ys[tid] = ks->yf[tid];
    yl[tid] = ks->yl[tid];
    vs[tid] = ks->vf[tid];
    as[tid] = ks->af[tid];
  }
  __syncthreads();
  const int p0 = (blockIdx.x * kStBlock + tid) * N;
  if (p0 >= a.P) return;
  const float cm1 = ks->cm1, sz = ks->sz, nu = ks->nu;
  const bool upd = ks->upd != 0;
  uint8_t label[N];
#pragma unroll
  for (int i = 0; i < N; ++i) label[i] = 0;
  for (int c = 0; c < a.C; ++c) {
    float u[N][KC], x[N];
    st_load<KC, TS, PAIR>(a, c, p0, u, x);
    const long long e = (long long)c * a.P + p0;
    float un[N][KC];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      float r = st_residual<KC>(x[i], u[i], ys, yl);
      if (upd) {
        float uv = 0.f, ua = 0.f;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          uv = fmaf(u[i][j], vs[j], uv);
          ua = fmaf(u[i][j], as[j], ua);
        }
        const float coef = fmaf(cm1, uv, -sz * (eta[e + i] - ua));
#pragma unroll
        for (int j = 0; j < KC; ++j) un[i][j] = fmaf(coef, vs[j], u[i][j]);
        if (a.labels_after_update) r = fmaf(-coef, nu, r);
      }
      if (fabsf(r) >= a.delta) label[i] = 1;
    }
    if (upd) {
      if constexpr (PAIR) {
        uint32_t* __restrict__ U = (uint32_t*)a.U;
#pragma unroll
        for (int j = 0; j < KC; ++j)
          if (j < a.k) U[((long long)j * a.ldU + e) >> 1] = pack_bf16_rne(un[0][j], un[1][j]);
      } else {
        TS* __restrict__ U = (TS*)a.U;
#pragma unroll
        for (int j = 0; j < KC; ++j)
          if (j < a.k) st_elem(U, (long long)j * a.ldU + e, un[0][j]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) a.lab[p0 + i] = label[i];
}

// Frame end: y and the frame counter (an accepted frame only).
__global__ void st_end(FrameArgs a, const StreamKS* __restrict__ ks) {
  const int t = threadIdx.x;
  if (ks->bad) {
    if (t == 0) a.stats->bad_frame = 1;
    return;
  }
  if (t < a.k) a.y[t] = ks->y[t];
  if (t == 0) {
    a.stats->bad_frame = 0;
    *a.nframe = *a.nframe + 1;
  }
}

// One frame: nblk workgroups of kStBlock threads, each thread one pixel (or
// one pixel pair with PAIR).  a.curv selects the CG curvature schedule: 0,
// d^T H d from a second pass over U per step; 1, H reduced with the gradient.
template <int KC, typename TS, bool PAIR>
static void st_frame_launch(const FrameArgs& a, StreamKS* ks, float* wc, float* eta, double* part, int nblk,
                            hipStream_t s) {
  hipLaunchKernelGGL(st_begin, dim3(1), dim3(64), 0, s, a, ks);
  for (int it = 0; it < a.J; ++it) {
    if (a.curv == 1) {
      hipLaunchKernelGGL((st_gradh<KC, TS, PAIR>), dim3(nblk), dim3(kStBlock), 0, s, a, (const StreamKS*)ks, part,
                         nblk);
      hipLaunchKernelGGL(st_hsum, dim3(st_nh<KC>()), dim3(256), 0, s, ks, (const double*)part, nblk);
      hipLaunchKernelGGL((st_step<KC>), dim3(1), dim3(64), 0, s, a, ks, it);
      continue;
    }
    hipLaunchKernelGGL((st_grad<KC, TS, PAIR>), dim3(nblk), dim3(kStBlock), 0, s, a, (const StreamKS*)ks, wc, part);
    hipLaunchKernelGGL((st_direction<KC>), dim3(1), dim3(kStRed), 0, s, a, ks, (const double*)part, nblk, it);
    hipLaunchKernelGGL((st_curv<KC, TS, PAIR>), dim3(nblk), dim3(kStBlock), 0, s, a, (const StreamKS*)ks,
                       (const float*)wc, part);
    hipLaunchKernelGGL(st_advance, dim3(1), dim3(kStRed), 0, s, a, ks, (const double*)part, nblk, it);
  }
  hipLaunchKernelGGL((st_eta<KC, TS, PAIR>), dim3(nblk), dim3(kStBlock), 0, s, a, (const StreamKS*)ks, eta, part);
  hipLaunchKernelGGL((st_geodesic<KC>), dim3(1), dim3(kStRed), 0, s, a, ks, (const double*)part, nblk);
  hipLaunchKernelGGL((st_update<KC, TS, PAIR>), dim3(nblk), dim3(kStBlock), 0, s, a, (const StreamKS*)ks,
                     (const float*)eta);
  hipLaunchKernelGGL(st_end, dim3(1), dim3(64), 0, s, a, (const StreamKS*)ks);
}

template <typename TS, bool PAIR>
static void st_frame_class(int kc, const FrameArgs& a, StreamKS* ks, float* wc, float* eta, double* part, int nblk,
                           hipStream_t s) {
  switch (kc) {
    case 2: st_frame_launch<2, TS, PAIR>(a, ks, wc, eta, part, nblk, s); break;
    case 4: st_frame_launch<4, TS, PAIR>(a, ks, wc, eta, part, nblk, s); break;
    case 5: st_frame_launch<5, TS, PAIR>(a, ks, wc, eta, part, nblk, s); break;
    case 8: st_frame_launch<8, TS, PAIR>(a, ks, wc, eta, part, nblk, s); break;
    case 10: st_frame_launch<10, TS, PAIR>(a, ks, wc, eta, part, nblk, s); break;
    case 12: st_frame_launch<12, TS, PAIR>(a, ks, wc, eta, part, nblk, s); break;
    case 15: st_frame_launch<15, TS, PAIR>(a, ks, wc, eta, part, nblk, s); break;
    default: st_frame_launch<16, TS, PAIR>(a, ks, wc, eta, part, nblk, s); break;
  }
}

static int st_class(int k) {
  return k <= 2 ? 2 : k <= 4 ? 4 : k <= 5 ? 5 : k <= 8 ? 8 : k <= 10 ? 10 : k <= 12 ? 12 : k <= 15 ? 15 : 16;
}

}  // namespace prost

// Device buffers of the streamed path: k-space state, per-entry w c and eta,
// per-workgroup partials.
pros_status prost_stream_alloc(pros_handle* h) {
  using namespace prost;
  const int nblk = (h->P + kStBlock - 1) / kStBlock;
  const size_t bytes = sizeof(StreamKS) + 2 * sizeof(float) * (size_t)h->m + sizeof(double) * (size_t)nblk * kStWide +
                       1024;
  hipError_t e = hipMalloc(&h->stream_ws, bytes);
  if (e != hipSuccess) return prost_host::set_error(PROS_ENOMEM, "streamed-frame buffers: %s", hipGetErrorString(e));
  e = hipMemsetAsync(h->stream_ws, 0, bytes, h->stream);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "streamed-frame buffers: %s", hipGetErrorString(e));
  h->stream_blocks = nblk;
  return PROS_OK;
}

pros_status prost_stream_frame(pros_handle* h, const prost::FrameArgs& a) {
  using namespace prost;
  char* base = (char*)h->stream_ws;
  StreamKS* ks = (StreamKS*)base;
  float* wc = (float*)(base + ((sizeof(StreamKS) + 255) / 256) * 256);
  float* eta = wc + h->m;
  double* part = (double*)(((uintptr_t)(eta + h->m) + 255) / 256 * 256);
  const int kc = st_class(h->k);
  if (h->prm.storage == PROS_BF16) {
    // pixel pairs: even P and every plane start 4-byte aligned (U's planes
    // are ldU apart with ldU a multiple of 64; the frame is the caller's)
    const bool pair = h->P % 2 == 0 && h->ldU % 2 == 0 && ((uintptr_t)a.x & 3u) == 0 && ((uintptr_t)a.U & 3u) == 0;
    if (pair)
      st_frame_class<uint16_t, true>(kc, a, ks, wc, eta, part, (h->P / 2 + kStBlock - 1) / kStBlock, h->stream);
    else
      st_frame_class<uint16_t, false>(kc, a, ks, wc, eta, part, h->stream_blocks, h->stream);
  } else {
    st_frame_class<float, false>(kc, a, ks, wc, eta, part, h->stream_blocks, h->stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    h->broken = true;
    h->broken_status = PROS_EHIP;
    return prost_host::set_error(PROS_EHIP, "streamed frame launch failed: %s", hipGetErrorString(e));
  }
  return PROS_OK;
}
