// Differentiable weighted smoothed cost h_{mu,w}(x - U y) for a batch of
// frames (Sec. 3.1, eqs. weightedLPnorm / spcacost):
//   f_b = sum_e w_e phi(X[b,e] - u_e . Y[b,:])
// and its adjoint for an upstream gradient g (length B):
//   dX[b,e] = g_b w_e phi'(r_{b,e})
//   dU[e,:] = -sum_b g_b w_e phi'(r_{b,e}) Y[b,:]   (B = 1, g = 1: eta y^T of Sec. 3.3)
//   dY[b,:] = -g_b sum_e w_e phi'(r_{b,e}) u_e
//   dmu     = sum_b g_b sum_e w_e dphi/dmu(r_{b,e})
// Layouts (row-major): U (m, k), Y (B, k), X (B, m), w (m) or NULL.
// The per-entry derivative code is the cost functor the frame kernel uses.
// Reductions are deterministic: per-workgroup partials in float64, summed in
// a fixed order by a finishing kernel.  The backward's contraction of the
// per-entry factors with U (dY) runs on the matrix cores in float32.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/prost.h"
#include "prost_device.hpp"
#include "prost_host.hpp"

namespace prost {

constexpr int kLpBlock = 256;        // rows of U per workgroup, one per thread
constexpr int kLpWaves = kLpBlock / 64;
constexpr int kLpChunkF = 32;        // frames per pass, forward
constexpr int kLpChunkB = 16;        // frames per pass, backward (LDS for s)
constexpr int kLpPad = kLpBlock + 4; // LDS row stride (16-byte aligned, spreads banks)

typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ CostParams make_cp(int form, float p, float mu) {
  CostParams cp;
  cp.form = form;
  cp.p = p;
  cp.half_p = 0.5f * p;
  cp.mu = mu;
  cp.inv_mu = 1.0f / mu;
  cp.half_p_m1 = 0.5f * p - 1.0f;
  cp.inv_p = 1.0f / p;
  return cp;
}

// dphi/dmu from c = phi'/r: lp: (p/2) s^(p/2-1) = c/2;  log: -r^2/(mu s) = -r^2 c / (2 mu)
__device__ __forceinline__ float dphi_dmu(float r, float c, const CostParams& cp) {
  return (cp.form == 0) ? 0.5f * c : -r * r * c * 0.5f * cp.inv_mu;
}

// Stage the workgroup's rows of U (row-major, K per row) transposed into
// LDS with coalesced reads; rows past the end are zero.
template <int K>
__device__ __forceinline__ void stage_rows(const float* __restrict__ U, long long e0, int nrow, float (*uT)[kLpPad]) {
  for (int q = thread_index(); q < kLpBlock * K; q += kLpBlock) {
    const int row = q / K, j = q - row * K;
    uT[j][row] = (row < nrow) ? U[e0 * K + q] : 0.f;
  }
}

// Frames [b0, b0 + nb) of Y into LDS.
template <int K, int CH>
__device__ __forceinline__ void stage_frames(const float* __restrict__ Y, int b0, int nb, float (*ys)[K]) {
  for (int q = thread_index(); q < nb * K; q += kLpBlock) ys[q / K][q % K] = Y[(long long)b0 * K + q];
}

// Frame entries of this thread's row for frames b .. b + kLpSub - 1 (0 past
// the last frame or row): one coalesced load per frame across the workgroup.
constexpr int kLpSub = 8;   // frames per prefetch step
__device__ __forceinline__ void fetch_frames(float (&buf)[kLpSub], const float* __restrict__ X, long long m,
                                             long long e, bool valid, int b, int B) {
#pragma unroll
  for (int i = 0; i < kLpSub; ++i) buf[i] = (valid && b + i < B) ? X[(long long)(b + i) * m + e] : 0.f;
}

// Forward: each thread owns one row e (u_e in registers) and walks the
// frames in passes of kLpChunkF, eight at a time, with the next eight
// frames' entries requested before the current ones are used (the loads of
// the first eight are in flight while U and Y are staged), so memory and
// arithmetic overlap within every workgroup.  Per frame the workgroup's sum
// of w phi(r) is formed with one in-place reduce-scatter per pass and float64
// across wavefronts.  Partials: part[b * nblk + workgroup].
template <int K>
__global__ __launch_bounds__(kLpBlock) void lpcost_fwd_kernel(const float* __restrict__ U, const float* __restrict__ Y,
                                                              const float* __restrict__ X, const float* __restrict__ w,
                                                              int m, int B, int form, float p, const float* __restrict__ mu_p,
                                                              double* __restrict__ part) {
  constexpr int CH = kLpChunkF;
  constexpr int NS = CH / kLpSub;
  __shared__ __align__(16) float uT[K][kLpPad];
  __shared__ float ys[CH][K];
  __shared__ double red[kLpWaves][CH];
  // A run-time form here: with the form a compile-time constant the compiler
  // hoists every frame's LDS reads of y ahead of the arithmetic and needs
  // 256 VGPRs (one wavefront per SIMD, 2x slower); the backward gains from it.
  const CostParams cp = make_cp(form, p, *mu_p);
  const int tid = thread_index(), lane = tid & 63, wv = tid >> 6;
  const int nblk = gridDim.x;
  const long long e0 = (long long)blockIdx.x * kLpBlock;
  const int nrow = (int)((long long)m - e0 < kLpBlock ? (long long)m - e0 : kLpBlock);
  const bool valid = tid < nrow;
  const long long e = e0 + tid;
  const float wt = valid ? (w ? w[e] : 1.0f) : 0.f;
  float xb[2][kLpSub];
  fetch_frames(xb[0], X, m, e, valid, 0, B);
  float u[K];
  for (int b0 = 0; b0 < B; b0 += CH) {
    const int nb = min(CH, B - b0);
    __syncthreads();
    if (b0 == 0) stage_rows<K>(U, e0, nrow, uT);
    stage_frames<K, CH>(Y, b0, nb, ys);
    __syncthreads();
    if (b0 == 0) {
#pragma unroll
      for (int j = 0; j < K; ++j) u[j] = uT[j][tid];
    }
    float acc[CH];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      fetch_frames(xb[(st + 1) & 1], X, m, e, valid, b0 + (st + 1) * kLpSub, B);   // the next eight
#pragma unroll
      for (int i = 0; i < kLpSub; ++i) {
        const int bl = st * kLpSub + i;
        float r = xb[st & 1][i];
#pragma unroll
        for (int j = 0; j < K; ++j) r = fmaf(-u[j], ys[bl][j], r);
        float phi, c;
        cost_eval(r, cp, phi, c);
        acc[bl] = (bl < nb) ? wt * phi : 0.f;
      }
    }
    int comp;
    const float v = wave_reduce_scatter<CH>(acc, comp);
    if (wave_rs_owner<CH>(lane)) red[wv][comp] = (double)v;   // each component once per wavefront
    __syncthreads();
    if (tid < nb) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < kLpWaves; ++q) sum += red[q][tid];
      part[(size_t)(b0 + tid) * nblk + blockIdx.x] = sum;
    }
  }
}

// Backward: per frame each thread forms s = g w phi'(r) for its row, writes
// dX, accumulates its dU row and dmu in registers, and leaves s in LDS; after
// each pass of kLpChunkB frames the workgroup's share of dY (pass x K) is
// formed from LDS, one output per thread, rows in order.  Frame entries are
// prefetched eight frames ahead as in the forward kernel.  Partials
// (output q = b K + j of dY, then dmu at q = B K): part[q * nblk + workgroup].
template <int K, int FORM>
__global__ __launch_bounds__(kLpBlock) void lpcost_bwd_kernel(const float* __restrict__ U, const float* __restrict__ Y,
                                                              const float* __restrict__ X, const float* __restrict__ w,
                                                              int m, int B, float p, const float* __restrict__ mu_p,
                                                              const float* __restrict__ gout, float* __restrict__ dX,
                                                              float* __restrict__ dU, double* __restrict__ part) {
  constexpr int CH = kLpChunkB;
  constexpr int NS = CH / kLpSub;
  __shared__ __align__(16) float uT[K][kLpPad];
  __shared__ __align__(16) float sdl[CH][kLpPad];
  __shared__ float ys[CH][K];
  __shared__ float gs[CH];
  __shared__ double redm[kLpWaves];
  __shared__ double dyw[kLpWaves][16][17];   // per-wavefront dY tiles [frame][j]
  static_assert(CH == 16 && K <= 16 && kLpBlock == 64 * kLpWaves, "one 16 x 16 tile per wavefront");
  const CostParams cp = make_cp(FORM, p, *mu_p);   // the form is a compile-time constant: no per-entry branch
  const int tid = thread_index(), lane = tid & 63, wv = tid >> 6;
  const int nblk = gridDim.x;
  const long long e0 = (long long)blockIdx.x * kLpBlock;
  const int nrow = (int)((long long)m - e0 < kLpBlock ? (long long)m - e0 : kLpBlock);
  const bool valid = tid < nrow;
  const long long e = e0 + tid;
  const float wt = valid ? (w ? w[e] : 1.0f) : 0.f;
  float u[K], du[K];
#pragma unroll
  for (int j = 0; j < K; ++j) du[j] = 0.f;
  float dmu = 0.f;
  float xb[2][kLpSub];
  fetch_frames(xb[0], X, m, e, valid, 0, B);
  for (int b0 = 0; b0 < B; b0 += CH) {
    const int nb = min(CH, B - b0);
    __syncthreads();
    if (b0 == 0) stage_rows<K>(U, e0, nrow, uT);
    stage_frames<K, CH>(Y, b0, nb, ys);
    if (tid < nb) gs[tid] = gout[b0 + tid];
    __syncthreads();
    if (b0 == 0) {
#pragma unroll
      for (int j = 0; j < K; ++j) u[j] = uT[j][tid];
    }
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      fetch_frames(xb[(st + 1) & 1], X, m, e, valid, b0 + (st + 1) * kLpSub, B);   // the next eight
#pragma unroll
      for (int i = 0; i < kLpSub; ++i) {
        const int bl = st * kLpSub + i;
        float sd = 0.f;
        if (bl < nb && valid) {
          float r = xb[st & 1][i];
#pragma unroll
          for (int j = 0; j < K; ++j) r = fmaf(-u[j], ys[bl][j], r);
          float phi, c;
          cost_eval(r, cp, phi, c);
          const float gw = gs[bl] * wt;
          sd = gw * c * r;                         // g w phi'(r)
          if (dX) dX[(long long)(b0 + bl) * m + e] = sd;
          dmu = fmaf(gw, dphi_dmu(r, c, cp), dmu);
#pragma unroll
          for (int j = 0; j < K; ++j) du[j] = fmaf(-sd, ys[bl][j], du[j]);
        }
        sdl[bl][tid] = sd;   // 0 past the last frame or row
      }
    }
    __syncthreads();
    // dY share of this workgroup: -sum_rows s[b][row] u[row][j], a 16 x 256
    // by 256 x K product on the matrix cores: wavefront w multiplies its 64
    // rows in 16 steps of v_mfma_f32_16x16x4f32 (A = s[frame][4 rows], B =
    // u[4 rows][j], float32 accumulation), and the four wavefronts' 16 x 16
    // tiles are added in order in float64.  Frames past nb and columns past
    // K only reach outputs that are not written.
    {
      const int i16 = lane & 15, k4 = lane >> 4;
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < 16; ++st) {
        const int row = wv * 64 + st * 4 + k4;
        const float av = sdl[i16][row];
        const float bv = (i16 < K) ? uT[i16 < K ? i16 : 0][row] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) dyw[wv][k4 * 4 + v][i16] = (double)acc[v];   // D[frame][j]
    }
    __syncthreads();
    for (int q = tid; q < nb * K; q += kLpBlock) {
      const int bl = q / K, j = q - bl * K;
      double sum = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < kLpWaves; ++w2) sum += dyw[w2][bl][j];
      part[(size_t)((size_t)b0 * K + q) * nblk + blockIdx.x] = -sum;
    }
  }
  if (dU) {   // coalesced store of the workgroup's dU rows through LDS
    static_assert(CH * kLpPad >= kLpBlock * K, "dU staging fits the s buffer");
    __syncthreads();
    float* buf = &sdl[0][0];
#pragma unroll
    for (int j = 0; j < K; ++j) buf[tid * K + j] = du[j];
    __syncthreads();
    for (int q = tid; q < nrow * K; q += kLpBlock) dU[e0 * K + q] = buf[q];
  }
  const float dm = wave_sum(dmu);
  if (lane == 0) redm[wv] = (double)dm;
  __syncthreads();
  if (tid == 0) {
    double v = 0.0;
    for (int q = 0; q < kLpWaves; ++q) v += redm[q];
    part[(size_t)B * K * nblk + blockIdx.x] = v;
  }
}

// out[q] = sum over workgroups b of part[q * nblk + b] (q < n0 to out0, the
// rest to out1), one workgroup per output: thread t adds partials t, t + 256,
// ... in order (contiguous, coalesced), then fixed-order wavefront and
// workgroup sums.
__global__ __launch_bounds__(256) void lpcost_finish(const double* __restrict__ part, int nblk, int n, int n0,
                                                     float* __restrict__ out0, float* __restrict__ out1) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  const int t = threadIdx.x;
  const double* row = part + (size_t)q * nblk;
  double s = 0.0;
  for (int b = t; b < nblk; b += 256) s += row[b];
  s = wave_sum(s);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  if (t == 0) {
    const double v = (red[0] + red[1]) + (red[2] + red[3]);
    if (q < n0) {
      if (out0) out0[q] = (float)v;
    } else if (out1) {
      out1[q - n0] = (float)v;
    }
  }
}

static int lp_blocks(int m) { return (m + kLpBlock - 1) / kLpBlock; }

// Partial sums of pros_lpcost_bwd_noalloc: a file-scope device array, one
// copy per GPU.  Calls on one GPU share it (they must not overlap).
static __device__ __align__(256) unsigned char scratch[PROS_LPCOST_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];   // device address of `scratch`, per device

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.
static pros_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return prost_host::set_error(PROS_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return prost_host::set_error(PROS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PROS_OK;
}

}  // namespace prost

using namespace prost;

#define PROST_K_SWITCH(k, CALL)                                                              \
  switch (k) {                                                                               \
    case 1: { constexpr int KK = 1; CALL; } break;   case 2: { constexpr int KK = 2; CALL; } break;   \
    case 3: { constexpr int KK = 3; CALL; } break;   case 4: { constexpr int KK = 4; CALL; } break;   \
    case 5: { constexpr int KK = 5; CALL; } break;   case 6: { constexpr int KK = 6; CALL; } break;   \
    case 7: { constexpr int KK = 7; CALL; } break;   case 8: { constexpr int KK = 8; CALL; } break;   \
    case 9: { constexpr int KK = 9; CALL; } break;   case 10: { constexpr int KK = 10; CALL; } break; \
    case 11: { constexpr int KK = 11; CALL; } break; case 12: { constexpr int KK = 12; CALL; } break; \
    case 13: { constexpr int KK = 13; CALL; } break; case 14: { constexpr int KK = 14; CALL; } break; \
    case 15: { constexpr int KK = 15; CALL; } break; case 16: { constexpr int KK = 16; CALL; } break; \
    default: break;                                                                          \
  }

extern "C" {

size_t pros_lpcost_workspace_size(int32_t m, int32_t k, int32_t B) {
  if (m <= 0 || k < 1 || k > PROS_MAX_K || B <= 0) return 0;
  const size_t nblk = (size_t)lp_blocks(m);
  return sizeof(double) * (nblk * ((size_t)B * k + 1) + nblk * (size_t)B) + 256;
}

static pros_status lp_check(const float* U, const float* Y, const float* X, const float* mu, int32_t m, int32_t k,
                            int32_t B, int32_t cost, float p, void* ws, size_t ws_bytes) {
  if (!U || !Y || !X || !mu || !ws) return prost_host::set_error(PROS_EINVAL, "NULL tensor or workspace");
  if (m <= 0 || B <= 0 || k < 1 || k > PROS_MAX_K) return prost_host::set_error(PROS_EINVAL, "bad sizes m=%d k=%d B=%d", m, k, B);
  if (cost != PROS_COST_LP && cost != PROS_COST_LOG) return prost_host::set_error(PROS_EINVAL, "unknown cost");
  if (cost == PROS_COST_LP && !(p > 0.f && p <= 2.f)) return prost_host::set_error(PROS_EINVAL, "p must be in (0, 2]");
  if (ws_bytes < pros_lpcost_workspace_size(m, k, B)) return prost_host::set_error(PROS_EINVAL, "workspace too small");
  return PROS_OK;
}

pros_status pros_lpcost_fwd(const float* U, const float* Y, const float* X, const float* w, const float* mu,
                            int32_t m, int32_t k, int32_t B, int32_t cost, float p, float* f, void* workspace,
                            size_t workspace_bytes, void* hip_stream) {
  pros_status st = lp_check(U, Y, X, mu, m, k, B, cost, p, workspace, workspace_bytes);
  if (st != PROS_OK) return st;
  if (!f) return prost_host::set_error(PROS_EINVAL, "f is NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  double* part = (double*)workspace;
  const int nblk = lp_blocks(m);
  const int form = (cost == PROS_COST_LOG) ? 1 : 0;
  PROST_K_SWITCH(k, hipLaunchKernelGGL((lpcost_fwd_kernel<KK>), dim3(nblk), dim3(kLpBlock), 0, s, U, Y, X, w, m, B,
                                       form, p, mu, part));
  hipLaunchKernelGGL(lpcost_finish, dim3(B), dim3(256), 0, s, (const double*)part, nblk, B, B, f, (float*)nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "lpcost forward launch: %s", hipGetErrorString(e));
  return PROS_OK;
}

static pros_status lp_bwd_launch(const float* U, const float* Y, const float* X, const float* w, const float* mu,
                                 int32_t m, int32_t k, int32_t B, int32_t cost, float p, const float* gout,
                                 float* dX, float* dU, float* dY, float* dmu, double* part, hipStream_t s) {
  const int nblk = lp_blocks(m);
  const int form = (cost == PROS_COST_LOG) ? 1 : 0;
  if (form)
    PROST_K_SWITCH(k, hipLaunchKernelGGL((lpcost_bwd_kernel<KK, 1>), dim3(nblk), dim3(kLpBlock), 0, s, U, Y, X, w, m,
                                         B, p, mu, gout, dX, dU, part))
  else
    PROST_K_SWITCH(k, hipLaunchKernelGGL((lpcost_bwd_kernel<KK, 0>), dim3(nblk), dim3(kLpBlock), 0, s, U, Y, X, w, m,
                                         B, p, mu, gout, dX, dU, part))
  if (dY || dmu) {
    const int n = B * k + 1;
    hipLaunchKernelGGL(lpcost_finish, dim3(n), dim3(256), 0, s, (const double*)part, nblk, n, B * k, dY, dmu);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "lpcost backward launch: %s", hipGetErrorString(e));
  return PROS_OK;
}

pros_status pros_lpcost_bwd(const float* U, const float* Y, const float* X, const float* w, const float* mu,
                            int32_t m, int32_t k, int32_t B, int32_t cost, float p, const float* gout, float* dX,
                            float* dU, float* dY, float* dmu, void* workspace, size_t workspace_bytes,
                            void* hip_stream) {
  pros_status st = lp_check(U, Y, X, mu, m, k, B, cost, p, workspace, workspace_bytes);
  if (st != PROS_OK) return st;
  if (!gout) return prost_host::set_error(PROS_EINVAL, "gout is NULL");
  return lp_bwd_launch(U, Y, X, w, mu, m, k, B, cost, p, gout, dX, dU, dY, dmu, (double*)workspace,
                       (hipStream_t)hip_stream);
}

// The backward without a workspace argument: its partial sums live in
// `scratch`, a fixed device array of the library (one per GPU, held until
// the process ends).  Host code never passes the array's name to a kernel
// (in host code it is a stand-in, not a device address): the device address
// is taken once per device with hipGetSymbolAddress and kept here.
pros_status pros_lpcost_bwd_noalloc(const float* U, const float* Y, const float* X, const float* w, const float* mu,
                                    int32_t m, int32_t k, int32_t B, int32_t cost, float p, const float* gout,
                                    float* dX, float* dU, float* dY, float* dmu, void* hip_stream) {
  const size_t need = pros_lpcost_workspace_size(m, k, B);
  if (need == 0) return prost_host::set_error(PROS_EINVAL, "bad sizes m=%d k=%d B=%d", m, k, B);
  if (need > (size_t)PROS_LPCOST_SCRATCH_BYTES)
    return prost_host::set_error(PROS_EINVAL,
                                 "m=%d k=%d B=%d needs %zu bytes of partial sums; the fixed scratch holds %zu "
                                 "(use pros_lpcost_bwd with a workspace)",
                                 m, k, B, need, (size_t)PROS_LPCOST_SCRATCH_BYTES);
  void* part = nullptr;
  pros_status st = scratch_address(&part);
  if (st != PROS_OK) return st;
  st = lp_check(U, Y, X, mu, m, k, B, cost, p, part, (size_t)PROS_LPCOST_SCRATCH_BYTES);
  if (st != PROS_OK) return st;
  if (!gout) return prost_host::set_error(PROS_EINVAL, "gout is NULL");
  return lp_bwd_launch(U, Y, X, w, mu, m, k, B, cost, p, gout, dX, dU, dY, dmu, (double*)part,
                       (hipStream_t)hip_stream);
}

}  // extern "C"
