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
// a fixed order by a finishing kernel.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/prost.h"
#include "prost_device.hpp"
#include "prost_host.hpp"

namespace prost {

constexpr int kLpChunk = 32;   // frames of Y staged in LDS at a time

template <int K>
struct LpRows {
  static constexpr int R = (K <= 8) ? 8 : 4;   // rows per thread
};

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

template <int K>
__global__ __launch_bounds__(kBlock) void lpcost_fwd_kernel(const float* __restrict__ U, const float* __restrict__ Y,
                                                            const float* __restrict__ X, const float* __restrict__ w,
                                                            int m, int B, int form, float p, const float* __restrict__ mu_p,
                                                            double* __restrict__ part) {
  constexpr int R = LpRows<K>::R;
  __shared__ float ys[kLpChunk][K];
  __shared__ double red[kWaves][kLpChunk];
  const CostParams cp = make_cp(form, p, *mu_p);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long long row0 = (long long)blockIdx.x * kBlock * R;
  float u[R][K], wt[R];
  long long ex[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const long long e = row0 + s * kBlock + tid;
    ex[s] = e;
    wt[s] = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j) u[s][j] = 0.f;
    if (e < m) {
      wt[s] = w ? w[e] : 1.0f;
#pragma unroll
      for (int j = 0; j < K; ++j) u[s][j] = U[e * K + j];
    }
  }
  for (int b0 = 0; b0 < B; b0 += kLpChunk) {
    const int nb = min(kLpChunk, B - b0);
    __syncthreads();
    for (int q = tid; q < nb * K; q += kBlock) ys[q / K][q % K] = Y[(long long)(b0 + q / K) * K + q % K];
    __syncthreads();
    for (int bl = 0; bl < nb; ++bl) {
      const float* xb = X + (long long)(b0 + bl) * m;
      float acc = 0.f;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        if (ex[s] < m) {
          float r = xb[ex[s]];
#pragma unroll
          for (int j = 0; j < K; ++j) r = fmaf(-u[s][j], ys[bl][j], r);
          float phi, c;
          cost_eval(r, cp, phi, c);
          acc = fmaf(wt[s], phi, acc);
        }
      }
      acc = wave_sum(acc);
      if (lane == 0) red[wv][bl] = (double)acc;
    }
    __syncthreads();
    if (tid < nb) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) v += red[q][tid];
      part[(size_t)blockIdx.x * B + b0 + tid] = v;
    }
  }
}

__global__ void lpcost_fwd_finish(const double* __restrict__ part, int nblk, int B, float* __restrict__ f) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int q = 0; q < nblk; ++q) s += part[(size_t)q * B + b];
  f[b] = (float)s;
}

template <int K>
__global__ __launch_bounds__(kBlock) void lpcost_bwd_kernel(const float* __restrict__ U, const float* __restrict__ Y,
                                                            const float* __restrict__ X, const float* __restrict__ w,
                                                            int m, int B, int form, float p, const float* __restrict__ mu_p,
                                                            const float* __restrict__ gout, float* __restrict__ dX,
                                                            float* __restrict__ dU, double* __restrict__ part_dy,
                                                            double* __restrict__ part_dmu) {
  constexpr int R = LpRows<K>::R;
  __shared__ float ys[kLpChunk][K];
  __shared__ float gs[kLpChunk];
  __shared__ double red[kWaves][kLpChunk * K];
  __shared__ double redm[kWaves];
  const CostParams cp = make_cp(form, p, *mu_p);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long long row0 = (long long)blockIdx.x * kBlock * R;
  float u[R][K], du[R][K], wt[R];
  long long ex[R];
  float dmu = 0.f;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const long long e = row0 + s * kBlock + tid;
    ex[s] = e;
    wt[s] = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      u[s][j] = 0.f;
      du[s][j] = 0.f;
    }
    if (e < m) {
      wt[s] = w ? w[e] : 1.0f;
#pragma unroll
      for (int j = 0; j < K; ++j) u[s][j] = U[e * K + j];
    }
  }
  for (int b0 = 0; b0 < B; b0 += kLpChunk) {
    const int nb = min(kLpChunk, B - b0);
    __syncthreads();
    for (int q = tid; q < nb * K; q += kBlock) ys[q / K][q % K] = Y[(long long)(b0 + q / K) * K + q % K];
    if (tid < nb) gs[tid] = gout[b0 + tid];
    __syncthreads();
    for (int bl = 0; bl < nb; ++bl) {
      const long long boff = (long long)(b0 + bl) * m;
      const float g = gs[bl];
      float dy[K];
#pragma unroll
      for (int j = 0; j < K; ++j) dy[j] = 0.f;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        if (ex[s] < m) {
          float r = X[boff + ex[s]];
#pragma unroll
          for (int j = 0; j < K; ++j) r = fmaf(-u[s][j], ys[bl][j], r);
          float phi, c;
          cost_eval(r, cp, phi, c);
          const float sd = g * wt[s] * c * r;          // g w phi'(r)
          if (dX) dX[boff + ex[s]] = sd;
          dmu = fmaf(g * wt[s], dphi_dmu(r, c, cp), dmu);
#pragma unroll
          for (int j = 0; j < K; ++j) {
            du[s][j] = fmaf(-sd, ys[bl][j], du[s][j]);
            dy[j] = fmaf(-sd, u[s][j], dy[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float v = wave_sum(dy[j]);
        if (lane == 0) red[wv][bl * K + j] = (double)v;
      }
    }
    __syncthreads();
    for (int q = tid; q < nb * K; q += kBlock) {
      double v = 0.0;
#pragma unroll
      for (int wq = 0; wq < kWaves; ++wq) v += red[wq][q];
      part_dy[(size_t)blockIdx.x * B * K + (size_t)b0 * K + q] = v;
    }
  }
  if (dU) {
#pragma unroll
    for (int s = 0; s < R; ++s)
      if (ex[s] < m)
#pragma unroll
        for (int j = 0; j < K; ++j) dU[ex[s] * K + j] = du[s][j];
  }
  const float dm = wave_sum(dmu);
  if (lane == 0) redm[wv] = (double)dm;
  __syncthreads();
  if (tid == 0) {
    double v = 0.0;
    for (int q = 0; q < kWaves; ++q) v += redm[q];
    part_dmu[blockIdx.x] = v;
  }
}

__global__ void lpcost_bwd_finish(const double* __restrict__ part_dy, const double* __restrict__ part_dmu, int nblk,
                                  int BK, float* __restrict__ dY, float* __restrict__ dmu) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < BK && dY) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part_dy[(size_t)b * BK + q];
    dY[q] = (float)s;
  }
  if (q == 0 && dmu) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part_dmu[b];
    *dmu = (float)s;
  }
}

static int lp_blocks_k(int k, int m) {
  return (k <= 8) ? (int)((m + kBlock * 8LL - 1) / (kBlock * 8LL)) : (int)((m + kBlock * 4LL - 1) / (kBlock * 4LL));
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
  const size_t nblk = (size_t)lp_blocks_k(k, m);
  return sizeof(double) * (nblk * (size_t)B * k + nblk * (size_t)B + nblk) + 256;
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
  const int nblk = lp_blocks_k(k, m);
  const int form = (cost == PROS_COST_LOG) ? 1 : 0;
  PROST_K_SWITCH(k, hipLaunchKernelGGL((lpcost_fwd_kernel<KK>), dim3(nblk), dim3(kBlock), 0, s, U, Y, X, w, m, B,
                                       form, p, mu, part));
  hipLaunchKernelGGL(lpcost_fwd_finish, dim3((B + 255) / 256), dim3(256), 0, s, (const double*)part, nblk, B, f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "lpcost forward launch: %s", hipGetErrorString(e));
  return PROS_OK;
}

pros_status pros_lpcost_bwd(const float* U, const float* Y, const float* X, const float* w, const float* mu,
                            int32_t m, int32_t k, int32_t B, int32_t cost, float p, const float* gout, float* dX,
                            float* dU, float* dY, float* dmu, void* workspace, size_t workspace_bytes,
                            void* hip_stream) {
  pros_status st = lp_check(U, Y, X, mu, m, k, B, cost, p, workspace, workspace_bytes);
  if (st != PROS_OK) return st;
  if (!gout) return prost_host::set_error(PROS_EINVAL, "gout is NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  const int nblk = lp_blocks_k(k, m);
  double* part_dy = (double*)workspace;
  double* part_dmu = part_dy + (size_t)nblk * B * k;
  const int form = (cost == PROS_COST_LOG) ? 1 : 0;
  PROST_K_SWITCH(k, hipLaunchKernelGGL((lpcost_bwd_kernel<KK>), dim3(nblk), dim3(kBlock), 0, s, U, Y, X, w, m, B,
                                       form, p, mu, gout, dX, dU, part_dy, part_dmu));
  const int BK = B * k;
  hipLaunchKernelGGL(lpcost_bwd_finish, dim3((BK + 255) / 256), dim3(256), 0, s, (const double*)part_dy,
                     (const double*)part_dmu, nblk, BK, dY, dmu);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "lpcost backward launch: %s", hipGetErrorString(e));
  return PROS_OK;
}

}  // extern "C"
