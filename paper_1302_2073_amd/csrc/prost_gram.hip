// Re-orthonormalisation of U in float64 on the GPU (precision form).
//
// U drifts off the Stiefel manifold (Sec. 2.1, eq. stiefeldef) when it is
// stored in float32 or bfloat16.  Since only span(U) matters (Sec. 3.2), U is
// replaced by its nearest orthonormal matrix, the polar factor
//   U <- U G^{-1/2},  G = U^T U,
// and y <- G^{1/2} y keeps U y unchanged to first order.  Three kernels:
//   gram_partial: per-workgroup float64 partial sums of the upper triangle of G
//   gram_solve:   one wavefront: fixed-order sum, cyclic Jacobi eigensolver of
//                 G (float64), G^{-1/2}, G^{1/2}, y update
//   gram_apply:   u_e <- u_e G^{-1/2} row by row in float64, rounded to storage
#include <hip/hip_runtime.h>

#include "prost_device.hpp"
#include "prost_host.hpp"

namespace prost {

constexpr int kGramRows = 256;                  // rows per LDS tile
constexpr int kGramPairs = kMaxK * (kMaxK + 1) / 2;
constexpr int kGramBlocks = 512;

template <typename TS>
__global__ __launch_bounds__(256) void gram_partial(const TS* __restrict__ U, long long ldU, int m, int k,
                                                    double* __restrict__ part) {
  __shared__ double tile[kGramRows][kMaxK + 1];
  // pair index -> (i, j), i <= j, fixed for the launch
  int pi = -1, pj = -1;
  {
    int t = threadIdx.x, i = 0;
    while (i < k && t >= k - i) { t -= k - i; ++i; }
    if (i < k) { pi = i; pj = i + t; }
  }
  double acc = 0.0;
  for (long long r0 = (long long)blockIdx.x * kGramRows; r0 < m; r0 += (long long)gridDim.x * kGramRows) {
    const int rows = (int)min((long long)kGramRows, (long long)m - r0);
    __syncthreads();
    for (int j = 0; j < k; ++j) {
      const int e = threadIdx.x;
      tile[e][j] = (e < rows) ? (double)ld_elem(U, (long long)j * ldU + r0 + e) : 0.0;
    }
    __syncthreads();
    if (pi >= 0) {
      for (int e = 0; e < rows; ++e) acc = fma(tile[e][pi], tile[e][pj], acc);
    }
  }
  if (threadIdx.x < kGramPairs) part[(size_t)blockIdx.x * kGramPairs + threadIdx.x] = (pi >= 0) ? acc : 0.0;
}

// One wavefront.  ws layout: [0, 256) G^{-1/2} (row-major k x k, stride 16).
__global__ __launch_bounds__(64) void gram_solve(const double* __restrict__ part, int nblocks, int k,
                                                 double* __restrict__ y, double* __restrict__ ws) {
  __shared__ double A[kMaxK][kMaxK];
  __shared__ double Vm[kMaxK][kMaxK];
  __shared__ double cs[2];
  const int l = threadIdx.x;
  // fixed-order sum of the partials; thread owns pairs l, l+64, l+128
  for (int q = l; q < kGramPairs; q += 64) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * kGramPairs + q];
    int t = q, i = 0;
    while (i < k && t >= k - i) { t -= k - i; ++i; }
    if (i < k) { A[i][i + t] = s; A[i + t][i] = s; }
  }
  if (l < kMaxK)
    for (int j = 0; j < kMaxK; ++j) Vm[l][j] = (l == j) ? 1.0 : 0.0;
  __syncthreads();
  // cyclic Jacobi: rotate (p, q) pairs until the off-diagonal mass vanishes
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        if (i != j) off += A[i][j] * A[i][j];
        else dia += A[i][j] * A[i][j];
      }
    if (!(off > 1e-32 * dia)) break;
    for (int p = 0; p < k - 1; ++p) {
      for (int q = p + 1; q < k; ++q) {
        if (l == 0) {
          const double apq = A[p][q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0) {
            const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
          cs[0] = c;
          cs[1] = s;
        }
        __syncthreads();
        const double c = cs[0], s = cs[1];
        if (s != 0.0) {
          // A <- J^T A J with J the (p, q) rotation; V <- V J
          if (l < k) {
            const double akp = A[l][p], akq = A[l][q];
            A[l][p] = c * akp - s * akq;
            A[l][q] = s * akp + c * akq;
          }
          __syncthreads();
          if (l < k) {
            const double apk = A[p][l], aqk = A[q][l];
            A[p][l] = c * apk - s * aqk;
            A[q][l] = s * apk + c * aqk;
            const double vkp = Vm[l][p], vkq = Vm[l][q];
            Vm[l][p] = c * vkp - s * vkq;
            Vm[l][q] = s * vkp + c * vkq;
          }
        }
        __syncthreads();
      }
    }
  }
  // G^{-1/2} = V diag(lam^{-1/2}) V^T, G^{1/2} = V diag(lam^{1/2}) V^T
  __shared__ double lam[kMaxK];
  __shared__ double yn[kMaxK];
  __shared__ int degenerate;
  if (l == 0) degenerate = 0;
  __syncthreads();
  if (l < k) {
    lam[l] = A[l][l];
    if (!(A[l][l] > 1e-300)) atomicOr(&degenerate, 1);
  }
  __syncthreads();
  if (degenerate) {   // rank-deficient U: leave U and y unchanged
    if (l < k)
      for (int j = 0; j < k; ++j) ws[l * kMaxK + j] = (l == j) ? 1.0 : 0.0;
    return;
  }
  if (l < k) {
    for (int j = 0; j < k; ++j) {
      double mneg = 0.0;
      for (int i = 0; i < k; ++i) mneg += Vm[l][i] * Vm[j][i] / sqrt(lam[i]);
      ws[l * kMaxK + j] = mneg;
    }
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      double mpos = 0.0;
      for (int i = 0; i < k; ++i) mpos += Vm[l][i] * Vm[j][i] * sqrt(lam[i]);
      s += mpos * y[j];
    }
    yn[l] = s;
  }
  __syncthreads();
  if (l < k) y[l] = yn[l];
}

template <int K, typename TS>
__global__ __launch_bounds__(256) void gram_apply(TS* __restrict__ U, long long ldU, int m,
                                                  const double* __restrict__ ws) {
  __shared__ double M[K][K];
  for (int q = threadIdx.x; q < K * K; q += 256) M[q / K][q % K] = ws[(q / K) * kMaxK + (q % K)];
  __syncthreads();
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < m; e += (long long)gridDim.x * 256) {
    // an offset the compiler cannot see is zero: the LDS reads of M stay in
    // the loop instead of being hoisted into (K * K * 2) registers and spilled
    int z = 0;
    asm volatile("" : "+v"(z));
    const double* Ml = &M[0][0] + z;
    double u[K];
#pragma unroll
    for (int i = 0; i < K; ++i) u[i] = (double)ld_elem(U, (long long)i * ldU + e);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < K; ++i) s = fma(u[i], Ml[i * K + j], s);
      st_elem(U, (long long)j * ldU + e, (float)s);
    }
  }
}

template <typename TS>
static hipError_t launch_apply(int k, TS* U, long long ldU, int m, const double* ws, int blocks, hipStream_t st) {
#define PROST_APPLY_CASE(KK) \
  case KK: hipLaunchKernelGGL((gram_apply<KK, TS>), dim3(blocks), dim3(256), 0, st, U, ldU, m, ws); break;
  switch (k) {
    PROST_APPLY_CASE(1) PROST_APPLY_CASE(2) PROST_APPLY_CASE(3) PROST_APPLY_CASE(4)
    PROST_APPLY_CASE(5) PROST_APPLY_CASE(6) PROST_APPLY_CASE(7) PROST_APPLY_CASE(8)
    PROST_APPLY_CASE(9) PROST_APPLY_CASE(10) PROST_APPLY_CASE(11) PROST_APPLY_CASE(12)
    PROST_APPLY_CASE(13) PROST_APPLY_CASE(14) PROST_APPLY_CASE(15) PROST_APPLY_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef PROST_APPLY_CASE
  return hipGetLastError();
}

}  // namespace prost

pros_status prost_reorth_launch(pros_handle* h) {
  using namespace prost;
  const int nb = (int)std::min<long long>(kGramBlocks, ((long long)h->m + kGramRows - 1) / kGramRows);
  if (!h->reorth_ws) {
    hipError_t e = hipMalloc(&h->reorth_ws, sizeof(double) * ((size_t)kGramBlocks * kGramPairs + 256));
    if (e != hipSuccess) return prost_host::set_error(PROS_ENOMEM, "re-orthonormalisation workspace: %s", hipGetErrorString(e));
  }
  double* part = (double*)h->reorth_ws;
  double* ws = part + (size_t)kGramBlocks * kGramPairs;
  const bool bf = h->prm.storage == PROS_BF16;
  if (bf)
    hipLaunchKernelGGL((gram_partial<uint16_t>), dim3(nb), dim3(256), 0, h->stream, (const uint16_t*)h->U, h->ldU, h->m, h->k, part);
  else
    hipLaunchKernelGGL((gram_partial<float>), dim3(nb), dim3(256), 0, h->stream, (const float*)h->U, h->ldU, h->m, h->k, part);
  hipLaunchKernelGGL(gram_solve, dim3(1), dim3(64), 0, h->stream, (const double*)part, nb, h->k, h->y, ws);
  const int ab = (int)std::min<long long>(2048, ((long long)h->m + 255) / 256);
  hipError_t e = bf ? launch_apply<uint16_t>(h->k, (uint16_t*)h->U, h->ldU, h->m, ws, ab, h->stream)
                    : launch_apply<float>(h->k, (float*)h->U, h->ldU, h->m, ws, ab, h->stream);
  if (e != hipSuccess) {
    h->broken = true;
    h->broken_status = PROS_EHIP;
    return prost_host::set_error(PROS_EHIP, "re-orthonormalisation launch failed: %s", hipGetErrorString(e));
  }
  return PROS_OK;
}
