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

// ---------------------------------------------------------------------------
// Initialization of U (Sec. 3.4): the orthonormal factor of the reduced QR
// decomposition of a random m x k matrix A.  A is drawn on the device from a
// counter-based generator (Philox4x32-10, Salmon et al., SC'11) with
// Box-Muller, so that the draw is reproducible per (seed, stream) and
// independent of the launch; Q = A R^{-1} comes from CholeskyQR2 in float64
// (two passes of G = A^T A, G = R^T R, A <- A R^{-1}), whose R has a
// positive diagonal, i.e. the QR factor with diag(R) > 0.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void philox_round10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned long long a = (unsigned long long)c[0] * 0xD2511F53ull;
    const unsigned long long b = (unsigned long long)c[2] * 0xCD9E8D57ull;
    const uint32_t w0 = (uint32_t)(b >> 32) ^ c[1] ^ k0;
    const uint32_t w2 = (uint32_t)(a >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)b;
    c[3] = (uint32_t)a;
    c[0] = w0;
    c[2] = w2;
  }
}

// Entry e = j m + i of the column-major m x k matrix: pair q = e / 2 is one
// generator call with counter (q lo, q hi, stream, 0) and key (seed lo, seed
// hi); its two 64-bit words give uniforms (z / 2^11 + 1/2) 2^-53 in (0, 1),
// and Box-Muller gives the cosine (even e) and sine (odd e) normal variates.
__global__ __launch_bounds__(256) void gauss_fill(double* __restrict__ A, long long n, unsigned long long seed,
                                                  uint32_t stream_index) {
  const long long npair = (n + 1) / 2;
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < npair; q += (long long)gridDim.x * 256) {
    uint32_t c[4] = {(uint32_t)q, (uint32_t)((unsigned long long)q >> 32), stream_index, 0u};
    philox_round10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const unsigned long long za = (((unsigned long long)c[0] << 32) | c[1]) >> 11;
    const unsigned long long zb = (((unsigned long long)c[2] << 32) | c[3]) >> 11;
    const double ua = ((double)za + 0.5) * 0x1p-53;
    const double ub = ((double)zb + 0.5) * 0x1p-53;
    const double rad = sqrt(-2.0 * log(ua));
    const double ang = 2.0 * 3.141592653589793 * ub;
    A[2 * q] = rad * cos(ang);
    if (2 * q + 1 < n) A[2 * q + 1] = rad * sin(ang);
  }
}

// One wavefront: G from the partials (fixed order), Cholesky G = R^T R (R
// upper, by lane 0 in float64), R^{-1} (upper) into ws (k x k, stride 16).
// A non-positive pivot (rank-deficient A) sets *bad and leaves ws = I.
__global__ __launch_bounds__(64) void qr_chol_inv(const double* __restrict__ part, int nblocks, int k,
                                                  double* __restrict__ ws, int* __restrict__ bad) {
  __shared__ double G[kMaxK][kMaxK];
  __shared__ double R[kMaxK][kMaxK];
  __shared__ double Ri[kMaxK][kMaxK];
  const int l = threadIdx.x;
  for (int q = l; q < kGramPairs; q += 64) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * kGramPairs + q];
    int t = q, i = 0;
    while (i < k && t >= k - i) { t -= k - i; ++i; }
    if (i < k) { G[i][i + t] = s; G[i + t][i] = s; }
  }
  __syncthreads();
  if (l == 0) {
    int ok = 1;
    for (int i = 0; i < k && ok; ++i) {
      for (int j = 0; j < k; ++j) R[i][j] = 0.0;
      double d = G[i][i];
      for (int r = 0; r < i; ++r) d -= R[r][i] * R[r][i];
      if (!(d > 0.0)) { ok = 0; break; }
      const double rii = sqrt(d);
      R[i][i] = rii;
      for (int j = i + 1; j < k; ++j) {
        double v = G[i][j];
        for (int r = 0; r < i; ++r) v -= R[r][i] * R[r][j];
        R[i][j] = v / rii;
      }
    }
    // R^{-1} by back substitution, column by column
    for (int j = k - 1; ok && j >= 0; --j) {
      for (int i = 0; i < k; ++i) Ri[i][j] = 0.0;
      Ri[j][j] = 1.0 / R[j][j];
      for (int i = j - 1; i >= 0; --i) {
        double v = 0.0;
        for (int r = i + 1; r <= j; ++r) v += R[i][r] * Ri[r][j];
        Ri[i][j] = -v / R[i][i];
      }
    }
    for (int i = 0; i < kMaxK; ++i)
      for (int j = 0; j < kMaxK; ++j)
        ws[i * kMaxK + j] = (i < k && j < k) ? (ok ? Ri[i][j] : (i == j ? 1.0 : 0.0)) : 0.0;
    if (!ok) *bad = 1;
  }
}

// a_e <- a_e R^{-1} for every row of the float64 m x k matrix (in place).
template <int K>
__global__ __launch_bounds__(256) void qr_apply_f64(double* __restrict__ A, long long m,
                                                    const double* __restrict__ ws) {
  __shared__ double M[K][K];
  for (int q = threadIdx.x; q < K * K; q += 256) M[q / K][q % K] = ws[(q / K) * kMaxK + (q % K)];
  __syncthreads();
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < m; e += (long long)gridDim.x * 256) {
    int z = 0;
    asm volatile("" : "+v"(z));   // keeps the reads of M in the loop (see gram_apply)
    const double* Ml = &M[0][0] + z;
    double a[K];
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = A[(long long)i * m + e];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i <= j; ++i) s = fma(a[i], Ml[i * K + j], s);   // R^{-1} is upper triangular
      A[(long long)j * m + e] = s;
    }
  }
}

// U (storage type, leading dimension ldU) <- A rounded to nearest.
template <typename TS>
__global__ __launch_bounds__(256) void store_subspace(TS* __restrict__ U, long long ldU, const double* __restrict__ A,
                                                      long long m, int k) {
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < m * k; q += (long long)gridDim.x * 256) {
    const long long j = q / m, e = q - j * m;
    st_elem(U, j * ldU + e, (float)A[q]);
  }
}

static hipError_t qr_apply_launch(int k, double* A, long long m, const double* ws, int blocks, hipStream_t st) {
#define PROST_QR_CASE(KK) \
  case KK: hipLaunchKernelGGL((qr_apply_f64<KK>), dim3(blocks), dim3(256), 0, st, A, m, ws); break;
  switch (k) {
    PROST_QR_CASE(1) PROST_QR_CASE(2) PROST_QR_CASE(3) PROST_QR_CASE(4)
    PROST_QR_CASE(5) PROST_QR_CASE(6) PROST_QR_CASE(7) PROST_QR_CASE(8)
    PROST_QR_CASE(9) PROST_QR_CASE(10) PROST_QR_CASE(11) PROST_QR_CASE(12)
    PROST_QR_CASE(13) PROST_QR_CASE(14) PROST_QR_CASE(15) PROST_QR_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef PROST_QR_CASE
  return hipGetLastError();
}

}  // namespace prost

// The seeded orthonormal m x k matrix into A (device, float64, column-major,
// leading dimension m), on `st`; synchronises.  Scratch is allocated here.
pros_status prost_random_subspace(unsigned long long seed, uint32_t stream_index, long long m, int k, double* A,
                                  hipStream_t st) {
  using namespace prost;
  if (m < k || k < 1 || k > PROS_MAX_K) return prost_host::set_error(PROS_EINVAL, "need 1 <= k <= min(m, %d)", PROS_MAX_K);
  const int nb = (int)std::min<long long>(kGramBlocks, (m + kGramRows - 1) / kGramRows);
  double* part = nullptr;
  hipError_t e = hipMalloc((void**)&part, sizeof(double) * ((size_t)kGramBlocks * kGramPairs + 256) + 64);
  if (e != hipSuccess) return prost_host::set_error(PROS_ENOMEM, "initialization scratch: %s", hipGetErrorString(e));
  double* ws = part + (size_t)kGramBlocks * kGramPairs;
  int* bad = (int*)(ws + 256);
  const long long n = m * k;
  const int fb = (int)std::min<long long>(4096, ((n + 1) / 2 + 255) / 256);
  const int ab = (int)std::min<long long>(2048, (m + 255) / 256);
  e = hipMemsetAsync(bad, 0, sizeof(int), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gauss_fill, dim3(fb), dim3(256), 0, st, A, n, seed, stream_index);
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
      hipLaunchKernelGGL((gram_partial<double>), dim3(nb), dim3(256), 0, st, (const double*)A, m, (int)m, k, part);
      hipLaunchKernelGGL(qr_chol_inv, dim3(1), dim3(64), 0, st, (const double*)part, nb, k, ws, bad);
      e = qr_apply_launch(k, A, m, ws, ab, st);
    }
  }
  int hbad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(part);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "initialization of U: %s", hipGetErrorString(e));
  if (hbad) return prost_host::set_error(PROS_EINVAL, "random matrix is rank-deficient (m=%lld, k=%d)", m, k);
  return PROS_OK;
}

// U of a handle <- the seeded orthonormal matrix rounded to the storage type.
pros_status prost_init_subspace(pros_handle* h, unsigned long long seed, uint32_t stream_index) {
  using namespace prost;
  double* A = nullptr;
  hipError_t e = hipMalloc((void**)&A, sizeof(double) * (size_t)h->m * h->k);
  if (e != hipSuccess) return prost_host::set_error(PROS_ENOMEM, "initialization buffer: %s", hipGetErrorString(e));
  pros_status st = prost_random_subspace(seed, stream_index, h->m, h->k, A, h->stream);
  if (st == PROS_OK) {
    const int sb = (int)std::min<long long>(4096, ((long long)h->m * h->k + 255) / 256);
    if (h->prm.storage == PROS_BF16)
      hipLaunchKernelGGL((store_subspace<uint16_t>), dim3(sb), dim3(256), 0, h->stream, (uint16_t*)h->U, h->ldU,
                         (const double*)A, (long long)h->m, h->k);
    else
      hipLaunchKernelGGL((store_subspace<float>), dim3(sb), dim3(256), 0, h->stream, (float*)h->U, h->ldU,
                         (const double*)A, (long long)h->m, h->k);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) st = prost_host::set_error(PROS_EHIP, "initialization store: %s", hipGetErrorString(e));
  }
  (void)hipFree(A);
  return st;
}

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
