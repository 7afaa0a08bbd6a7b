// Segmentation quality against a ground-truth mask (the measures of Sec. 5:
// Recall, Specificity, FPR, FNR, PWC, Precision and F-measure follow from
// the four counts) and the delta sweep behind the ROC curves of Sec. 5.
// Counts are integers accumulated with atomics: order-independent, exact.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/prost.h"
#include "prost_device.hpp"
#include "prost_host.hpp"

namespace prost {

constexpr int kQBlock = 256;
constexpr int kMaxThresholds = 256;

// counts[0..3] += (TP, FP, TN, FN) of mask against truth over P pixels.
__global__ __launch_bounds__(kQBlock) void quality_count_kernel(const uint8_t* __restrict__ mask,
                                                                const uint8_t* __restrict__ truth, int P,
                                                                unsigned long long* __restrict__ counts) {
  __shared__ unsigned int c[4];
  if (threadIdx.x < 4) c[threadIdx.x] = 0u;
  __syncthreads();
  unsigned int tp = 0, fp = 0, tn = 0, fn = 0;
  for (int p = blockIdx.x * kQBlock + threadIdx.x; p < P; p += gridDim.x * kQBlock) {
    const bool m = mask[p] != 0, t = truth[p] != 0;
    tp += (m && t);
    fp += (m && !t);
    tn += (!m && !t);
    fn += (!m && t);
  }
  atomicAdd(&c[0], tp);
  atomicAdd(&c[1], fp);
  atomicAdd(&c[2], tn);
  atomicAdd(&c[3], fn);
  __syncthreads();
  if (threadIdx.x < 4 && c[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)c[threadIdx.x]);
}

// counts[4 i + 0..3] += (TP, FP, TN, FN) of the labels [s_p >= thr[i]],
// s_p = max_c score[c P + p], against truth.
__global__ __launch_bounds__(kQBlock) void roc_count_kernel(const float* __restrict__ score,
                                                            const uint8_t* __restrict__ truth, int P, int C,
                                                            const float* __restrict__ thr, int T,
                                                            unsigned long long* __restrict__ counts) {
  __shared__ unsigned int c[kMaxThresholds * 4];
  __shared__ float th[kMaxThresholds];
  for (int q = threadIdx.x; q < 4 * T; q += kQBlock) c[q] = 0u;
  for (int q = threadIdx.x; q < T; q += kQBlock) th[q] = thr[q];
  __syncthreads();
  for (int p = blockIdx.x * kQBlock + threadIdx.x; p < P; p += gridDim.x * kQBlock) {
    float s = score[p];
    for (int ch = 1; ch < C; ++ch) s = fmaxf(s, score[(size_t)ch * P + p]);
    const int t = truth[p] != 0;
    for (int i = 0; i < T; ++i) {
      const int m = s >= th[i];
      atomicAdd(&c[4 * i + (m ? (t ? 0 : 1) : (t ? 3 : 2))], 1u);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 4 * T; q += kQBlock)
    if (c[q]) atomicAdd(&counts[q], (unsigned long long)c[q]);
}

}  // namespace prost

using namespace prost;

static int q_grid(int P) {
  const int g = (P + kQBlock - 1) / kQBlock;
  return g < 1024 ? g : 1024;
}

extern "C" {

pros_status pros_quality_counts(pros_handle* h, const uint8_t* truth, int32_t on_device, int32_t filtered,
                                int64_t* counts) {
  pros_status st = prost_host::check_usable(h);
  if (st != PROS_OK) return st;
  if (!truth || !counts) return prost_host::set_error(PROS_EINVAL, "truth or counts is NULL");
  if (filtered) {
    st = prost_host::refresh_mask(h);
    if (st != PROS_OK) return st;
  }
  uint8_t* tdev = nullptr;
  unsigned long long* cdev = nullptr;
  hipError_t e = hipMalloc((void**)&cdev, 4 * sizeof(unsigned long long));
  if (e == hipSuccess && !on_device) e = hipMalloc((void**)&tdev, (size_t)h->P);
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(tdev, truth, (size_t)h->P, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(cdev, 0, 4 * sizeof(unsigned long long), h->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(quality_count_kernel, dim3(q_grid(h->P)), dim3(kQBlock), 0, h->stream,
                       (const uint8_t*)(filtered ? h->mask : h->lab), on_device ? truth : tdev, h->P, cdev);
    e = hipGetLastError();
  }
  unsigned long long hc[4] = {0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hc, cdev, sizeof(hc), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (tdev) (void)hipFree(tdev);
  if (cdev) (void)hipFree(cdev);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "quality counts: %s", hipGetErrorString(e));
  for (int i = 0; i < 4; ++i) counts[i] = (int64_t)hc[i];
  return PROS_OK;
}

pros_status pros_roc_counts(const float* scores, const uint8_t* truth, int32_t P, int32_t C, const float* thresholds,
                            int32_t T, int64_t* counts, void* hip_stream) {
  if (!scores || !truth || !thresholds || !counts)
    return prost_host::set_error(PROS_EINVAL, "NULL scores, truth, thresholds or counts");
  if (P < 1 || C < 1 || C > 4 || T < 1 || T > kMaxThresholds)
    return prost_host::set_error(PROS_EINVAL, "bad sizes P=%d C=%d T=%d (T <= %d)", P, C, T, kMaxThresholds);
  hipStream_t s = (hipStream_t)hip_stream;
  float* tdev = nullptr;
  unsigned long long* cdev = nullptr;
  const size_t nc = (size_t)4 * T;
  hipError_t e = hipMalloc((void**)&tdev, sizeof(float) * T);
  if (e == hipSuccess) e = hipMalloc((void**)&cdev, sizeof(unsigned long long) * nc);
  if (e == hipSuccess) e = hipMemcpyAsync(tdev, thresholds, sizeof(float) * T, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(cdev, 0, sizeof(unsigned long long) * nc, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(roc_count_kernel, dim3(q_grid(P)), dim3(kQBlock), 0, s, scores, truth, P, C,
                       (const float*)tdev, T, cdev);
    e = hipGetLastError();
  }
  std::vector<unsigned long long> hc(nc, 0ull);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), cdev, sizeof(unsigned long long) * nc, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (tdev) (void)hipFree(tdev);
  if (cdev) (void)hipFree(cdev);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "roc counts: %s", hipGetErrorString(e));
  for (size_t i = 0; i < nc; ++i) counts[i] = (int64_t)hc[i];
  return PROS_OK;
}

}  // extern "C"
