// Video ingest around the tracker.  Sec. 5.1 re-samples every sequence to
// one small resolution (160 x 120) before pROST runs, and Sec. 5.3 notes
// that a mask computed at the small size is upsampled for evaluation.
//
//  * resample_area_kernel: interleaved 8-bit frames (H x W x C, as a video
//    decoder delivers them) -> the tracker's planar frame (C planes of
//    dst_h x dst_w, float32 or bfloat16), each destination pixel the mean of
//    the source over its footprint (area averaging).  The weights are exact
//    integers: in units of 1/dst_w a source column c spans
//    [c dst_w, (c+1) dst_w) and destination column j spans
//    [j src_w, (j+1) src_w), so every overlap is an integer and the weighted
//    sum is exact in 64-bit integers; one division and one scaling in float64
//    give the value, rounded once to float32 (then to nearest-even bfloat16).
//  * mask_upsample_kernel: nearest neighbour, output pixel (i, j) copies the
//    source pixel containing its centre, floor((2i+1) h / (2 out_h)).
//  * pros_ingest: pinned host slots, a copy stream and events so that the
//    H2D copy of frame n+1 overlaps the tracking of frame n.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/prost.h"
#include "prost_device.hpp"
#include "prost_host.hpp"

namespace prost {

constexpr int kRsBlock = 64;   // destination pixels per workgroup (small grids: spread over the CUs)
constexpr int kMaxRsChannels = 4;

__device__ __forceinline__ long long lmin(long long a, long long b) { return a < b ? a : b; }
__device__ __forceinline__ long long lmax(long long a, long long b) { return a > b ? a : b; }

template <typename TS>
__device__ __forceinline__ void store_entry(TS* dst, size_t i, double v);
template <>
__device__ __forceinline__ void store_entry<float>(float* dst, size_t i, double v) {
  dst[i] = (float)v;
}
template <>
__device__ __forceinline__ void store_entry<uint16_t>(uint16_t* dst, size_t i, double v) {
  const float f = (float)v;
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (values are finite)
  dst[i] = (uint16_t)(u >> 16);
}

template <typename TS>
__global__ __launch_bounds__(kRsBlock) void resample_area_kernel(const uint8_t* __restrict__ src, int sw, int sh,
                                                                 int C, long long stride, TS* __restrict__ dst,
                                                                 int dw, int dh, double scale) {
  const long long p = (long long)blockIdx.x * kRsBlock + threadIdx.x;
  const long long P = (long long)dw * dh;
  if (p >= P) return;
  const int i = (int)(p / dw), j = (int)(p - (long long)i * dw);
  // footprint in scaled units: rows [i sh, (i+1) sh) / dh, columns [j sw, (j+1) sw) / dw
  const long long ya = (long long)i * sh, yb = ya + sh;
  const long long xa = (long long)j * sw, xb = xa + sw;
  const int r0 = (int)(ya / dh), r1 = (int)((yb - 1) / dh);
  const int c0 = (int)(xa / dw), c1 = (int)((xb - 1) / dw);
  unsigned long long acc[kMaxRsChannels] = {0ull, 0ull, 0ull, 0ull};
  for (int r = r0; r <= r1; ++r) {
    const long long lo = (long long)r * dh, hi = lo + dh;
    const unsigned long long wr = (unsigned long long)(lmin(hi, yb) - lmax(lo, ya));
    const uint8_t* row = src + (long long)r * stride;
    for (int c = c0; c <= c1; ++c) {
      const long long clo = (long long)c * dw, chi = clo + dw;
      const unsigned long long w = wr * (unsigned long long)(lmin(chi, xb) - lmax(clo, xa));
      const uint8_t* px = row + (long long)c * C;
      for (int ch = 0; ch < C; ++ch) acc[ch] += w * px[ch];
    }
  }
  const double inv_area = 1.0 / ((double)sw * (double)sh);
  for (int ch = 0; ch < C; ++ch) store_entry<TS>(dst, (size_t)ch * P + p, (double)acc[ch] * inv_area * scale);
}

__global__ __launch_bounds__(256) void mask_upsample_kernel(const uint8_t* __restrict__ mask, int w, int h,
                                                            uint8_t* __restrict__ out, int ow, int oh) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= (long long)ow * oh) return;
  const long long i = q / ow, j = q - i * ow;
  const long long r = ((2 * i + 1) * h) / (2LL * oh), c = ((2 * j + 1) * w) / (2LL * ow);
  out[q] = mask[r * w + c];
}

}  // namespace prost

using namespace prost;

static pros_status check_resample_args(const uint8_t* src, int32_t sw, int32_t sh, int32_t C, int64_t stride,
                                       const void* dst, int32_t dtype, int32_t dw, int32_t dh) {
  if (!src || !dst) return prost_host::set_error(PROS_EINVAL, "src or dst is NULL");
  if (sw < 1 || sh < 1 || dw < 1 || dh < 1 || sw > 32768 || sh > 32768 || dw > 32768 || dh > 32768)
    return prost_host::set_error(PROS_EINVAL, "sizes must be 1..32768 (src %dx%d, dst %dx%d)", sw, sh, dw, dh);
  if (C < 1 || C > kMaxRsChannels) return prost_host::set_error(PROS_EINVAL, "channels must be 1..4");
  if (stride < (int64_t)sw * C) return prost_host::set_error(PROS_EINVAL, "row stride below width * channels");
  if (dtype != PROS_F32 && dtype != PROS_BF16) return prost_host::set_error(PROS_EINVAL, "unknown dst dtype");
  return PROS_OK;
}

static hipError_t launch_resample(const uint8_t* src, int sw, int sh, int C, long long stride, void* dst, int dtype,
                                  int dw, int dh, double scale, hipStream_t s) {
  const long long P = (long long)dw * dh;
  const dim3 grid((unsigned)((P + kRsBlock - 1) / kRsBlock));
  if (dtype == PROS_F32)
    hipLaunchKernelGGL(resample_area_kernel<float>, grid, dim3(kRsBlock), 0, s, src, sw, sh, C, stride, (float*)dst,
                       dw, dh, scale);
  else
    hipLaunchKernelGGL(resample_area_kernel<uint16_t>, grid, dim3(kRsBlock), 0, s, src, sw, sh, C, stride,
                       (uint16_t*)dst, dw, dh, scale);
  return hipGetLastError();
}

static hipError_t launch_upsample(const uint8_t* mask, int w, int h, uint8_t* out, int ow, int oh, hipStream_t s) {
  const long long n = (long long)ow * oh;
  hipLaunchKernelGGL(mask_upsample_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mask, w, h, out, ow,
                     oh);
  return hipGetLastError();
}

struct pros_ingest {
  pros_handle* h = nullptr;
  int sw = 0, sh = 0, slots = 0, next = 0;
  double scale = 1.0 / 255.0;
  size_t bytes = 0;
  hipStream_t copy = nullptr;
  std::vector<uint8_t*> host, dev;
  std::vector<hipEvent_t> copied, consumed;
  std::vector<char> copy_pending, read_pending;
  void* frame = nullptr;       // resampled frame (storage type, m entries)
  uint8_t* up = nullptr;       // upsampled mask (sw * sh)
  bool slot_taken = false;     // pros_ingest_slot handed out `next`
};

static void free_ingest(pros_ingest* g) {
  if (!g) return;
  if (g->copy) (void)hipStreamSynchronize(g->copy);
  if (g->h) (void)hipStreamSynchronize(g->h->stream);
  for (uint8_t* p : g->host)
    if (p) (void)hipHostFree(p);
  for (uint8_t* p : g->dev)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : g->copied)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : g->consumed)
    if (e) (void)hipEventDestroy(e);
  if (g->frame) (void)hipFree(g->frame);
  if (g->up) (void)hipFree(g->up);
  if (g->copy) (void)hipStreamDestroy(g->copy);
  delete g;
}

extern "C" {

pros_status pros_resample_rgb8(const uint8_t* src, int32_t src_w, int32_t src_h, int32_t channels,
                               int64_t src_row_stride, void* dst, int32_t dst_dtype, int32_t dst_w, int32_t dst_h,
                               double scale, void* hip_stream) {
  pros_status st = check_resample_args(src, src_w, src_h, channels, src_row_stride, dst, dst_dtype, dst_w, dst_h);
  if (st != PROS_OK) return st;
  if (!(scale > 0.0) || !std::isfinite(scale)) return prost_host::set_error(PROS_EINVAL, "scale must be > 0");
  hipError_t e = launch_resample(src, src_w, src_h, channels, src_row_stride, dst, dst_dtype, dst_w, dst_h, scale,
                                 (hipStream_t)hip_stream);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "resample launch: %s", hipGetErrorString(e));
  return PROS_OK;
}

pros_status pros_mask_upsample(const uint8_t* mask, int32_t width, int32_t height, uint8_t* out, int32_t out_w,
                               int32_t out_h, void* hip_stream) {
  if (!mask || !out) return prost_host::set_error(PROS_EINVAL, "mask or out is NULL");
  if (width < 1 || height < 1 || out_w < 1 || out_h < 1 || width > 32768 || height > 32768 || out_w > 32768 ||
      out_h > 32768)
    return prost_host::set_error(PROS_EINVAL, "sizes must be 1..32768");
  hipError_t e = launch_upsample(mask, width, height, out, out_w, out_h, (hipStream_t)hip_stream);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "upsample launch: %s", hipGetErrorString(e));
  return PROS_OK;
}

pros_status pros_ingest_init(pros_handle* h, int32_t src_w, int32_t src_h, int32_t slots, double scale,
                             pros_ingest** out) {
  if (!out) return prost_host::set_error(PROS_EINVAL, "out is NULL");
  *out = nullptr;
  pros_status st = prost_host::check_usable(h);
  if (st != PROS_OK) return st;
  if (src_w < 1 || src_h < 1 || src_w > 32768 || src_h > 32768)
    return prost_host::set_error(PROS_EINVAL, "source size must be 1..32768");
  if (slots < 1 || slots > 16) return prost_host::set_error(PROS_EINVAL, "slots must be 1..16");
  if (!(scale > 0.0) || !std::isfinite(scale)) return prost_host::set_error(PROS_EINVAL, "scale must be > 0");
  pros_ingest* g = new pros_ingest();
  g->h = h;
  g->sw = src_w;
  g->sh = src_h;
  g->slots = slots;
  g->scale = scale;
  g->bytes = (size_t)src_w * src_h * h->C;
  g->host.assign(slots, nullptr);
  g->dev.assign(slots, nullptr);
  g->copied.assign(slots, nullptr);
  g->consumed.assign(slots, nullptr);
  g->copy_pending.assign(slots, 0);
  g->read_pending.assign(slots, 0);
  hipError_t e = hipStreamCreateWithFlags(&g->copy, hipStreamNonBlocking);
  for (int s = 0; s < slots && e == hipSuccess; ++s) {
    e = hipHostMalloc((void**)&g->host[s], g->bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&g->dev[s], g->bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->copied[s], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->consumed[s], hipEventDisableTiming);
  }
  const size_t es = h->prm.storage == PROS_BF16 ? 2 : 4;
  if (e == hipSuccess) e = hipMalloc(&g->frame, es * (size_t)h->m);
  if (e == hipSuccess) e = hipMalloc((void**)&g->up, (size_t)src_w * src_h);
  if (e != hipSuccess) {
    free_ingest(g);
    return prost_host::set_error(PROS_ENOMEM, "ingest buffers: %s", hipGetErrorString(e));
  }
  *out = g;
  return PROS_OK;
}

pros_status pros_ingest_slot(pros_ingest* g, uint8_t** host_slot) {
  if (!g || !host_slot) return prost_host::set_error(PROS_EINVAL, "NULL argument");
  const int s = g->next;
  if (g->copy_pending[s]) {   // the last copy out of this pinned buffer must be done before it is rewritten
    hipError_t e = hipEventSynchronize(g->copied[s]);
    if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "ingest slot wait: %s", hipGetErrorString(e));
    g->copy_pending[s] = 0;
  }
  g->slot_taken = true;
  *host_slot = g->host[s];
  return PROS_OK;
}

pros_status pros_ingest_submit(pros_ingest* g) {
  if (!g) return prost_host::set_error(PROS_EINVAL, "NULL argument");
  if (!g->slot_taken) return prost_host::set_error(PROS_ESTATE, "fill a slot from pros_ingest_slot first");
  pros_handle* h = g->h;
  pros_status st = prost_host::check_usable(h);
  if (st != PROS_OK) return st;
  if (!h->state_set) return prost_host::set_error(PROS_ESTATE, "set U with pros_set_state before the first frame");
  const int s = g->next;
  hipError_t e = hipSuccess;
  // the device slot must have been read by the previous resample from it
  if (g->read_pending[s]) e = hipStreamWaitEvent(g->copy, g->consumed[s], 0);
  if (e == hipSuccess) e = hipMemcpyAsync(g->dev[s], g->host[s], g->bytes, hipMemcpyHostToDevice, g->copy);
  if (e == hipSuccess) e = hipEventRecord(g->copied[s], g->copy);
  if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, g->copied[s], 0);
  if (e == hipSuccess)
    e = launch_resample(g->dev[s], g->sw, g->sh, h->C, (long long)g->sw * h->C, g->frame, h->prm.storage,
                        h->prm.width, h->prm.height, g->scale, h->stream);
  if (e == hipSuccess) e = hipEventRecord(g->consumed[s], h->stream);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "ingest: %s", hipGetErrorString(e));
  g->copy_pending[s] = 1;
  g->read_pending[s] = 1;
  g->slot_taken = false;
  g->next = (s + 1) % g->slots;
  return pros_track_frame(h, g->frame, h->prm.storage, 1);
}

pros_status pros_ingest_push(pros_ingest* g, const uint8_t* frame_rgb8) {
  if (!g || !frame_rgb8) return prost_host::set_error(PROS_EINVAL, "NULL argument");
  uint8_t* slot = nullptr;
  pros_status st = pros_ingest_slot(g, &slot);
  if (st != PROS_OK) return st;
  std::memcpy(slot, frame_rgb8, g->bytes);
  return pros_ingest_submit(g);
}

pros_status pros_ingest_mask(pros_ingest* g, uint8_t* out, int32_t filtered, int32_t on_device) {
  if (!g || !out) return prost_host::set_error(PROS_EINVAL, "NULL argument");
  pros_handle* h = g->h;
  pros_status st = prost_host::check_usable(h);
  if (st != PROS_OK) return st;
  if (filtered) {
    st = prost_host::refresh_mask(h);
    if (st != PROS_OK) return st;
  }
  const uint8_t* src = filtered ? h->mask : h->lab;
  hipError_t e = launch_upsample(src, h->prm.width, h->prm.height, on_device ? out : g->up, g->sw, g->sh, h->stream);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "upsample launch: %s", hipGetErrorString(e));
  if (on_device) return PROS_OK;
  st = prost_host::sync_and_check(h);
  if (st != PROS_OK && st != PROS_EBADFRAME) return st;
  e = hipMemcpy(out, g->up, (size_t)g->sw * g->sh, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return prost_host::set_error(PROS_EHIP, "mask copy: %s", hipGetErrorString(e));
  return st;
}

void pros_ingest_destroy(pros_ingest* g) { free_ingest(g); }

}  // extern "C"
