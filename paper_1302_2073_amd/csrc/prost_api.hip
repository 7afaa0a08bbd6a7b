// C ABI of the pROST per-frame hot path: handle management, state exchange,
// launch of the persistent frame kernel.  No torch types cross this boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <vector>

#include "../../include/prost.h"
#include "prost_frame.hpp"
#include "prost_kernels.hpp"
#include "prost_host.hpp"

using prost::FrameArgs;

namespace {
thread_local char g_last_error[512] = "";
}  // namespace

pros_status prost_host::set_error(pros_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return s;
}

#define fail prost_host::set_error

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      return fail(PROS_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                  __FILE__, __LINE__);                                                \
    }                                                                                 \
  } while (0)



namespace prost_host {

double effective_delta(const pros_params& p) {
  if (p.delta > 0.0) return p.delta;
  if (p.cost == PROS_COST_LOG) return std::sqrt(p.mu);
  return std::sqrt(p.mu / (1.0 - p.p));
}

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_to_f32(uint16_t b) {
  uint32_t u = ((uint32_t)b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

}  // namespace prost_host

using namespace prost_host;

// Mask of the latest frame on demand: 3x3 median of the raw labels and the
// count of foreground labels (integer atomics: order-independent).
__global__ void median_kernel(const uint8_t* __restrict__ lab, uint8_t* __restrict__ mask, int W, int H, int P,
                              long long* __restrict__ fg) {
  __shared__ unsigned cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int p0 = blockIdx.x * blockDim.x;
  const int npx = min((int)blockDim.x, P - p0);
  prost::median3x3_range(lab, mask, W, H, p0, npx);
  if ((int)threadIdx.x < npx && lab[p0 + threadIdx.x]) atomicAdd(&cnt, 1u);
  __syncthreads();
  if (threadIdx.x == 0 && cnt) atomicAdd((unsigned long long*)fg, (unsigned long long)cnt);
}

pros_status prost_host::refresh_mask(pros_handle* h) {
  if (!h->mask_stale) return PROS_OK;
  HIP_TRY(hipMemsetAsync(&h->stats->fg_pixels, 0, sizeof(long long), h->stream));
  hipLaunchKernelGGL(median_kernel, dim3((h->P + 255) / 256), dim3(256), 0, h->stream, (const uint8_t*)h->lab,
                     h->mask, h->prm.width, h->prm.height, h->P, (long long*)&h->stats->fg_pixels);
  HIP_TRY(hipGetLastError());
  h->mask_stale = false;
  return PROS_OK;
}

// Entry points keep the C linkage of their declarations in prost.h.

const char* pros_strerror(pros_status s) {
  switch (s) {
    case PROS_OK: return "ok";
    case PROS_EINVAL: return "invalid argument";
    case PROS_ENOMEM: return "out of memory";
    case PROS_EHIP: return "HIP runtime error";
    case PROS_ESTATE: return "invalid handle state";
    case PROS_EBADFRAME: return "frame contains NaN or Inf";
    case PROS_ETIMEOUT: return "persistent kernel timed out";
    case PROS_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char* pros_last_error(void) { return g_last_error; }

pros_status pros_params_default(pros_params* out, int32_t width, int32_t height, int32_t channels) {
  if (!out) return fail(PROS_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->width = width;
  out->height = height;
  out->channels = channels;
  out->k = 15;
  out->cg_iters = 5;
  out->cost = PROS_COST_LP;
  out->p = 0.25;
  out->mu = 1e-3;
  out->delta = 0.0;
  out->omega = 5e-5;
  out->t_init = 5e-3;
  out->t_min = 1e-4;
  out->i_init = 100;
  out->storage = PROS_F32;
  out->reorth_every = 0;
  out->labels_after_update = 1;
  out->weights_from_filtered = 0;
  return PROS_OK;
}

pros_status pros_validate(const pros_params* p) {
  if (!p) return fail(PROS_EINVAL, "params is NULL");
  if (p->width <= 0 || p->height <= 0) return fail(PROS_EINVAL, "width/height must be positive");
  if (p->channels < 1 || p->channels > 4) return fail(PROS_EINVAL, "channels must be 1..4");
  const long long P = (long long)p->width * p->height;
  if (P * p->channels > (1LL << 30)) return fail(PROS_EINVAL, "frame too large");
  if (p->k < 1 || p->k > PROS_MAX_K) return fail(PROS_EINVAL, "k must be 1..%d", PROS_MAX_K);
  if (p->k > P * p->channels) return fail(PROS_EINVAL, "k exceeds the frame size");
  if (p->cg_iters < 1 || p->cg_iters > PROS_MAX_CG) return fail(PROS_EINVAL, "cg_iters must be 1..%d", PROS_MAX_CG);
  if (p->cost != PROS_COST_LP && p->cost != PROS_COST_LOG) return fail(PROS_EINVAL, "unknown cost");
  if (p->cost == PROS_COST_LP && !(p->p > 0.0 && p->p <= 2.0)) return fail(PROS_EINVAL, "p must be in (0, 2]");
  if (!(p->mu > 0.0) || !std::isfinite(p->mu)) return fail(PROS_EINVAL, "mu must be > 0");
  if (p->cost == PROS_COST_LP && p->delta <= 0.0 && !(p->p < 1.0))
    return fail(PROS_EINVAL, "delta from mu needs p < 1");
  if (!std::isfinite(p->delta)) return fail(PROS_EINVAL, "delta must be finite");
  if (!(p->omega >= 0.0 && p->omega <= 1.0)) return fail(PROS_EINVAL, "omega must be in [0, 1]");
  if (!(p->t_init > 0.0) || !(p->t_min > 0.0) || !std::isfinite(p->t_init) || !std::isfinite(p->t_min))
    return fail(PROS_EINVAL, "t_init and t_min must be > 0");
  if (p->i_init < 1) return fail(PROS_EINVAL, "i_init must be >= 1");
  if (p->storage != PROS_F32 && p->storage != PROS_BF16) return fail(PROS_EINVAL, "unknown storage type");
  if (p->reorth_every < 0) return fail(PROS_EINVAL, "reorth_every must be >= 0");
  if (p->labels_after_update != 0 && p->labels_after_update != 1) return fail(PROS_EINVAL, "labels_after_update must be 0/1");
  if (p->weights_from_filtered != 0 && p->weights_from_filtered != 1) return fail(PROS_EINVAL, "weights_from_filtered must be 0/1");
  if (p->preprocess != 0 && p->preprocess != 1) return fail(PROS_EINVAL, "preprocess must be 0 or 1");
  if (p->ysolve < 0 || p->ysolve > 2) return fail(PROS_EINVAL, "ysolve must be 0 (CG), 1 (gradient descent) or 2 (IRLS)");
  if (p->ysolve == 2 && p->storage != PROS_F32) return fail(PROS_EINVAL, "the IRLS step needs float32 storage");
  return PROS_OK;
}

void prost_host::free_handle(pros_handle* h) {
  if (!h) return;
  void* ptrs[] = {h->U, h->xstage, h->lab, h->mask, h->y, h->nframe, h->stats, h->part, h->sync, h->reorth_ws,
                  h->pre_mean, h->pre_m2, h->pre_stat, (void*)h->seq, h->stream_ws};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete h;
}

int prost_host::tile_pixels(int storage, int NR, int channels, double scale, int threads) {
  const int full = threads * NR / channels;
  int tpw = (int)std::floor(threads * NR * scale / channels);
  tpw = std::max(1, std::min(tpw, full));
  if (storage == PROS_BF16 && tpw > 1) tpw &= ~1;
  return tpw;
}

// The frame's steps reduce H with the gradient (IRLS, or CG under the
// one-exchange curvature schedule): wide exchange slots, optional-feature
// kernels.
static bool wide_exchange(const pros_handle* h) { return h->prm.ysolve == 2 || h->curv == 1; }

constexpr int kSeqChunk = 256;   // frames per sequence launch (device pointer table)

size_t prost_host::part_bytes(const pros_handle* h, int G) {
  size_t d = (2 * (size_t)G + prost::kExtraSlots) * prost::kSlot;
  if (wide_exchange(h)) d += ((size_t)G + 16) * prost::kWideMax;
  return sizeof(double) * d;
}

bool prost_host::pair_layout(const pros_handle* h) {
  return h->prm.storage == PROS_BF16 && h->P % 2 == 0 && h->tpw % 2 == 0 && h->ldU % 2 == 0;
}

// Register rows per thread for a single stream.  A frame is latency-bound
// (its gang-wide exchanges), so the fastest tile is the smallest one whose
// gang still fits one workgroup per compute unit: more rows per thread only
// add work per workgroup.  Small frames are the exception: a gang of up to
// kSmallGang workgroups exchanges faster than a larger one (measured at
// 160x120x3: 29 workgroups 74 us per frame, 113 workgroups 81 us), so the
// smallest tile reaching such a gang wins, and a frame that fits one
// workgroup takes that tile (its reductions stay inside the workgroup, no
// memory round trip).  Frames too large for one workgroup per CU take the
// largest tile that is resident.  force_nr > 0 asks for one row count.
constexpr int kSmallGang = 32;
static pros_status choose_launch(pros_handle* h, int force_nr) {
  const int nrs[] = {1, 2, 4, 8, 16, 32};
  const void* best = nullptr;
  int bestNR = 0, bestG = 0, bestT = 0;
  const bool ext = h->prm.preprocess != 0 || h->score != nullptr || wide_exchange(h);
  h->streamed = false;
  if (force_nr == 0) {
    for (int NR : nrs) {
      const void* f = (h->prm.storage == PROS_BF16) ? prost::frame_kernel_bf16(h->k, NR, ext)
                                                    : prost::frame_kernel_f32(h->k, NR, ext);
      if (!f || prost::kBlock * NR < h->C) continue;
      const int tpw = prost_host::tile_pixels(h->prm.storage, NR, h->C, 1.0);
      if (tpw < h->P) continue;
      int occ = 0;
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, prost::kBlock, 0));
      if (occ < 1) continue;
      h->kfn = f;
      h->NR = NR;
      h->G = 1;
      h->tpw = tpw;
      return PROS_OK;
    }
    for (int NR : nrs) {
      const void* f = (h->prm.storage == PROS_BF16) ? prost::frame_kernel_bf16(h->k, NR, ext)
                                                    : prost::frame_kernel_f32(h->k, NR, ext);
      if (!f || prost::kBlock * NR < h->C) continue;
      const int tpw = prost_host::tile_pixels(h->prm.storage, NR, h->C, 1.0);
      const long long G = (h->P + tpw - 1) / tpw;
      if (G > kSmallGang || G > h->num_cu) continue;
      int occ = 0;
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, prost::kBlock, 0));
      if (occ < 1) continue;
      h->kfn = f;
      h->NR = NR;
      h->G = (int)G;
      h->tpw = tpw;
      return PROS_OK;
    }
  }
  for (int NR : nrs) {
    if (force_nr > 0 && NR != force_nr) continue;
    const void* f = (h->prm.storage == PROS_BF16) ? prost::frame_kernel_bf16(h->k, NR, ext)
                                                  : prost::frame_kernel_f32(h->k, NR, ext);
    if (!f) continue;
    if (prost::kBlock * NR < h->C) continue;
    const int tpw = prost_host::tile_pixels(h->prm.storage, NR, h->C, 1.0);
    const long long G = (h->P + tpw - 1) / tpw;
    int occ = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, prost::kBlock, 0));
    if (G > (long long)occ * h->num_cu) continue;   // not resident
    best = f; bestNR = NR; bestG = (int)G; bestT = tpw;
    if (G <= h->num_cu) break;                      // smallest tile at one workgroup per CU
  }
  if (!best) {
    // no resident gang holds the frame's register tiles: stream every pass
    // (default features only; the optional features need the tile kernels)
    const bool stream_ok = h->prm.preprocess == 0 && h->score == nullptr && h->prm.ysolve != 2;
    if (force_nr > 0 || !stream_ok)
      return fail(PROS_EUNSUPPORTED,
                  "frame of %d pixels x %d channels at k=%d does not fit the device's resident workgroups%s", h->P,
                  h->C, h->k, stream_ok ? "" : " (its streamed form has no pre-processing, scores or IRLS step)");
    h->streamed = true;
    h->kfn = nullptr;
    h->NR = 0;
    h->G = 1;
    h->tpw = h->P;
    return PROS_OK;
  }
  h->streamed = false;
  h->kfn = best;
  h->NR = bestNR;
  h->G = bestG;
  h->tpw = bestT;
  return PROS_OK;
}

pros_status prost_host::create_handle(const pros_params* prm, hipStream_t stream, int nr_force, int tpw_force,
                                      int g_force, pros_handle** out) {
  *out = nullptr;
  pros_status st = pros_validate(prm);
  if (st != PROS_OK) return st;
  pros_handle* h = new pros_handle();
  h->prm = *prm;
  h->P = prm->width * prm->height;
  h->C = prm->channels;
  h->m = h->P * h->C;
  h->k = prm->k;
  h->ldU = ((long long)h->m + 63) / 64 * 64;
  h->stream = stream;
  auto bail = [&](pros_status s) { free_handle(h); return s; };
#define INIT_TRY(expr)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      pros_status s_ = (e_ == hipErrorOutOfMemory) ? PROS_ENOMEM : PROS_EHIP;             \
      fail(s_, "%s failed: %s", #expr, hipGetErrorString(e_));                            \
      return bail(s_);                                                                    \
    }                                                                                     \
  } while (0)
  INIT_TRY(hipGetDevice(&h->device));
  INIT_TRY(hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device));
  int wclk_khz = 0;
  INIT_TRY(hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, h->device));
  if (wclk_khz <= 0) wclk_khz = 100000;
  h->timeout_ticks = (long long)wclk_khz * 1000LL * 2;  // 2 s per barrier wait
  if (g_force > 0) {             // launch owned by a batch
    h->NR = nr_force;
    h->tpw = tpw_force;
    h->G = g_force;
  } else {
    st = choose_launch(h, nr_force);
    if (st != PROS_OK) return bail(st);
    // small gangs: every workgroup reading all partials beats the two hops
    // (160x120x3 at 29 workgroups: 74 vs 84 us; 320x240x3 at 113: 91 vs 85)
    h->sync_mode = h->G <= 64 ? 3 : 2;
  }
  const size_t es = (prm->storage == PROS_BF16) ? 2 : 4;
  INIT_TRY(hipMalloc(&h->U, es * (size_t)h->ldU * h->k));
  INIT_TRY(hipMalloc(&h->xstage, es * (size_t)h->m));
  INIT_TRY(hipMalloc((void**)&h->lab, (size_t)h->P));
  INIT_TRY(hipMalloc((void**)&h->mask, (size_t)h->P));
  INIT_TRY(hipMalloc((void**)&h->y, sizeof(double) * PROS_MAX_K));
  INIT_TRY(hipMalloc((void**)&h->nframe, sizeof(long long)));
  INIT_TRY(hipMalloc((void**)&h->stats, sizeof(pros_stats)));
  INIT_TRY(hipMalloc((void**)&h->seq, sizeof(void*) * kSeqChunk));
  INIT_TRY(hipMalloc((void**)&h->part, prost_host::part_bytes(h, h->G)));
  INIT_TRY(hipMalloc((void**)&h->sync, 64));
  INIT_TRY(hipMemsetAsync(h->U, 0, es * (size_t)h->ldU * h->k, h->stream));
  INIT_TRY(hipMemsetAsync(h->lab, 0, (size_t)h->P, h->stream));
  INIT_TRY(hipMemsetAsync(h->mask, 0, (size_t)h->P, h->stream));
  INIT_TRY(hipMemsetAsync(h->y, 0, sizeof(double) * PROS_MAX_K, h->stream));
  INIT_TRY(hipMemsetAsync(h->nframe, 0, sizeof(long long), h->stream));
  INIT_TRY(hipMemsetAsync(h->stats, 0, sizeof(pros_stats), h->stream));
  INIT_TRY(hipMemsetAsync(h->sync, 0, 64, h->stream));
  if (prm->preprocess) {
    INIT_TRY(hipMalloc((void**)&h->pre_mean, sizeof(float) * (size_t)h->m));
    INIT_TRY(hipMalloc((void**)&h->pre_m2, sizeof(float) * (size_t)h->m));
    INIT_TRY(hipMalloc((void**)&h->pre_stat, 2 * sizeof(double)));
    INIT_TRY(hipMemsetAsync(h->pre_mean, 0, sizeof(float) * (size_t)h->m, h->stream));
    INIT_TRY(hipMemsetAsync(h->pre_m2, 0, sizeof(float) * (size_t)h->m, h->stream));
    INIT_TRY(hipMemsetAsync(h->pre_stat, 0, 2 * sizeof(double), h->stream));
  }
  // epoch-tagged exchange slots must start with tag 0 (the first exchange uses 1)
  INIT_TRY(hipMemsetAsync(h->part, 0, prost_host::part_bytes(h, h->G),
                          h->stream));
  if (h->streamed) {
    st = prost_stream_alloc(h);
    if (st != PROS_OK) return bail(st);
  }
  INIT_TRY(hipStreamSynchronize(h->stream));
#undef INIT_TRY
  *out = h;
  return PROS_OK;
}

pros_status pros_init(const pros_params* prm, void* hip_stream, pros_handle** out) {
  if (!out) return fail(PROS_EINVAL, "out is NULL");
  pros_status st = prost_host::create_handle(prm, (hipStream_t)hip_stream, 0, 0, 0, out);
  if (st != PROS_OK) return st;
  st = prost_init_subspace(*out, prm->seed, 0);   // U0 of Sec. 3.4
  if (st != PROS_OK) {
    free_handle(*out);
    *out = nullptr;
    return st;
  }
  (*out)->state_set = true;
  return PROS_OK;
}

pros_status pros_random_subspace(uint64_t seed, uint32_t stream_index, int64_t m, int32_t k, double* U,
                                 void* hip_stream) {
  if (!U) return fail(PROS_EINVAL, "U is NULL");
  if (m < 1 || k < 1 || k > PROS_MAX_K || m < k) return fail(PROS_EINVAL, "bad sizes m=%lld k=%d", (long long)m, k);
  return prost_random_subspace(seed, stream_index, m, k, U, (hipStream_t)hip_stream);
}

void pros_destroy(pros_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  free_handle(h);
}

pros_status prost_host::check_usable(pros_handle* h) {
  if (!h) return fail(PROS_EINVAL, "handle is NULL");
  if (h->broken) return fail(h->broken_status, "handle unusable after an earlier error");
  return PROS_OK;
}

// Synchronise and fold device-side error bits into a status.
pros_status prost_host::sync_and_check(pros_handle* h) {
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    h->broken = true;
    h->broken_status = PROS_EHIP;
    return fail(PROS_EHIP, "stream synchronisation failed: %s", hipGetErrorString(e));
  }
  unsigned bits[3] = {0, 0, 0};
  e = hipMemcpy(bits, h->sync, sizeof(bits), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    h->broken = true;
    h->broken_status = PROS_EHIP;
    return fail(PROS_EHIP, "reading the error word failed: %s", hipGetErrorString(e));
  }
  if (bits[2] & prost::kErrTimeout) {
    h->broken = true;
    h->broken_status = PROS_ETIMEOUT;
    return fail(PROS_ETIMEOUT, "a frame kernel timed out waiting for its workgroups");
  }
  if (bits[2] & prost::kErrBadFrame) {
    unsigned zero = 0;
    e = hipMemcpy(h->sync + 2, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      h->broken = true;
      h->broken_status = PROS_EHIP;
      return fail(PROS_EHIP, "clearing the error word failed: %s", hipGetErrorString(e));
    }
    return fail(PROS_EBADFRAME, "a frame with a non-finite entry was rejected");
  }
  return PROS_OK;
}

pros_status pros_sync(pros_handle* h) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  return sync_and_check(h);
}

pros_status pros_set_state(pros_handle* h, const double* U, const double* y, const uint8_t* labels, int64_t n) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (!U) return fail(PROS_EINVAL, "U is NULL");
  if (n < 0) return fail(PROS_EINVAL, "n must be >= 0");
  for (long long i = 0; i < (long long)h->m * h->k; ++i)
    if (!std::isfinite(U[i])) return fail(PROS_EINVAL, "U has a non-finite entry");
  if (y)
    for (int j = 0; j < h->k; ++j)
      if (!std::isfinite(y[j])) return fail(PROS_EINVAL, "y has a non-finite entry");
  HIP_TRY(hipStreamSynchronize(h->stream));
  const bool bf = h->prm.storage == PROS_BF16;
  const size_t es = bf ? 2 : 4;
  std::vector<unsigned char> buf(es * (size_t)h->ldU * h->k, 0);
  for (int j = 0; j < h->k; ++j) {
    for (int e = 0; e < h->m; ++e) {
      const float v = (float)U[(size_t)j * h->m + e];
      const size_t o = (size_t)j * h->ldU + e;
      if (bf) {
        const uint16_t b = bf16_rne(v);
        std::memcpy(&buf[o * 2], &b, 2);
      } else {
        std::memcpy(&buf[o * 4], &v, 4);
      }
    }
  }
  HIP_TRY(hipMemcpy(h->U, buf.data(), buf.size(), hipMemcpyHostToDevice));
  double yv[PROS_MAX_K] = {0};
  if (y)
    for (int j = 0; j < h->k; ++j) yv[j] = y[j];
  HIP_TRY(hipMemcpy(h->y, yv, sizeof(yv), hipMemcpyHostToDevice));
  if (labels) {
    std::vector<uint8_t> l(labels, labels + h->P);
    for (auto& v : l) v = v ? 1 : 0;
    HIP_TRY(hipMemcpy(h->lab, l.data(), (size_t)h->P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->mask, l.data(), (size_t)h->P, hipMemcpyHostToDevice));
  } else {
    HIP_TRY(hipMemset(h->lab, 0, (size_t)h->P));
    HIP_TRY(hipMemset(h->mask, 0, (size_t)h->P));
  }
  long long nn = n;
  HIP_TRY(hipMemcpy(h->nframe, &nn, sizeof(nn), hipMemcpyHostToDevice));
  HIP_TRY(hipDeviceSynchronize());
  h->submitted = n;
  h->state_set = true;
  h->mask_stale = true;
  return PROS_OK;
}

pros_status pros_get_state(pros_handle* h, double* U, double* y, uint8_t* labels, int64_t* n) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  st = sync_and_check(h);
  if (st != PROS_OK && st != PROS_EBADFRAME) return st;
  pros_status pending = st;
  const bool bf = h->prm.storage == PROS_BF16;
  if (U) {
    const size_t es = bf ? 2 : 4;
    std::vector<unsigned char> buf(es * (size_t)h->ldU * h->k);
    HIP_TRY(hipMemcpy(buf.data(), h->U, buf.size(), hipMemcpyDeviceToHost));
    for (int j = 0; j < h->k; ++j)
      for (int e = 0; e < h->m; ++e) {
        const size_t o = (size_t)j * h->ldU + e;
        double v;
        if (bf) {
          uint16_t b;
          std::memcpy(&b, &buf[o * 2], 2);
          v = bf16_to_f32(b);
        } else {
          float f;
          std::memcpy(&f, &buf[o * 4], 4);
          v = f;
        }
        U[(size_t)j * h->m + e] = v;
      }
  }
  if (y) {
    double yv[PROS_MAX_K];
    HIP_TRY(hipMemcpy(yv, h->y, sizeof(yv), hipMemcpyDeviceToHost));
    for (int j = 0; j < h->k; ++j) y[j] = yv[j];
  }
  if (labels) HIP_TRY(hipMemcpy(labels, h->lab, (size_t)h->P, hipMemcpyDeviceToHost));
  if (n) {
    long long nn;
    HIP_TRY(hipMemcpy(&nn, h->nframe, sizeof(nn), hipMemcpyDeviceToHost));
    *n = nn;
  }
  return pending;
}

FrameArgs prost_host::make_args(pros_handle* h, const void* x) {
  FrameArgs a;
  std::memset(&a, 0, sizeof(a));
  const pros_params& p = h->prm;
  a.U = h->U;
  a.x = x;
  a.lab = h->lab;
  a.mask = h->mask;
  a.y = h->y;
  a.nframe = h->nframe;
  a.stats = h->stats;
  a.part = h->part;
  a.sync = h->sync;
  a.ldU = h->ldU;
  a.m = h->m;
  a.P = h->P;
  a.C = h->C;
  a.W = p.width;
  a.H = p.height;
  a.k = h->k;
  a.G = h->G;
  a.tpw = h->tpw;
  a.cp.form = (p.cost == PROS_COST_LOG) ? 1 : 0;
  a.cp.p = (float)p.p;
  a.cp.half_p = (float)(0.5 * p.p);
  a.cp.mu = (float)p.mu;
  a.cp.inv_mu = (float)(1.0 / p.mu);
  a.cp.half_p_m1 = (float)(0.5 * p.p - 1.0);
  a.cp.inv_p = (float)(1.0 / p.p);
  a.delta = (float)effective_delta(p);
  a.omega = (float)p.omega;
  a.t_init = p.t_init;
  a.t_min = p.t_min;
  a.tau = -std::log(p.t_min / p.t_init) / (double)p.i_init;
  a.J = p.cg_iters;
  a.labels_after_update = p.labels_after_update;
  a.weights_from_filtered = p.weights_from_filtered;
  a.timeout = h->timeout_ticks;
  a.sync_mode = h->sync_mode;
  a.curv = h->curv;
  a.trace = h->trace;
  a.pair_aligned = (pair_layout(h) && ((uintptr_t)x & 3u) == 0) ? 1 : 0;
  a.pre_mean = h->pre_mean;
  a.pre_m2 = h->pre_m2;
  a.pre_stat = h->pre_stat;
  a.i_init = p.i_init;
  a.score = h->score;
  a.ysolve = p.ysolve;
  a.seq = nullptr;
  a.nseq = 1;
  return a;
}


// Launch frame kernel fn for a.nseq frames (a.x, then a.seq[1 ..]) and run a
// re-orthonormalisation when one is due after them.
static pros_status launch_frames(pros_handle* h, FrameArgs& a, const void* fn) {
  void* args[] = {&a};
  hipError_t e = h->coop ? hipLaunchCooperativeKernel(fn, dim3(h->G), dim3(prost::kBlock), args, 0, h->stream)
                         : hipLaunchKernel(fn, dim3(h->G), dim3(prost::kBlock), args, 0, h->stream);
  if (e != hipSuccess) {
    h->broken = true;
    h->broken_status = PROS_EHIP;
    return fail(PROS_EHIP, "frame kernel launch failed: %s", hipGetErrorString(e));
  }
  h->submitted += a.nseq;
  h->mask_stale = true;
  if (h->prm.reorth_every > 0 && h->submitted % h->prm.reorth_every == 0) {
    pros_status st = prost_reorth_launch(h);
    if (st != PROS_OK) return st;
  }
  return PROS_OK;
}

// One frame of the streamed path (weights from the filtered mask need the
// previous frame's median first), then a re-orthonormalisation when due.
static pros_status stream_frame(pros_handle* h, const FrameArgs& a) {
  if (h->prm.weights_from_filtered) {
    pros_status st = prost_host::refresh_mask(h);
    if (st != PROS_OK) return st;
  }
  pros_status st = prost_stream_frame(h, a);
  if (st != PROS_OK) return st;
  h->submitted += 1;
  h->mask_stale = true;
  if (h->prm.reorth_every > 0 && h->submitted % h->prm.reorth_every == 0) return prost_reorth_launch(h);
  return PROS_OK;
}

pros_status pros_track_frame(pros_handle* h, const void* frame, int32_t dtype, int32_t on_device) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (!frame) return fail(PROS_EINVAL, "frame is NULL");
  if (dtype != PROS_F32 && dtype != PROS_BF16) return fail(PROS_EINVAL, "unknown frame dtype");
  if (!h->state_set) return fail(PROS_ESTATE, "set U with pros_set_state before the first frame");
  const void* x = frame;
  if (on_device) {
    if (dtype != h->prm.storage) return fail(PROS_EINVAL, "device frames must have the storage dtype");
  } else {
    const bool bf = h->prm.storage == PROS_BF16;
    const size_t es = bf ? 2 : 4;
    std::vector<unsigned char> tmp;
    const void* src = frame;
    if (dtype == PROS_F32) {
      const float* f = (const float*)frame;
      for (int e = 0; e < h->m; ++e)
        if (!std::isfinite(f[e])) return fail(PROS_EBADFRAME, "frame entry %d is not finite", e);
      if (bf) {
        tmp.resize(es * h->m);
        for (int e = 0; e < h->m; ++e) {
          const uint16_t b = bf16_rne(f[e]);
          std::memcpy(&tmp[(size_t)e * 2], &b, 2);
        }
        src = tmp.data();
      }
    } else {
      const uint16_t* b = (const uint16_t*)frame;
      for (int e = 0; e < h->m; ++e)
        if ((b[e] & 0x7f80u) == 0x7f80u) return fail(PROS_EBADFRAME, "frame entry %d is not finite", e);
      if (!bf) {
        tmp.resize(es * h->m);
        for (int e = 0; e < h->m; ++e) {
          const float f = bf16_to_f32(b[e]);
          std::memcpy(&tmp[(size_t)e * 4], &f, 4);
        }
        src = tmp.data();
      }
    }
    HIP_TRY(hipMemcpyAsync(h->xstage, src, es * (size_t)h->m, hipMemcpyHostToDevice, h->stream));
    if (!tmp.empty()) HIP_TRY(hipStreamSynchronize(h->stream));
    x = h->xstage;
  }
  FrameArgs a = make_args(h, x);
  if (h->streamed) return stream_frame(h, a);
  return launch_frames(h, a, h->kfn);
}

pros_status pros_track_frames(pros_handle* h, const void* const* frames, int32_t count, int32_t dtype) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (!frames || count < 1) return fail(PROS_EINVAL, "frames is NULL or count < 1");
  if (dtype != h->prm.storage) return fail(PROS_EINVAL, "device frames must have the storage dtype");
  if (!h->state_set) return fail(PROS_ESTATE, "set U with pros_set_state before the first frame");
  for (int i = 0; i < count; ++i)
    if (!frames[i]) return fail(PROS_EINVAL, "frame %d is NULL", i);
  // frames that depend on more than the tile's own state between frames
  // (filtered-mask weights, pre-processing statistics, scores, the wide
  // exchange) run one launch each
  const void* fseq = h->streamed ? nullptr : prost::frame_kernel_seq(h->prm.storage == PROS_BF16, h->k, h->NR);
  const bool seq_ok = fseq && !h->prm.weights_from_filtered && h->pre_mean == nullptr && h->score == nullptr &&
                      !wide_exchange(h);
  if (!seq_ok) {
    for (int i = 0; i < count; ++i) {
      st = pros_track_frame(h, frames[i], dtype, 1);
      if (st != PROS_OK) return st;
    }
    return PROS_OK;
  }
  for (int i = 0; i < count;) {
    long long len = std::min(count - i, kSeqChunk);
    if (h->prm.reorth_every > 0)   // end the launch where a re-orthonormalisation is due
      len = std::min<long long>(len, h->prm.reorth_every - h->submitted % h->prm.reorth_every);
    HIP_TRY(hipMemcpyAsync(h->seq, frames + i, sizeof(void*) * (size_t)len, hipMemcpyHostToDevice, h->stream));
    FrameArgs a = make_args(h, frames[i]);
    a.seq = (const void* const*)h->seq;
    a.nseq = (int)len;
    for (long long f = 1; f < len; ++f)
      if (((uintptr_t)frames[i + f] & 3u) != 0) a.pair_aligned = 0;
    st = launch_frames(h, a, fseq);
    if (st != PROS_OK) return st;
    i += (int)len;
  }
  return PROS_OK;
}

pros_status pros_get_mask(pros_handle* h, uint8_t* out, int32_t filtered, int32_t on_device) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (!out) return fail(PROS_EINVAL, "out is NULL");
  if (filtered) {
    st = prost_host::refresh_mask(h);
    if (st != PROS_OK) return st;
  }
  const uint8_t* src = filtered ? h->mask : h->lab;
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(out, src, (size_t)h->P, hipMemcpyDeviceToDevice, h->stream));
    return PROS_OK;
  }
  st = sync_and_check(h);
  if (st != PROS_OK && st != PROS_EBADFRAME) return st;
  HIP_TRY(hipMemcpy(out, src, (size_t)h->P, hipMemcpyDeviceToHost));
  return st;
}

pros_status pros_get_stats(pros_handle* h, pros_stats* out) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (!out) return fail(PROS_EINVAL, "out is NULL");
  st = prost_host::refresh_mask(h);
  if (st != PROS_OK) return st;
  st = sync_and_check(h);
  if (st != PROS_OK && st != PROS_EBADFRAME) return st;
  HIP_TRY(hipMemcpy(out, h->stats, sizeof(pros_stats), hipMemcpyDeviceToHost));
  return st;
}

pros_status pros_get_launch_info(pros_handle* h, pros_launch_info* out) {
  if (!h || !out) return fail(PROS_EINVAL, "NULL argument");
  if (h->streamed) {   // one launch per pass: no register tile, no gang exchange
    // bfloat16 with even P takes pixel pairs (for 4-byte aligned frames)
    const bool pairs = h->prm.storage == PROS_BF16 && h->P % 2 == 0 && h->ldU % 2 == 0;
    out->threads = 256;
    out->pixels_per_wg = pairs ? 512 : 256;
    out->workgroups = (h->P + out->pixels_per_wg - 1) / out->pixels_per_wg;
    out->rows_per_thread = 0;
    out->barriers_per_frame = 0;
    out->sync_mode = -1;
    out->curvature = h->curv;
    return PROS_OK;
  }
  out->workgroups = h->G;
  out->threads = prost::kBlock;
  out->rows_per_thread = h->NR;
  out->pixels_per_wg = h->tpw;
  out->barriers_per_frame = (wide_exchange(h) ? 1 : 2) * h->prm.cg_iters + 1;
  out->sync_mode = h->sync_mode;
  out->curvature = h->curv;
  return PROS_OK;
}

// Clear the exchange slots and restart the epoch and arrival counters (after
// any change of the gang; stale tags must never match a new epoch).
pros_status prost_host::reset_exchange(pros_handle* h) {
  HIP_TRY(hipMemsetAsync(h->part, 0, prost_host::part_bytes(h, h->G), h->stream));
  HIP_TRY(hipMemsetAsync(h->sync, 0, 16, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return PROS_OK;
}

pros_status pros_set_launch(pros_handle* h, int32_t rows_per_thread, int32_t sync_mode) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (rows_per_thread == -1) {   // the streamed form, whatever the frame's size
    if (h->prm.preprocess || h->score || h->prm.ysolve == 2)
      return fail(PROS_EUNSUPPORTED, "the streamed form has no pre-processing, scores or IRLS step");
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (!h->stream_ws) {
      st = prost_stream_alloc(h);
      if (st != PROS_OK) return st;
    }
    h->streamed = true;
    return PROS_OK;
  }
  if (sync_mode < 0 || sync_mode > 3) return fail(PROS_EINVAL, "sync_mode must be 0..3");
  if (sync_mode == 0 && wide_exchange(h))
    return fail(PROS_EINVAL, "the wide exchange (IRLS, curvature schedule 1) needs a tagged exchange (sync_mode 1..3)");
  if (rows_per_thread != 0 && rows_per_thread != 1 && rows_per_thread != 2 && rows_per_thread != 4 &&
      rows_per_thread != 8 && rows_per_thread != 16 && rows_per_thread != 32)
    return fail(PROS_EINVAL, "rows_per_thread must be 0 (automatic), 1, 2, 4, 8, 16 or 32");
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int oldG = h->G;
  st = choose_launch(h, rows_per_thread);
  if (st != PROS_OK) return st;
  if (h->G > oldG) {
    (void)hipFree(h->part);
    h->part = nullptr;
    hipError_t e = hipMalloc((void**)&h->part, prost_host::part_bytes(h, h->G));
    if (e != hipSuccess) {
      h->broken = true;
      h->broken_status = PROS_ENOMEM;
      return fail(PROS_ENOMEM, "partials: %s", hipGetErrorString(e));
    }
  }
  h->sync_mode = sync_mode;
  return prost_host::reset_exchange(h);
}

pros_status pros_set_dispatch(pros_handle* h, int32_t cooperative) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (cooperative != 0 && cooperative != 1) return fail(PROS_EINVAL, "cooperative must be 0 or 1");
  h->coop = cooperative != 0;
  return PROS_OK;
}

pros_status pros_set_curvature(pros_handle* h, int32_t schedule) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (schedule != 0 && schedule != 1) return fail(PROS_EINVAL, "curvature schedule must be 0 or 1");
  if (h->streamed) {   // one launch per pass: both schedules, any storage, no exchange slots
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->curv = schedule;
    return PROS_OK;
  }
  if (schedule == 1 && h->prm.storage != PROS_F32)
    return fail(PROS_EUNSUPPORTED, "curvature schedule 1 needs float32 storage");
  if (schedule == 1 && h->sync_mode == 0)
    return fail(PROS_EINVAL, "curvature schedule 1 needs a tagged exchange (sync_mode 1..3)");
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int old = h->curv;
  h->curv = schedule;
  st = choose_launch(h, h->NR);   // same tile; kernel with or without the wide exchange
  if (st != PROS_OK) {
    h->curv = old;
    return st;
  }
  (void)hipFree(h->part);        // the wide exchange has its own slots
  h->part = nullptr;
  hipError_t e = hipMalloc((void**)&h->part, prost_host::part_bytes(h, h->G));
  if (e != hipSuccess) {
    h->broken = true;
    h->broken_status = PROS_ENOMEM;
    return fail(PROS_ENOMEM, "partials: %s", hipGetErrorString(e));
  }
  return prost_host::reset_exchange(h);
}

pros_status pros_set_score_output(pros_handle* h, float* device_scores) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (h->streamed) return fail(PROS_EUNSUPPORTED, "the frame is streamed (it does not fit resident register tiles)");
  HIP_TRY(hipStreamSynchronize(h->stream));
  float* old = h->score;
  h->score = device_scores;
  st = choose_launch(h, h->NR);   // same tile, kernel with or without the optional features
  if (st != PROS_OK) h->score = old;
  return st;
}

pros_status pros_debug_trace(pros_handle* h, long long* device_buffer) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  h->trace = device_buffer;
  return PROS_OK;
}

pros_status pros_set_preprocess(pros_handle* h, const double* mean, const double* m2, int64_t count) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (!h->pre_mean) return fail(PROS_ESTATE, "the handle was created without pre-processing");
  if (count < 0) return fail(PROS_EINVAL, "count must be >= 0");
  std::vector<float> mf((size_t)h->m, 0.f), vf((size_t)h->m, 0.f);
  double sum = 0.0;
  for (int e = 0; e < h->m; ++e) {
    if (mean) mf[e] = (float)mean[e];
    if (m2) vf[e] = (float)m2[e];
    if (!std::isfinite(mf[e]) || !std::isfinite(vf[e]) || vf[e] < 0.f)
      return fail(PROS_EINVAL, "pre-processing entry %d is not finite or has a negative deviation sum", e);
    sum += (double)vf[e];
  }
  const double stat[2] = {sum, (double)count};
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(h->pre_mean, mf.data(), sizeof(float) * (size_t)h->m, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->pre_m2, vf.data(), sizeof(float) * (size_t)h->m, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->pre_stat, stat, sizeof(stat), hipMemcpyHostToDevice));
  return PROS_OK;
}

pros_status pros_get_preprocess(pros_handle* h, double* mean, double* m2, int64_t* count, double* scale) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  if (!h->pre_mean) return fail(PROS_ESTATE, "the handle was created without pre-processing");
  st = sync_and_check(h);
  if (st != PROS_OK && st != PROS_EBADFRAME) return st;
  std::vector<float> buf((size_t)h->m);
  if (mean) {
    HIP_TRY(hipMemcpy(buf.data(), h->pre_mean, sizeof(float) * (size_t)h->m, hipMemcpyDeviceToHost));
    for (int e = 0; e < h->m; ++e) mean[e] = buf[e];
  }
  if (m2) {
    HIP_TRY(hipMemcpy(buf.data(), h->pre_m2, sizeof(float) * (size_t)h->m, hipMemcpyDeviceToHost));
    for (int e = 0; e < h->m; ++e) m2[e] = buf[e];
  }
  double stat[2];
  HIP_TRY(hipMemcpy(stat, h->pre_stat, sizeof(stat), hipMemcpyDeviceToHost));
  if (count) *count = (int64_t)stat[1];
  if (scale) {
    const double var = stat[1] >= 2.0 ? stat[0] / ((double)h->m * (stat[1] - 1.0)) : 0.0;
    *scale = var > 0.0 ? std::sqrt(var) : 1.0;
  }
  return st;
}

pros_status pros_reorthonormalize(pros_handle* h) {
  pros_status st = check_usable(h);
  if (st != PROS_OK) return st;
  return prost_reorth_launch(h);
}


