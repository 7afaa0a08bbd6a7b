// Batched form: many independent video streams advance by one frame each in
// ONE persistent cooperative launch.
//
// Every stream is split into workgroup tiles exactly as in the single-stream
// kernel and owns a gang of workgroups for the frame's gang-wide reductions.
// The launch is a fixed grid of resident workgroups; a host-built schedule
// assigns each workgroup a sequence of (stream, tile) items, one per round.
// Gangs of one round are disjoint sets of workgroups, so every gang is
// resident; streams of a round do not wait for each other, and a workgroup
// moves to its next item as soon as its current stream's frame is done.
//
// One kernel serves every stream with k <= K: columns k..K-1 of the register
// tile are zero, which leaves the method's arithmetic unchanged (their
// gradient entries, directions, y entries and geodesic components are all 0).
#pragma once

#include "prost_frame.hpp"

namespace prost {
inline namespace PROST_BLOCK_NS {

struct BatchItem {
  int stream;   // -1: idle slot
  int tile;
};

// Subspace-dimension classes with a batch kernel, and register rows per
// thread for a budget of about `budget` 32-bit registers of U per thread:
// one float32 row entry or one bfloat16 row-pair entry per register.
constexpr int kBatchClasses[] = {2, 4, 5, 8, 10, 12, 15, 16};
constexpr int kNumBatchClasses = 8;

__host__ __device__ constexpr int batch_nr(int budget, int K) {
  return (budget / K >= 16) ? 16 : (budget / K < 1 ? 1 : budget / K);
}
__host__ __device__ constexpr int batch_nr_bf16(int budget, int K) {
  return 2 * batch_nr(budget, K);
}
// The LDS form (register_budget kBudgetLds, bfloat16, k class >= 10): the
// register tile of budget 128, plus the row pairs whose K words and two
// residuals per thread fit the LDS left beside the frame scratch (at most 16
// pairs in all).  A 640x480x3 k = 15 stream then needs 82 workgroups
// instead of 113, so three such streams share a round instead of two.
constexpr int kBudgetLds = 192;
constexpr int kLdsBytes = 160 * 1024;
__host__ __device__ constexpr int batch_lds_np(int K) { return batch_nr(128, K); }
__host__ __device__ constexpr int batch_lds_nl(int K) {
  const int fit = (kLdsBytes - (int)sizeof(FrameSmem) - 1024) / ((K + 2) * 4 * kBlock);
  const int room = 16 - batch_lds_np(K);
  return fit < room ? fit : room;
}
__host__ __device__ constexpr bool batch_lds_form(int K) { return K >= 10; }

__host__ __device__ constexpr int batch_rows(int storage_bf16, int budget, int K) {
  if (budget == kBudgetLds) return 2 * (batch_lds_np(K) + batch_lds_nl(K));
  return storage_bf16 ? batch_nr_bf16(budget, K) : batch_nr(budget, K);
}

__host__ __device__ constexpr int batch_class(int k) {
  return k <= 2 ? 2 : k <= 4 ? 4 : k <= 5 ? 5 : k <= 8 ? 8 : k <= 10 ? 10 : k <= 12 ? 12 : k <= 15 ? 15 : 16;
}

// A stream descriptor copied into scalar registers (its words are uniform
// across the workgroup), as kernel arguments are: held in vector registers
// the fields would take room from the register tile.
__device__ __forceinline__ FrameArgs load_uniform(const FrameArgs* __restrict__ p) {
  static_assert(sizeof(FrameArgs) % 4 == 0, "descriptor of 32-bit words");
  FrameArgs a;
  const int* src = (const int*)p;
  int w[sizeof(FrameArgs) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(FrameArgs) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
  __builtin_memcpy(&a, w, sizeof(FrameArgs));
  return a;
}

// SEQ: every item advances its stream by a.nseq frames of its ring with the
// tile kept in registers (several batch steps per launch).
template <typename TS, int K, int NR, bool EXT, int NL = 0, bool SEQ = false>
__global__ __launch_bounds__(kBlock, 2) void batch_kernel(const FrameArgs* __restrict__ descs,
                                                       const BatchItem* __restrict__ items, int rounds) {
  __shared__ FrameSmem sm;
  __shared__ uint32_t lt[NL > 0 ? NL * (K + 2) * kBlock : 1];   // LDS row pairs of the tile and their residuals
  for (int r = 0; r < rounds; ++r) {
    const BatchItem it = items[(size_t)r * gridDim.x + blockIdx.x];
    if (it.stream < 0) continue;
    const FrameArgs a = load_uniform(descs + it.stream);
    if (!run_tile<K, NR, TS, EXT, false, NL, SEQ>(a, it.tile, sm, lt)) return;
  }
}

// The multi-step form of class K at register budget 128 (default features).
template <int K>
const void* batch_kernel_seq(int storage_bf16) {
  return storage_bf16 ? (const void*)&batch_kernel<uint16_t, K, batch_nr_bf16(128, K), false, 0, true>
                      : (const void*)&batch_kernel<float, K, batch_nr(128, K), false, 0, true>;
}

// The LDS form of class K (bfloat16, default features).
template <int K>
const void* batch_kernel_lds() {
  static_assert(batch_lds_form(K), "LDS form for k class >= 10");
  constexpr int NL = batch_lds_nl(K);
  static_assert(NL >= 1 && sizeof(FrameSmem) + NL * (K + 2) * 4 * kBlock + 1024 <= kLdsBytes, "LDS budget");
  return (const void*)&batch_kernel<uint16_t, K, 2 * batch_lds_np(K), false, NL>;
}

}  // inline namespace PROST_BLOCK_NS

// Kernel for (storage, class K, budget, optional features compiled in);
// nullptr if not built.
const void* batch_kernel_ptr(int storage_bf16, int K, int budget, bool ext);
const void* batch_kernel_seq_ptr(int storage_bf16, int K);
// The 256-thread build (two workgroups per CU) at register budget 128 with
// the default features: one step per launch, and the multi-step form;
// nullptr if not built for (storage, class K).
const void* batch256_kernel_ptr(int storage_bf16, int K);
const void* batch256_kernel_seq_ptr(int storage_bf16, int K);

}  // namespace prost
