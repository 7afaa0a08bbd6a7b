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
__host__ __device__ constexpr int batch_rows(int storage_bf16, int budget, int K) {
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

template <typename TS, int K, int NR, bool EXT>
__global__ __launch_bounds__(kBlock, 2) void batch_kernel(const FrameArgs* __restrict__ descs,
                                                       const BatchItem* __restrict__ items, int rounds) {
  __shared__ FrameSmem sm;
  for (int r = 0; r < rounds; ++r) {
    const BatchItem it = items[(size_t)r * gridDim.x + blockIdx.x];
    if (it.stream < 0) continue;
    const FrameArgs a = load_uniform(descs + it.stream);
    if (!run_tile<K, NR, TS, EXT>(a, it.tile, sm)) return;
  }
}

// Kernel for (storage, class K, budget, optional features compiled in);
// nullptr if not built.
const void* batch_kernel_ptr(int storage_bf16, int K, int budget, bool ext);

}  // namespace prost
