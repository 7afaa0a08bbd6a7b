// Batched form: many independent video streams (uneven resolution and k)
// advance by one frame each in ONE persistent cooperative launch.
//
// Every stream is split into workgroup tiles exactly as in the single-stream
// kernel and owns a gang of workgroups for the frame's gang-wide reductions.
// The launch is a fixed grid of resident workgroups; a host-built schedule
// assigns each workgroup a sequence of (stream, tile) items, one per round.
// Gangs of one round are disjoint sets of workgroups, so every gang is
// resident; streams of a round do not wait for each other, and a workgroup
// moves to its next item as soon as its current stream's frame is done.
#pragma once

#include "prost_frame.hpp"

namespace prost {

struct BatchItem {
  int stream;   // -1: idle slot
  int tile;
};

// Register rows per thread for subspace dimension K at a register budget of
// about BUDGET floats of U per thread.
template <int BUDGET>
struct BatchNR {
  template <int K>
  static constexpr int nr() {
    return (BUDGET / K >= 16) ? 16 : (BUDGET / K >= 12) ? 12 : (BUDGET / K >= 8) ? 8 : 4;
  }
};

template <typename TS, int BUDGET>
__device__ __forceinline__ bool batch_dispatch(const FrameArgs& a, int tile, FrameSmem& sm) {
  using NRs = BatchNR<BUDGET>;
  switch (a.k) {
#define PROST_BATCH_CASE(KK) \
    case KK: return frame_tile<KK, NRs::template nr<KK>(), TS>(a, tile, sm);
    PROST_BATCH_CASE(1) PROST_BATCH_CASE(2) PROST_BATCH_CASE(3) PROST_BATCH_CASE(4)
    PROST_BATCH_CASE(5) PROST_BATCH_CASE(6) PROST_BATCH_CASE(7) PROST_BATCH_CASE(8)
    PROST_BATCH_CASE(9) PROST_BATCH_CASE(10) PROST_BATCH_CASE(11) PROST_BATCH_CASE(12)
    PROST_BATCH_CASE(13) PROST_BATCH_CASE(14) PROST_BATCH_CASE(15) PROST_BATCH_CASE(16)
#undef PROST_BATCH_CASE
    default: return true;
  }
}

template <typename TS, int BUDGET>
__global__ __launch_bounds__(kBlock) void batch_kernel(const FrameArgs* __restrict__ descs,
                                                       const BatchItem* __restrict__ items, int rounds) {
  __shared__ FrameSmem sm;
  for (int r = 0; r < rounds; ++r) {
    const BatchItem it = items[(size_t)r * gridDim.x + blockIdx.x];
    if (it.stream < 0) continue;
    const FrameArgs a = descs[it.stream];
    if (!batch_dispatch<TS, BUDGET>(a, it.tile, sm)) return;
  }
}

}  // namespace prost
