// Lookup of the frame-kernel instantiations (one translation unit per
// storage type so that they compile in parallel).
#pragma once

namespace prost {
// Frame kernel for exact subspace dimension K (1..16) and NR register rows
// per thread (1, 2, 4, 8; 16 only for K <= 8).  nullptr when not built.
const void* frame_kernel_f32(int K, int NR);
const void* frame_kernel_bf16(int K, int NR);
}  // namespace prost
