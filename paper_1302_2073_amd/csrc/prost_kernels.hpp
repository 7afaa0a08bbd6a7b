// Lookup of the frame-kernel instantiations (one translation unit per
// storage type so that they compile in parallel).
#pragma once

namespace prost {
// Frame kernel for exact subspace dimension K (1..16) and NR register rows
// per thread (float32: 1, 2, 4, 8, 16 for K <= 8; bfloat16: 2, 4, 8, 16,
// 32 for K <= 8), with or without the optional features (pre-processing, label scores).  nullptr when
// not built.
const void* frame_kernel_f32(int K, int NR, bool ext);
const void* frame_kernel_bf16(int K, int NR, bool ext);
// The sequence form (several frames per launch, default features) of the
// same tile; nullptr when not built.
const void* frame_kernel_seq(int bf16, int K, int NR);
}  // namespace prost
