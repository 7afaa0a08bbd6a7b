// Dispatch from (storage, K, NR) to a frame-kernel instantiation.
#include "prost_kernels.hpp"

namespace prost {
const void* frame_kernel_f32_g0(int K, int NR, bool ext);
const void* frame_kernel_f32_g1(int K, int NR, bool ext);
const void* frame_kernel_f32_g2(int K, int NR, bool ext);
const void* frame_kernel_f32_g3(int K, int NR, bool ext);
const void* frame_kernel_bf16_g0(int K, int NR, bool ext);
const void* frame_kernel_bf16_g1(int K, int NR, bool ext);
const void* frame_kernel_bf16_g2(int K, int NR, bool ext);
const void* frame_kernel_bf16_g3(int K, int NR, bool ext);
const void* frame_kernel_seq_f32_g0(int K, int NR);
const void* frame_kernel_seq_f32_g1(int K, int NR);
const void* frame_kernel_seq_f32_g2(int K, int NR);
const void* frame_kernel_seq_f32_g3(int K, int NR);
const void* frame_kernel_seq_bf16_g0(int K, int NR);
const void* frame_kernel_seq_bf16_g1(int K, int NR);
const void* frame_kernel_seq_bf16_g2(int K, int NR);
const void* frame_kernel_seq_bf16_g3(int K, int NR);

const void* frame_kernel_f32(int K, int NR, bool ext) {
  if (K < 1 || K > 16) return nullptr;
  switch ((K - 1) / 4) {
    case 0: return frame_kernel_f32_g0(K, NR, ext);
    case 1: return frame_kernel_f32_g1(K, NR, ext);
    case 2: return frame_kernel_f32_g2(K, NR, ext);
    default: return frame_kernel_f32_g3(K, NR, ext);
  }
}

const void* frame_kernel_bf16(int K, int NR, bool ext) {
  if (K < 1 || K > 16) return nullptr;
  switch ((K - 1) / 4) {
    case 0: return frame_kernel_bf16_g0(K, NR, ext);
    case 1: return frame_kernel_bf16_g1(K, NR, ext);
    case 2: return frame_kernel_bf16_g2(K, NR, ext);
    default: return frame_kernel_bf16_g3(K, NR, ext);
  }
}

const void* frame_kernel_seq(int bf16, int K, int NR) {
  if (K < 1 || K > 16) return nullptr;
  switch ((K - 1) / 4) {
    case 0: return bf16 ? frame_kernel_seq_bf16_g0(K, NR) : frame_kernel_seq_f32_g0(K, NR);
    case 1: return bf16 ? frame_kernel_seq_bf16_g1(K, NR) : frame_kernel_seq_f32_g1(K, NR);
    case 2: return bf16 ? frame_kernel_seq_bf16_g2(K, NR) : frame_kernel_seq_f32_g2(K, NR);
    default: return bf16 ? frame_kernel_seq_bf16_g3(K, NR) : frame_kernel_seq_f32_g3(K, NR);
  }
}
}  // namespace prost
