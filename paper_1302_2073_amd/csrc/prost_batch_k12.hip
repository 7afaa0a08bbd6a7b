// Batched-form kernels for subspace class K = 12 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k12(int storage_bf16, int budget) {
  if (storage_bf16)
    return budget == 64 ? (const void*)&batch_kernel<uint16_t, 12, batch_nr_bf16(64, 12)>
                        : (const void*)&batch_kernel<uint16_t, 12, batch_nr_bf16(128, 12)>;
  return budget == 64 ? (const void*)&batch_kernel<float, 12, batch_nr(64, 12)>
                      : (const void*)&batch_kernel<float, 12, batch_nr(128, 12)>;
}
}  // namespace prost
