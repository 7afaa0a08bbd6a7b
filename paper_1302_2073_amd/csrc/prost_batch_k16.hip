// Batched-form kernels for subspace class K = 16 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k16(int storage_bf16, int budget, bool ext) {
  if (budget == kBudgetLds) return (storage_bf16 && !ext) ? batch_kernel_lds<16>() : nullptr;
  if (storage_bf16)
    return ext ? (budget == 64 ? (const void*)&batch_kernel<uint16_t, 16, batch_nr_bf16(64, 16), true>
                               : (const void*)&batch_kernel<uint16_t, 16, batch_nr_bf16(128, 16), true>)
               : (budget == 64 ? (const void*)&batch_kernel<uint16_t, 16, batch_nr_bf16(64, 16), false>
                               : (const void*)&batch_kernel<uint16_t, 16, batch_nr_bf16(128, 16), false>);
  return ext ? (budget == 64 ? (const void*)&batch_kernel<float, 16, batch_nr(64, 16), true>
                             : (const void*)&batch_kernel<float, 16, batch_nr(128, 16), true>)
             : (budget == 64 ? (const void*)&batch_kernel<float, 16, batch_nr(64, 16), false>
                             : (const void*)&batch_kernel<float, 16, batch_nr(128, 16), false>);
}
const void* batch_kernel_seq_k16(int storage_bf16) { return batch_kernel_seq<16>(storage_bf16); }
}  // namespace prost
