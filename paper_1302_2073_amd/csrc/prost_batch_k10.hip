// Batched-form kernels for subspace class K = 10 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k10(int storage_bf16, int budget, bool ext) {
  if (budget == kBudgetLds) return (storage_bf16 && !ext) ? batch_kernel_lds<10>() : nullptr;
  if (storage_bf16)
    return ext ? (budget == 64 ? (const void*)&batch_kernel<uint16_t, 10, batch_nr_bf16(64, 10), true>
                               : (const void*)&batch_kernel<uint16_t, 10, batch_nr_bf16(128, 10), true>)
               : (budget == 64 ? (const void*)&batch_kernel<uint16_t, 10, batch_nr_bf16(64, 10), false>
                               : (const void*)&batch_kernel<uint16_t, 10, batch_nr_bf16(128, 10), false>);
  return ext ? (budget == 64 ? (const void*)&batch_kernel<float, 10, batch_nr(64, 10), true>
                             : (const void*)&batch_kernel<float, 10, batch_nr(128, 10), true>)
             : (budget == 64 ? (const void*)&batch_kernel<float, 10, batch_nr(64, 10), false>
                             : (const void*)&batch_kernel<float, 10, batch_nr(128, 10), false>);
}
const void* batch_kernel_seq_k10(int storage_bf16) { return batch_kernel_seq<10>(storage_bf16); }
}  // namespace prost
