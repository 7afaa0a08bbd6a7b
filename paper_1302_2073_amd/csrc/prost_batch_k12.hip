// Batched-form kernels for subspace class K = 12 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k12(int storage_bf16, int budget, bool ext) {
  if (budget == kBudgetLds) return (storage_bf16 && !ext) ? batch_kernel_lds<12>() : nullptr;
  if (storage_bf16)
    return ext ? (budget == 64 ? (const void*)&batch_kernel<uint16_t, 12, batch_nr_bf16(64, 12), true>
                               : (const void*)&batch_kernel<uint16_t, 12, batch_nr_bf16(128, 12), true>)
               : (budget == 64 ? (const void*)&batch_kernel<uint16_t, 12, batch_nr_bf16(64, 12), false>
                               : (const void*)&batch_kernel<uint16_t, 12, batch_nr_bf16(128, 12), false>);
  return ext ? (budget == 64 ? (const void*)&batch_kernel<float, 12, batch_nr(64, 12), true>
                             : (const void*)&batch_kernel<float, 12, batch_nr(128, 12), true>)
             : (budget == 64 ? (const void*)&batch_kernel<float, 12, batch_nr(64, 12), false>
                             : (const void*)&batch_kernel<float, 12, batch_nr(128, 12), false>);
}
const void* batch_kernel_seq_k12(int storage_bf16) { return batch_kernel_seq<12>(storage_bf16); }
}  // namespace prost
