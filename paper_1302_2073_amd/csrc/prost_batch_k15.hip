// Batched-form kernels for subspace class K = 15 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k15(int storage_bf16, int budget, bool ext) {
  if (budget == kBudgetLds) return (storage_bf16 && !ext) ? batch_kernel_lds<15>() : nullptr;
  if (storage_bf16)
    return ext ? (budget == 64 ? (const void*)&batch_kernel<uint16_t, 15, batch_nr_bf16(64, 15), true>
                               : (const void*)&batch_kernel<uint16_t, 15, batch_nr_bf16(128, 15), true>)
               : (budget == 64 ? (const void*)&batch_kernel<uint16_t, 15, batch_nr_bf16(64, 15), false>
                               : (const void*)&batch_kernel<uint16_t, 15, batch_nr_bf16(128, 15), false>);
  return ext ? (budget == 64 ? (const void*)&batch_kernel<float, 15, batch_nr(64, 15), true>
                             : (const void*)&batch_kernel<float, 15, batch_nr(128, 15), true>)
             : (budget == 64 ? (const void*)&batch_kernel<float, 15, batch_nr(64, 15), false>
                             : (const void*)&batch_kernel<float, 15, batch_nr(128, 15), false>);
}
const void* batch_kernel_seq_k15(int storage_bf16) { return batch_kernel_seq<15>(storage_bf16); }
}  // namespace prost
