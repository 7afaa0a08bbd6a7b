// Batched-form kernels for subspace class K = 5 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k5(int storage_bf16, int budget, bool ext) {
  if (budget == kBudgetLds) return nullptr;   // no LDS form below k class 10
  if (storage_bf16)
    return ext ? (budget == 64 ? (const void*)&batch_kernel<uint16_t, 5, batch_nr_bf16(64, 5), true>
                               : (const void*)&batch_kernel<uint16_t, 5, batch_nr_bf16(128, 5), true>)
               : (budget == 64 ? (const void*)&batch_kernel<uint16_t, 5, batch_nr_bf16(64, 5), false>
                               : (const void*)&batch_kernel<uint16_t, 5, batch_nr_bf16(128, 5), false>);
  return ext ? (budget == 64 ? (const void*)&batch_kernel<float, 5, batch_nr(64, 5), true>
                             : (const void*)&batch_kernel<float, 5, batch_nr(128, 5), true>)
             : (budget == 64 ? (const void*)&batch_kernel<float, 5, batch_nr(64, 5), false>
                             : (const void*)&batch_kernel<float, 5, batch_nr(128, 5), false>);
}
const void* batch_kernel_seq_k5(int storage_bf16) { return batch_kernel_seq<5>(storage_bf16); }
}  // namespace prost
