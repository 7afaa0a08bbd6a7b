// Batched-form kernels for subspace class K = 2 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k2(int storage_bf16, int budget, bool ext) {
  if (budget == kBudgetLds) return nullptr;   // no LDS form below k class 10
  if (storage_bf16)
    return ext ? (budget == 64 ? (const void*)&batch_kernel<uint16_t, 2, batch_nr_bf16(64, 2), true>
                               : (const void*)&batch_kernel<uint16_t, 2, batch_nr_bf16(128, 2), true>)
               : (budget == 64 ? (const void*)&batch_kernel<uint16_t, 2, batch_nr_bf16(64, 2), false>
                               : (const void*)&batch_kernel<uint16_t, 2, batch_nr_bf16(128, 2), false>);
  return ext ? (budget == 64 ? (const void*)&batch_kernel<float, 2, batch_nr(64, 2), true>
                             : (const void*)&batch_kernel<float, 2, batch_nr(128, 2), true>)
             : (budget == 64 ? (const void*)&batch_kernel<float, 2, batch_nr(64, 2), false>
                             : (const void*)&batch_kernel<float, 2, batch_nr(128, 2), false>);
}
const void* batch_kernel_seq_k2(int storage_bf16) { return batch_kernel_seq<2>(storage_bf16); }
}  // namespace prost
