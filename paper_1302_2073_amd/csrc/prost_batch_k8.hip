// Batched-form kernels for subspace class K = 8 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k8(int storage_bf16, int budget, bool ext) {
  if (budget == kBudgetLds) return nullptr;   // no LDS form below k class 10
  if (storage_bf16)
    return ext ? (budget == 64 ? (const void*)&batch_kernel<uint16_t, 8, batch_nr_bf16(64, 8), true>
                               : (const void*)&batch_kernel<uint16_t, 8, batch_nr_bf16(128, 8), true>)
               : (budget == 64 ? (const void*)&batch_kernel<uint16_t, 8, batch_nr_bf16(64, 8), false>
                               : (const void*)&batch_kernel<uint16_t, 8, batch_nr_bf16(128, 8), false>);
  return ext ? (budget == 64 ? (const void*)&batch_kernel<float, 8, batch_nr(64, 8), true>
                             : (const void*)&batch_kernel<float, 8, batch_nr(128, 8), true>)
             : (budget == 64 ? (const void*)&batch_kernel<float, 8, batch_nr(64, 8), false>
                             : (const void*)&batch_kernel<float, 8, batch_nr(128, 8), false>);
}
const void* batch_kernel_seq_k8(int storage_bf16) { return batch_kernel_seq<8>(storage_bf16); }
}  // namespace prost
