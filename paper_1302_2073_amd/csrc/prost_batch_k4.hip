// Batched-form kernels for subspace class K = 4 (both storage types, both
// register budgets).
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_k4(int storage_bf16, int budget, bool ext) {
  if (budget == kBudgetLds) return nullptr;   // no LDS form below k class 10
  if (storage_bf16)
    return ext ? (budget == 64 ? (const void*)&batch_kernel<uint16_t, 4, batch_nr_bf16(64, 4), true>
                               : (const void*)&batch_kernel<uint16_t, 4, batch_nr_bf16(128, 4), true>)
               : (budget == 64 ? (const void*)&batch_kernel<uint16_t, 4, batch_nr_bf16(64, 4), false>
                               : (const void*)&batch_kernel<uint16_t, 4, batch_nr_bf16(128, 4), false>);
  return ext ? (budget == 64 ? (const void*)&batch_kernel<float, 4, batch_nr(64, 4), true>
                             : (const void*)&batch_kernel<float, 4, batch_nr(128, 4), true>)
             : (budget == 64 ? (const void*)&batch_kernel<float, 4, batch_nr(64, 4), false>
                             : (const void*)&batch_kernel<float, 4, batch_nr(128, 4), false>);
}
const void* batch_kernel_seq_k4(int storage_bf16) { return batch_kernel_seq<4>(storage_bf16); }
}  // namespace prost
