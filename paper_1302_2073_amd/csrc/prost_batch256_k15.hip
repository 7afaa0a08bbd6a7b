// Batched-form kernels of subspace class K = 15 built for 256-thread
// workgroups (two workgroups, of two different streams, share each CU, so
// one stream's tile can run while the other waits on a gang exchange);
// register budget 128, default features, both storage types.
#define PROST_BLOCK 256
#include "prost_batch.hpp"

namespace prost {
const void* batch256_kernel_k15(int storage_bf16) {
  return storage_bf16 ? (const void*)&batch_kernel<uint16_t, 15, batch_nr_bf16(128, 15), false>
                      : (const void*)&batch_kernel<float, 15, batch_nr(128, 15), false>;
}
const void* batch256_kernel_seq_k15(int storage_bf16) { return batch_kernel_seq<15>(storage_bf16); }
}  // namespace prost
