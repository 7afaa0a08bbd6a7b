// Batched-form kernel instantiation: bf16 storage, register budget 64.
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_bf16_b64() { return (const void*)&batch_kernel<uint16_t, 64>; }
}  // namespace prost
