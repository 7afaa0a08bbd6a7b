// Batched-form kernel instantiation: bf16 storage, register budget 128.
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_bf16_b128() { return (const void*)&batch_kernel<uint16_t, 128>; }
}  // namespace prost
