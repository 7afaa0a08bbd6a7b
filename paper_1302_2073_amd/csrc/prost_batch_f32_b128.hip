// Batched-form kernel instantiation: f32 storage, register budget 128.
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_f32_b128() { return (const void*)&batch_kernel<float, 128>; }
}  // namespace prost
