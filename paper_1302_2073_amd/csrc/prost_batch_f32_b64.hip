// Batched-form kernel instantiation: f32 storage, register budget 64.
#include "prost_batch.hpp"

namespace prost {
const void* batch_kernel_f32_b64() { return (const void*)&batch_kernel<float, 64>; }
}  // namespace prost
