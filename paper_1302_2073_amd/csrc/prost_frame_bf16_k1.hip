// Frame-kernel instantiations: bf16 storage, k = 1..4.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_GROUP(frame_kernel_bf16_g0, uint16_t, 1)
}  // namespace prost
