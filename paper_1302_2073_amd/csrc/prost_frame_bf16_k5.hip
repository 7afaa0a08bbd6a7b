// Frame-kernel instantiations: bf16 storage, k = 5..8.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_GROUP(frame_kernel_bf16_g1, uint16_t, 5)
}  // namespace prost
