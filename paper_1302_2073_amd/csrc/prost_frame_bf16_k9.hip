// Frame-kernel instantiations: bf16 storage, k = 9..12.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_GROUP(frame_kernel_bf16_g2, uint16_t, 9)
}  // namespace prost
