// Frame-kernel instantiations: f32 storage, k = 9..12.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_GROUP(frame_kernel_f32_g2, float, 9)
}  // namespace prost
