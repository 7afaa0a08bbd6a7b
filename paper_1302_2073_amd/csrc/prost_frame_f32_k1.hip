// Frame-kernel instantiations: f32 storage, k = 1..4.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_GROUP(frame_kernel_f32_g0, float, 1)
}  // namespace prost
