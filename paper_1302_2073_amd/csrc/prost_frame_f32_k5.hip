// Frame-kernel instantiations: f32 storage, k = 5..8.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_GROUP(frame_kernel_f32_g1, float, 5)
}  // namespace prost
