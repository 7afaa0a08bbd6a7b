// Frame-kernel instantiations of the sequence form: f32 storage, k = 13..16.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_SEQ_GROUP(frame_kernel_seq_f32_g3, float, 13)
}  // namespace prost
