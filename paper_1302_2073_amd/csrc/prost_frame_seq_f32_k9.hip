// Frame-kernel instantiations of the sequence form: f32 storage, k = 9..12.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_SEQ_GROUP(frame_kernel_seq_f32_g2, float, 9)
}  // namespace prost
