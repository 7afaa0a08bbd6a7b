// Frame-kernel instantiations of the sequence form: f32 storage, k = 5..8.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_SEQ_GROUP(frame_kernel_seq_f32_g1, float, 5)
}  // namespace prost
