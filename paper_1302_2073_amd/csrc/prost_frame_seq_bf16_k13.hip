// Frame-kernel instantiations of the sequence form: bf16 storage, k = 13..16.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_SEQ_GROUP(frame_kernel_seq_bf16_g3, uint16_t, 13)
}  // namespace prost
