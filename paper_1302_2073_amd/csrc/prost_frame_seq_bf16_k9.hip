// Frame-kernel instantiations of the sequence form: bf16 storage, k = 9..12.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_SEQ_GROUP(frame_kernel_seq_bf16_g2, uint16_t, 9)
}  // namespace prost
