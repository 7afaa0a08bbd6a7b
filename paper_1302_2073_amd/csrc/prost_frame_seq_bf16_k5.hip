// Frame-kernel instantiations of the sequence form: bf16 storage, k = 5..8.
#include "prost_frame_inst.hpp"

namespace prost {
PROST_FRAME_SEQ_GROUP(frame_kernel_seq_bf16_g1, uint16_t, 5)
}  // namespace prost
