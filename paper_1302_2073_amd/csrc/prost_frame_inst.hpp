// Instantiation helper: PROST_FRAME_GROUP(name, TS, K0) defines
// name(K, NR, ext) returning the frame kernel for K in [K0, K0+3], or nullptr
// for a row count that is not built.  float32 tiles: NR in {1, 2, 4, 8}
// (16 for K <= 8); bfloat16 tiles hold row pairs: NR in {2, 4, 8, 16}
// (32 for K <= 8).
#pragma once
#include "prost_frame.hpp"

namespace prost {
inline namespace PROST_BLOCK_NS {

template <typename TS, int KK, bool EXT, bool SEQ = false>
const void* frame_kernel_nr(int NR) {
  constexpr int KS = (KK <= 8) ? KK : 1;   // widest tile only for small K
  if constexpr (sizeof(TS) == 2) {
    switch (NR) {
      case 2: return (const void*)&frame_kernel<KK, 2, TS, EXT, SEQ>;
      case 4: return (const void*)&frame_kernel<KK, 4, TS, EXT, SEQ>;
      case 8: return (const void*)&frame_kernel<KK, 8, TS, EXT, SEQ>;
      case 16: return (const void*)&frame_kernel<KK, 16, TS, EXT, SEQ>;
      case 32: return (KK <= 8) ? (const void*)&frame_kernel<KS, 32, TS, EXT, SEQ> : nullptr;
      default: return nullptr;
    }
  } else {
    switch (NR) {
      case 1: return (const void*)&frame_kernel<KK, 1, TS, EXT, SEQ>;
      case 2: return (const void*)&frame_kernel<KK, 2, TS, EXT, SEQ>;
      case 4: return (const void*)&frame_kernel<KK, 4, TS, EXT, SEQ>;
      case 8: return (const void*)&frame_kernel<KK, 8, TS, EXT, SEQ>;
      case 16: return (KK <= 8) ? (const void*)&frame_kernel<KS, 16, TS, EXT, SEQ> : nullptr;
      default: return nullptr;
    }
  }
}

}  // inline namespace PROST_BLOCK_NS
}  // namespace prost

#define PROST_FRAME_GROUP(name, TS, K0)                                                   \
  const void* name(int K, int NR, bool ext) {                                             \
    switch (K) {                                                                          \
      case K0 + 0: return ext ? frame_kernel_nr<TS, K0 + 0, true>(NR) : frame_kernel_nr<TS, K0 + 0, false>(NR); \
      case K0 + 1: return ext ? frame_kernel_nr<TS, K0 + 1, true>(NR) : frame_kernel_nr<TS, K0 + 1, false>(NR); \
      case K0 + 2: return ext ? frame_kernel_nr<TS, K0 + 2, true>(NR) : frame_kernel_nr<TS, K0 + 2, false>(NR); \
      case K0 + 3: return ext ? frame_kernel_nr<TS, K0 + 3, true>(NR) : frame_kernel_nr<TS, K0 + 3, false>(NR); \
      default: return nullptr;                                                            \
    }                                                                                     \
  }

// The sequence form (default features only): name(K, NR).
#define PROST_FRAME_SEQ_GROUP(name, TS, K0)                         \
  const void* name(int K, int NR) {                                 \
    switch (K) {                                                    \
      case K0 + 0: return frame_kernel_nr<TS, K0 + 0, false, true>(NR); \
      case K0 + 1: return frame_kernel_nr<TS, K0 + 1, false, true>(NR); \
      case K0 + 2: return frame_kernel_nr<TS, K0 + 2, false, true>(NR); \
      case K0 + 3: return frame_kernel_nr<TS, K0 + 3, false, true>(NR); \
      default: return nullptr;                                      \
    }                                                               \
  }
