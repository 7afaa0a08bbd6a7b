// Instantiation helper: PROST_FRAME_GROUP(name, TS, K0) defines
// name(K, NR) returning the frame kernel for K in [K0, K0+3].
#pragma once
#include "prost_frame.hpp"

#define PROST_FRAME_NR(KK, TS)                                                         \
  switch (NR) {                                                                        \
    case 1: return (const void*)&frame_kernel<KK, 1, TS>;                              \
    case 2: return (const void*)&frame_kernel<KK, 2, TS>;                              \
    case 4: return (const void*)&frame_kernel<KK, 4, TS>;                              \
    case 8: return (const void*)&frame_kernel<KK, 8, TS>;                              \
    case 16: return (KK <= 8) ? (const void*)&frame_kernel<(KK <= 8 ? KK : 1), 16, TS> \
                              : nullptr;                                               \
    default: return nullptr;                                                           \
  }

#define PROST_FRAME_GROUP(name, TS, K0)                 \
  const void* name(int K, int NR) {                     \
    switch (K) {                                        \
      case K0 + 0: PROST_FRAME_NR(K0 + 0, TS)           \
      case K0 + 1: PROST_FRAME_NR(K0 + 1, TS)           \
      case K0 + 2: PROST_FRAME_NR(K0 + 2, TS)           \
      case K0 + 3: PROST_FRAME_NR(K0 + 3, TS)           \
      default: return nullptr;                          \
    }                                                   \
  }
