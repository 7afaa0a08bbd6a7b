// Device-side building blocks of the pROST frame kernels (gfx950).
//
// * storage conversions (float32 / bfloat16 with round-to-nearest-even),
// * the per-entry cost functor phi and its majoriser weight c = phi'/r
//   (Sec. 3.1, eqs. smoothlpnorm / weightedLPnorm),
// * deterministic wave / workgroup / gang reductions,
// * the gang barrier used by the persistent frame kernel: one atomic arrival
//   per workgroup on a monotone counter, bounded spin, error word.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Threads per workgroup of the persistent kernels: 512 (8 wavefronts, one
// workgroup per CU) by default; a translation unit that defines PROST_BLOCK
// as 256 before including this header builds its kernels for 256-thread
// workgroups (4 wavefronts, two workgroups of different streams per CU).
// Everything below lives in a namespace named after the block size, so the
// two builds never share a definition.
#ifndef PROST_BLOCK
#define PROST_BLOCK 512
#endif
#if PROST_BLOCK == 512
#define PROST_BLOCK_NS b512
#elif PROST_BLOCK == 256
#define PROST_BLOCK_NS b256
#else
#error "PROST_BLOCK must be 256 or 512"
#endif

namespace prost {
inline namespace PROST_BLOCK_NS {

constexpr int kBlock = PROST_BLOCK;    // threads per workgroup
constexpr int kWaves = kBlock / 64;    // wavefronts per workgroup
constexpr int kMaxK = 16;
constexpr int kSlot = 32;              // doubles per workgroup partial slot

// error bits in sync[2]
constexpr unsigned kErrTimeout = 1u;
constexpr unsigned kErrBadFrame = 2u;

// Thread index through an opaque move.  In a persistent loop over tiles the
// compiler would otherwise hoist all index arithmetic derived from it out of
// the loop and keep the results live across whole frames, taking registers
// from the register-resident tile.
__device__ __forceinline__ int thread_index() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// ---------------------------------------------------------------------------
// storage
// ---------------------------------------------------------------------------
__device__ __forceinline__ float ld_elem(const float* p, long long i) { return p[i]; }
__device__ __forceinline__ double ld_elem(const double* p, long long i) { return p[i]; }
__device__ __forceinline__ float ld_elem(const uint16_t* p, long long i) {
  return __uint_as_float(((uint32_t)p[i]) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ void st_elem(float* p, long long i, float v) { p[i] = v; }
__device__ __forceinline__ void st_elem(uint16_t* p, long long i, float v) { p[i] = f32_to_bf16_rne(v); }

// ---------------------------------------------------------------------------
// cost functor
// ---------------------------------------------------------------------------
struct CostParams {
  float p;        // lp exponent
  float half_p;   // p / 2
  float mu;       // smoothing
  float inv_mu;   // 1 / mu
  float half_p_m1;  // p / 2 - 1
  float inv_p;    // 1 / p
  int form;       // 0: (r^2+mu)^(p/2), 1: log(1 + r^2/mu)
};

// phi(r) and c(r) = phi'(r)/r.  lp: c = p s^(p/2-1) with s = r^2 + mu and
// phi = s^(p/2) = c s / p (two transcendental instructions: log2, exp2).
// log: phi = log(1 + r^2/mu), c = 2/s.
__device__ __forceinline__ void cost_eval(float r, const CostParams& cp, float& phi, float& c) {
  const float s = fmaf(r, r, cp.mu);
  if (cp.form == 0) {
    c = cp.p * __builtin_amdgcn_exp2f(cp.half_p_m1 * __builtin_amdgcn_logf(s));
    phi = c * s * cp.inv_p;
  } else {
    phi = 0.69314718055994531f * __builtin_amdgcn_logf(fmaf(r * r, cp.inv_mu, 1.0f));
    c = 2.0f * __builtin_amdgcn_rcpf(s);
  }
}

// ---------------------------------------------------------------------------
// reductions (fixed order: identical results in every workgroup and run)
// ---------------------------------------------------------------------------
// Cross-lane moves in the vector unit (gfx950): DPP row rotations (lane l of
// a 16-lane row reads lane l - r mod 16 for row_ror:r) and quad permutations,
// and the permlane swaps that trade the upper 32 (16 of each 32) lanes of one
// register with the lower ones of another.  Every lane must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)b, CTRL, 0xf, 0xf, false);
  const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128, kRowRor12 = 0x12C;
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E;   // quad_perm [1,0,3,2], [2,3,0,1]

// v of lane l plus v of lane l ^ 32 (W = 32) or l ^ 16 (W = 16), the same
// sum in both lanes of a pair.
template <int W>
__device__ __forceinline__ float swap_sum(float v) {
  const auto r = (W == 32) ? __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false)
                           : __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int W>
__device__ __forceinline__ double swap_sum(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const auto lo = (W == 32) ? __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false)
                            : __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = (W == 32) ? __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false)
                            : __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  const double x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return x + y;
}

// Sum over each 16-lane row, in every lane of the row: partners l ^ 8, then
// l - 4 mod 16 (with the first step, the sum over l, l ^ 4, l ^ 8, l ^ 12),
// then l ^ 2 and l ^ 1.  Each step adds the same two values in both lanes of
// a pair, so every lane of the row holds the same total.
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
  v += dpp_mov<kRowRor8>(v);
  v += dpp_mov<kRowRor4>(v);
  v += dpp_mov<kQuadXor2>(v);
  v += dpp_mov<kQuadXor1>(v);
  return v;
}
// Sum over the 64 lanes, in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v = swap_sum<32>(v);
  v = swap_sum<16>(v);
  return row16_sum(v);
}

constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : 32; }
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Reduce-scatter of L values across the 64 lanes of a wavefront: at each of
// log2(P) stages (P = L rounded up to a power of two) a lane keeps one half of
// its values and adds its partner's copy of that half, so the work halves
// every stage (P - 1 exchanges instead of 6 L); the lane bits left over are
// then summed over (all-reduce).  The exchanges stay in the vector unit:
// partners across lane bit 5 or 4 trade both halves in one
// v_permlane32_swap / v_permlane16_swap, partners across bits 3, 0 and 1 are
// reached with DPP (row_ror:8, quad_perm), and the last all-reduce bit, 2,
// with row_ror:12 (lane l reads lane l - 12 mod 16 of its row), which gives
// the partner l + 4 to the lanes with bit 2 clear: those lanes own the
// results.  Stage order: bits 5, 4, 3, 0, 1, then 2.  On return every owner
// lane (wave_rs_owner) holds the wavefront total of component `comp`, each
// component in exactly one owner.  Fixed order, deterministic.
constexpr int kRsOrder[6] = {5, 4, 3, 0, 1, 2};

// One reduce-scatter stage across lane bit b for the value pair (lo, hi):
// lanes with the bit clear end with lo + partner's lo, the others with
// hi + partner's hi.
__device__ __forceinline__ float rs_stage(int b, float lo, float hi, int lane) {
  if (b == 5 || b == 4) {
    const auto r = (b == 5) ? __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false)
                            : __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool up = (lane >> b) & 1;
  const float send = up ? lo : hi, keep = up ? hi : lo;
  return keep + (b == 3 ? dpp_mov<kRowRor8>(send) : b == 0 ? dpp_mov<kQuadXor1>(send) : dpp_mov<kQuadXor2>(send));
}

// One all-reduce stage across lane bit b (bit 2: right in the lanes with bit
// 2 clear only).
__device__ __forceinline__ float ar_stage(int b, float v) {
  if (b == 5 || b == 4) {
    const auto r = (b == 5) ? __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false)
                            : __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  return v + (b == 3 ? dpp_mov<kRowRor8>(v) : b == 0 ? dpp_mov<kQuadXor1>(v) : b == 1 ? dpp_mov<kQuadXor2>(v)
                                                                     : dpp_mov<kRowRor12>(v));
}

template <int L>
__device__ __forceinline__ float wave_reduce_scatter(float (&a)[L], int& comp) {
  constexpr int P = pow2_at_least(L);
  constexpr int S = ilog2(P);
  static_assert(S <= 5, "at most 32 components");
  const int lane = thread_index() & 63;
  int base = 0;
#pragma unroll
  for (int st = 0; st < S; ++st) {
    const int half = P >> (st + 1);
    const int b = kRsOrder[st];
#pragma unroll
    for (int i = 0; i < half; ++i) {      // in place; entries >= L are zero
      const float lo = a[i];
      const float hi = (i + half < L) ? a[(i + half < L) ? i + half : 0] : 0.f;
      a[i] = rs_stage(b, lo, hi, lane);
    }
    if ((lane >> b) & 1) base += half;
  }
#pragma unroll
  for (int st = S; st < 6; ++st) a[0] = ar_stage(kRsOrder[st], a[0]);
  comp = base;
  return a[0];
}

// The lanes that hold each component of wave_reduce_scatter<L> once: those
// whose all-reduced bits are clear.
template <int L>
__device__ __forceinline__ bool wave_rs_owner(int lane) {
  constexpr int S = ilog2(pow2_at_least(L));
  int mask = 0;
#pragma unroll
  for (int st = S; st < 6; ++st) mask |= 1 << kRsOrder[st];
  return (lane & mask) == 0;
}

__device__ __forceinline__ long long now_ticks() { return wall_clock64(); }

// Epoch tags carried in the low 8 mantissa bits of a float64 partial sum:
// an aligned 8-byte store is single-copy atomic, so a reader that sees the
// current tag also sees the value written with it, without a flag or fence.
// Clearing 8 of 52 mantissa bits changes a sum by at most 2^-44 relative.
__device__ __forceinline__ double tag_value(double v, unsigned ep) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return __longlong_as_double((long long)((b & ~0xFFull) | (ep & 0xFFu)));
}
__device__ __forceinline__ unsigned tag_of(double v) {
  return (unsigned)((unsigned long long)__double_as_longlong(v) & 0xFFull);
}
__device__ __forceinline__ double untag(double v) {
  return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v) & ~0xFFull));
}
__device__ __forceinline__ double ld_tagged(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_tagged(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Gang barrier.  Every workgroup of the gang calls it the same number of
// times; `target` = base + G * (index of this barrier + 1).  Thread 0 makes
// the workgroup's prior global writes visible at device scope, arrives, and
// spins (bounded by `timeout` wall-clock ticks, also leaving early when an
// error bit is set).  Returns false in every thread when the gang must abort.
__device__ __forceinline__ bool gang_barrier(unsigned* sync, unsigned target, long long timeout,
                                             int* s_ctl) {
  __syncthreads();
  if (thread_index() == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(&sync[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = now_ticks();
    int ok = 1;
    unsigned spins = 0;
    while ((int)(__hip_atomic_load(&sync[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 63u) == 0) {
        if (__hip_atomic_load(&sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout) { ok = 0; break; }
        if (now_ticks() - t0 > timeout) {
          __hip_atomic_fetch_or(&sync[2], kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ctl[0] = ok;
  }
  __syncthreads();
  return s_ctl[0] != 0;
}

}  // inline namespace PROST_BLOCK_NS
}  // namespace prost
