// Host-side definitions shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/prost.h"
#include "prost_device.hpp"

struct pros_handle {
  pros_params prm;
  int P = 0, C = 0, m = 0, k = 0;
  long long ldU = 0;
  int device = 0;
  int num_cu = 0;
  hipStream_t stream = nullptr;
  // device memory
  void* U = nullptr;
  void* xstage = nullptr;
  uint8_t* lab = nullptr;
  uint8_t* mask = nullptr;
  double* y = nullptr;
  long long* nframe = nullptr;
  pros_stats* stats = nullptr;
  double* part = nullptr;
  unsigned* sync = nullptr;
  void* reorth_ws = nullptr;
  float* pre_mean = nullptr;    // pre-processing: running average (m), or NULL
  float* pre_m2 = nullptr;      // sum of squared deviations (m)
  double* pre_stat = nullptr;   // [0] entry sum of pre_m2, [1] initialization frames accumulated
  float* score = nullptr;       // caller's buffer for per-entry label scores (m floats), or NULL
  void** seq = nullptr;         // device table of the frames of a sequence launch
  // launch configuration
  const void* kfn = nullptr;
  int G = 0, tpw = 0, NR = 0;
  int sync_mode = 2;       // 0: counter barrier, 1: tagged gather/broadcast, 2: two-level tagged, 3: tagged all-read
  int curv = 0;            // CG curvature schedule: 0 = second pass per step, 1 = H with the gradient
  bool coop = true;        // cooperative launch (co-residency guaranteed) or an ordinary dispatch
  long long* trace = nullptr;   // optional per-tile timestamps (diagnostics)
  bool mask_stale = true;       // mask not yet computed from the latest labels
  long long timeout_ticks = 0;
  // frames too large for a resident gang: every pass streams U (prost_stream.hip)
  bool streamed = false;
  void* stream_ws = nullptr;    // k-space state, per-entry w c and eta, per-workgroup partials
  int stream_blocks = 0;        // workgroups of a streamed pass
  // host bookkeeping
  long long submitted = 0;
  bool state_set = false;
  bool broken = false;
  pros_status broken_status = PROS_OK;
};

namespace prost {
inline namespace PROST_BLOCK_NS {
struct FrameArgs;
}
}  // namespace prost

namespace prost_host {
double effective_delta(const pros_params& p);
// Allocate and zero a tracker's device state.  g_force > 0 fixes the tile
// configuration (used by batches); otherwise it is chosen for the frame kernel.
pros_status create_handle(const pros_params* prm, hipStream_t stream, int nr_force, int tpw_force, int g_force,
                          pros_handle** out);
void free_handle(pros_handle* h);
pros_status check_usable(pros_handle* h);
pros_status sync_and_check(pros_handle* h);
prost::FrameArgs make_args(pros_handle* h, const void* x);
pros_status reset_exchange(pros_handle* h);
// Compute the mask (and foreground count) of the latest labels if a frame
// kernel has not done so yet.  Queued on the handle's stream.
pros_status refresh_mask(pros_handle* h);
// Pixels per workgroup tile for NR register rows per thread (a fraction
// `scale` of the full tile); even for bfloat16 storage so that row pairs
// stay inside one colour plane.
int tile_pixels(int storage, int NR, int channels, double scale, int threads = prost::kBlock);
// bfloat16 row pairs can be accessed as aligned 32-bit words in U (frame
// alignment is checked separately).
bool pair_layout(const pros_handle* h);
// Bytes of the exchange buffer for a gang of G workgroups: the regular
// slots, plus the wide region of the IRLS step when the stream uses it.
size_t part_bytes(const pros_handle* h, int G);

uint16_t bf16_rne(float f);
float bf16_to_f32(uint16_t b);
pros_status set_error(pros_status s, const char* fmt, ...);
}  // namespace prost_host

pros_status prost_reorth_launch(pros_handle* h);
// Seeded orthonormal m x k float64 matrix (Sec. 3.4 initialization) into a
// device buffer; and a handle's U set from it (rounded to the storage type).
pros_status prost_random_subspace(unsigned long long seed, uint32_t stream_index, long long m, int k, double* A,
                                  hipStream_t st);
pros_status prost_init_subspace(pros_handle* h, unsigned long long seed, uint32_t stream_index);
// The streamed path for frames whose register tiles do not fit the device.
pros_status prost_stream_alloc(pros_handle* h);
pros_status prost_stream_frame(pros_handle* h, const prost::FrameArgs& a);
