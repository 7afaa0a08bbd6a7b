// Batched form (C ABI): n independent streams, one persistent cooperative
// launch per batch step, optional hipGraph replay, and a schedule tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/prost.h"
#include "prost_batch.hpp"
#include "prost_host.hpp"

namespace prost {
const void* batch_kernel_k2(int, int, bool);
const void* batch_kernel_k4(int, int, bool);
const void* batch_kernel_k5(int, int, bool);
const void* batch_kernel_k8(int, int, bool);
const void* batch_kernel_k10(int, int, bool);
const void* batch_kernel_k12(int, int, bool);
const void* batch_kernel_k15(int, int, bool);
const void* batch_kernel_k16(int, int, bool);
const void* batch_kernel_seq_k2(int);
const void* batch_kernel_seq_k4(int);
const void* batch_kernel_seq_k5(int);
const void* batch_kernel_seq_k8(int);
const void* batch_kernel_seq_k10(int);
const void* batch_kernel_seq_k12(int);
const void* batch_kernel_seq_k15(int);
const void* batch_kernel_seq_k16(int);

const void* batch256_kernel_k15(int);
const void* batch256_kernel_seq_k15(int);

const void* batch256_kernel_ptr(int bf16, int K) { return K == 15 ? batch256_kernel_k15(bf16) : nullptr; }
const void* batch256_kernel_seq_ptr(int bf16, int K) { return K == 15 ? batch256_kernel_seq_k15(bf16) : nullptr; }

const void* batch_kernel_seq_ptr(int bf16, int K) {
  switch (K) {
    case 2: return batch_kernel_seq_k2(bf16);
    case 4: return batch_kernel_seq_k4(bf16);
    case 5: return batch_kernel_seq_k5(bf16);
    case 8: return batch_kernel_seq_k8(bf16);
    case 10: return batch_kernel_seq_k10(bf16);
    case 12: return batch_kernel_seq_k12(bf16);
    case 15: return batch_kernel_seq_k15(bf16);
    case 16: return batch_kernel_seq_k16(bf16);
    default: return nullptr;
  }
}

const void* batch_kernel_ptr(int bf16, int K, int budget, bool ext) {
  switch (K) {
    case 2: return batch_kernel_k2(bf16, budget, ext);
    case 4: return batch_kernel_k4(bf16, budget, ext);
    case 5: return batch_kernel_k5(bf16, budget, ext);
    case 8: return batch_kernel_k8(bf16, budget, ext);
    case 10: return batch_kernel_k10(bf16, budget, ext);
    case 12: return batch_kernel_k12(bf16, budget, ext);
    case 15: return batch_kernel_k15(bf16, budget, ext);
    case 16: return batch_kernel_k16(bf16, budget, ext);
    default: return nullptr;
  }
}
}  // namespace prost

using prost::BatchItem;
using prost::FrameArgs;

#define fail prost_host::set_error

namespace {
constexpr int kBudgets[] = {64, 128, prost::kBudgetLds};
}  // namespace

struct pros_batch {
  int n = 0;
  int storage = PROS_F32;
  int kclass = 16;               // compiled subspace class covering every stream's k
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;   // graphs are captured here, replayed on `stream`
  int num_cu = 0;
  std::vector<pros_handle*> hs;
  // launch
  int budget = 128;
  int wg_per_cu = 2;
  int threads = prost::kBlock;   // threads per workgroup of the launch (512, or the 256-thread build)
  int nwg = 0;
  int rounds = 0;
  int strategy = 0;
  int sync_mode = 2;
  double tile_scale = 1.0;
  const void* kfn = nullptr;
  FrameArgs* d_descs = nullptr;
  BatchItem* d_items = nullptr;
  const void** d_xtab = nullptr;
  int ring = 1;
  bool frames_set = false;
  std::vector<char> frames_aligned;   // per stream: every ring frame 4-byte aligned
  std::vector<FrameArgs> descs;
  std::vector<BatchItem> items;
  // graph
  bool use_graph = false;
  bool coop = true;              // cooperative launch, or an ordinary dispatch of the resident grid
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph_seq = nullptr;       // the multi-step launch (seq_steps steps), captured likewise
  hipGraphExec_t gexec_seq = nullptr;
  bool broken = false;
  bool ext = false;              // a stream uses the optional features
  // multi-step launches: descriptors with nseq = seq_steps
  FrameArgs* d_descs_seq = nullptr;
  int seq_steps = 0;
  long long descs_version = 0, seq_version = -1;
  // per-call frames (pros_batch_track_frames): two pinned copies of the
  // frame table, each reusable once the copy queued from it has run
  const void** h_xstage[2] = {nullptr, nullptr};
  hipEvent_t xstage_done[2] = {nullptr, nullptr};
  int xstage_next = 0;
};

static void drop_graph(pros_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->gexec_seq) (void)hipGraphExecDestroy(b->gexec_seq);
  if (b->graph_seq) (void)hipGraphDestroy(b->graph_seq);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->gexec_seq = nullptr;
  b->graph_seq = nullptr;
}

// Capture one launch of `fn` over `descs` on the private capture stream and
// instantiate it.
static pros_status capture_launch(pros_batch* b, const void* fn, FrameArgs* descs, hipGraph_t* g_out,
                                  hipGraphExec_t* x_out);

static void free_batch(pros_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  for (pros_handle* h : b->hs) prost_host::free_handle(h);
  if (b->d_descs) (void)hipFree(b->d_descs);
  if (b->d_descs_seq) (void)hipFree(b->d_descs_seq);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_xtab) (void)hipFree((void*)b->d_xtab);
  for (int i = 0; i < 2; ++i) {
    if (b->xstage_done[i]) (void)hipEventDestroy(b->xstage_done[i]);
    if (b->h_xstage[i]) (void)hipHostFree((void*)b->h_xstage[i]);
  }
  delete b;
}

// Build the (round, workgroup) -> (stream, tile) schedule for the current
// launch parameters.  strategy 0: first-fit by decreasing gang size;
// strategy 1: first-fit in stream order.
static pros_status build_schedule(pros_batch* b) {
  const int nwg = b->nwg;
  std::vector<int> order(b->n);
  std::iota(order.begin(), order.end(), 0);
  if (b->strategy == 0)
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->hs[a]->G > b->hs[c]->G; });
  std::vector<int> used;   // slots used per round
  std::vector<BatchItem> items;
  for (int s : order) {
    const int G = b->hs[s]->G;
    if (G > nwg) return fail(PROS_EUNSUPPORTED, "stream %d needs %d resident workgroups, the launch has %d", s, G, nwg);
    // gangs are packed back to back: with round-robin placement of
    // consecutive workgroups over the XCDs, the tiles t = x (mod 8) of a
    // gang (one group of the two-hop exchange) land on one XCD wherever the
    // gang starts
    auto start = [&](int rr) { return used[rr]; };
    int r = 0;
    while (r < (int)used.size() && start(r) + G > nwg) ++r;
    if (r == (int)used.size()) {
      used.push_back(0);
      items.resize(used.size() * (size_t)nwg, BatchItem{-1, 0});
    }
    const int s0 = start(r);
    for (int t = 0; t < G; ++t) items[(size_t)r * nwg + s0 + t] = BatchItem{s, t};
    used[r] = s0 + G;
  }
  b->rounds = (int)used.size();
  b->items.swap(items);
  return PROS_OK;
}

// (Re)create the per-stream tile configuration, descriptors and schedule.
static pros_status configure(pros_batch* b, int budget, int wg_per_cu, double tile_scale, int strategy, int sync_mode,
                             int threads) {
  bool ext = false;
  for (pros_handle* h : b->hs) {
    ext = ext || (h->pre_mean != nullptr);
  }
  if (threads != prost::kBlock && threads != 256) return fail(PROS_EINVAL, "threads must be 256 or %d", prost::kBlock);
  const void* f = nullptr;
  if (threads == 256) {
    if (budget != 128 || ext || wg_per_cu != 2)
      return fail(PROS_EUNSUPPORTED, "256-thread workgroups: register budget 128, two per CU, default features");
    f = prost::batch256_kernel_ptr(b->storage == PROS_BF16, b->kclass);
  } else {
    f = prost::batch_kernel_ptr(b->storage == PROS_BF16, b->kclass, budget, ext);
  }
  if (!f) return fail(PROS_EUNSUPPORTED, "no batch kernel for k class %d (%d threads)", b->kclass, threads);
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, threads, 0);
  if (e != hipSuccess) return fail(PROS_EHIP, "occupancy query: %s", hipGetErrorString(e));
  if (occ < 1) return fail(PROS_EUNSUPPORTED, "batch kernel cannot be resident");
  const int wpc = std::min(occ, wg_per_cu);
  const int nwg = wpc * b->num_cu;
  for (pros_handle* h : b->hs) {
    const int NR = prost::batch_rows(b->storage == PROS_BF16, budget, b->kclass);
    const int tpw = prost_host::tile_pixels(b->storage, NR, h->C, tile_scale, threads);
    const int G = (h->P + tpw - 1) / tpw;
    if (G > nwg) return fail(PROS_EUNSUPPORTED, "a %dx%dx%d stream at k=%d needs %d workgroups (> %d)",
                             h->prm.width, h->prm.height, h->C, h->k, G, nwg);
    if (G != h->G) {   // partial buffer sized by the gang
      (void)hipFree(h->part);
      h->part = nullptr;
      e = hipMalloc((void**)&h->part, prost_host::part_bytes(h, G));
      if (e != hipSuccess) return fail(PROS_ENOMEM, "partials: %s", hipGetErrorString(e));
    }
    h->NR = NR;
    h->tpw = tpw;
    h->G = G;
    h->sync_mode = sync_mode;
    pros_status rs = prost_host::reset_exchange(h);
    if (rs != PROS_OK) return rs;
  }
  b->budget = budget;
  b->threads = threads;
  b->wg_per_cu = wpc;
  b->nwg = nwg;
  b->kfn = f;
  b->tile_scale = tile_scale;
  b->strategy = strategy;
  b->sync_mode = sync_mode;
  pros_status st = build_schedule(b);
  if (st != PROS_OK) return st;
  b->descs.resize(b->n);
  for (int s = 0; s < b->n; ++s) {
    FrameArgs a = prost_host::make_args(b->hs[s], nullptr);
    a.xtab = b->d_xtab + (size_t)s * b->ring;
    a.ring = b->ring;
    a.pair_aligned = (prost_host::pair_layout(b->hs[s]) && b->frames_aligned[s]) ? 1 : 0;
    b->descs[s] = a;
  }
  if (b->d_items) (void)hipFree(b->d_items);
  b->d_items = nullptr;
  e = hipMalloc((void**)&b->d_items, sizeof(BatchItem) * b->items.size());
  if (e != hipSuccess) return fail(PROS_ENOMEM, "schedule: %s", hipGetErrorString(e));
  e = hipMemcpy(b->d_items, b->items.data(), sizeof(BatchItem) * b->items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(PROS_EHIP, "schedule upload: %s", hipGetErrorString(e));
  e = hipMemcpy(b->d_descs, b->descs.data(), sizeof(FrameArgs) * b->n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(PROS_EHIP, "descriptor upload: %s", hipGetErrorString(e));
  ++b->descs_version;
  b->ext = ext;
  drop_graph(b);
  return PROS_OK;
}

static pros_status launch(pros_batch* b, hipStream_t on, const void* fn = nullptr, FrameArgs* descs = nullptr) {
  FrameArgs* d = descs ? descs : b->d_descs;
  BatchItem* it = b->d_items;
  int rounds = b->rounds;
  void* args[] = {&d, &it, &rounds};
  if (!fn) fn = b->kfn;
  hipError_t e = b->coop ? hipLaunchCooperativeKernel(fn, dim3(b->nwg), dim3(b->threads), args, 0, on)
                         : hipLaunchKernel(fn, dim3(b->nwg), dim3(b->threads), args, 0, on);
  if (e != hipSuccess) {
    b->broken = true;
    return fail(PROS_EHIP, "batch kernel launch: %s", hipGetErrorString(e));
  }
  return PROS_OK;
}

static pros_status capture_launch(pros_batch* b, const void* fn, FrameArgs* descs, hipGraph_t* g_out,
                                  hipGraphExec_t* x_out) {
  hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return fail(PROS_EHIP, "begin capture: %s", hipGetErrorString(e));
  pros_status ls = launch(b, b->capture_stream, fn, descs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->capture_stream, &g);
  if (ls != PROS_OK) return ls;
  if (e != hipSuccess) {
    b->broken = true;
    return fail(PROS_EHIP, "end capture: %s", hipGetErrorString(e));
  }
  *g_out = g;
  e = hipGraphInstantiate(x_out, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    b->broken = true;
    return fail(PROS_EHIP, "graph instantiate: %s", hipGetErrorString(e));
  }
  return PROS_OK;
}

static pros_status check_batch(pros_batch* b) {
  if (!b) return fail(PROS_EINVAL, "batch is NULL");
  if (b->broken) return fail(PROS_EHIP, "batch unusable after an earlier error");
  return PROS_OK;
}

static pros_status check_stream(pros_batch* b, int32_t s) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (s < 0 || s >= b->n) return fail(PROS_EINVAL, "stream index %d out of range", s);
  return PROS_OK;
}

extern "C" {

pros_status pros_batch_init(const pros_params* per_stream, int32_t n, void* hip_stream, pros_batch** out) {
  if (!out) return fail(PROS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!per_stream || n < 1) return fail(PROS_EINVAL, "need at least one stream");
  const int storage = per_stream[0].storage;
  for (int s = 0; s < n; ++s) {
    pros_status st = pros_validate(&per_stream[s]);
    if (st != PROS_OK) {
      char why[256];
      std::snprintf(why, sizeof(why), "%s", pros_last_error());
      return fail(st, "stream %d: %s", s, why);
    }
    if (per_stream[s].storage != storage) return fail(PROS_EINVAL, "all streams of a batch share one storage type");
    if (per_stream[s].reorth_every != 0)
      return fail(PROS_EINVAL, "stream %d: use pros_batch_reorthonormalize in a batch", s);
    if (per_stream[s].ysolve == 2)
      return fail(PROS_EINVAL, "stream %d: the IRLS step runs in the single-stream kernel only", s);
  }
  pros_batch* b = new pros_batch();
  b->n = n;
  b->storage = storage;
  b->frames_aligned.assign(n, 1);
  b->stream = (hipStream_t)hip_stream;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    free_batch(b);
    return fail(PROS_EHIP, "device query: %s", hipGetErrorString(e));
  }
  int kmax = 1;
  for (int s = 0; s < n; ++s) kmax = std::max(kmax, (int)per_stream[s].k);
  b->kclass = prost::batch_class(kmax);
  e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    free_batch(b);
    return fail(PROS_EHIP, "capture stream: %s", hipGetErrorString(e));
  }
  for (int s = 0; s < n; ++s) {
    pros_handle* h = nullptr;
    const int NR = prost::batch_rows(storage == PROS_BF16, 128, b->kclass);
    const int tpw = prost_host::tile_pixels(storage, NR, per_stream[s].channels, 1.0);
    const int P = per_stream[s].width * per_stream[s].height;
    pros_status st = prost_host::create_handle(&per_stream[s], b->stream, NR, tpw, (P + tpw - 1) / tpw, &h);
    if (st != PROS_OK) {
      free_batch(b);
      return st;
    }
    b->hs.push_back(h);
    st = prost_init_subspace(h, per_stream[s].seed, (uint32_t)s);   // U0 of Sec. 3.4, stream s
    if (st != PROS_OK) {
      free_batch(b);
      return st;
    }
    h->state_set = true;
  }
  e = hipMalloc((void**)&b->d_descs, sizeof(FrameArgs) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_xtab, sizeof(void*) * n);
  if (e != hipSuccess) {
    free_batch(b);
    return fail(PROS_ENOMEM, "batch tables: %s", hipGetErrorString(e));
  }
  pros_status st = configure(b, 128, 2, 1.0, 0, 2, prost::kBlock);   // sync mode 2 suits every stream
  if (st != PROS_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return PROS_OK;
}

void pros_batch_destroy(pros_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
}

pros_status pros_batch_set_state(pros_batch* b, int32_t s, const double* U, const double* y, const uint8_t* labels,
                                 int64_t n) {
  pros_status st = check_stream(b, s);
  if (st != PROS_OK) return st;
  return pros_set_state(b->hs[s], U, y, labels, n);
}

pros_status pros_batch_get_state(pros_batch* b, int32_t s, double* U, double* y, uint8_t* labels, int64_t* n) {
  pros_status st = check_stream(b, s);
  if (st != PROS_OK) return st;
  return pros_get_state(b->hs[s], U, y, labels, n);
}

pros_status pros_batch_set_preprocess(pros_batch* b, int32_t s, const double* mean, const double* m2,
                                      int64_t count) {
  pros_status st = check_stream(b, s);
  if (st != PROS_OK) return st;
  return pros_set_preprocess(b->hs[s], mean, m2, count);
}

pros_status pros_batch_get_preprocess(pros_batch* b, int32_t s, double* mean, double* m2, int64_t* count,
                                      double* scale) {
  pros_status st = check_stream(b, s);
  if (st != PROS_OK) return st;
  return pros_get_preprocess(b->hs[s], mean, m2, count, scale);
}

pros_status pros_batch_set_frames(pros_batch* b, const void* const* frames, int32_t ring) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (!frames || ring < 1) return fail(PROS_EINVAL, "frames is NULL or ring < 1");
  for (int i = 0; i < b->n * ring; ++i)
    if (!frames[i]) return fail(PROS_EINVAL, "frame pointer %d is NULL", i);
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail(PROS_EHIP, "sync: %s", hipGetErrorString(e));
  bool descs_changed = false;
  if (ring != b->ring) {
    (void)hipFree((void*)b->d_xtab);
    b->d_xtab = nullptr;
    e = hipMalloc((void**)&b->d_xtab, sizeof(void*) * (size_t)b->n * ring);
    if (e != hipSuccess) return fail(PROS_ENOMEM, "frame table: %s", hipGetErrorString(e));
    b->ring = ring;
    for (int s = 0; s < b->n; ++s) {
      b->descs[s].xtab = b->d_xtab + (size_t)s * ring;
      b->descs[s].ring = ring;
    }
    descs_changed = true;
    drop_graph(b);
  }
  for (int s = 0; s < b->n; ++s) {
    bool al = true;
    for (int i = 0; i < ring; ++i) al = al && (((uintptr_t)frames[(size_t)s * ring + i] & 3u) == 0);
    b->frames_aligned[s] = al ? 1 : 0;
    const int pa = (prost_host::pair_layout(b->hs[s]) && al) ? 1 : 0;
    if (b->descs[s].pair_aligned != pa) {
      b->descs[s].pair_aligned = pa;
      descs_changed = true;
    }
  }
  if (descs_changed) {   // descriptors are read by the kernel at run time (also from a graph)
    e = hipMemcpy(b->d_descs, b->descs.data(), sizeof(FrameArgs) * b->n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(PROS_EHIP, "descriptor upload: %s", hipGetErrorString(e));
    ++b->descs_version;
  }
  e = hipMemcpy((void*)b->d_xtab, frames, sizeof(void*) * (size_t)b->n * ring, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(PROS_EHIP, "frame table upload: %s", hipGetErrorString(e));
  b->frames_set = true;
  return PROS_OK;
}

pros_status pros_batch_track(pros_batch* b) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (!b->frames_set) return fail(PROS_ESTATE, "register frames with pros_batch_set_frames first");
  for (pros_handle* h : b->hs)
    if (!h->state_set) return fail(PROS_ESTATE, "set every stream's U before the first batch step");
  if (b->use_graph) {
    if (!b->gexec) {
      st = capture_launch(b, b->kfn, b->d_descs, &b->graph, &b->gexec);
      if (st != PROS_OK) return st;
    }
    hipError_t e = hipGraphLaunch(b->gexec, b->stream);
    if (e != hipSuccess) {
      b->broken = true;
      return fail(PROS_EHIP, "graph launch: %s", hipGetErrorString(e));
    }
  } else {
    st = launch(b, b->stream);
    if (st != PROS_OK) return st;
  }
  for (pros_handle* h : b->hs) {
    ++h->submitted;
    h->mask_stale = true;
  }
  return PROS_OK;
}

pros_status pros_batch_track_frames(pros_batch* b, const void* const* frames) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (!frames) return fail(PROS_EINVAL, "frames is NULL");
  for (int s = 0; s < b->n; ++s)
    if (!frames[s]) return fail(PROS_EINVAL, "frame pointer %d is NULL", s);
  // The kernels' descriptors depend on the ring length and on whether each
  // stream's frame is 4-byte aligned; a change goes through the synchronous
  // registration.
  bool same = b->frames_set && b->ring == 1;
  for (int s = 0; same && s < b->n; ++s) same = (((uintptr_t)frames[s] & 3u) == 0) == (b->frames_aligned[s] != 0);
  if (!same) {
    st = pros_batch_set_frames(b, frames, 1);
    if (st != PROS_OK) return st;
    return pros_batch_track(b);
  }
  const int i = b->xstage_next;
  hipError_t e = hipSuccess;
  if (!b->h_xstage[i]) {
    e = hipHostMalloc((void**)&b->h_xstage[i], sizeof(void*) * (size_t)b->n, hipHostMallocDefault);
    if (e != hipSuccess) return fail(PROS_ENOMEM, "pinned frame table: %s", hipGetErrorString(e));
    e = hipEventCreateWithFlags(&b->xstage_done[i], hipEventDisableTiming);
    if (e != hipSuccess) return fail(PROS_EHIP, "event: %s", hipGetErrorString(e));
  } else {
    e = hipEventSynchronize(b->xstage_done[i]);   // the copy queued from this table two calls ago has run
    if (e != hipSuccess) return fail(PROS_EHIP, "event wait: %s", hipGetErrorString(e));
  }
  std::memcpy((void*)b->h_xstage[i], frames, sizeof(void*) * (size_t)b->n);
  // stream-ordered: the previous step's kernel has finished reading the
  // table when the copy runs, and this step's launch reads the new one
  e = hipMemcpyAsync((void*)b->d_xtab, (const void*)b->h_xstage[i], sizeof(void*) * (size_t)b->n,
                     hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->xstage_done[i], b->stream);
  if (e != hipSuccess) return fail(PROS_EHIP, "frame table upload: %s", hipGetErrorString(e));
  b->xstage_next = 1 - i;
  return pros_batch_track(b);
}

pros_status pros_batch_track_steps(pros_batch* b, int32_t steps) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (steps < 1 || steps > 4096) return fail(PROS_EINVAL, "steps must be 1..4096");
  if (steps == 1) return pros_batch_track(b);
  if (!b->frames_set) return fail(PROS_ESTATE, "register frames with pros_batch_set_frames first");
  bool filtered = false;
  for (pros_handle* h : b->hs) {
    if (!h->state_set) return fail(PROS_ESTATE, "set every stream's U before the first batch step");
    filtered = filtered || h->prm.weights_from_filtered;
  }
  const void* fn = (b->threads == 256) ? prost::batch256_kernel_seq_ptr(b->storage == PROS_BF16, b->kclass)
                                       : prost::batch_kernel_seq_ptr(b->storage == PROS_BF16, b->kclass);
  if (!fn || b->budget != 128 || b->ext || filtered) {   // one launch per step
    for (int i = 0; i < steps; ++i) {
      st = pros_batch_track(b);
      if (st != PROS_OK) return st;
    }
    return PROS_OK;
  }
  hipError_t e = hipSuccess;
  if (!b->d_descs_seq) e = hipMalloc((void**)&b->d_descs_seq, sizeof(FrameArgs) * b->n);
  if (e != hipSuccess) return fail(PROS_ENOMEM, "descriptors: %s", hipGetErrorString(e));
  if (b->seq_steps != steps || b->seq_version != b->descs_version) {
    std::vector<FrameArgs> d = b->descs;
    for (FrameArgs& a : d) a.nseq = steps;
    e = hipStreamSynchronize(b->stream);   // a running launch may still read the table
    if (e == hipSuccess) e = hipMemcpy(b->d_descs_seq, d.data(), sizeof(FrameArgs) * b->n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(PROS_EHIP, "descriptor upload: %s", hipGetErrorString(e));
    b->seq_steps = steps;
    b->seq_version = b->descs_version;
    if (b->gexec_seq) (void)hipGraphExecDestroy(b->gexec_seq);
    if (b->graph_seq) (void)hipGraphDestroy(b->graph_seq);
    b->gexec_seq = nullptr;
    b->graph_seq = nullptr;
  }
  if (b->use_graph) {   // the multi-step launch replayed from its own graph
    if (!b->gexec_seq) {
      st = capture_launch(b, fn, b->d_descs_seq, &b->graph_seq, &b->gexec_seq);
      if (st != PROS_OK) return st;
    }
    e = hipGraphLaunch(b->gexec_seq, b->stream);
    if (e != hipSuccess) {
      b->broken = true;
      return fail(PROS_EHIP, "graph launch: %s", hipGetErrorString(e));
    }
  } else {
    st = launch(b, b->stream, fn, b->d_descs_seq);
    if (st != PROS_OK) return st;
  }
  for (pros_handle* h : b->hs) {
    h->submitted += steps;
    h->mask_stale = true;
  }
  return PROS_OK;
}

pros_status pros_batch_set_dispatch(pros_batch* b, int32_t cooperative) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (cooperative != 0 && cooperative != 1) return fail(PROS_EINVAL, "cooperative must be 0 or 1");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail(PROS_EHIP, "sync: %s", hipGetErrorString(e));
  b->coop = cooperative != 0;
  drop_graph(b);   // a captured launch keeps its launch kind
  return PROS_OK;
}

pros_status pros_batch_use_graph(pros_batch* b, int32_t on) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  b->use_graph = on != 0;
  if (!b->use_graph) drop_graph(b);
  return PROS_OK;
}

pros_status pros_batch_sync(pros_batch* b) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  pros_status worst = PROS_OK;
  for (pros_handle* h : b->hs) {
    st = pros_sync(h);
    if (st != PROS_OK && worst == PROS_OK) worst = st;
  }
  return worst;
}

pros_status pros_batch_get_mask(pros_batch* b, int32_t s, uint8_t* out, int32_t filtered, int32_t on_device) {
  pros_status st = check_stream(b, s);
  if (st != PROS_OK) return st;
  return pros_get_mask(b->hs[s], out, filtered, on_device);
}

pros_status pros_batch_get_stats(pros_batch* b, int32_t s, pros_stats* out) {
  pros_status st = check_stream(b, s);
  if (st != PROS_OK) return st;
  return pros_get_stats(b->hs[s], out);
}

pros_status pros_batch_reorthonormalize(pros_batch* b) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  for (pros_handle* h : b->hs) {
    st = pros_reorthonormalize(h);
    if (st != PROS_OK) return st;
  }
  return PROS_OK;
}

pros_status pros_batch_get_config(pros_batch* b, pros_batch_config* out) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (!out) return fail(PROS_EINVAL, "out is NULL");
  out->register_budget = b->budget;
  out->workgroups_per_cu = b->wg_per_cu;
  out->tile_scale = b->tile_scale;
  out->strategy = b->strategy;
  out->sync_mode = b->sync_mode;
  out->workgroups = b->nwg;
  out->rounds = b->rounds;
  out->threads = b->threads;
  return PROS_OK;
}

pros_status pros_batch_configure(pros_batch* b, const pros_batch_config* cfg) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (!cfg) return fail(PROS_EINVAL, "cfg is NULL");
  if (cfg->register_budget != 64 && cfg->register_budget != 128 && cfg->register_budget != prost::kBudgetLds)
    return fail(PROS_EINVAL, "register_budget must be 64, 128 or %d", prost::kBudgetLds);
  if (cfg->workgroups_per_cu < 1 || cfg->workgroups_per_cu > 8) return fail(PROS_EINVAL, "workgroups_per_cu must be 1..8");
  if (!(cfg->tile_scale > 0.0 && cfg->tile_scale <= 1.0)) return fail(PROS_EINVAL, "tile_scale must be in (0, 1]");
  if (cfg->strategy < 0 || cfg->strategy > 1) return fail(PROS_EINVAL, "strategy must be 0 or 1");
  if (cfg->sync_mode < 0 || cfg->sync_mode > 3) return fail(PROS_EINVAL, "sync_mode must be 0..3");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail(PROS_EHIP, "sync: %s", hipGetErrorString(e));
  return configure(b, cfg->register_budget, cfg->workgroups_per_cu, cfg->tile_scale, cfg->strategy, cfg->sync_mode,
                   cfg->threads == 0 ? prost::kBlock : cfg->threads);
}

// Device-side copy of every stream's state, so that tuning leaves the
// trackers where they were.
struct Snapshot {
  std::vector<void*> bufs;
  ~Snapshot() {
    for (void* p : bufs)
      if (p) (void)hipFree(p);
  }
};

static size_t state_bytes(const pros_handle* h, int which) {
  const size_t es = (h->prm.storage == PROS_BF16) ? 2 : 4;
  switch (which) {
    case 0: return es * (size_t)h->ldU * h->k;
    case 1: return sizeof(double) * PROS_MAX_K;
    case 2: return (size_t)h->P;
    case 3: return (size_t)h->P;
    case 4: return sizeof(long long);
    case 5: return h->pre_mean ? sizeof(float) * (size_t)h->m : 0;
    case 6: return h->pre_m2 ? sizeof(float) * (size_t)h->m : 0;
    default: return h->pre_stat ? 2 * sizeof(double) : 0;
  }
}
constexpr int kStateItems = 8;   // U, y, labels, mask, frame counter, pre-processing (3)

static void* state_ptr(pros_handle* h, int which) {
  switch (which) {
    case 0: return h->U;
    case 1: return h->y;
    case 2: return h->lab;
    case 3: return h->mask;
    case 4: return h->nframe;
    case 5: return h->pre_mean;
    case 6: return h->pre_m2;
    default: return h->pre_stat;
  }
}

static pros_status snapshot(pros_batch* b, Snapshot& sn, bool restore) {
  if (!restore) sn.bufs.assign((size_t)b->n * kStateItems, nullptr);
  for (int s = 0; s < b->n; ++s)
    for (int w = 0; w < kStateItems; ++w) {
      void*& buf = sn.bufs[(size_t)s * kStateItems + w];
      const size_t nb = state_bytes(b->hs[s], w);
      if (nb == 0) continue;
      hipError_t e = hipSuccess;
      if (!restore) e = hipMalloc(&buf, nb);
      if (e == hipSuccess)
        e = restore ? hipMemcpyAsync(state_ptr(b->hs[s], w), buf, nb, hipMemcpyDeviceToDevice, b->stream)
                    : hipMemcpyAsync(buf, state_ptr(b->hs[s], w), nb, hipMemcpyDeviceToDevice, b->stream);
      if (e != hipSuccess) return fail(PROS_ENOMEM, "tuner snapshot: %s", hipGetErrorString(e));
    }
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail(PROS_EHIP, "tuner sync: %s", hipGetErrorString(e));
  return PROS_OK;
}

extern "C" pros_status pros_batch_tune(pros_batch* b, int32_t steps, pros_batch_config* best, double* best_ms) {
  pros_status st = check_batch(b);
  if (st != PROS_OK) return st;
  if (steps < 1) return fail(PROS_EINVAL, "steps must be >= 1");
  if (!b->frames_set) return fail(PROS_ESTATE, "register frames with pros_batch_set_frames first");
  for (pros_handle* h : b->hs)
    if (!h->state_set) return fail(PROS_ESTATE, "set every stream's U before tuning");
  Snapshot sn;
  st = snapshot(b, sn, false);
  if (st != PROS_OK) return st;
  const bool graph = b->use_graph;
  b->use_graph = false;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(PROS_EHIP, "event creation failed");
  double bestt = 1e300;
  pros_batch_config bc{};
  // 0.95 and 0.9 spread gangs that leave compute units idle over more of them
  // (640x480x3 bfloat16 at k = 15: 113 workgroups per stream at 1.0, 126 at
  // 0.9, two streams on 252 of 256 compute units, 2 % faster per step)
  const double scales[] = {1.0, 0.95, 0.9, 0.75, 0.5};
  const int wpcs[] = {1, 2};
  const int thr[] = {prost::kBlock, 256};
  for (int sm = 0; sm < 4; ++sm)
  for (int threads : thr)
  for (int budget : kBudgets)
    for (int wpc : wpcs)
      for (double sc : scales)
        for (int strat = 0; strat < 2; ++strat) {
          if (configure(b, budget, wpc, sc, strat, sm, threads) != PROS_OK) continue;   // does not fit
          if (b->wg_per_cu != wpc) continue;                               // duplicate of a smaller grid
          st = launch(b, b->stream);                                        // warm-up
          for (int i = 0; i < steps && st == PROS_OK; ++i) {
            if (i == 0) (void)hipEventRecord(e0, b->stream);
            st = launch(b, b->stream);
          }
          (void)hipEventRecord(e1, b->stream);
          hipError_t e = hipEventSynchronize(e1);
          if (st != PROS_OK || e != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return st != PROS_OK ? st : fail(PROS_EHIP, "tuner: %s", hipGetErrorString(e));
          }
          pros_status ds = pros_batch_sync(b);
          if (ds != PROS_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return ds;
          }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          const double per = ms / steps;
          if (per < bestt) {
            bestt = per;
            bc.register_budget = budget;
            bc.workgroups_per_cu = wpc;
            bc.tile_scale = sc;
            bc.strategy = strat;
            bc.sync_mode = sm;
            bc.threads = threads;
          }
          st = snapshot(b, sn, true);
          if (st != PROS_OK) break;
        }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->use_graph = graph;
  if (st != PROS_OK) return st;
  if (bestt >= 1e300) return fail(PROS_EUNSUPPORTED, "no candidate configuration fits");
  st = configure(b, bc.register_budget, bc.workgroups_per_cu, bc.tile_scale, bc.strategy, bc.sync_mode, bc.threads);
  if (st != PROS_OK) return st;
  if (best) pros_batch_get_config(b, best);
  if (best_ms) *best_ms = bestt;
  return PROS_OK;
}

}  // extern "C"
