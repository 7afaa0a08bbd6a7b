/*
 * prost.h -- C ABI of the MI355X (gfx950) pROST per-frame hot path.
 *
 * pROST (Seidel, Hage, Kleinsteuber, arXiv:1302.2073) tracks a background
 * subspace U (m x k, orthonormal columns) of a video online.  Every frame x
 * (m = channels * width * height entries) is processed in three steps
 * (Sec. 3.3 "An online alternating minimization algorithm"):
 *   Step 1  y = argmin_y h_{mu,w}(x - U y)            eq. (onlinestep1),
 *           a few conjugate-gradient steps on the weighted smoothed cost
 *           h_{mu,w}(r) = sum_i w_i (r_i^2 + mu)^(p/2)  eq. (weightedLPnorm);
 *   Step 2  one descent step of U along the Grassmann geodesic eq. (geodesic)
 *           using the closed-form rank-one SVD of the projected gradient
 *           eq. (svd) and the step-size rule of Sec. 3.4;
 *   Step 3  segmentation: pixel i is foreground when max over colour channels
 *           of |x_i - u_i^T y| >= delta (Sec. 3.4 "Color images"); the labels
 *           set the weights w (1 or omega) of the next frame
 *           eq. (pixelweighting); a 3x3 median filter gives the output mask
 *           (Sec. 3.4 "Pre- and post-processing").
 *
 * Layout.  Frames are planar: all P = width*height pixels of channel 0, then
 * channel 1, ... ; each plane row-major (pixel p = row*width + col, entry
 * e = c*P + p), as x = [x_R; x_G; x_B] of Sec. 3.4.  Masks are P bytes (0/1).
 * State exchanged through pros_get_state / pros_set_state is float64 on the
 * host: U column-major m x k (column j at U + j*m), y of length k.
 *
 * Ownership.  A handle owns all device memory it uses (U, y, labels, mask,
 * partial sums, staging).  Callers own every buffer they pass in.  Device
 * pointers passed in must stay valid and unmodified until the work queued on
 * the handle's stream has completed.
 *
 * Asynchrony and errors.  Work is queued on the HIP stream given at init
 * (NULL = the default stream).  pros_track_frame returns without waiting;
 * errors detected on the device (a non-finite frame, a kernel that timed out
 * waiting for its peers) are reported by the next call that synchronises
 * (pros_get_mask, pros_get_state, pros_get_stats, pros_sync).  No function
 * throws; every function returns a pros_status.  After PROS_EHIP or
 * PROS_ETIMEOUT the handle must be destroyed.  A handle is not thread-safe.
 */
#ifndef PROST_H
#define PROST_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define PROS_API __attribute__((visibility("default")))
#else
#define PROS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pros_status {
  PROS_OK = 0,
  PROS_EINVAL = -1,        /* invalid argument or parameter set */
  PROS_ENOMEM = -2,        /* device or host allocation failed */
  PROS_EHIP = -3,          /* a HIP runtime call failed (handle unusable) */
  PROS_ESTATE = -4,        /* call not valid in the current handle state */
  PROS_EBADFRAME = -5,     /* frame had a NaN/Inf entry; state left unchanged */
  PROS_ETIMEOUT = -6,      /* a persistent kernel gave up waiting (handle unusable) */
  PROS_EUNSUPPORTED = -7   /* size/option outside what the library supports */
} pros_status;

typedef enum pros_dtype { PROS_F32 = 0, PROS_BF16 = 1 } pros_dtype;

/* Per-entry cost phi(r):
 *   PROS_COST_LP : (r^2 + mu)^(p/2), eq. (smoothlpnorm), 0 < p <= 2;
 *   PROS_COST_LOG: log(1 + r^2/mu), the p -> 0 limit of the lp form. */
typedef enum pros_cost { PROS_COST_LP = 0, PROS_COST_LOG = 1 } pros_cost;

enum { PROS_MAX_K = 16, PROS_MAX_CG = 16 };

typedef struct pros_params {
  int32_t width, height, channels; /* channels 1..4 */
  int32_t k;                       /* subspace dimension, 1..PROS_MAX_K */
  int32_t cg_iters;                /* CG steps per frame (Sec. 5.1: 5), 1..PROS_MAX_CG */
  int32_t cost;                    /* pros_cost */
  double p;                        /* lp exponent (Sec. 5.1: 0.25) */
  double mu;                       /* smoothing mu > 0 */
  double delta;                    /* threshold; <= 0 selects eq. (opt_mu2):
                                      sqrt(mu/(1-p)) (lp) or sqrt(mu) (log) */
  double omega;                    /* foreground weight in [0,1] (Sec. 5.1: 5e-5) */
  double t_init, t_min;            /* step-size rule of Sec. 3.4 */
  int32_t i_init;                  /* frames to decay from t_init to t_min */
  int32_t storage;                 /* pros_dtype of U and of device frames */
  int32_t reorth_every;            /* re-orthonormalise U every N frames; 0 = never */
  int32_t labels_after_update;     /* 1: labels use the updated U (default) */
  int32_t weights_from_filtered;   /* 1: weights from the median-filtered mask */
  int32_t preprocess;              /* 1: Sec. 3.4 pre-processing. During the first
                                      i_init frames each frame joins a running
                                      per-entry average; every frame has that
                                      average subtracted and is divided by the
                                      standard deviation of the mean-subtracted
                                      entries of the earlier initialization
                                      frames (1 before two frames are in); both
                                      freeze after i_init frames.  0: frames are
                                      used as given (default). */
  int32_t ysolve;                  /* Step 1 solver: 0 = nonlinear CG with the
                                      Polak-Ribiere-plus direction (default),
                                      1 = gradient descent (d = -g), both with
                                      the majoriser step; Sec. 3.3 compares
                                      the two.  2 = iteratively reweighted
                                      least squares: each step is the full
                                      step -H^-1 g of the quadratic majoriser
                                      (H = U^T diag(w c) U), the classical
                                      reading of the majorise-minimise scheme
                                      of Sec. 3.3; float32 storage, a tagged
                                      exchange (sync_mode 1..3) and the
                                      single-stream tracker only (a batch
                                      refuses it).
                                      A singular H ends the solve with the
                                      current y. */
  uint64_t seed;                   /* U0 = orthonormal factor of the reduced QR
                                      of a random m x k matrix drawn from this
                                      seed (Sec. 3.4, Initialization; see
                                      pros_random_subspace); default 0 */
} pros_params;

typedef struct pros_stats {
  int64_t frame;                 /* 0-based index of the frame described */
  int32_t cg_steps;              /* CG steps taken (< cg_iters only at an exact stop) */
  int32_t restarts;              /* steps whose PR+ direction was reset to -g */
  int32_t updated;               /* 1 if U moved (zeta > 0 and nu > 0) */
  int32_t bad_frame;             /* 1 if the frame was rejected (non-finite) */
  double f[PROS_MAX_CG + 1];     /* cost at y_0 .. y_{cg_steps} */
  double alpha[PROS_MAX_CG];     /* CG step lengths */
  double beta[PROS_MAX_CG];      /* PR+ coefficients */
  double t;                      /* step size of the frame (Sec. 3.4) */
  double sigma;                  /* ||pi(eta)|| ||y||, eq. (svd) */
  double theta;                  /* geodesic angle sigma * t */
  double zeta;                   /* ||pi(eta)|| */
  double nu;                     /* ||y|| */
  int64_t fg_pixels;             /* pixels labelled foreground (raw labels); set
                                    when the mask is computed on demand */
} pros_stats;

typedef struct pros_handle pros_handle;

/* Initialization of U (Sec. 3.4): U = the orthonormal factor Q (diag(R) > 0)
 * of the reduced QR decomposition of an m x k matrix A of independent
 * standard normal entries.  A is drawn from a counter-based generator, so it
 * is the same for every launch and device: entry e = j m + i of A (column j,
 * row i) belongs to pair q = e / 2, one Philox4x32-10 call (Salmon, Moraes,
 * Dror, Shaw, SC'11) with counter (q mod 2^32, q div 2^32, stream_index, 0)
 * and key (seed mod 2^32, seed div 2^32); its words (w0, w1, w2, w3) give the
 * uniforms u_a = ((w0 2^32 + w1) div 2^11 + 1/2) 2^-53 and u_b likewise from
 * (w2, w3), and Box-Muller gives sqrt(-2 ln u_a) cos(2 pi u_b) for even e and
 * sqrt(-2 ln u_a) sin(2 pi u_b) for odd e.  Q is formed in float64 on the GPU
 * by CholeskyQR2.  U: caller-owned device memory, m x k float64,
 * column-major with leading dimension m.  Work runs on `hip_stream`;
 * synchronises (temporary device scratch is allocated and freed).  Errors:
 * PROS_EINVAL for NULL U or sizes outside 1 <= k <= min(m, PROS_MAX_K), or a
 * rank-deficient draw; PROS_ENOMEM; PROS_EHIP.  pros_init and
 * pros_batch_init (stream index = the stream's position in the batch) set
 * each tracker's U from it. */
PROS_API pros_status pros_random_subspace(uint64_t seed, uint32_t stream_index, int64_t m, int32_t k, double* U,
                                          void* hip_stream);

/* Fill *out with the Sec. 5.1 benchmark parameters for a width x height x
 * channels video (k=15, 5 CG steps, p=0.25, omega=5e-5, t_init=5e-3,
 * t_min=1e-4, i_init=100, mu=1e-3, FP32 storage).  Returns PROS_EINVAL on a
 * NULL pointer. */
PROS_API pros_status pros_params_default(pros_params* out, int32_t width, int32_t height, int32_t channels);

/* Validate a parameter set without touching the GPU.  PROS_EINVAL names no
 * field; pros_last_error() gives the reason. */
PROS_API pros_status pros_validate(const pros_params* prm);

/* Create a tracker.  Allocates the device state on the current HIP device and
 * initialises it on `hip_stream` (a hipStream_t, NULL = default), then
 * synchronises: U = U0 of Sec. 3.4 drawn from prm->seed (stream index 0 of
 * pros_random_subspace, rounded to the storage type), y = 0, labels = mask
 * = 0, frame counter 0, so frames can be tracked right away;
 * pros_set_state replaces any of it.  On error *out is NULL.
 * Frames whose tiles of U fit the resident workgroups' registers (on
 * MI355X at k = 15: up to 349 440 pixels x 3 channels in FP32 storage,
 * 698 880 in BF16) run the persistent frame kernel, U kept on chip for the
 * whole frame.  Larger frames run the streamed form: the same arithmetic,
 * one launch per dependent pass, U and the frame read from HBM in every
 * pass (pros_get_launch_info reports sync_mode -1); it has the default
 * features only, so pre-processing (preprocess = 1) or the IRLS step
 * (ysolve = 2) with such a frame gives PROS_EUNSUPPORTED, before any
 * allocation, as does pros_set_score_output on a streamed handle. */
PROS_API pros_status pros_init(const pros_params* prm, void* hip_stream, pros_handle** out);

/* Release all device memory of the handle (waits for its stream).  NULL is
 * accepted. */
PROS_API void pros_destroy(pros_handle* h);

/* Load tracker state from host float64 arrays: U (m x k column-major,
 * required), y (k, NULL = zeros), labels (P bytes, NULL = zeros; also used as
 * the previous filtered mask), frame counter n >= 0.  U is rounded to the
 * storage type.  Synchronous. */
PROS_API pros_status pros_set_state(pros_handle* h, const double* U, const double* y,
                           const uint8_t* labels, int64_t n);

/* Copy the tracker state to host buffers (any may be NULL): U as float64
 * m x k column-major, y (k), raw labels (P bytes), frame counter.
 * Synchronises the stream and reports pending device errors. */
PROS_API pros_status pros_get_state(pros_handle* h, double* U, double* y, uint8_t* labels, int64_t* n);

/* Process one frame (Steps 1-3 of Sec. 3.3 and the median).  `frame` holds m
 * entries of type `dtype` (PROS_F32 or PROS_BF16, must equal the storage
 * type when on_device = 1).  on_device = 0: host memory, copied to a device
 * staging buffer before returning (rejected with PROS_EBADFRAME if an entry
 * is not finite); on_device = 1: device memory read in place by the queued
 * kernels.  Asynchronous. */
PROS_API pros_status pros_track_frame(pros_handle* h, const void* frame, int32_t dtype, int32_t on_device);

/* A buffered sequence: frames[0 .. count-1] (a host array of device
 * pointers, each m entries of the storage dtype) are processed in order,
 * exactly as count calls of pros_track_frame(h, frames[i], dtype, 1) would
 * (same results, bit for bit), but up to 256 frames share one launch of the
 * persistent kernel: every workgroup keeps its tile of U in registers from
 * one frame to the next (U is still written every frame) and the next
 * frame's weights come from the labels it has just produced, so neither the
 * launch nor the reload of U is paid per frame.  Every frame's 3x3 mask is
 * formed, as in single launches, when the next frame has passed its first
 * gang exchange (the last one by pros_get_mask); a launch ends where a
 * re-orthonormalisation is due.
 * Options whose state crosses tiles between frames (weights_from_filtered,
 * pre-processing, score output, the IRLS step or curvature schedule 1) fall
 * back to one launch per frame.  The frames must stay unmodified until the
 * work is done.  Asynchronous. */
PROS_API pros_status pros_track_frames(pros_handle* h, const void* const* frames, int32_t count, int32_t dtype);

/* Segmentation quality (the measures of Sec. 5 follow from these counts:
 * Recall = TP/(TP+FN), Specificity = TN/(TN+FP), FPR = FP/(FP+TN),
 * FNR = FN/(TP+FN), PWC = 100 (FN+FP)/(TP+FN+FP+TN), Precision =
 * TP/(TP+FP), F-measure = 2 Pr Re/(Pr+Re)).
 *
 * pros_set_score_output: the frame kernel also writes |r'_e| (the Step 3
 * residual whose per-pixel maximum over channels is compared with delta)
 * for every entry to `device_scores` (m floats, caller-owned, channel-major
 * like a frame; NULL stops it).  Synchronises.
 *
 * pros_quality_counts: counts[0..3] = (TP, FP, TN, FN) of the latest mask
 * (filtered = 1) or raw labels (0) against `truth` (P bytes, nonzero =
 * foreground; device pointer when on_device, else host).  Synchronises.
 *
 * pros_roc_counts: the delta sweep of Sec. 5 without re-running the
 * tracker: for each of T <= 256 thresholds (host array),
 * counts[4 i .. 4 i + 3] = (TP, FP, TN, FN) of the labels
 * [max_c scores[c P + p] >= thresholds[i]] against truth (device arrays of
 * C P floats and P bytes).  Queued on hip_stream, then synchronises. */
PROS_API pros_status pros_set_score_output(pros_handle* h, float* device_scores);
PROS_API pros_status pros_quality_counts(pros_handle* h, const uint8_t* truth, int32_t on_device, int32_t filtered,
                                         int64_t* counts);
PROS_API pros_status pros_roc_counts(const float* scores, const uint8_t* truth, int32_t P, int32_t C,
                                     const float* thresholds, int32_t T, int64_t* counts, void* hip_stream);

/* Pre-processing statistics (handles created with preprocess = 1):
 * per-entry running average and sum of squared deviations (m doubles each,
 * entry order of a frame; NULL sets zeros) over `count` initialization
 * frames.  Stored in float32 on the device; the entry sum of the squared
 * deviations is recomputed here.  Synchronises.  PROS_ESTATE when the handle
 * has no pre-processing. */
PROS_API pros_status pros_set_preprocess(pros_handle* h, const double* mean, const double* m2, int64_t count);

/* Read them back (each output may be NULL); *scale is the standard
 * deviation the next frame will be divided by.  Synchronises. */
PROS_API pros_status pros_get_preprocess(pros_handle* h, double* mean, double* m2, int64_t* count, double* scale);

/* Copy the latest mask: filtered = 1 gives the 3x3-median mask F, 0 the raw
 * labels.  The median of a frame's labels is computed at the start of the
 * next frame's kernel, or here (one small kernel) when the mask of the
 * latest frame is asked for first.  out holds P bytes on the host (on_device = 0, synchronises) or on
 * the device (on_device = 1, queued on the stream). */
PROS_API pros_status pros_get_mask(pros_handle* h, uint8_t* out, int32_t filtered, int32_t on_device);

/* Statistics of the last processed frame.  Synchronises. */
PROS_API pros_status pros_get_stats(pros_handle* h, pros_stats* out);

/* Wait for the handle's queued work and report pending device errors. */
PROS_API pros_status pros_sync(pros_handle* h);

/* Re-orthonormalise U now (nearest orthonormal basis U (U^T U)^{-1/2},
 * accumulated and solved in float64 on the GPU; y <- (U^T U)^{1/2} y so that
 * U y is unchanged to first order).  Asynchronous.  Also run automatically
 * every reorth_every frames. */
PROS_API pros_status pros_reorthonormalize(pros_handle* h);

/* Launch configuration chosen for the handle (for diagnostics).  A
 * streamed handle reports sync_mode -1, rows_per_thread 0 and the workgroups
 * of one pass (256 threads, one pixel each, or a pixel pair each in bfloat16
 * storage with even P and a 4-byte aligned frame). */
typedef struct pros_launch_info {
  int32_t workgroups;        /* persistent workgroups of the frame kernel */
  int32_t threads;           /* threads per workgroup */
  int32_t rows_per_thread;   /* register-resident rows of U per thread */
  int32_t pixels_per_wg;     /* pixels of one workgroup tile */
  int32_t barriers_per_frame;/* gang-wide reductions per frame */
  int32_t sync_mode;         /* gang exchange, as in pros_set_launch */
  int32_t curvature;         /* CG curvature schedule, as in pros_set_curvature */
} pros_launch_info;
PROS_API pros_status pros_get_launch_info(pros_handle* h, pros_launch_info* out);

/* ---------------------------------------------------------------------------
 * Batched form.  n independent streams (own resolution, k, parameters; one
 * storage type) advance by one frame each per pros_batch_track, in ONE
 * persistent cooperative kernel launch: every stream's frame is the same
 * Steps 1-3 + median as pros_track_frame (Sec. 3.3, 3.4), its workgroup
 * tiles form a gang for the frame's reductions, and a host-built schedule
 * packs the gangs onto the resident workgroups in rounds.  Frames are read
 * from a caller-registered ring of device frames: stream s reads
 * frames[s * ring + (n_s % ring)] where n_s is its frame counter.  Every
 * stream starts from its own seeded U0 (pros_batch_init); pros_batch_set_state
 * replaces it.  A stream whose gang does not fit the resident workgroups (a
 * frame beyond the single-stream resident bound, see pros_init) is refused
 * with PROS_EUNSUPPORTED: the batched form has no streamed form.
 * Errors as for single streams; a failed launch makes the batch unusable.
 * ------------------------------------------------------------------------- */
typedef struct pros_batch pros_batch;

typedef struct pros_batch_config {
  int32_t register_budget;   /* floats of U held in registers per thread: 64 or 128;
                                192 = the LDS form (bfloat16, k class 10..16, default
                                features): the 128 tile in registers plus 3-4
                                row pairs per thread in LDS (one workgroup per
                                CU) */
  int32_t workgroups_per_cu; /* resident workgroups per CU used by the launch */
  double tile_scale;         /* (0, 1]: fraction of the register tile each workgroup fills */
  int32_t strategy;          /* 0: gangs packed by decreasing size, 1: in stream order */
  int32_t sync_mode;         /* gang exchange, as in pros_set_launch */
  int32_t workgroups;        /* out: resident workgroups of the launch */
  int32_t rounds;            /* out: rounds of the schedule */
  int32_t threads;           /* threads per workgroup: 512 (0 selects it), or 256 with
                                register budget 128 and workgroups_per_cu 2 (two
                                workgroups of different streams share a CU, so one
                                computes while the other waits on an exchange;
                                k class 15, default features) */
} pros_batch_config;

/* Create a batch of n streams (per_stream[0..n-1]; reorth_every must be 0,
 * use pros_batch_reorthonormalize).  Stream s starts from U0 of Sec. 3.4
 * drawn from per_stream[s].seed with stream index s (pros_random_subspace),
 * so equal seeds still give distinct subspaces.  Work runs on hip_stream;
 * synchronises. */
PROS_API pros_status pros_batch_init(const pros_params* per_stream, int32_t n, void* hip_stream, pros_batch** out);
PROS_API void pros_batch_destroy(pros_batch* b);
/* Same contract as pros_set_state / pros_get_state for stream s. */
PROS_API pros_status pros_batch_set_state(pros_batch* b, int32_t s, const double* U, const double* y,
                                 const uint8_t* labels, int64_t n);
PROS_API pros_status pros_batch_get_state(pros_batch* b, int32_t s, double* U, double* y, uint8_t* labels, int64_t* n);
/* Same contract as pros_set_preprocess / pros_get_preprocess for stream s
 * (a stream created with preprocess = 1; PROS_ESTATE otherwise). */
PROS_API pros_status pros_batch_set_preprocess(pros_batch* b, int32_t s, const double* mean, const double* m2,
                                               int64_t count);
PROS_API pros_status pros_batch_get_preprocess(pros_batch* b, int32_t s, double* mean, double* m2, int64_t* count,
                                               double* scale);
/* Register the frame ring: n * ring device pointers (host array; stream s,
 * slot i at frames[s * ring + i]), each m_s entries of the storage type.
 * The pointed-to frames must stay valid while batch steps run.  Synchronous. */
PROS_API pros_status pros_batch_set_frames(pros_batch* b, const void* const* frames, int32_t ring);
/* One batch step: every stream processes its next frame.  Asynchronous. */
PROS_API pros_status pros_batch_track(pros_batch* b);
/* One batch step on the frames given for this call (Sec. 3.3: each stream's
 * new frame arrives online): frames[s] is stream s's device frame (m_s
 * entries of the storage type) for this step, n pointers in a host array
 * that may be reused as soon as the call returns.  The frames themselves
 * must stay valid until the step has run (pros_batch_sync).  The table of
 * frame pointers is updated in stream order (from pinned staging), so
 * consecutive calls queue without waiting, also with hipGraph replay; the
 * first call, a change from a ring registered with pros_batch_set_frames,
 * or a change in a frame's 4-byte alignment registers the frames
 * synchronously (ring of 1).  Errors as pros_batch_track; PROS_EINVAL for a
 * NULL pointer.  Asynchronous otherwise. */
PROS_API pros_status pros_batch_track_frames(pros_batch* b, const void* const* frames);
/* `steps` batch steps (1..4096) with the same results as `steps` calls of
 * pros_batch_track, in one launch: every (stream, tile) item of the
 * schedule advances its stream by `steps` frames of the ring with its tile
 * of U kept in registers between them (as pros_track_frames does for one
 * stream).  For frames buffered ahead (the ring holds them).  Register
 * budget 128 and the default features only; otherwise one launch per
 * step.  Asynchronous. */
PROS_API pros_status pros_batch_track_steps(pros_batch* b, int32_t steps);
/* 1: capture the launch into a hipGraph on first use and replay it; the
 * multi-step launch of pros_batch_track_steps gets a graph of its own (per
 * step count), recaptured when the step count, the frame ring or the launch
 * configuration changes. */
PROS_API pros_status pros_batch_use_graph(pros_batch* b, int32_t on);
PROS_API pros_status pros_batch_sync(pros_batch* b);
PROS_API pros_status pros_batch_get_mask(pros_batch* b, int32_t s, uint8_t* out, int32_t filtered, int32_t on_device);
PROS_API pros_status pros_batch_get_stats(pros_batch* b, int32_t s, pros_stats* out);
/* Re-orthonormalise every stream's U (as pros_reorthonormalize). */
PROS_API pros_status pros_batch_reorthonormalize(pros_batch* b);
/* Current launch configuration / apply one (resizes tiles, rebuilds the
 * schedule; synchronises). */
PROS_API pros_status pros_batch_get_config(pros_batch* b, pros_batch_config* out);
PROS_API pros_status pros_batch_configure(pros_batch* b, const pros_batch_config* cfg);
/* Autotuner: time `steps` batch steps (after one warm-up step) for every
 * candidate configuration (register budget x workgroups per CU x tile scale
 * x strategy), restoring every stream's state after each candidate, then
 * apply the fastest.  Needs registered frames.  Reports the chosen
 * configuration and its time per step (ms). */
PROS_API pros_status pros_batch_tune(pros_batch* b, int32_t steps, pros_batch_config* best, double* best_ms);

/* ---------------------------------------------------------------------------
 * Differentiable cost.  h_{mu,w}(x - U y) of eqs. (weightedLPnorm),
 * (spcacost) for a batch of B frames sharing U, and its adjoint.  For B = 1
 * and an upstream gradient of 1, dU is the Euclidean gradient eta y^T of
 * Sec. 3.3 (Step 2).
 *
 * All pointers are device pointers to row-major float32 arrays:
 *   U (m, k), Y (B, k), X (B, m), w (m) or NULL for w = 1, mu (1 value, so
 *   that it can be a tensor with a gradient), f (B), gout (B),
 *   dX (B, m), dU (m, k), dY (B, k), dmu (1); any output of the backward may
 *   be NULL to skip writing it.
 * `workspace` is caller-owned device memory of at least
 * pros_lpcost_workspace_size(m, k, B) bytes (partial sums; contents need
 * not be initialised).  Work is queued on `hip_stream`; results are
 * deterministic (fixed-order float64 reductions).  1 <= k <= PROS_MAX_K.
 * Errors: PROS_EINVAL for NULL inputs, bad sizes or a small workspace.
 * ------------------------------------------------------------------------- */
PROS_API size_t pros_lpcost_workspace_size(int32_t m, int32_t k, int32_t B);

/* f_b = sum_e w_e phi(X[b,e] - U[e,:] . Y[b,:]). */
PROS_API pros_status pros_lpcost_fwd(const float* U, const float* Y, const float* X, const float* w, const float* mu,
                            int32_t m, int32_t k, int32_t B, int32_t cost, float p, float* f,
                            void* workspace, size_t workspace_bytes, void* hip_stream);

/* Adjoint of pros_lpcost_fwd for the upstream gradient gout:
 * dX[b,e] = gout_b w_e phi'(r), dU[e,:] = -sum_b gout_b w_e phi'(r) Y[b,:],
 * dY[b,:] = -gout_b sum_e w_e phi'(r) U[e,:], dmu = sum_b gout_b sum_e w_e dphi/dmu. */
PROS_API pros_status pros_lpcost_bwd(const float* U, const float* Y, const float* X, const float* w, const float* mu,
                            int32_t m, int32_t k, int32_t B, int32_t cost, float p, const float* gout,
                            float* dX, float* dU, float* dY, float* dmu,
                            void* workspace, size_t workspace_bytes, void* hip_stream);

/* Bytes of the fixed device scratch behind pros_lpcost_bwd_noalloc (8 MiB). */
#define PROS_LPCOST_SCRATCH_BYTES (8u << 20)

/* pros_lpcost_bwd without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as
 * pros_lpcost_bwd, bit for bit; the partial sums go to a fixed scratch array
 * inside the library instead: one per GPU, PROS_LPCOST_SCRATCH_BYTES bytes,
 * held until the process ends.  No call allocates: the array's device
 * address is looked up once per device (the first call made with that
 * device current) and kept.  Every call on one GPU uses the same array, and
 * its contents after a call are that call's partials (nothing in it has to
 * start at zero); calls that overlap on one GPU (two host threads, or two
 * streams without ordering between them) race and give wrong results.
 * Errors: PROS_EINVAL when pros_lpcost_workspace_size(m, k, B) exceeds
 * PROS_LPCOST_SCRATCH_BYTES (m = 230400, k = 10, B = 32 needs 2.5 MB) or for
 * the argument errors of pros_lpcost_bwd; PROS_EHIP when the array's address
 * cannot be looked up. */
PROS_API pros_status pros_lpcost_bwd_noalloc(const float* U, const float* Y, const float* X, const float* w,
                                             const float* mu, int32_t m, int32_t k, int32_t B, int32_t cost, float p,
                                             const float* gout, float* dX, float* dU, float* dY, float* dmu,
                                             void* hip_stream);

/* Launch tuning of a single-stream handle.  pros_init chooses automatically:
 * one workgroup if the frame fits one, else the smallest tile reaching a
 * gang of <= 32 workgroups, else the smallest tile whose gang fits one
 * workgroup per compute unit; exchange 3 for gangs of <= 64 workgroups, 2
 * above.  This call overrides it: rows_per_thread (0 = automatic tile; else
 * 1, 2, 4, 8, 16 (k <= 8 for float32) or, for bfloat16 storage, whose tiles
 * hold row pairs, 2, 4, 8, 16 or 32 (k <= 8); the frame's pixels must fit
 * the resident workgroups) and the gang exchange used for the frame's
 * reductions:
 * 0 = one arrival counter per gang and every workgroup reading all partial
 * sums, 1 = epoch-tagged partial sums gathered by the gang's first
 * workgroup and broadcast back, 2 = the same in two levels (groups of
 * tiles t = x mod 8; every workgroup reads the 8 group sums),
 * 3 = every workgroup reads all tagged partials (one hop, G^2 reads).
 * Results agree to float64 rounding.  rows_per_thread = -1 selects the
 * streamed form (one launch per pass, U read from HBM every pass; see
 * pros_init) for any frame size; sync_mode is then ignored.
 * Synchronises. */
PROS_API pros_status pros_set_launch(pros_handle* h, int32_t rows_per_thread, int32_t sync_mode);

/* Dispatch of the persistent kernels.  A frame's gang of workgroups waits on
 * itself at every exchange, so all of its workgroups must be resident at
 * once.  cooperative = 1 (default): hipLaunchCooperativeKernel, which
 * guarantees it; on this device each such launch costs about 17 us more
 * than an ordinary one (measured: 19.6 vs 2.7 us per launch of an empty
 * kernel of 113-256 workgroups).  cooperative = 0: an ordinary launch.  The
 * grid is already sized to what the device holds at once (occupancy query
 * at configuration), so on a device running nothing else every workgroup
 * starts immediately; if other work holds compute units, waiting
 * workgroups end the frame through the bounded exchange waits with
 * PROS_ETIMEOUT (no hang) and the handle becomes unusable.  Use 0 on a
 * dedicated device.  pros_batch_set_dispatch does the same for a batch
 * (and drops a captured graph).  Results are identical either way. */
PROS_API pros_status pros_set_dispatch(pros_handle* h, int32_t cooperative);
PROS_API pros_status pros_batch_set_dispatch(pros_batch* b, int32_t cooperative);

/* Curvature schedule of the Step 1 solver (Sec. 3.3): how d^T H d of the
 * majoriser step alpha = -g.d / d^T H d, H = U^T diag(w c) U, is formed.
 * 0 (default): a second pass per step sums w c (u_e . d)^2 after the
 * direction is known (two gang exchanges per step, 2 J + 1 per frame);
 * 1: the gradient pass also reduces the k (k + 1) / 2 entries of H, and the
 * direction, d^T H d and the step follow from the one (wide) exchange
 * (J + 1 per frame; k (k + 1) / 2 more multiply-adds per entry).  The same
 * method: the two agree to float32 rounding of the sums.  Schedule 1 needs
 * float32 storage (PROS_EUNSUPPORTED otherwise) and a tagged exchange
 * (sync_mode 1..3).  The IRLS solver (ysolve = 2) always reduces H.
 * Synchronises; the tile (rows per thread) is kept.  On a streamed handle
 * (frames beyond the resident tiles) both schedules are available in either
 * storage type: schedule 1 reads U once per CG step instead of twice. */
PROS_API pros_status pros_set_curvature(pros_handle* h, int32_t schedule);

/* ---------------------------------------------------------------------------
 * Video ingest.  Sec. 5.1 re-samples every sequence to one small resolution
 * (160 x 120) before tracking; Sec. 5.3 brings the mask computed at the
 * small size back up for evaluation.
 *
 * pros_resample_rgb8: `src` (device) holds an interleaved 8-bit frame,
 * src_h rows of src_w pixels of `channels` (1..4) bytes, rows src_row_stride
 * bytes apart (as a video decoder writes it).  `dst` (device, m =
 * channels * dst_w * dst_h entries of dst_dtype, PROS_F32 or PROS_BF16)
 * receives the tracker's planar frame: for each channel plane and
 * destination pixel, scale times the mean of the source over the pixel's
 * footprint (area averaging; the source is piecewise constant over its
 * pixels).  Weights are exact integers and the sums exact, so the value is
 * the correctly rounded float64 mean, rounded once to float32 (then to
 * nearest-even bfloat16).  Any sizes 1..32768 (shrinking or enlarging).
 * Asynchronous on hip_stream; PROS_EINVAL for bad sizes or NULL pointers,
 * before any device work.
 *
 * pros_mask_upsample: `mask` (device, height x width bytes) to `out`
 * (device, out_h x out_w bytes) by nearest neighbour: out pixel (i, j)
 * copies the source pixel containing its centre, row
 * floor((2i+1) height / (2 out_h)), column floor((2j+1) width / (2 out_w)).
 * Asynchronous on hip_stream.
 *
 * pros_ingest: frames from host memory, pipelined.  pros_ingest_init binds
 * a pipeline to a tracker whose frame is the resampled size (its
 * width x height, its channels) for source frames src_w x src_h
 * (interleaved 8-bit, rows packed), with `slots` (1..16) pinned host
 * buffers and device buffers and its own copy stream.  pros_ingest_slot
 * hands out the next pinned buffer to fill (waits only if that buffer's
 * previous copy is still in flight); pros_ingest_submit copies it to the
 * device on the copy stream and queues resample + pros_track_frame on the
 * tracker's stream behind the copy (events order the two streams), so the
 * copy of the next frame overlaps the tracking of this one.
 * pros_ingest_push = slot + memcpy + submit.  pros_ingest_mask writes the
 * latest mask (filtered = 1: 3x3 median, 0: raw labels) upsampled to the
 * source size (src_w x src_h bytes; device when on_device, queued; host
 * otherwise, synchronises).  The pipeline owns its buffers; destroy it
 * before its tracker.  Not thread-safe. */
typedef struct pros_ingest pros_ingest;
PROS_API pros_status pros_resample_rgb8(const uint8_t* src, int32_t src_w, int32_t src_h, int32_t channels,
                                        int64_t src_row_stride, void* dst, int32_t dst_dtype, int32_t dst_w,
                                        int32_t dst_h, double scale, void* hip_stream);
PROS_API pros_status pros_mask_upsample(const uint8_t* mask, int32_t width, int32_t height, uint8_t* out,
                                        int32_t out_w, int32_t out_h, void* hip_stream);
PROS_API pros_status pros_ingest_init(pros_handle* h, int32_t src_w, int32_t src_h, int32_t slots, double scale,
                                      pros_ingest** out);
PROS_API pros_status pros_ingest_slot(pros_ingest* g, uint8_t** host_slot);
PROS_API pros_status pros_ingest_submit(pros_ingest* g);
PROS_API pros_status pros_ingest_push(pros_ingest* g, const uint8_t* frame_rgb8);
PROS_API pros_status pros_ingest_mask(pros_ingest* g, uint8_t* out, int32_t filtered, int32_t on_device);
PROS_API void pros_ingest_destroy(pros_ingest* g);

/* Diagnostics: record wall-clock timestamps (64 per workgroup tile, int64,
 * device memory of at least 64 * workgroups entries) around every gang-wide
 * exchange of the following frames; NULL stops recording. */
PROS_API pros_status pros_debug_trace(pros_handle* h, long long* device_buffer);

/* Text for a status code (static storage). */
PROS_API const char* pros_strerror(pros_status s);
/* Detail of the last error on the calling thread (static thread storage). */
PROS_API const char* pros_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PROST_H */
