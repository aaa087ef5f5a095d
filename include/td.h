/*
 * td.h - lazy, seed-consistent windowed diffusion sampling of an unbounded
 * latent plane (InfiniteDiffusion) on one AMD Instinct MI355X (gfx950).
 *
 * The library answers queries J_t[R] of the infinite image produced by the
 * InfiniteDiffusion update (Sec. 3.2, Eq. 2; formal restatement in the
 * appendix "Formal Properties") with the lazy, memoising query algorithm of
 * Sec. 3.3 (Alg. 1), the window-range function kappa of the appendix's
 * window-range algorithm, and the Laplacian decode of Sec. 5.2.
 *
 * Conventions for every call:
 *  - Coordinates are int64 pixel indices; x is the column, y the row.  A
 *    region [x0, x0+w) x [y0, y0+h) needs 1 <= w, h <= 2^20, w*h <= 2^26
 *    and |x0|, |y0| < 2^31 - 2^22 (so every window index of its dependency
 *    cone fits in int32 window units).
 *  - Latent outputs are float32, planar [C][h][w] (C = latent channels);
 *    height outputs are float32 [h][w] in metres.
 *  - Every call returns td_status; nothing throws across the ABI.  On error,
 *    td_last_error(ctx) describes the failure.  A query that fails after
 *    its arguments were accepted (an allocation, a launch) drops the
 *    context's cache, which only ever changes speed, never values; the
 *    context stays usable.
 *  - A context is not thread-safe: one caller at a time.
 *  - Buffers are owned by the caller; the context owns its weights, its
 *    device cache and its workspaces, all freed by td_destroy.
 *  - Device pointers are HIP device addresses on the context's device;
 *    streams are hipStream_t passed as void* (NULL = the context's own
 *    stream where a call has a context, else the device's default stream;
 *    TD_STREAM_DEFAULT always names the device's default stream).
 */
#ifndef TD_H
#define TD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Stream argument naming the device's default (null) stream; the value of
 * HIP's hipStreamLegacy handle.  Work enqueued with it is ordered with
 * everything the caller put on the default stream. */
#define TD_STREAM_DEFAULT ((void *)1)

typedef struct td_ctx td_ctx;

typedef enum {
  TD_OK = 0,
  TD_E_INVAL = -1,   /* bad argument: size, level, buffer length, option   */
  TD_E_NOMEM = -2,   /* device or host allocation failed                   */
  TD_E_DEVICE = -3,  /* HIP runtime error                                  */
  TD_E_IO = -4,      /* weight file missing or unreadable                  */
  TD_E_FORMAT = -5,  /* weight file malformed or describes an unknown model */
  TD_E_STATE = -6    /* call not valid now (e.g. query before weights)     */
} td_status;

/* Per-context counters.  windows_evaluated[t] counts denoiser (Phi)
 * evaluations at level t since the last td_cache_clear / td_load_weights. */
typedef struct {
  uint64_t hits;          /* windows of a query's cone found in the cache  */
  uint64_t misses;        /* windows that had to be evaluated              */
  uint64_t evictions;     /* cache entries dropped by the LRU              */
  uint64_t bytes_used;    /* device bytes held by cached contributions     */
  uint64_t bytes_budget;  /* current budget                                */
  uint64_t batches;       /* batched denoiser rounds launched              */
  uint64_t queries;       /* td_sample_region* calls served                */
  uint64_t denoiser_evals;/* network evaluations (windows x Euler steps)   */
  uint64_t windows_evaluated[64];
  uint64_t judge_fallbacks;/* consistency windows that fell back to the    */
                           /* teacher's plain sample (td_set_judge)        */
} td_cache_stats_t;

/* Elevation query level: decoded height in metres on full-resolution pixels
 * (factor 8 finer than the latent), Sec. 5.2. */
#define TD_LEVEL_HEIGHT (-1)

/* Create a context on HIP device `hip_device`. */
td_status td_create(int hip_device, td_ctx **out);

/* Free every device and host resource of the context (NULL is a no-op). */
void td_destroy(td_ctx *ctx);

/* Load a .tdw weight file: 4-byte magic "TDW1", uint32 header length, JSON
 * header (denoiser architecture or analytic kind, EDM sampler constants,
 * window size/stride/offset/epsilon, decode constants, tensor table), zero
 * padding to 64 bytes, then little-endian float32 tensors.  Replaces any
 * previous model and clears the cache (cached contributions are
 * model-specific).  TD_E_IO if unreadable, TD_E_FORMAT if malformed; on
 * any error the context keeps its previous model (or none) and its cache. */
td_status td_load_weights(td_ctx *ctx, const char *path);

/* Hierarchy (Sec. 5.1; DAGs of infinite tensors, infinite-tensor appendix):
 * make `parent`'s final latent J_0 the conditioning of `child`.  A model
 * whose header has "cond" = {channels C_y, factor f} reads, for each window,
 * concat(c_in x, y) where y is the parent's J_0 (same seed) nearest-
 * upsampled by f: child pixel (X, Y) takes parent pixel (floor(X/f),
 * floor(Y/f)).  A query of the child first samples the parent (through the
 * parent's own cache, on the parent's stream) on the parent-resolution cover
 * of the child's new windows; a parent may itself be conditioned (chains).
 * Both contexts must be on one device; the parent is not owned and must
 * stay alive while linked (td_destroy of either unlinks).  NULL unlinks.
 * Clears the child's cache; a later td_load_weights or "precision" change
 * of the parent clears it again at the child's next query.  TD_E_INVAL for
 * a cycle or another device; a child query without a linked parent whose
 * channels equal C_y gives TD_E_STATE. */
td_status td_set_conditioning(td_ctx *child, td_ctx *parent);

/* Few-step consistency sampling with a fallback (Sec. 3.4 lets Phi be a
 * few-step consistency model; the paper's distilled core model takes two
 * steps): for a model whose sampler kind is "consistency", every window of
 * every step is also denoised by `teacher` at the same noise level (one
 * teacher network evaluation), and a window whose estimate differs from the
 * teacher's by more than `threshold` in RMS over the window (all pixels and
 * channels, FP32) falls back to the plain sampler: it takes the teacher's
 * plain sample J_0 on the window's region for the same seed, computed by
 * the teacher context's own lazy sampler and cache (Sec. 5.3: the plain
 * sampler stands behind the distilled two-step model).  td_cache_stats
 * counts those windows in judge_fallbacks.  The teacher needs the student's
 * channels and window layout; its one-step network runs on the student's
 * stream in the teacher's workspace, its fallback samples on its own
 * stream, both ordered after the teacher's own work (do not query the
 * teacher from another thread meanwhile).  NULL teacher turns the judge off.
 * Clears the student's cache; reloading the teacher clears it again at the
 * student's next query.  TD_E_INVAL if the student is not a consistency
 * model, threshold < 0 or the devices differ; TD_E_STATE at query time if
 * the teacher's layout does not match. */
td_status td_set_judge(td_ctx *student, td_ctx *teacher, float threshold);

/* J_level[R] for seed `seed` (Alg. 1 applied recursively from J_T = sigma_0 G).
 * level in [0, T] (T = blend levels, "levels" in td_get_info; T = sampler
 * steps K unless the weight file truncates T, Sec. 3.4, in which case Phi
 * of a level runs several window-local Euler steps; 0 = final latent,
 * T = scaled noise),
 * or TD_LEVEL_HEIGHT for decoded elevation on the full-resolution region.
 * `out` is a host buffer of out_len floats, at least C*w*h (latent) or w*h
 * (height); the call blocks until the result is in `out`.  Values depend
 * only on (weights, seed, level, region), never on the cache or on earlier
 * queries (seed consistency, Sec. 3.5). */
td_status td_sample_region(td_ctx *ctx, uint64_t seed, int64_t x0, int64_t y0,
                           int32_t w, int32_t h, int32_t level, float *out,
                           size_t out_len);

/* As td_sample_region, but `dev_out` is device memory and the work is
 * enqueued on `hip_stream` (NULL: the context's stream).  Host-side planning
 * runs synchronously; the result is ready when the stream reaches the end
 * of the enqueued work. */
td_status td_sample_region_async(td_ctx *ctx, uint64_t seed, int64_t x0,
                                 int64_t y0, int32_t w, int32_t h,
                                 int32_t level, float *dev_out, size_t out_len,
                                 void *hip_stream);

/* Byte budget of the device cache of window contributions (Sec. 3.3, the
 * per-window contribution store with LRU eviction).  Entries beyond the
 * budget are evicted least-recently-used first at the end of each query
 * level; a query may exceed it transiently by its own working set.  Any
 * budget, including 0, gives identical results. */
td_status td_cache_set_budget(td_ctx *ctx, size_t bytes);

/* Drop every cached contribution and reset the counters. */
td_status td_cache_clear(td_ctx *ctx);

/* Copy the counters into *out. */
td_status td_cache_stats(td_ctx *ctx, td_cache_stats_t *out);

/* Copy the cached contribution W_i (x) Phi(J_{t+1}[R_i]) of window
 * (ix, iy) at level t for `seed` into the host buffer `out` ([H][H][C]
 * float32, row-major, out_len >= H*H*C).  TD_E_INVAL if not cached. */
td_status td_cache_peek(td_ctx *ctx, uint64_t seed, int32_t level, int64_t ix,
                        int64_t iy, float *out, size_t out_len);

/* Options: "batch" = max windows per batched denoiser round, 1..2^20
 * (default: as many as a 32 GB workspace holds for 4-channel networks, at
 * most 1024, else a 16 GB one, at most 4096; the context allocates the
 * workspace for this many windows at its first query and keeps it);
 * "cache_budget" = as td_cache_set_budget; "precision" = 0 FP32 network
 * (default), 1 BF16 convolution operands with FP32 accumulation (GroupNorm
 * statistics, attention, the input/output layers, blend, Euler update and
 * decode stay FP32), 2 as 1 but with OCP FP8 e4m3 weights scaled per
 * output channel (FP32 scale applied to the FP32 accumulator); changing it
 * clears the cache; "timing" = 1 records every kernel
 * launch between HIP events on its stream (see td_kernel_stats), 0 stops.
 * TD_E_INVAL for unknown keys. */
td_status td_set_option(td_ctx *ctx, const char *key, int64_t value);

/* Model facts: "channels", "steps" (K), "levels" (T), "window", "stride", "offset",
 * "factor" (decode), "params", "batch", "precision", "cond_channels" and
 * "cond_factor" (0 for an unconditioned model), "noise_step" (counter word
 * of the model's J_T noise).  TD_E_INVAL for unknown keys. */
td_status td_get_info(td_ctx *ctx, const char *key, int64_t *value);

/* Denoiser D(x; sigma_k) of the loaded model on `n` windows (EDM
 * preconditioning, the definition of Phi's network call): x_dev and
 * out_dev are device arrays [n][H][H][C] float32 (H = window size), k in
 * [0, K-1] selects sigma_k of the schedule.  cond_dev: the windows'
 * conditioning [n][H][H][C_y] float32 for a conditioned model, NULL
 * otherwise (TD_E_INVAL if that does not match the model).  Synchronous.
 * For checking the network apart from the sampler. */
td_status td_denoise_windows(td_ctx *ctx, const float *x_dev,
                             const float *cond_dev, int32_t n, int32_t k,
                             float *out_dev);

/* The model's own sampler steps k0 .. k1-1 (0 <= k0 < k1 <= K, EDM Euler)
 * on `n` windows independently, without blending: x_dev [n][H][H][C] holds
 * the windows at sigma_k0, out_dev receives them at sigma_k1 (k1 = K: the
 * sample).  With k0 = 0 and x = sigma_0 G this is the plain sampler on a
 * single window (the teacher output of distillation).  out_dev may equal
 * x_dev.  Synchronous.  TD_E_INVAL for consistency or conditioned models. */
td_status td_denoise_steps(td_ctx *ctx, const float *x_dev, int32_t n, int32_t k0, int32_t k1, float *out_dev);

/* scale * G(seed, x, y, c, step) on [x0, x0+w) x [y0, y0+h), written to
 * dev_out as [h][w][channels] float32 on `hip_stream` (NULL: default
 * stream): the seed noise of the seeds paragraph of the formal appendix
 * with any counter word `step` (0 is J_T's; the student's re-noising uses
 * 1).  accumulate = 0 overwrites dev_out; accumulate = 1 adds the noise to
 * what dev_out holds (dev_out += scale * G: the re-noising x + sigma G of
 * multistep consistency sampling, used by distillation).  Asynchronous.
 * TD_E_INVAL for a null buffer, empty sides, more than 2^30 pixels or an
 * accumulate value other than 0 or 1. */
td_status td_noise_region(uint64_t seed, int64_t x0, int64_t y0, int32_t w, int32_t h, int32_t channels,
                          uint32_t step, float scale, int32_t accumulate, float *dev_out, void *hip_stream);

/* Laplacian decode (Sec. 5.2, with the signed-sqrt inverse of the
 * signed-sqrt appendix) of a latent held in device memory, [lh][lw][C]
 * float32 with latent origin (lx0, ly0), onto the full-resolution region
 * [X0, X0+W) x [Y0, Y0+H): out_dev is [H][W] float32.  The latent must
 * cover the 17-pixel apron; TD_E_INVAL otherwise.  Enqueued on hip_stream.
 * The decode and td_lap_encode use one scratch buffer of the context: calls
 * on different streams must be ordered by the caller. */
td_status td_lap_decode(td_ctx *ctx, const float *latent_dev, int64_t lx0,
                        int64_t ly0, int32_t lw, int32_t lh, int64_t X0,
                        int64_t Y0, int32_t W, int32_t H, float *out_dev,
                        void *hip_stream);

/* td_lap_decode without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments, kernels and results, but its
 * scratch is a fixed 16 MiB array per GPU, set up by td_create, instead of
 * the context's grown buffer.  The decode needs 2 n_x n_y floats of it,
 * n_x by n_y being the latent pixels the region's low band spans plus the
 * 15-pixel blur radius on each side (about W/8 + 32 by H/8 + 32); the array
 * holds 2^22 floats.  Every square region the library accepts (up to 2^26
 * px) fits; a long strip may not (2^20 x 64 px needs 2 x 5.2 M floats), and
 * then the call gives TD_E_INVAL and launches nothing.  Per-launch timing is
 * not recorded.  Every call on one GPU shares that GPU's array (it keeps
 * the last call's contents; the decode writes all of it before reading):
 * calls that overlap on one GPU, on any streams or contexts, race and must
 * be ordered by the caller. */
td_status td_lap_decode_noalloc(td_ctx *ctx, const float *latent_dev, int64_t lx0, int64_t ly0, int32_t lw,
                                int32_t lh, int64_t X0, int64_t Y0, int32_t W, int32_t H, float *out_dev,
                                void *hip_stream);

/* Laplacian encode (Sec. 5.2; the inverse construction the decode undoes):
 * elevation height_dev [H][W] float32 on the 8-aligned full-resolution
 * region [X0, X0+W) x [Y0, Y0+H) -> z = sign(h) sqrt|h|, L = G5 * down8(z)
 * (valid), and per output latent pixel the low band L / sigma_low and the
 * residual coefficients <z - up8(L), beta_k> / sigma_res (k = 1..3) of its
 * 8x8 block, written to latent_dev [oh][ow][C] float32 (channels beyond 4
 * zero).  The output shrinks by the blur radius plus one block on each
 * side: geom receives {ox0, oy0, ow, oh} = {X0/8 + R + 1, Y0/8 + R + 1,
 * W/8 - 2R - 2, H/8 - 2R - 2} with R the blur radius of the loaded weights.
 * latent_dev may be NULL to query geom only.  TD_E_INVAL for an unaligned
 * or too small region or latent_len < ow * oh * C.  Enqueued on hip_stream
 * (NULL: the context's stream). */
td_status td_lap_encode(td_ctx *ctx, const float *height_dev, int64_t X0,
                        int64_t Y0, int32_t W, int32_t H, float *latent_dev,
                        size_t latent_len, int64_t geom[4], void *hip_stream);

/* Window-range function kappa of the formal appendix for one axis pair:
 * windows [ix*stride+offset, +size) meeting [x0,x0+w) x [y0,y0+h).
 * Writes {ix_min, ix_max, iy_min, iy_max}; returns TD_OK, or TD_E_INVAL if
 * the range is empty (region between windows) or an argument is invalid.
 * Host-only; needs no context or device. */
td_status td_kappa(int64_t x0, int64_t y0, int64_t w, int64_t h, int32_t size,
                   int32_t stride, int32_t offset, int64_t out[4]);

/* Number of denoiser evaluations a cold query of region R at level t needs
 * with K steps: sum over levels of |kappa(R_l)| along the dependency cone
 * (constant-time random access bound, appendix).  Host-only. */
td_status td_cone_windows(int64_t x0, int64_t y0, int64_t w, int64_t h,
                          int32_t level, int32_t steps, int32_t size,
                          int32_t stride, int32_t offset, uint64_t *count);

/* Per kernel class, totals over the launches recorded while "timing" was
 * on: launch count, summed event-measured duration, and the algorithmic
 * FLOPs and HBM bytes the launches had to do (what the method requires, not
 * what the hardware counted). */
typedef struct {
  char name[32];      /* e.g. "conv3x3_mfma_f32", "blend", "noise_philox" */
  uint64_t launches;
  double ms;
  double flops;
  double bytes;
} td_kernel_stat_t;

/* Copy up to `cap` class totals into out, set *count to the number of
 * classes with launches; reset != 0 clears the totals afterwards.  Waits for
 * the recorded launches to finish.  TD_E_STATE if timing is off. */
td_status td_kernel_stats(td_ctx *ctx, td_kernel_stat_t *out, int32_t cap,
                          int32_t *count, int32_t reset);

/* ------------------------------------------------------------- serving --
 * A request loop over one context with continuous batching.  Queries are
 * admitted in arrival order while fewer than max_inflight are in flight and
 * their worst-case device footprint (cone contributions + level canvases)
 * fits hbm_budget bytes (a query that alone exceeds it is admitted when
 * nothing else is in flight).  Each td_server_progress round builds the
 * level inputs that are ready and runs one batched denoiser call over ready
 * windows of one level, taken from any in-flight queries (windows shared by
 * several queries are evaluated once).  Results equal those of the same
 * queries made one at a time (seed consistency, Sec. 3.5; Parallelization
 * theorem of the appendix).  The server uses the context's model, cache
 * and stream; one thread drives it.  After a td_server_progress error the
 * server refuses further rounds (TD_E_STATE); td_server_destroy then also
 * drops the context's cache (windows in flight may never have been
 * written). */
typedef struct td_server td_server;

typedef struct {
  uint64_t seed;
  int64_t x0, y0;
  int32_t w, h;
  int32_t level;      /* latent level 0..T-1 */
  float *dev_out;     /* device buffer [C][h][w], owned by the caller */
  size_t out_len;
} td_request;

typedef struct {
  uint64_t submitted, admitted, completed;
  uint64_t rounds;           /* batched denoiser rounds */
  uint64_t batched_windows;  /* windows evaluated by the server */
  uint64_t in_flight, queued;
  uint64_t mem_in_flight;    /* admitted footprint (bytes) */
  uint64_t canvas_bytes;     /* device bytes of the canvas pool */
} td_server_stats_t;

td_status td_server_create(td_ctx *ctx, size_t hbm_budget, int32_t max_inflight,
                           td_server **out);
/* Waits for the device, releases unfinished queries, frees the server. */
void td_server_destroy(td_server *srv);
/* Queue a query (copied); *ticket identifies it.  Non-blocking. */
td_status td_server_submit(td_server *srv, const td_request *req,
                           uint64_t *ticket);
/* Run `rounds` scheduling rounds; *in_flight = admitted + queued queries
 * not yet complete.  Enqueues work and returns without waiting for it. */
td_status td_server_progress(td_server *srv, int32_t rounds, int32_t *in_flight);
/* *done = 1 once the query's result is in its buffer (then *latency_ms is
 * the time from submission to observed completion and the ticket is
 * released); TD_E_INVAL for an unknown ticket. */
td_status td_server_poll(td_server *srv, uint64_t ticket, int32_t *done,
                         double *latency_ms);
td_status td_server_stats(td_server *srv, td_server_stats_t *out);

/* Description of the last error on ctx (owned by ctx, valid until the next
 * call); "" if none.  Safe on NULL. */
const char *td_last_error(const td_ctx *ctx);

/* ---------------------------------------------------------------- training
 * Hand-written forward and backward of a window UNet denoiser, for
 * distilling a few-step student (Sec. 5.1: the core model is distilled into
 * a two-step consistency model; the student here is distilled on (noise
 * window, teacher output) pairs).  The network is the sampler's (EDM
 * preconditioning around the UNet of the weight file's header); parameters
 * are one flat float32 device buffer laid out as the file's data section
 * (tensor i at float offset offset_i / 4, conv weights [co][ci][kh][kw]),
 * so a file's data can be loaded, trained and written back as it is.
 * Gradients use the same layout.  FP32 by default (BF16 convolution
 * operands with td_train_set_precision); all reductions run in a fixed
 * order (deterministic gradients).  One trainer is not thread-safe;
 * calls are asynchronous on the HIP stream `stream` (NULL: the device's
 * default stream). */
typedef struct td_trainer td_trainer;

/* Trainer for the UNet of weight file `path` (its architecture and tensor
 * table; the values are not read).  TD_E_FORMAT for analytic or
 * conditioned models. */
td_status td_train_create(int hip_device, const char *path, td_trainer **out);
void td_train_destroy(td_trainer *tr);
const char *td_train_last_error(const td_trainer *tr);

/* 0 (default): FP32 convolutions.  1: BF16 operands (activations and
 * weights, converted from the FP32 masters at every forward) for the
 * forward and data-gradient convolutions, FP32 accumulation; weight
 * gradients, GroupNorm, attention and the optimizer stay FP32.
 * TD_E_INVAL for other values. */
td_status td_train_set_precision(td_trainer *tr, int32_t precision);

/* Length in floats of the flat parameter buffer (the data section). */
td_status td_train_param_count(td_trainer *tr, size_t *n);

/* D = D_theta(x; sigma) for n windows x [n][H][H][C] float32 (device), out
 * D the same shape.  Keeps the activations the next td_train_backward
 * needs (one pending backward per trainer). */
td_status td_train_forward(td_trainer *tr, const float *params, const float *x, int32_t n, double sigma, float *D,
                           void *stream);

/* Adds dL/dparams to grads (same layout as params) for the dL/dD of the
 * last forward, which must have used the same params pointer
 * (TD_E_STATE otherwise). */
td_status td_train_backward(td_trainer *tr, const float *params, const float *dD, float *grads, void *stream);

/* Weighted mean squared error over n floats: dD = weight 2 (D - y) / n;
 * *loss (nullable; synchronises) = weight mean((D - y)^2). */
td_status td_train_mse(td_trainer *tr, const float *D, const float *y, size_t n, float weight, float *dD,
                       double *loss, void *stream);

/* AdamW step `step` (>= 1) on n floats: bias-corrected moments m, v
 * (device, zero-initialised by the caller), decoupled weight decay
 * params -= lr (m_hat / (sqrt(v_hat) + eps) + weight_decay params). */
td_status td_train_adamw(td_trainer *tr, float *params, const float *grads, float *m, float *v, size_t n, float lr,
                         float beta1, float beta2, float eps, float weight_decay, int32_t step, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TD_H */
