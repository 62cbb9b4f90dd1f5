/*
 * lego_raster.h -- C ABI of the MI355X (gfx950) differentiable Gaussian
 * rasterizer: RGB + depth + 16-d language feature, forward and backward.
 *
 * What it computes.  LEGO-SLAM (arXiv 2511.16144) renders its
 * language-embedded Gaussians Theta = {p, q, s, alpha, c, f in R^16}
 * with the usual 3D Gaussian Splatting rasterizer into an RGB image and a feature map
 * (Sec. III-B.1), uses the rendered depth in the L1 depth term of its mapping
 * loss (Sec. III-B.3, Eq. (1)), optimises Theta through the renderer over
 * several iterations per keyframe (Sec. III-B.3) and refines keyframe poses by
 * the same rendering loss (Sec. III-B.2).  This library is that renderer and
 * its exact gradient.  Per pixel (readings where the paper is silent):
 *   s = exp(log_scale), q normalised, o = sigmoid(logit);
 *   EWA screen covariance Sigma' = J R_cw R(q) diag(s^2) R(q)^T R_cw^T J^T
 *     + eps I (J: pinhole Jacobian with the view-angle clamp);
 *   contributors: m2 = d^T Sigma'^{-1} d <= cutoff2 and
 *     alpha = min(alpha_max, o exp(-m2/2)) >= alpha_min, in (z, index) order;
 *   front to back, T' = T (1 - alpha), stop before T' < T_eps,
 *     Y += alpha T [rgb, z, f];  background 0.
 *
 * Conventions shared by every call.
 *   - All pointers named "device" are HIP device memory owned by the caller;
 *     the library never frees them.  Structure-of-arrays planes: a field
 *     written [k][n] is k contiguous planes of n values.
 *   - Cameras are world->camera (R_cw row-major, t_cw), OpenCV axes (x right,
 *     y down, z forward); pixel (i, j) is evaluated at its centre (i, j).
 *   - Every call enqueues work on the given stream and returns without
 *     waiting for it, except where its comment says it synchronises: an
 *     eager forward performs one 4-byte device->host read (the pair count);
 *     lgs_prune, the count / stage-time queries, lgs_graph_create,
 *     lgs_graph_status, lgs_autotune and the destroy calls synchronise.  Releasing a state is
 *     stream-ordered: its device buffers return to the context's cache and
 *     are handed out again only behind the work already enqueued on that
 *     stream.
 *   - Errors are returned as lgs_status; details via lgs_last_error().  No
 *     call throws.  Arguments are validated on the host: NULL pointers,
 *     n < 0, image sides outside [1, 2048], n_views outside [1, 1024],
 *     unknown dtype, tile not in {8, 16, 32}, misaligned (< 4-byte) pointers.
 *   - Gaussians with a non-finite input, a zero quaternion, or camera depth
 *     <= z_near are culled: no contribution and zero gradient.
 *   - One context serves one stream at a time; calls on a shared context are
 *     not thread-safe.
 */
#ifndef LEGO_RASTER_H
#define LEGO_RASTER_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LGS_OK = 0,
  LGS_ERR_INVALID_ARG = 1,  /* bad argument (see lgs_last_error) */
  LGS_ERR_HIP = 2,          /* a HIP runtime call failed */
  LGS_ERR_CAPACITY = 3,     /* pair buffer too small (graph mode) */
  LGS_ERR_UNSUPPORTED = 4,  /* valid but not supported by this build */
  LGS_ERR_STATE = 5,        /* object used in the wrong state */
  LGS_STATUS_INT32 = 0x7fffffff  /* not a status: makes every int32 a value of the type */
} lgs_status;

typedef enum {
  LGS_F32 = 0,
  LGS_BF16 = 1,
  LGS_DTYPE_INT32 = 0x7fffffff  /* not a dtype: makes every int32 a value of the type */
} lgs_dtype;

/* Bits of lgs_settings.profile. */
enum { LGS_PROFILE_EVENTS = 1, LGS_PROFILE_COUNTS = 2 };

/* Pinhole camera and world->camera pose (Sec. III-A: T_k in SE(3)). */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R_cw[9];   /* row-major */
  float t_cw[3];
} lgs_camera;

/* Rasterizer constants (the paper publishes none; defaults are the readings
 * listed beside each field) and execution tunables.  Results do not depend on
 * the tunables: the forward is bitwise identical for every tile size. */
typedef struct {
  float z_near;     /* 0.2     near-plane cull */
  float eps2d;      /* 0.3     px^2 added to Sigma' diagonal */
  float fov_clamp;  /* 1.3     Jacobian view-angle clamp factor */
  float alpha_max;  /* 0.99    alpha clamp */
  float alpha_min;  /* 1/255   smallest alpha that contributes */
  float T_eps;      /* 1e-4    stop before T' < T_eps */
  float cutoff2;    /* 9.0     largest m2 that contributes */
  int32_t tile;     /* 16      binning tile side: 8, 16 or 32 */
  int32_t chunk;    /* 4       8x8 pixel blocks per work-group (1, 2, 4, 8) */
  int32_t order;    /* 0       work order of the compositing kernels' per-XCD queues:
                     *         0 raster order, neighbouring tiles on different XCDs;
                     *         1 descending tile-list length; 2 descending list length
                     *         with each 128 x 128-px region on one XCD (the tiles
                     *         of a region share that XCD's L2) */
  int32_t profile;  /* 0       bit LGS_PROFILE_EVENTS: record HIP events around each
                     *         stage (lgs_state_stage_ms, lgs_graph_stage_ms);
                     *         bit LGS_PROFILE_COUNTS: run the compositing kernels'
                     *         counting variants, which fill the work counts of
                     *         lgs_counts (fwd_evals .. bwd_written; 0 otherwise) */
} lgs_settings;

/* Gaussians: SoA planes, n of each (Sec. III-B.1, Theta).  means [3][n],
 * log_scales [3][n], quats [4][n] (w, x, y, z; need not be unit),
 * opacity_logits [n] are FP32; rgb [3][n] and feat [D][n] are FP32 or BF16
 * (appearance_dtype).  All device pointers.  feat_dim D is the language
 * feature dimension: 8 or a multiple of 16 up to 128 (0 means 16; the paper
 * uses 16 and its ablation varies it).  Features are rendered in groups of
 * 16 channels: each group beyond the first repeats the compositing passes
 * (the blend weights do not depend on the features), so the cost of the
 * compositing kernels grows with ceil(D / 16). */
typedef struct {
  int64_t n;
  const float *means, *log_scales, *quats, *opacity_logits;
  const void *rgb, *feat;
  lgs_dtype appearance_dtype;
  int32_t feat_dim;
} lgs_gaussians;

/* Per-view images, FP32 planes of the view's H x W pixels (device):
 * rgb [3][H][W], depth [H][W], feat [D][H][W], final_T [H][W].
 * n_contrib [H][W] (int32, optional, may be NULL) receives each pixel's
 * contributor count.  As a backward input (dL/dY) rgb/depth/feat hold the
 * upstream gradients and final_T (dL/dT) may be NULL. */
typedef struct {
  float *rgb, *depth, *feat, *final_T;
  int32_t *n_contrib;
} lgs_images;

/* Parameter gradients, FP32 SoA planes shaped like the inputs (device):
 * means [3][n], log_scales [3][n], quats [4][n], opacity_logits [n],
 * rgb [3][n], feat [D][n] (always FP32, w.r.t. the stored values, summed
 * over views), and twist [n_views][6] = dL/d(rho, phi) of the left pose
 * perturbation T_cw <- Exp(xi) T_cw at xi = 0 (may be NULL). */
typedef struct {
  float *means, *log_scales, *quats, *opacity_logits, *rgb, *feat;
  float *twist;
} lgs_grads;

typedef struct lgs_context lgs_context;
typedef struct lgs_fwd_state lgs_fwd_state;
typedef struct lgs_graph lgs_graph;

/* Work counts of a forward (and of its backward once run), for measurement
 * and tests.  The compositing kernels' counts (fwd_evals .. bwd_written) are
 * collected only with the LGS_PROFILE_COUNTS bit of settings.profile (they
 * read 0 otherwise): counting in the entry loops costs those kernels
 * several percent, so the timed variants do not count. */
typedef struct {
  int64_t n_visible;    /* visible (view, Gaussian) pairs */
  int64_t n_pairs;      /* (tile, Gaussian) pairs after binning */
  int64_t n_slots;      /* (8x8 block, Gaussian) gradient slots */
  int64_t n_tiles;      /* binning tiles over all views */
  int64_t n_items;      /* 8x8 blocks (work items) over all views */
  int64_t fwd_evals;    /* (pixel, list entry) evaluations, forward compositing */
  int64_t fwd_contrib;  /* ... of which contributed */
  int64_t bwd_evals;    /* (pixel, list entry) evaluations, backward compositing */
  int64_t bwd_contrib;  /* ... of which contributed */
  int64_t fwd_entries;  /* list entries visited by a wave (8x8 block), forward */
  int64_t bwd_entries;  /* ... backward */
  int64_t bwd_written;  /* partial records the backward wrote (visited, some pixel contributed) */
} lgs_counts;

const char *lgs_status_string(lgs_status s);
/* Last error text of a context (never NULL; "" when none). */
const char *lgs_last_error(const lgs_context *ctx);
lgs_settings lgs_default_settings(void);

/* Context: owns the device workspace (records, sort buffers, partials) of
 * every state it creates.  hip_device is made current by every call. */
lgs_status lgs_context_create(int hip_device, lgs_context **out);
void lgs_context_destroy(lgs_context *ctx);

/* Forward render of n_views views (Sec. III-B.1 render of I^ and F_render;
 * Eq. (1) depth D^).  cams[n_views] and out[n_views] are host arrays of
 * structs whose image pointers are device memory.  On success *state_out
 * holds what lgs_backward needs; release it with lgs_state_release.  The
 * Gaussian arrays must stay unmodified until the backward has run.
 * LGS_ERR_UNSUPPORTED when n > 2^30, when n rounded up to a power of two
 * exceeds 2^26 (BF16 appearance) or 2^25 (FP32), or n_views times it
 * exceeds 2^27 (the compositing kernels address their records by 32-bit
 * byte offsets), or for more than 2^31 8x8 pixel blocks. */
lgs_status lgs_forward(lgs_context *ctx, const lgs_settings *st,
                       const lgs_gaussians *g, int32_t n_views,
                       const lgs_camera *cams, const lgs_images *out,
                       lgs_fwd_state **state_out, hipStream_t stream);

/* Vector-Jacobian product of the forward that produced `state` (the
 * gradient step of Sec. III-B.3 map optimisation and of the Sec. III-B.2
 * pose refinement).  grad_out[n_views] holds dL/dY per view (final_T may be
 * NULL).  Every plane of `grads` is overwritten.  Deterministic: no
 * atomics in the gradient reduction.  Enqueued on `stream` without a host
 * wait (the host tables it uploads are kept alive by the state). */
lgs_status lgs_backward(lgs_context *ctx, const lgs_fwd_state *state,
                        const lgs_gaussians *g, const lgs_images *grad_out,
                        lgs_grads *grads, hipStream_t stream);

/* The backward of the mapping loss of Eq. (1) without its D-SSIM term:
 * computes dL/dY of L = sum over views of mean|RGB-RGB*| + w_depth mean|D-D*|
 * + w_feat mean|F-F*| (sign(0) = 0, loss_w = {1, w_depth, w_feat}) inside
 * the backward compositing kernel from the forward's images `out` (the
 * buffers lgs_forward wrote) and `targets` (device planes; final_T
 * ignored), then back-propagates it like lgs_backward.  Deterministic. */
lgs_status lgs_backward_l1(lgs_context *ctx, const lgs_fwd_state *state,
                           const lgs_gaussians *g, const lgs_images *out,
                           const lgs_images *targets, const float loss_w[3],
                           lgs_grads *grads, hipStream_t stream);

/* The mapping loss of Eq. (1) with the D-SSIM term of its photometric part
 * (Sec. III-B.3), and its gradient with respect to the rendered images:
 *   L = sum over views of  w_rgb ((1 - lam) mean|I - I*| + lam (1 - SSIM))
 *                          + w_depth mean|D - D*| + w_feat mean|F - F*|,
 * loss_w = {w_rgb, w_depth, w_feat}, lam = ssim_lambda in [0, 1] (the 3D
 * Gaussian Splatting convention is 0.2).  SSIM is the mean over the three
 * colour channels and every pixel of the SSIM map under an 11 x 11 Gaussian
 * window (sigma 1.5, weights summing to 1, zero padding at the border),
 * C1 = 0.01^2, C2 = 0.03^2 (images in [0, 1]).  sign(0) = 0 in the L1
 * terms.
 *   cams[n_views]    only width and height are read
 *   feat_dim         D, feature planes of the images (as lgs_gaussians;
 *                    0 means 16); the feature term is a mean over D planes
 *   out, targets     rendered and observed images (device FP32 planes;
 *                    final_T and n_contrib ignored)
 *   grad             receives dL/dY: rgb [3][H][W], depth, feat [D][H][W]
 *                    (device, overwritten; final_T and n_contrib ignored);
 *                    it may be passed to lgs_backward as grad_out
 *   terms            NULL, or device FP32 [n_views][4] receiving per view
 *                    mean|I-I*|, 1 - SSIM (0 when ssim_lambda = 0: the SSIM
 *                    stencil is skipped), mean|D-D*|, mean|F-F*|
 * Enqueued on `stream` (the context keeps a small view table and partial
 * sums; calls on one context are ordered by its stream).  Deterministic.
 * LGS_ERR_INVALID_ARG for NULL or misaligned planes, non-finite weights or
 * ssim_lambda outside [0, 1]. */
lgs_status lgs_loss(lgs_context *ctx, int32_t n_views, const lgs_camera *cams,
                    int32_t feat_dim, const lgs_images *out, const lgs_images *targets,
                    const float loss_w[3], float ssim_lambda,
                    const lgs_images *grad, float *terms, hipStream_t stream);

/* The feature-distillation loss of Eq. (2) through the decoder D_theta
 * (Sec. III-B.3), and its gradients.  D_theta is read as a 1x1 convolution,
 * one affine map R^16 -> R^C per pixel, Z(p) = W F(p) + b:
 *   L = w_feat * mean over C x H x W of |Z - F_gt|   (sign(0) = 0)
 *   grad_feat   = dL/dF        [16][H][W]  (overwritten)
 *   grad_weight = dL/dW        [C][16]     (overwritten)
 *   grad_bias   = dL/db        [C]         (overwritten)
 *   loss        = L            device scalar, or NULL
 * feat F [16][H][W], weight W [C][16] (row-major), bias b [C]: FP32 device
 * arrays; target F_gt [C][H][W] in target_dtype (BF16 or FP32), device.
 * out_dim C: 256 or 512.  The products run on the matrix cores with the
 * FP32 operands split into two BF16 terms each (relative error of Z about
 * 2^-16 of |W||F|; the signs are exact).  Enqueued on `stream` (the context
 * keeps a small partial-sum buffer; calls on one context are ordered by its
 * stream).  Deterministic (fixed-order reductions).  Targets must be finite:
 * BF16 targets enter a matrix product as they are, so a non-finite one turns
 * its channel's results over its 32-pixel chunk into NaN.
 * LGS_ERR_INVALID_ARG for NULL or misaligned arrays, sizes < 1 or a
 * non-finite w_feat; LGS_ERR_UNSUPPORTED for another out_dim. */
lgs_status lgs_decoder_l1(lgs_context *ctx, int32_t width, int32_t height,
                          int32_t out_dim, const float *feat,
                          const float *weight, const float *bias,
                          const void *target, lgs_dtype target_dtype,
                          float w_feat, float *grad_feat, float *grad_weight,
                          float *grad_bias, float *loss, hipStream_t stream);

/* The loss of lgs_decoder_l1 over several views in one launch: the sum over
 * views v of w_feat * mean over C x height[v] x width[v] of |Z_v - F_gt,v|
 * (each view normalised by its own size, as the per-view Eq. (2) terms are
 * summed over the views of a step), with the shared weight and bias.
 *   width, height  host int32 [n_views], each >= 1
 *   feat, target, grad_feat   host arrays of n_views device pointers, the
 *                  per-view planes of lgs_decoder_l1 (grad_feat[v] = dL/dF_v,
 *                  overwritten)
 *   grad_weight, grad_bias, loss   as in lgs_decoder_l1, summed over views
 * The host arrays are read during the call only.  Results equal the sums of
 * lgs_decoder_l1 over the views up to FP32 summation order.  n_views 1..16
 * (LGS_ERR_UNSUPPORTED above 16, LGS_ERR_INVALID_ARG below 1); otherwise the
 * errors of lgs_decoder_l1, for every view. */
lgs_status lgs_decoder_l1_views(lgs_context *ctx, int32_t n_views,
                                const int32_t *width, const int32_t *height,
                                int32_t out_dim, const float *const *feat,
                                const float *weight, const float *bias,
                                const void *const *target,
                                lgs_dtype target_dtype, float w_feat,
                                float *const *grad_feat, float *grad_weight,
                                float *grad_bias, float *loss,
                                hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as lgs_decoder_l1, same arguments and results (the same
 * kernels and, up to 256 work-groups, the same launch), with no allocation.
 * Its per-work-group partial sums live in a fixed device array of 256 x 8768
 * floats (8.98 MB) that the library holds on every GPU it runs on until the
 * process ends (its address is resolved once per device at
 * lgs_context_create); it calls no hipMalloc, hipFree or allocating library
 * routine.  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (other streams, other contexts, other threads) race and must be
 * ordered by the caller.  LGS_ERR_CAPACITY if the partial sums would exceed
 * the array (not reachable with out_dim <= 512), otherwise the errors of
 * lgs_decoder_l1. */
lgs_status lgs_decoder_l1_noalloc(lgs_context *ctx, int32_t width,
                                  int32_t height, int32_t out_dim,
                                  const float *feat, const float *weight,
                                  const float *bias, const void *target,
                                  lgs_dtype target_dtype, float w_feat,
                                  float *grad_feat, float *grad_weight,
                                  float *grad_bias, float *loss,
                                  hipStream_t stream);

/* Language-guided pruning (Sec. III-C, Eq. (4)) combined with the geometric
 * criteria.  The paper publishes neither K nor the thresholds; the defaults
 * (lgs_default_prune_params) are readings:
 *   k           16     neighbours examined per Gaussian (1..32): the k
 *                      nearest other Gaussians by distance of the means,
 *                      ties by index
 *   tau_dist    0.02   redundant only if closer than this (scene units)
 *   tau_sim     0.9    ... and cosine similarity of the 16-d features above
 *                      this (0 when either feature is zero)
 *   min_opacity 0.005  geometric: sigmoid(logit) below this
 *   max_scale   0.3    geometric: exp(largest log-scale) above this
 * Of a redundant pair the dominated Gaussian is marked (smaller opacity
 * logit; equal logits: the larger index), so one of the two survives.
 * Non-finite means, logits or log-scales fail the geometric test.
 * Uses means, log_scales, opacity_logits and feat of `g` (rgb unused).
 *   mask    device uint8 [n]: bit 0 redundant (Eq. (4)), bit 1 geometric;
 *           prune where non-zero (overwritten)
 *   counts  NULL or host int64 [3]: redundant, geometric, pruned (either)
 * Distances and similarities are evaluated in FP64.  Synchronises with
 * `stream` (two small readbacks).  LGS_ERR_INVALID_ARG for bad parameters
 * or NULL arrays; LGS_ERR_UNSUPPORTED when a mean lies more than 2^20 cells
 * of tau_dist from the origin along an axis. */
typedef struct {
  int32_t k;
  float tau_dist, tau_sim, min_opacity, max_scale;
} lgs_prune_params;
lgs_prune_params lgs_default_prune_params(void);
lgs_status lgs_prune(lgs_context *ctx, const lgs_gaussians *g,
                     const lgs_prune_params *params, uint8_t *mask,
                     int64_t counts[3], hipStream_t stream);

/* Counts of the state's forward and, once enqueued, its backward (read when
 * asked for: synchronises with the device). */
lgs_status lgs_state_counts(const lgs_fwd_state *state, lgs_counts *out);
/* With the LGS_PROFILE_EVENTS bit of settings.profile on the forward, after
 * its backward: elapsed milliseconds of ms[0..4] = projection + depth sort +
 * scans, pair emission + tile sort, forward compositing kernel, backward
 * compositing kernel, gradient reduction + projection backward (HIP events
 * on the caller's stream).  Synchronises. */
lgs_status lgs_state_stage_ms(const lgs_fwd_state *state, float ms[5]);
/* Frees the state without waiting: its device buffers go back to the
 * context's cache behind the work already enqueued on the state's stream
 * (a later call on another stream waits for that work on the device). */
lgs_status lgs_state_release(lgs_context *ctx, lgs_fwd_state *state);

/* Whole mapping-loss step as one captured hipGraph: forward, gradient of the
 * loss of Eq. (1), backward.  With ssim_lambda = 0 the loss is the L1 form
 * (sum over views of w_rgb mean|RGB-RGB*| + w_depth mean|D-D*| + w_feat
 * mean|F-F*|, sign(0) = 0) whose gradient the backward compositing kernel
 * forms itself (the eager lgs_forward + lgs_backward_l1 computes the same
 * step); with ssim_lambda in (0, 1] it is the loss of lgs_loss, whose
 * kernel writes dL/dY into graph-owned planes before the backward (the
 * eager lgs_forward + lgs_loss + lgs_backward computes the same step).
 * targets[n_views] (device planes, final_T ignored), out[n_views] and grads
 * are bound at creation;
 * every launch recomputes them from the current contents of the Gaussian
 * arrays.  pair_capacity bounds the (tile, Gaussian) pairs; a launch that
 * would exceed it writes nothing valid and lgs_graph_status then returns
 * LGS_ERR_CAPACITY (re-create with a larger capacity).  Creation waits for
 * its own uploads on `stream` before returning, so the graph may then be
 * launched on any stream. */
lgs_status lgs_graph_create(lgs_context *ctx, const lgs_settings *st,
                            const lgs_gaussians *g, int32_t n_views,
                            const lgs_camera *cams, const lgs_images *targets,
                            const float loss_w[3], float ssim_lambda,
                            const lgs_images *out, const lgs_grads *grads,
                            int64_t pair_capacity, hipStream_t stream,
                            lgs_graph **graph_out);
lgs_status lgs_graph_launch(lgs_graph *graph, hipStream_t stream);
/* Synchronises with the graph's last launch; LGS_ERR_CAPACITY after an
 * overflowing launch, else LGS_OK. */
lgs_status lgs_graph_status(lgs_graph *graph);
/* Work counts of the graph's last launch (synchronises with it). */
lgs_status lgs_graph_counts(lgs_graph *graph, lgs_counts *out);
/* With the LGS_PROFILE_EVENTS bit of settings.profile at creation, the step
 * is captured as five graphs, one per stage, which lgs_graph_launch launches
 * back to back with HIP events recorded between them on the launching stream
 * (same results as the one-graph form).  Elapsed milliseconds of the last
 * launch's stages,
 * ms[0..4] = projection + depth sort + scans, pair emission + tile sort,
 * forward compositing, backward compositing (with the loss gradient: fused
 * L1, or the lgs_loss kernel), gradient reduction + projection backward.  Synchronises. */
lgs_status lgs_graph_stage_ms(lgs_graph *graph, float ms[5]);
void lgs_graph_destroy(lgs_graph *graph);

/* Autotuner (Sec. III-B.3: the mapping step, repeated over many iterations
 * per keyframe window): for every (tile, chunk, order) setting on the given
 * workload, captures the L1 mapping step as one graph (lgs_graph_create,
 * ssim_lambda 0, pair_capacity as there) and times it on `stream` with HIP
 * events (median of 7 launches after 2 warm-up launches: device time only),
 * and returns the fastest in *best_out (other fields copied from *st).
 * Settings are visited in a fixed order and a later one wins only when it is
 * more than 1 % faster, so settings within noise of each other resolve to the
 * same choice.  `out` and `grads` are overwritten.  Synchronises.  With
 * cache_path non-NULL the result is stored in / read from a small JSON file
 * keyed by the Gaussian count, appearance dtype, feature dimension, loss form
 * and view sizes. */
lgs_status lgs_autotune(lgs_context *ctx, const lgs_settings *st,
                        const lgs_gaussians *g, int32_t n_views,
                        const lgs_camera *cams, const lgs_images *targets,
                        const float loss_w[3], const lgs_images *out,
                        const lgs_grads *grads, int64_t pair_capacity,
                        hipStream_t stream, const char *cache_path,
                        lgs_settings *best_out);

#ifdef __cplusplus
}
#endif
#endif /* LEGO_RASTER_H */
