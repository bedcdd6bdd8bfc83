/*
 * gs2d: differentiable 2D Gaussian surfel rasterizer for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libgs2d.so.  The rasterizer renders colour, depth, normal and opacity
 * images from 2D Gaussian surfels seen by a pinhole camera, and returns gradients
 * to every surfel parameter and to the camera pose as an se(3) 6-vector.  The
 * method is the one of "Globally Consistent RGB-D SLAM with 2D Gaussian
 * Splatting" (Zhong et al., 2025): Sec. "2D Gaussian Splatting" (eq:Puv, eq:hc,
 * eq:homo, eq:wth, eq:alpha_blending) for the forward pass, Sec. "Camera Pose
 * Optimization" (eq:derivatives) for the pose gradient, and Sec. "Tracking and
 * Keyframe Selection" (eq:LD, eq:normal_mask, eq:opacity_mask, eq:tracking_loss)
 * for the tracking loss.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Surfels   float32 structure-of-arrays [15][n], row-major, rows:
 *           mu.xyz (0-2), t_u.xyz (3-5), t_v.xyz (6-8), s_u (9), s_v (10),
 *           opacity (11), r g b (12-14).  Scales and opacity are used as given
 *           (post-activation); colour is a plain RGB triple (no spherical
 *           harmonics).  The surfel normal is t_u x t_v (not re-normalised).
 * Pose      float32 [12], row-major 3x4 [R | t] mapping world points into the
 *           camera frame (x right, y down, z forward).  Pose gradients are with
 *           respect to a left perturbation Exp(tau) T, tau = (rho, phi):
 *           translation first, rotation vector second.
 * Camera    pinhole (fx, fy, cx, cy); pixel (x, y) is sampled at the integer
 *           image coordinates x, y.
 * Images    float32 planar, row-major: rgb [3][H][W], depth [H][W],
 *           normal [3][H][W], alpha [H][W].  Depth is the blended camera z of
 *           each ray-splat intersection (not divided by alpha); background is 0.
 * Rules     a (pixel, surfel) pair is composited when min(u^2+v^2, 2|p-c|^2)
 *           <= 9 (c: projected centre, the second term a low-pass filter that
 *           the options can turn off), its depth is >= z_near and
 *           alpha = min(0.99, o G) >= 1/255; compositing stops before the
 *           surfel that would drop transmittance below 1e-4; surfels are
 *           ordered by float32 camera depth of their centre, ties by index.
 *
 * Memory: every array argument is a device pointer owned by the caller unless
 * marked "host".  Inputs are only read.  The library allocates only context
 * workspace, never while the stream is being captured into a graph.  Calls on
 * one context must be serialised by the caller (one context per stream).
 *
 * Errors: every int-returning call returns GS2D_OK (0) or a negative code; see
 * gs2d_error_string.  After GS2D_ERR_HIP the underlying hipError_t is kept in
 * the context (gs2d_last_hip_error).
 */
#ifndef GS2D_H
#define GS2D_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS2D_API __attribute__((visibility("default")))

#define GS2D_OK 0
#define GS2D_ERR_INVALID_ARG (-1)
#define GS2D_ERR_OOM (-2)
#define GS2D_ERR_HIP (-3)
#define GS2D_ERR_CAPACITY (-4)   /* tile-pair capacity exceeded on the device */
#define GS2D_ERR_STATE (-5)      /* backward called without a matching forward */
#define GS2D_ERR_UNSUPPORTED (-6)
#define GS2D_ERR_NONFINITE (-7)    /* a surfel, pose, loss or gradient was not finite */
#define GS2D_ERR_DEVICE_CHECK (-8) /* a device check of a GS2D_DEVICE_CHECKS build failed */

/* Most views (or tracking problems) one batched call may take. */
#define GS2D_MAX_VIEWS 32

/* Flags for gs2d_render_backward. */
#define GS2D_ACCUMULATE 1        /* add into d_params / d_pose instead of overwriting */

typedef struct gs2d_ctx gs2d_ctx;

typedef struct gs2d_camera {
  int32_t width, height;
  float fx, fy, cx, cy;
} gs2d_camera;

typedef struct gs2d_options {
  int32_t tile_w, tile_h;    /* screen tile: 8x8, 16x8, 16x16 (default) or 32x16 */
  int32_t batch;             /* surfels staged per LDS batch: 32, 64, 128 (default) or 256 */
  int32_t filter;            /* 1 (default): low-pass filter branch; 0: plain 3-sigma footprint */
  float z_near;              /* default 0.2: centre cull and per-pixel depth cut */
  int64_t pair_capacity;     /* tile-pair capacity; 0 (default): grow on demand */
  int32_t keep_unsorted;     /* 1: keep a copy of the pairs before the tile sort (tests) */
  int32_t profile;           /* 1: time kernel families with HIP events and count blend work;
                                2: time them only (the blend kernels then run the same code as
                                without profiling); calls outside graph capture only; see
                                gs2d_get_profile */
} gs2d_options;

/* Counters of the last forward pass (gs2d_get_counts synchronises the stream). */
typedef struct gs2d_counts {
  int64_t n_surfels;         /* surfels given to the last render */
  int64_t n_visible;         /* surfels that touch at least one tile */
  int64_t n_pairs;           /* (tile, surfel) pairs after duplication */
  int64_t pair_capacity;     /* current pair capacity */
  int32_t overflow;          /* 1: the last render exceeded the capacity (outputs invalid) */
  int32_t n_tiles;
  int32_t nonfinite;         /* 1: the last render met a surfel or pose with a value that is
                                not finite; those surfels (all of a bad view) were culled */
  int32_t device_checks;     /* bits of the device checks that failed since the context was
                                created (always 0 unless built with GS2D_DEVICE_CHECKS):
                                1 tile rectangle outside its view's grid, 2 pair tile key out
                                of range, 4 pair slot past the capacity, 8 sorted key out of
                                range, 16 blended tile or range invalid */
} gs2d_counts;

/* One view of a batched render: its surfels [15][n], camera, pose [12] and outputs
 * (planar images of the view's size; any may be NULL).  Views may share a surfel
 * buffer (a window of keyframes over one map) or not (independent problems). */
typedef struct gs2d_view {
  const float* params;
  int64_t n;
  gs2d_camera camera;
  const float* pose;
  float* rgb;
  float* depth;
  float* normal;
  float* alpha;
  /* optional [n] out: each surfel's contribution to this view, the sum over pixels of
   * its blending weight (Sec. "Tracking and Keyframe Selection", eq:contribution);
   * float atomics, so the summation order varies between runs.  NULL: not wanted. */
  float* contrib;
  /* optional [H][W] outs, the depth channel's variants: depth_norm = D / O (0 where
   * O = 0); depth_median = the depth of the last composited intersection whose
   * incoming transmittance exceeds 1/2, where the accumulated opacity reaches one half
   * (the last composited one if it never does; 0 with none).  NULL: not wanted. */
  float* depth_norm;
  float* depth_median;
} gs2d_view;

/* Gradients of one view for gs2d_render_backward_batch: image gradients in (any may
 * be NULL, meaning zero), d_params [15][n] and d_pose [6] out (NULL: not wanted). */
typedef struct gs2d_view_grad {
  const float* d_rgb;
  const float* d_depth;
  const float* d_normal;
  const float* d_alpha;
  float* d_params;
  float* d_pose;
} gs2d_view_grad;

/* One independent tracking problem of gs2d_track_batch. */
typedef struct gs2d_track_problem {
  const float* params;       /* [15][n] */
  int64_t n;
  gs2d_camera camera;
  float* pose;               /* [12] in: start pose, out: final pose */
  const float* tgt_rgb;      /* [3][H][W] */
  const float* tgt_depth;    /* [H][W] */
  /* Warm-start fallback (both device pointers, or both NULL for none): a pose [12] and
   * its unmasked tracking loss [1] (use_masks = 0, the same lambda_d), as
   * gs2d_warm_start_propose gives for the start pose.  The first iteration compares the
   * unmasked loss at the problem's own start pose with it; if that is larger (or not
   * finite), the pose becomes the fallback pose before the second iteration, with no
   * step taken (the first entries of the histories record the rejected pose's loss and
   * gradient, and the fallback pose); status then has GS2D_TRACK_FELL_BACK set. */
  const float* fallback_pose;
  const float* fallback_loss;
} gs2d_track_problem;

/* Kernel-family timings (options.profile = 1 or 2) and blend work counters (profile = 1). */
#define GS2D_PROFILE_FAMILIES 13
typedef struct gs2d_profile {
  double ms[GS2D_PROFILE_FAMILIES];          /* summed event time per family since the last reset */
  int64_t launches[GS2D_PROFILE_FAMILIES];   /* timed calls per family */
  int64_t fwd_evaluated;     /* (pixel, surfel) evaluations performed by the forward blend */
  int64_t fwd_covering;      /* ... of which inside the footprint (rho <= 9, depth >= z_near) */
  int64_t bwd_evaluated;     /* the same for the backward blend */
  int64_t bwd_covering;
} gs2d_profile;

/* Arguments of gs2d_track: n_iters tracking iterations, each a forward render at the
 * current pose, the tracking loss against (tgt_rgb, tgt_depth), a pose-only backward
 * and one AdamW step on tau followed by T <- Exp(tau) T (tau reset to 0, moments kept). */
typedef struct gs2d_track_args {
  const float* params;       /* [15][n] */
  int64_t n;
  gs2d_camera camera;
  float* pose;               /* [12] in: start pose, out: final pose */
  const float* tgt_rgb;      /* [3][H][W] */
  const float* tgt_depth;    /* [H][W] */
  float lambda_d;            /* depth weight of the tracking loss */
  int32_t use_masks;         /* 1: normal and opacity masks of the tracking loss */
  int32_t n_iters;
  float lr[6];               /* per-component learning rates (rho then phi) */
  float beta1, beta2, eps, weight_decay;
  int32_t use_graph;         /* 1: capture one iteration into a HIP graph and replay it */
  float* pose_history;       /* [n_iters][12] pose after each step, or NULL */
  float* loss_history;       /* [n_iters] loss before each step, or NULL */
  double* grad_history;      /* [n_iters][6] pose gradient (rho, phi) each step consumed, FP64
                                as the step uses it, or NULL */
  /* Divergence guard: after this many iterations in a row without a loss below the
   * lowest one so far, the problem stops and its pose returns to the pose of that
   * lowest loss; the remaining iterations leave it there (0: never stop). */
  int32_t diverge_patience;
  /* [n_problems] out (device, int32) or NULL: each problem's end state, 0 every
   * iteration stepped, 1 stopped by the divergence guard, 2 stopped on a loss or
   * pose gradient that is not finite (the pose is the last finite one); plus
   * GS2D_TRACK_FELL_BACK (4) when the warm-start fallback replaced the start pose. */
  int32_t* status;
  /* gs2d_track only: the warm-start fallback of its problem (see gs2d_track_problem);
   * gs2d_track_batch reads each problem's own. */
  const float* fallback_pose;
  const float* fallback_loss;
} gs2d_track_args;
#define GS2D_TRACK_FELL_BACK 4

/* Build flags of the loaded library: GS2D_BUILD_DEVICE_CHECKS when it was compiled
 * with GS2D_DEVICE_CHECKS (the debug build whose kernels check their indices and
 * record failures in gs2d_counts.device_checks; gs2d_track then returns
 * GS2D_ERR_DEVICE_CHECK). */
#define GS2D_BUILD_DEVICE_CHECKS 1
GS2D_API int gs2d_build_info(void);

/* Fill *opt with the defaults listed above. */
GS2D_API int gs2d_default_options(gs2d_options* opt);

/* Create a context on HIP device `device` (opt may be NULL for defaults).  The
 * context owns all workspace.  Returns INVALID_ARG for an unsupported tile or batch. */
GS2D_API int gs2d_create(gs2d_ctx** ctx, int device, const gs2d_options* opt);

/* Free the context and its workspace (never caller memory).  NULL is accepted. */
GS2D_API int gs2d_destroy(gs2d_ctx* ctx);

/* Forward render (Sec. "2D Gaussian Splatting": eq:homo for the ray-splat
 * intersection, eq:alpha_blending for compositing).  params [15][n], pose [12]
 * (device); camera by value from the host.  Overwrites rgb [3][H][W],
 * depth [H][W], normal [3][H][W], alpha [H][W]; any of them may be NULL.
 * Saves the forward state in the context and returns its generation number in
 * *generation (host, may be NULL).  n == 0 renders a blank image. */
GS2D_API int gs2d_render(gs2d_ctx* ctx, const float* params, int64_t n, const gs2d_camera* camera,
                         const float* pose, float* rgb, float* depth, float* normal, float* alpha,
                         uint32_t* generation, hipStream_t stream);

/* Reverse mode of the render with generation `generation` (else GS2D_ERR_STATE)
 * for the given image gradients (any may be NULL, meaning zero).
 * d_params [15][n] receives dL/d(surfel parameters) in the world frame; NULL
 * selects the pose-only mode, in which no per-surfel gradient is formed.
 * d_pose [6] receives dL/dtau for a left perturbation of the pose, the paper's
 * eq:derivatives (dL/dmu_c [I, -mu_c^x] plus dL/dR_c against [0, -R_c[:,k]^x]).
 * flags: GS2D_ACCUMULATE adds to d_params and d_pose instead of overwriting.
 * With d_params the per-surfel sums are added with float atomics, so d_params and
 * d_pose can differ in their last bits between runs; the pose-only mode sums in a
 * fixed order and is bitwise repeatable.  Needs the GPU to hold 64 B per (view,
 * surfel) item of accumulator rows (grown on demand; GS2D_ERR_CAPACITY when
 * that would happen under stream capture). */
GS2D_API int gs2d_render_backward(gs2d_ctx* ctx, const float* d_rgb, const float* d_depth,
                                  const float* d_normal, const float* d_alpha, float* d_params,
                                  float* d_pose, uint32_t generation, int32_t flags,
                                  hipStream_t stream);

/* Batched forward render of n_views (1..GS2D_MAX_VIEWS) views in one launch per
 * kernel: pairs of every (view, surfel) item keyed by a global tile index that
 * places each view's tiles after the previous view's, one tile sort, one depth
 * order of every tile's list, and one blend grid over all tiles of all views.  Each view's images equal
 * what gs2d_render gives for that view alone, bit for bit. */
GS2D_API int gs2d_render_batch(gs2d_ctx* ctx, const gs2d_view* views, int32_t n_views, uint32_t* generation,
                               hipStream_t stream);

/* Reverse mode of the batched render `generation`; grads has one entry per view.
 * Views that share a d_params buffer accumulate into it (the first overwrites unless
 * GS2D_ACCUMULATE).  Each view's d_pose is its own left-perturbation gradient. */
GS2D_API int gs2d_render_backward_batch(gs2d_ctx* ctx, const gs2d_view_grad* grads, int32_t n_views,
                                        uint32_t generation, int32_t flags, hipStream_t stream);

/* Tracking loss of Sec. "Tracking and Keyframe Selection" (eq:tracking_loss):
 * L = (1/HW) sum_p M_n M_o (|rgb - tgt_rgb|_1 + lambda_d |depth - tgt_depth|),
 * M_n = [normal . ray > 0] (eq:normal_mask), M_o = [alpha > 0.95]
 * (eq:opacity_mask); use_masks = 0 drops both masks.  Inputs are images of
 * `camera`'s size.  Writes the loss to *loss (device scalar) and its gradients,
 * masks held constant and d|x|/dx = 0 at 0, to d_rgb [3][H][W] and d_depth [H][W]. */
GS2D_API int gs2d_tracking_loss(gs2d_ctx* ctx, const gs2d_camera* camera, const float* rgb,
                                const float* depth, const float* normal, const float* alpha,
                                const float* tgt_rgb, const float* tgt_depth, float lambda_d,
                                int32_t use_masks, float* loss, float* d_rgb, float* d_depth,
                                hipStream_t stream);

/* Weights and masks of gs2d_image_loss. */
typedef struct gs2d_loss_weights {
  float w_rgb, w_depth, w_normal;
  int32_t normal_mask;   /* 1: M_n = [normal . ray > 0] (eq:normal_mask) */
  int32_t opacity_mask;  /* 1: M_o = [alpha > 0.95] (eq:opacity_mask) */
} gs2d_loss_weights;

/* Masked L1 image loss: L = (1/HW) sum_p M (w_rgb |rgb - tgt_rgb|_1 + w_depth |depth -
 * tgt_depth| + w_normal |normal - tgt_normal|_1), M the product of the selected masks
 * (1 with none).  The tracking loss (eq:tracking_loss) is (1, lambda_d, 0) with both
 * masks; the unmasked single-frame L1 over colour, depth and normal is (1, 1, 1); the
 * mapping window's colour and depth terms (Sec. "Mapping", w_d = 0.5) under the opacity
 * mask are (1, 0.5, 0) with opacity_mask only.  rgb/tgt_rgb may be NULL when w_rgb = 0
 * and d_rgb is NULL, normal/tgt_normal when w_normal = 0, d_normal is NULL and the
 * normal mask is off.  Writes *loss (device scalar) and, where not NULL, the gradients
 * (masks constant, d|x|/dx = 0 at 0) to d_rgb [3][H][W], d_depth [H][W], d_normal
 * [3][H][W]. */
GS2D_API int gs2d_image_loss(gs2d_ctx* ctx, const gs2d_camera* camera, const float* rgb, const float* depth,
                             const float* normal, const float* alpha, const float* tgt_rgb, const float* tgt_depth,
                             const float* tgt_normal, const gs2d_loss_weights* weights, float* loss, float* d_rgb,
                             float* d_depth, float* d_normal, hipStream_t stream);

/* One view of gs2d_image_loss_batch: its camera and the images, targets and gradient
 * outputs of gs2d_image_loss (same NULL rules). */
typedef struct gs2d_loss_view {
  gs2d_camera camera;
  const float *rgb, *depth, *normal, *alpha;
  const float *tgt_rgb, *tgt_depth, *tgt_normal;
  float *d_rgb, *d_depth, *d_normal;
} gs2d_loss_view;

/* gs2d_image_loss of n_views (1..GS2D_MAX_VIEWS) views with one set of weights, in one
 * launch for all views and one for their reductions: losses [n_views] (device)
 * receives each view's loss; each view's gradients as gs2d_image_loss writes them.
 * Results equal n_views calls of gs2d_image_loss, bit for bit. */
GS2D_API int gs2d_image_loss_batch(gs2d_ctx* ctx, const gs2d_loss_view* views, int32_t n_views,
                                   const gs2d_loss_weights* weights, float* losses, hipStream_t stream);

/* Largest image (width x height) gs2d_image_loss_noalloc takes. */
#define GS2D_NOALLOC_MAX_PIXELS (1 << 24)

/* gs2d_image_loss without a context, for callers that cannot allocate device memory:
 * code under HIP graph capture, serving loops, harnesses that forbid hipMalloc.  Same
 * arguments (other than the context), NULL rules, results and launches as
 * gs2d_image_loss, on the device that is current for the calling thread.  It calls no
 * allocating routine: its scratch memory (a one-view descriptor table and one partial
 * sum per 256 pixels, 257 KiB) is a fixed array in the library's device code, one copy
 * per GPU, held until the process ends; the first call on a device looks up that
 * copy's address.  Images of more than GS2D_NOALLOC_MAX_PIXELS pixels return
 * GS2D_ERR_CAPACITY before any work.  Every call on one GPU shares that GPU's copy:
 * calls that overlap on one GPU (on different streams, or from different threads)
 * race and must be serialised by the caller.  GS2D_ERR_HIP if the address lookup or a
 * launch fails. */
GS2D_API int gs2d_image_loss_noalloc(const gs2d_camera* camera, const float* rgb, const float* depth,
                                     const float* normal, const float* alpha, const float* tgt_rgb,
                                     const float* tgt_depth, const float* tgt_normal,
                                     const gs2d_loss_weights* weights, float* loss, float* d_rgb, float* d_depth,
                                     float* d_normal, hipStream_t stream);

/* Relocalisation error of Sec. "Loop Detection and Relocalization" (eq:tracking_error):
 * e_t = (1/HW) sum_p M_n M_o |depth - tgt_depth|, the depth term of the tracking loss
 * with its masks (M_n = [normal . ray > 0], M_o = [alpha > 0.95]), computed on the
 * depth re-rendered at the optimised pose.  Inputs are images of `camera`'s size;
 * writes *error (device scalar). */
GS2D_API int gs2d_tracking_error(gs2d_ctx* ctx, const gs2d_camera* camera, const float* depth, const float* normal,
                                 const float* alpha, const float* tgt_depth, float* error, hipStream_t stream);

/* Run the tracking loop described at gs2d_track_args (the pose update of Sec.
 * "Tracking and Keyframe Selection": AdamW on the pose, surfels frozen).  The
 * first call sizes the pair buffers on the start pose (one synchronising render).
 * With use_graph the iteration is captured once on a stream of the context and
 * replayed; the instantiated graph is kept and reused by later calls with the same
 * buffers and hyper-parameters.  Returns after the work has completed (the call
 * synchronises).  On a pair overflow the loop restarts from the start pose with
 * larger buffers (up to 3 attempts, then GS2D_ERR_CAPACITY).  GS2D_ERR_NONFINITE
 * when a surfel or the pose held a value that is not finite (such surfels are culled
 * from every render) or a problem stopped on a non-finite loss or gradient; the poses
 * and histories are still written (a stopped problem keeps its last finite pose). */
GS2D_API int gs2d_track(gs2d_ctx* ctx, const gs2d_track_args* args, hipStream_t stream);

/* n_problems (1..GS2D_MAX_VIEWS) independent tracking problems stepped together:
 * every iteration renders all of them in one batched launch per kernel, computes
 * each one's tracking loss, runs one batched pose-only backward and one AdamW + Exp
 * step per problem.  `common` supplies lambda_d, use_masks, n_iters, the optimizer
 * constants and use_graph (its params/n/camera/pose/target fields are ignored);
 * its pose_history is [n_iters][n_problems][12], loss_history [n_iters][n_problems] and
 * grad_history [n_iters][n_problems][6].
 * Same graph caching, synchronisation and restart rules as gs2d_track. */
GS2D_API int gs2d_track_batch(gs2d_ctx* ctx, const gs2d_track_problem* problems, int32_t n_problems,
                              const gs2d_track_args* common, hipStream_t stream);

/* pose_out = Exp(tau) pose_in for tau = (rho, phi) [6] and 3x4 poses [12] (device;
 * pose_out may alias pose_in).  The left perturbation of the paper's manifold
 * derivative (Sec. "Camera Pose Optimization"); Exp in closed form, FP64 inside. */
GS2D_API int gs2d_pose_exp(gs2d_ctx* ctx, const float* tau, const float* pose_in, float* pose_out,
                           hipStream_t stream);

/* d_tau = J_l(tau)^T d_pose (device [6] each): pulls the left-perturbation gradient
 * at Exp(tau) T back to tau, J_l the SE(3) left Jacobian (identity at tau = 0). */
GS2D_API int gs2d_pose_tau_grad(gs2d_ctx* ctx, const float* tau, const float* d_pose, float* d_tau,
                                hipStream_t stream);

/* Result of gs2d_autotune. */
typedef struct gs2d_tuning {
  int32_t tile_w, tile_h, batch;
  float ms;                  /* best mean fwd + bwd time (ms), the backward as flags select */
  int32_t n_candidates;
  int32_t from_cache;        /* 1: the choice came from the context's cache */
} gs2d_tuning;

/* Autotuner: for every tile shape {8x8, 16x8, 16x16, 32x16} x LDS batch {32, 64, 128,
 * 256}, time `reps` repetitions (after one warm-up) of the tracking iteration that
 * gs2d_track runs on (params, n, camera, pose): the sorts, the fused walk (forward
 * blend, tracking loss and pose-only backward) and the pose step, against the render
 * at `pose` as target, on a copy of the pose (the caller's pose is only read).  Keep
 * the fastest in the context (its later renders and tracking calls use it) and cache
 * it for this (width, height, power-of-two class of n, flags).  flags:
 * GS2D_TUNE_FULL_BACKWARD times the forward render and the backward to all surfel
 * parameters instead (the mapping side's workload; it needs 60 B per surfel of device
 * memory while it runs).  The images do not depend on the choice.  Synchronises
 * `stream`; not capturable. */
#define GS2D_TUNE_FULL_BACKWARD 1

GS2D_API int gs2d_autotune(gs2d_ctx* ctx, const float* params, int64_t n, const gs2d_camera* camera,
                           const float* pose, int32_t reps, int32_t flags, gs2d_tuning* out, hipStream_t stream);

/* Counters of the last render; synchronises `stream`. */
GS2D_API int gs2d_get_counts(gs2d_ctx* ctx, gs2d_counts* out, hipStream_t stream);

/* Copy an internal buffer of the last render to host memory (diagnostics and tests).
 * which: 0 sorted tile keys (uint32 [n_pairs]), 1 the tiles' surfel ids (uint32 [n_pairs];
 * within each tile ascending in (depth key, id)), 2 tile ranges (uint32 [n_tiles][2]),
 * 3 per-surfel depth keys (uint32 [n]: float32 camera depth bits, 0xFFFFFFFF for
 * surfels that touch no tile), 4 per-surfel tile rect (uint16 [n][4]: x0, x1, y0, y1,
 * inclusive; empty: x0 > x1), 5 per-pixel final transmittance (float [H][W]),
 * 6 per-pixel list length (uint32 [H][W]), 7 unsorted tile keys, 8 unsorted surfel ids
 * (uint32 [n_pairs], emitted in surfel order before the tile sort; only with
 * options.keep_unsorted = 1), 10 the pose gradient of each problem's last tracking
 * iteration (double [32][6]; available after gs2d_track / gs2d_track_batch, without a
 * forward).
 * *bytes (host) is the buffer size in; the bytes copied out.  Synchronises `stream`. */
GS2D_API int gs2d_debug_copy(gs2d_ctx* ctx, int32_t which, void* host_dst, size_t* bytes,
                             hipStream_t stream);

/* Name of profile family i (0 <= i < GS2D_PROFILE_FAMILIES), NULL otherwise. */
GS2D_API const char* gs2d_profile_family(int i);

/* Collect the profile since the last reset (synchronises `stream`); reset != 0
 * clears it afterwards.  GS2D_ERR_UNSUPPORTED when options.profile = 0. */
GS2D_API int gs2d_get_profile(gs2d_ctx* ctx, gs2d_profile* out, int32_t reset, hipStream_t stream);

/* Last hipError_t recorded by the context (0 if none). */
GS2D_API int gs2d_last_hip_error(gs2d_ctx* ctx);

/* Static description of an error code. */
GS2D_API const char* gs2d_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* GS2D_H */
