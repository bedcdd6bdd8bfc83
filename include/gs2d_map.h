/* The mapping side around the rasterizer: the mapping loss with its image
 * gradients, covisibility and keyframe selection, contribution pruning with stable
 * compaction, the per-splat map state, and map correction after pose-graph
 * optimisation.
 *
 * Per-splat contributions come from the forward render (gs2d_view.contrib,
 * eq:contribution).  Every pointer is caller-owned device memory; every call is
 * asynchronous on `stream` and allocates nothing.  Errors: GS2D_ERR_INVALID_ARG for
 * null pointers where data is required or negative sizes, GS2D_ERR_HIP for a failed
 * launch.  None of these calls needs a rasterizer context.
 */
#ifndef GS2D_MAP_H
#define GS2D_MAP_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs2d.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Weights of the mapping loss's four terms.  The table of parameters gives 0.125 to
 * the SSIM term (so 0.875 to the L1 term), w_d = 0.5 and w_n = 0.02: the defaults. */
typedef struct gs2d_mapping_weights {
  float w_l1, w_ssim, w_d, w_n;
} gs2d_mapping_weights;

/* Floats of workspace gs2d_mapping_loss needs for a width x height image. */
GS2D_API int64_t gs2d_mapping_loss_workspace(int32_t width, int32_t height);

/* Mapping loss of Sec. "Mapping" on one view's rendered images (planar float32:
 * rgb [3][H][W], depth [H][W], normal [3][H][W]) against the observed tgt_rgb and
 * tgt_depth:
 *   L_m = (1/HW) sum_p [ w_l1 |rgb - tgt_rgb|_1 + w_ssim (1 - SSIM(p))
 *                        + w_d |depth - tgt_depth| + w_n (1 - N_D(p) . normal(p)) ],
 * with SSIM(p) the mean over RGB of the SSIM map (11 x 11 Gaussian window, sigma 1.5,
 * zero outside the image, C1 = 0.01^2, C2 = 0.03^2) and N_D the normals of the
 * rendered depth (eq:normal_fromD): the normalised cross product of the central
 * differences X(x+1, y) - X(x-1, y) and X(x, y+1) - X(x, y-1) of the back-projected
 * pixels X = depth ((x - cx)/fx, (y - cy)/fy, 1), x the column; 0 on the image border
 * and where the cross product vanishes.  weights NULL: the defaults above.
 * Writes loss (device float [5]) = {L_m, and the image means of |d rgb|_1,
 * 1 - SSIM, |d depth| and 1 - N_D . N}, and the gradients of L_m to the three
 * rendered images (d|x|/dx = 0 at 0) to d_rgb, d_depth, d_normal (overwritten).
 * work: device float [gs2d_mapping_loss_workspace(W, H)].  Deterministic: fixed-order
 * sums, no atomics. */
GS2D_API int gs2d_mapping_loss(const gs2d_camera* camera, const float* rgb, const float* depth, const float* normal,
                               const float* tgt_rgb, const float* tgt_depth, const gs2d_mapping_weights* weights,
                               float* loss, float* d_rgb, float* d_depth, float* d_normal, float* work,
                               hipStream_t stream);

/* Words of workspace gs2d_covisibility needs for n splats (at most 2048). */
GS2D_API int64_t gs2d_covisibility_workspace(int64_t n);

/* Covisibility of two views over the same n splats (Sec. "Tracking and Keyframe
 * Selection"): G_V = {k : contrib_V[k] > threshold} (the paper's visibility uses 0.5);
 * counts (device uint32 [2], overwritten) = {|G_A & G_B|, |G_A | G_B|}.  The score
 * S_cov = counts[0] / counts[1] (0 when counts[1] = 0).  work: device uint32
 * [gs2d_covisibility_workspace(n)], per-workgroup partial counts (no atomics, so the
 * counts do not depend on scheduling). */
GS2D_API int gs2d_covisibility(const float* contrib_a, const float* contrib_b, int64_t n, float threshold,
                               uint32_t* counts, uint32_t* work, hipStream_t stream);

/* Keyframe test (Sec. "Tracking and Keyframe Selection"): *is_keyframe (device
 * int32) = 1 when S_cov from `counts` is below c_k, or when the translation vectors of
 * the world-to-camera poses pose_cur and pose_kf (device [12], [R|t] row-major) are
 * more than d_k apart; else 0.  The score and the distance are evaluated in double. */
GS2D_API int gs2d_keyframe_test(const uint32_t* counts, const float* pose_cur, const float* pose_kf, double c_k,
                                double d_k, int32_t* is_keyframe, hipStream_t stream);

/* Pruning (Sec. "Mapping"): remove[k] (device uint8 [n]) = 1 when splat k is
 * associated with keyframe `frame` (closest_frame[k] == frame) and its contribution
 * from that keyframe, contrib[k], is below `threshold` (0.5 in the paper); else 0. */
GS2D_API int gs2d_prune_mask(const float* contrib, const int32_t* closest_frame, int32_t frame, float threshold,
                             int64_t n, uint8_t* remove, hipStream_t stream);

/* Words of workspace gs2d_compact needs for n splats. */
GS2D_API int64_t gs2d_compact_workspace(int64_t n);

/* Stable compaction: the columns k < n with remove[k] == 0 (remove NULL: all) of
 * n_planes planes of 32-bit values (in: [n_planes][in_stride]) to the front of
 * out ([n_planes][out_stride], out_stride >= the kept count; in and out must not
 * overlap), in their order; *n_out (device uint32) = the kept count.  work: device
 * uint32 [gs2d_compact_workspace(n)].  The surfel parameters [15][n] and the map
 * state arrays compact with one call each (their strides may differ). */
GS2D_API int gs2d_compact(const void* in, int64_t in_stride, int32_t n_planes, int64_t n, const uint8_t* remove,
                          void* out, int64_t out_stride, uint32_t* n_out, uint32_t* work, hipStream_t stream);

/* Map state after keyframe `frame` (Sec. "Mapping", eq:map), in place:
 *   1. with loop_frame >= 0 (the keyframes after a loop with keyframe loop_frame): an
 *      inactive splat that is visible (contrib > 0.5) and has t_closest > loop_frame
 *      becomes active with t_last = frame;
 *   2. every active visible splat gets t_last = frame, and t_closest = frame and
 *      d_closest = its distance to the keyframe's camera centre when that is below
 *      d_closest;
 *   3. an active splat with frame - t_last > inactive_after becomes inactive.
 * params [15][n] (the centre mu in rows 0-2); contrib [n] from the keyframe's render;
 * pose_kf device [12] world-to-camera; t_closest, t_last, active int32 [n] (active:
 * 0 or 1, 32-bit so that the state compacts with gs2d_compact); d_closest float [n]
 * (metres).  Distances are evaluated in double. */
GS2D_API int gs2d_map_state_update(const float* params, int64_t n, const float* contrib, const float* pose_kf,
                                   int32_t frame, int32_t inactive_after, int32_t loop_frame, int32_t* t_closest,
                                   float* d_closest, int32_t* t_last, int32_t* active, hipStream_t stream);

/* Map correction (Sec. "Map Correction"): each splat with 0 <= closest_frame[k] <
 * n_frames moves with its keyframe's pose increment Delta T = T^o T^-1 (T, T^o the
 * keyframe's camera-to-world poses before and after the pose-graph optimisation; for
 * world-to-camera poses pass (T^o)^-1 T).  delta: device float [n_frames][12], [R|t]
 * row-major, acting on world points:
 * mu <- dR mu + dt, t_u <- dR t_u, t_v <- dR t_v, in place on params [15][n]; other
 * splats are left as they are.  Evaluated in double. */
GS2D_API int gs2d_map_correct(float* params, int64_t n, const int32_t* closest_frame, const float* delta,
                              int32_t n_frames, hipStream_t stream);

/* Arguments of gs2d_params_adam.  lr: one learning rate per parameter group, in the
 * order mu, t_u, t_v, scales, opacity, colour; step: the 1-based step number t of the
 * bias corrections. */
typedef struct gs2d_adam_args {
  float lr[6];
  float beta1, beta2, eps, weight_decay;
  int32_t step;
  float s_min, o_min, o_max;
} gs2d_adam_args;

/* One Adam step over the surfel parameters params [15][n] with their gradient grad
 * [15][n] and moments m, v [15][n] (all device float, updated in place): per entry
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + weight_decay p),
 * then the scales (rows 9-10) clamped to >= s_min and the opacity (row 11) to
 * [o_min, o_max].  The map's optimiser of Sec. "Mapping" (the paper does not state its
 * constants; Adam is the optimiser of 2D Gaussian splatting maps).  Float32. */
GS2D_API int gs2d_params_adam(float* params, const float* grad, float* m, float* v, int64_t n,
                              const gs2d_adam_args* args, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GS2D_MAP_H */
