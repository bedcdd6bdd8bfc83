/* Learned pose warm start for tracking: a small BF16 convolutional network on the
 * matrix cores that proposes an se(3) twist from the residual between the frame
 * rendered at the start pose and the observed RGB-D frame.
 *
 * This is an extension of the paper's method, not a step of it: the paper's
 * tracking (Sec. "Tracking and Keyframe Selection") starts at the previous pose
 * and iterates eq:tracking_loss with AdamW.  Here T_0 = Exp(tau_hat) T_start,
 * with tau_hat in the left-perturbation convention of the pose gradient
 * (eq:derivatives), and the plain iterations start from T_0 -- or from T_start
 * when T_0 does not lower the tracking loss (the fallback).
 *
 * Network (all sizes fixed):
 *   input   R, G, B, depth of (rendered - observed), each averaged over 8 x 8 pixel
 *           blocks: [4][60][80] per frame (frames of 640 x 480; other sizes whose
 *           width is 80 k and height 60 k are averaged over k x k blocks);
 *   conv    4->32 k5, 32->64 k3, 64->128 k3, 128->128 k3, stride 2, zero padding
 *           k/2, ReLU after each: [128][4][5];
 *   fc      2560->256 (ReLU) -> 6: the twist normalised as (rho / 0.1 m,
 *           phi / (8 deg in radians)).
 * Parameters: one flat FP32 vector of GS2D_WS_PARAMS = 900,326 values, layer by
 * layer the weight then the bias; conv weights [co][ci][ky][kx], fc weights [o][i].
 * Precision: BF16 weights (copies of the FP32 master vector) and activations,
 * round-to-nearest-even after every layer (and for every layer's input gradient
 * in training), FP32 accumulation, FP32 biases, FP32 output and weight gradients.
 *
 * Memory: every pointer argument is caller-owned device memory unless stated.
 * The network object owns its master weights, BF16 copies, AdamW moments and
 * activation workspace for up to max_batch frames.  One object per stream; calls
 * on one object must not overlap.
 */
#ifndef GS2D_WARM_H
#define GS2D_WARM_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs2d.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GS2D_WS_PARAMS 900326
#define GS2D_WS_IN_C 4
#define GS2D_WS_IN_H 60
#define GS2D_WS_IN_W 80
#define GS2D_WS_OUT 6

typedef struct gs2d_ws gs2d_ws;

typedef struct gs2d_ws_adamw {
  float lr;            /* learning rate */
  float beta1, beta2;  /* moment decays */
  float eps;
  float weight_decay;  /* decoupled: theta <- theta (1 - lr wd) - lr m_hat / (sqrt(v_hat) + eps) */
} gs2d_ws_adamw;

/* Number of parameters (GS2D_WS_PARAMS). */
GS2D_API int64_t gs2d_ws_param_count(void);

/* Create a network on `device` for batches of up to max_batch (1..4096) frames.
 * Its parameters are zero until gs2d_ws_set_params. */
GS2D_API int gs2d_ws_create(gs2d_ws** net, int device, int32_t max_batch);
GS2D_API int gs2d_ws_destroy(gs2d_ws* net);

/* Load the FP32 master parameters from theta (device [GS2D_WS_PARAMS]), refresh
 * the BF16 copies and reset the AdamW state. */
GS2D_API int gs2d_ws_set_params(gs2d_ws* net, const float* theta, hipStream_t stream);
/* Copy the FP32 master parameters to theta (device [GS2D_WS_PARAMS]). */
GS2D_API int gs2d_ws_get_params(gs2d_ws* net, float* theta, hipStream_t stream);

/* Network inputs of `batch` frames: input[b] = the block means of (rgb[b] - tgt_rgb[b],
 * depth[b] - tgt_depth[b]).  Images are planar, frame after frame: rgb [batch][3][H][W],
 * depth [batch][H][W]; input is FP32 [batch][4][60][80].  width must be a multiple
 * of 80 and height of 60 with the same factor (the block side). */
GS2D_API int gs2d_ws_residual(const float* rgb, const float* depth, const float* tgt_rgb,
                              const float* tgt_depth, int32_t width, int32_t height, int32_t batch,
                              float* input, hipStream_t stream);

/* Forward pass: out (device FP32 [batch][6]) = the normalised twist for input
 * (device FP32 [batch][4][60][80]; rounded to BF16 on entry). */
GS2D_API int gs2d_ws_forward(gs2d_ws* net, const float* input, int32_t batch, float* out,
                             hipStream_t stream);

/* Forward and backward of the mean squared error between the output and `target`
 * (device FP32 [batch][6], normalised twists) over batch x 6 values.  loss (device
 * FP32 scalar) and out (device [batch][6]) may be NULL; grad (device FP32
 * [GS2D_WS_PARAMS], NULL: kept only inside the network for gs2d_ws_adamw_step)
 * receives dL/dtheta in the flat parameter layout. */
GS2D_API int gs2d_ws_gradient(gs2d_ws* net, const float* input, const float* target, int32_t batch,
                              float* loss, float* out, float* grad, hipStream_t stream);

/* One AdamW step of the master parameters with the gradient of the last
 * gs2d_ws_gradient call (bias-corrected moments), then the BF16 copies. */
GS2D_API int gs2d_ws_adamw_step(gs2d_ws* net, const gs2d_ws_adamw* opt, hipStream_t stream);

/* Warm start of one tracking problem: render at pose_start (device [12], world to
 * camera [R|t]), form the residual against (tgt_rgb [3][H][W], tgt_depth [H][W]),
 * run the network, T_0 = Exp(tau_hat) T_start, render at T_0 and keep T_0 only if
 * its tracking loss (lambda_d, use_masks as gs2d_tracking_loss) is not larger than
 * at T_start.  Pass use_masks = 0: the masked loss of a pose that sees nothing is 0
 * (the opacity mask drops every pixel), so only the unmasked loss can reject it.
 * pose_out (device [12]) receives the chosen pose; info (device FP32 [4], nullable)
 * = {loss at T_start, loss at T_0, 1 if T_0 was kept else 0, 0}.  Image workspace
 * for one frame belongs to the network object; the renders may synchronise `stream`
 * as gs2d_render does when the context's pair buffers must grow. */
GS2D_API int gs2d_warm_start(gs2d_ctx* ctx, gs2d_ws* net, const float* params, int64_t n,
                             const gs2d_camera* camera, const float* pose_start, const float* tgt_rgb,
                             const float* tgt_depth, float lambda_d, int32_t use_masks, float* pose_out,
                             float* info, hipStream_t stream);

/* The proposal half of gs2d_warm_start, for tracking that makes the fallback decision
 * itself: render at pose_start, the residual, the network, and pose_out (device [12]) =
 * T_0 = Exp(tau_hat) T_start; start_loss (device FP32 [1]) receives the unmasked
 * tracking loss at T_start (lambda_d).  Pass (pose_start, start_loss) as the tracking
 * problem's fallback (gs2d_track_problem.fallback_pose, .fallback_loss) and pose_out as
 * its start pose: the first tracking iteration, which renders at T_0 anyway, rejects
 * T_0 if its unmasked loss is larger, so no render at T_0 is spent here. */
GS2D_API int gs2d_warm_start_propose(gs2d_ctx* ctx, gs2d_ws* net, const float* params, int64_t n,
                                     const gs2d_camera* camera, const float* pose_start, const float* tgt_rgb,
                                     const float* tgt_depth, float lambda_d, float* pose_out, float* start_loss,
                                     hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GS2D_WARM_H */
