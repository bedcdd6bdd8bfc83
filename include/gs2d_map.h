/* Map bookkeeping around the rasterizer: covisibility and keyframe selection,
 * contribution pruning with stable compaction, the per-splat map state, and map
 * correction after pose-graph optimisation.
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

#ifdef __cplusplus
}
#endif

#endif /* GS2D_MAP_H */
