"""Map bookkeeping around the rasterizer: visibility, covisibility and keyframe
selection, pruning, the per-splat map state, and map correction.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing in the product path.
Plain NumPy definitions in float64 (counts are integers), each following the passage
it cites:

* visibility (Sec. "Tracking and Keyframe Selection", eq:contribution): a splat is
  visible from view V when its contribution C_k^V exceeds 0.5;
* covisibility of two views: |G_A & G_B| / |G_A | G_B| over the visible sets;
* keyframe selection: a new keyframe when the covisibility with the last keyframe is
  below c_k = 0.9, or when the translation vectors of the two world-to-camera poses
  are more than d_k = 15 cm apart;
* pruning (Sec. "Mapping"): splats associated with a sampled keyframe r (closest
  frame t^c = r) whose contribution from r falls below 0.5 are removed;
* map state (Sec. "Mapping", eq:map): for keyframe n, active splats that are visible
  get t^l = n, and t^c = n with d^c the new distance when their distance to the
  keyframe's camera centre is below d^c; active splats not seen for more than a set
  number of keyframes become inactive; within the keyframes after a loop with
  keyframe h, an inactive splat that is visible and has t^c > h becomes active again
  with t^l = n;
* map correction (Sec. "Map Correction"): each splat moves with the pose increment
  Delta T = T^o T^-1 of its closest keyframe, mu' = Delta T mu and R' = Delta R R (here
  the tangent vectors t_u, t_v, the columns of R that span the splat).
"""

from __future__ import annotations

import numpy as np

VISIBLE = 0.5       # eq:contribution: visible when C > 0.5
COVIS_KF = 0.9      # c_k
DIST_KF = 0.15      # d_k (metres)
PRUNE = 0.5         # removed when the contribution falls below 0.5


def visible(contrib, threshold: float = VISIBLE):
    return np.asarray(contrib) > threshold


def covisibility_counts(contrib_a, contrib_b, threshold: float = VISIBLE):
    """(|G_A & G_B|, |G_A | G_B|) as integers."""
    a, b = visible(contrib_a, threshold), visible(contrib_b, threshold)
    return int(np.count_nonzero(a & b)), int(np.count_nonzero(a | b))


def covisibility(contrib_a, contrib_b, threshold: float = VISIBLE) -> float:
    """S_cov(A, B); 0 when neither view sees a splat (no overlap to speak of)."""
    inter, union = covisibility_counts(contrib_a, contrib_b, threshold)
    return inter / union if union else 0.0


def is_keyframe(score: float, pose_cur, pose_kf, c_k: float = COVIS_KF, d_k: float = DIST_KF) -> bool:
    """Poses are world-to-camera [R|t] (3x4); the distance is between their t."""
    t_cur = np.asarray(pose_cur, dtype=np.float64).reshape(3, 4)[:, 3]
    t_kf = np.asarray(pose_kf, dtype=np.float64).reshape(3, 4)[:, 3]
    return bool(score < c_k or np.linalg.norm(t_cur - t_kf) > d_k)


def prune_mask(contrib, closest_frame, frame: int, threshold: float = PRUNE):
    """True for splats to remove: associated with `frame` and contributing < 0.5."""
    return (np.asarray(closest_frame) == frame) & (np.asarray(contrib) < threshold)


def compact(planes, keep):
    """The kept columns of each [k, n] plane, in their order."""
    keep = np.asarray(keep, dtype=bool)
    return [np.asarray(p)[..., keep] for p in planes]


def camera_centre(pose_cw):
    """World position of the camera of a world-to-camera pose: -R^T t."""
    T = np.asarray(pose_cw, dtype=np.float64).reshape(3, 4)
    return -T[:, :3].T @ T[:, 3]


def state_update(params, contrib, pose_kf, n: int, t_closest, d_closest, t_last, active, inactive_after: int,
                 loop_frame: int | None = None):
    """Map state after keyframe n; returns new (t_closest, d_closest, t_last, active).

    Order: reactivation (within the keyframes after a loop with keyframe `loop_frame`),
    then the visible active splats' last and closest frames, then deactivation.
    """
    t_c = np.array(t_closest, dtype=np.int64)
    d_c = np.array(d_closest, dtype=np.float64)
    t_l = np.array(t_last, dtype=np.int64)
    act = np.array(active, dtype=bool)
    vis = visible(contrib)
    if loop_frame is not None:
        back = ~act & vis & (t_c > loop_frame)
        act[back] = True
        t_l[back] = n
    seen = act & vis
    t_l[seen] = n
    mu = np.asarray(params, dtype=np.float64)[0:3]
    dist = np.linalg.norm(mu - camera_centre(pose_kf)[:, None], axis=0)
    closer = seen & (dist < d_c)
    d_c[closer] = dist[closer]
    t_c[closer] = n
    act[act & (n - t_l > inactive_after)] = False
    return t_c, d_c, t_l, act


def correct(params, closest_frame, delta_T):
    """mu' = dR mu + dt and t_u' = dR t_u, t_v' = dR t_v with the increment of each
    splat's closest keyframe (delta_T [K, 3, 4]); splats whose closest frame is outside
    0..K-1 are left as they are."""
    p = np.array(params, dtype=np.float64, copy=True)
    D = np.asarray(delta_T, dtype=np.float64).reshape(-1, 3, 4)
    f = np.asarray(closest_frame, dtype=np.int64)
    ok = (f >= 0) & (f < D.shape[0])
    R, t = D[f[ok], :, :3], D[f[ok], :, 3]
    for rows in (slice(0, 3), slice(3, 6), slice(6, 9)):
        v = p[rows][:, ok].T
        v2 = np.einsum("kij,kj->ki", R, v)
        if rows.start == 0:
            v2 = v2 + t
        p[rows][:, ok] = v2.T
    return p
