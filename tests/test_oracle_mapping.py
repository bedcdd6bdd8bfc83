"""CPU pins of the oracle's contribution and map bookkeeping (oracle/mapping.py).

Each pin checks the oracle against something other than itself: the rendered opacity
image (a different accumulation of the same weights), a two-surfel closed form,
Python set algebra, and hand-worked cases.
"""

import numpy as np

import oracle
import synth
from oracle import mapping as om


def test_contribution_sums_to_rendered_opacity():
    """sum_k C_k = sum_p sum_k w_k(p) = sum_p O(p) (eq:contribution against eq:alpha_blending)."""
    for seed in (0, 3):
        s = synth.random_surfels(2000, seed=seed)
        c = oracle.contribution(s.params, s.camera, s.pose)["contrib"]
        o = oracle.render(s.params, s.camera, s.pose)["alpha"]
        assert abs(c.sum() - o.sum()) <= 1e-9 * max(1.0, o.sum())
        assert np.all(c >= 0.0)


def test_contribution_of_a_surfel_behind_its_twin():
    """Two identical surfels: the first (by index at equal depth) has weight alpha(p), the
    second alpha(p) (1 - alpha(p)), where alpha is the single surfel's opacity image."""
    s = synth.single_surfel(scale=0.1)
    one = oracle.render(s.params, s.camera, s.pose)["alpha"]
    twin = np.concatenate([s.params, s.params], axis=1)
    c = oracle.contribution(twin, s.camera, s.pose)["contrib"]
    assert np.isclose(c[0], one.sum(), rtol=1e-12)
    assert np.isclose(c[1], (one * (1.0 - one)).sum(), rtol=1e-12)


def test_covisibility_against_sets():
    g = np.random.default_rng(0)
    ca, cb = g.uniform(0, 1, 5000), g.uniform(0, 1, 5000)
    A = {i for i in range(5000) if ca[i] > 0.5}
    B = {i for i in range(5000) if cb[i] > 0.5}
    assert om.covisibility_counts(ca, cb) == (len(A & B), len(A | B))
    assert om.covisibility(ca, cb) == len(A & B) / len(A | B)
    # the threshold is strict, and no visible splat gives 0
    assert om.covisibility_counts([0.5, 0.6], [0.5, 0.4]) == (0, 1)
    assert om.covisibility([0.1, 0.2], [0.3, 0.5]) == 0.0


def test_keyframe_rule():
    I = np.hstack([np.eye(3), np.zeros((3, 1))])
    near = I.copy()
    near[:, 3] = [0.1, 0.0, 0.05]  # 11.2 cm
    far = I.copy()
    far[:, 3] = [0.12, 0.1, 0.05]  # 16.4 cm
    assert not om.is_keyframe(0.95, near, I)
    assert om.is_keyframe(0.85, near, I)       # covisibility below 0.9
    assert om.is_keyframe(0.95, far, I)        # more than 15 cm
    far[:, 3] = [0.1, 0.1, 0.0]
    assert not om.is_keyframe(0.95, far, I)    # 14.1 cm


def test_prune_mask_and_compaction():
    contrib = np.array([0.2, 0.7, 0.4, 0.49, 0.9])
    closest = np.array([3, 3, 2, 3, 3])
    rm = om.prune_mask(contrib, closest, 3)
    np.testing.assert_array_equal(rm, [True, False, False, True, False])
    planes = [np.arange(15 * 5, dtype=np.float64).reshape(15, 5), np.array([10, 11, 12, 13, 14])]
    kept = om.compact(planes, ~rm)
    np.testing.assert_array_equal(kept[0], planes[0][:, [1, 2, 4]])
    np.testing.assert_array_equal(kept[1], [11, 12, 14])


def test_state_update_worked_example():
    """Keyframe n = 10 at the world origin looking down +z (identity pose)."""
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    mu = np.array([[0, 0, 1.0], [0, 0, 2.0], [0, 0, 3.0], [0, 0, 0.5], [0, 0, 4.0]]).T
    params = np.zeros((15, 5))
    params[0:3] = mu
    contrib = np.array([0.9, 0.9, 0.1, 0.8, 0.7])
    t_c = np.array([2, 4, 4, 1, 8])
    d_c = np.array([0.5, 3.0, 1.0, 1.0, 9.0])
    t_l = np.array([9, 9, 1, 3, 9])
    act = np.array([True, True, True, False, False])
    # splat 0: visible, but 1.0 m is not closer than 0.5 m: t_l = 10 only
    # splat 1: visible and 2.0 < 3.0: closest -> (10, 2.0)
    # splat 2: not visible; last seen 9 keyframes ago > 5: inactive
    # splat 3: inactive, visible, t_c = 1 is not after the loop keyframe 6: stays inactive
    # splat 4: inactive, visible, t_c = 8 > 6: active again, then seen from 4.0 m < 9.0
    tc, dc, tl, a = om.state_update(params, contrib, pose, 10, t_c, d_c, t_l, act, inactive_after=5, loop_frame=6)
    np.testing.assert_array_equal(tc, [2, 10, 4, 1, 10])
    np.testing.assert_allclose(dc, [0.5, 2.0, 1.0, 1.0, 4.0])
    np.testing.assert_array_equal(tl, [10, 10, 1, 3, 10])
    np.testing.assert_array_equal(a, [True, True, False, False, True])


def test_camera_centre():
    R = synth.look_at_pose([1.0, 2.0, 3.0], [0.0, 0.0, 0.0])
    np.testing.assert_allclose(om.camera_centre(R), [1.0, 2.0, 3.0], atol=1e-12)


def test_correction_is_rigid_per_keyframe():
    g = np.random.default_rng(1)
    s = synth.random_surfels(200, seed=2)
    closest = g.integers(0, 3, 200)
    closest[:5] = 7  # no increment for frame 7: unchanged
    from oracle import se3

    D = np.stack([se3.exp(g.normal(size=6) * 0.1)[:3] for _ in range(3)])
    p2 = om.correct(s.params, closest, D)
    np.testing.assert_array_equal(p2[:, :5], s.params[:, :5].astype(np.float64))
    np.testing.assert_array_equal(p2[9:], s.params[9:].astype(np.float64))  # scales, opacity, colour
    for k in range(3):
        m = closest == k
        a, b = s.params[0:3, m].astype(np.float64), p2[0:3, m]
        da = np.linalg.norm(a[:, :, None] - a[:, None, :], axis=0)
        db = np.linalg.norm(b[:, :, None] - b[:, None, :], axis=0)
        np.testing.assert_allclose(db, da, atol=1e-12)
        q = s.params.astype(np.float64)
        np.testing.assert_allclose(np.sum(p2[3:6, m] * p2[6:9, m], axis=0),
                                   np.sum(q[3:6, m] * q[6:9, m], axis=0), atol=1e-12)
    # applying the inverse increments restores the map
    Dinv = np.stack([np.hstack([d[:, :3].T, -(d[:, :3].T @ d[:, 3])[:, None]]) for d in D])
    np.testing.assert_allclose(om.correct(p2, closest, Dinv), s.params.astype(np.float64), atol=1e-12)
    # a worked case: 90 deg about z, then 1 m along x
    Dz = np.array([[[0.0, -1.0, 0.0, 1.0], [1.0, 0.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]]])
    q = np.zeros((15, 1))
    q[0:3, 0] = [1.0, 0.0, 2.0]
    q[3:6, 0] = [1.0, 0.0, 0.0]
    q[6:9, 0] = [0.0, 1.0, 0.0]
    q2 = om.correct(q, [0], Dz)
    np.testing.assert_allclose(q2[0:9, 0], [1.0, 1.0, 2.0, 0.0, 1.0, 0.0, -1.0, 0.0, 0.0], atol=1e-15)
