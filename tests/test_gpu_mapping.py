"""GPU: per-surfel contribution and the map bookkeeping (include/gs2d_map.h) against
the oracle (oracle.contribution, oracle/mapping.py).

Contributions come from the forward render and are compared with the FP64 oracle's,
excluding surfels seen at pixels within a decision margin (their composited sets may
differ in float32).  The bookkeeping kernels get seeded synthetic inputs and must give
the oracle's integers and flags exactly, and its distances and corrected parameters to
float32 rounding.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import mapping as om
from tests.gpu_common import ROOM_CAM, dev, host, room_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_00970_amd as p
    from paper_2506_00970_amd import mapstate

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return p, mapstate


def _contrib(r, params, cam, pose):
    outs = r.render_batch([(dev(params), cam, dev(np.asarray(pose).reshape(12)))], contribution=True)
    torch.cuda.synchronize()
    return host(outs[0].contrib), host(outs[0].alpha)


@pytest.mark.parametrize("scene", ["random", "room"])
def test_contribution_matches_oracle(pkg, scene):
    p, _ = pkg
    r = p.Rasterizer()
    if scene == "random":
        s = synth.random_surfels(2000, seed=4)
        params, cam, pose = s.params, s.camera, s.pose
    else:
        room, pose = room_scene(300_000, seed=2, cam_seed=2)
        params, cam = room.params, ROOM_CAM
    c, alpha = _contrib(r, params, cam, pose)
    ref = oracle.contribution(params, cam, pose)
    keep = ~ref["touched"]
    print(scene, "surfels", len(c), "excluded", int((~keep).sum()), "visible", int((ref["contrib"] > 0.5).sum()))
    err = np.abs(c - ref["contrib"])
    tol = 1e-4 * np.maximum(ref["contrib"], 1.0)
    assert np.all(err[keep] <= tol[keep]), float((err[keep] / tol[keep]).max())
    # the GPU's own sum: sum_k C_k = sum_p O(p) (float32 sums of the same weights)
    assert abs(c.sum() - alpha.sum()) <= 1e-4 * alpha.sum()
    # visibility agrees wherever the oracle's contribution is not within the bar of 0.5
    clear = keep & (np.abs(ref["contrib"] - 0.5) > 1e-4)
    np.testing.assert_array_equal(c[clear] > 0.5, ref["contrib"][clear] > 0.5)


def test_contribution_batch_equals_single(pkg):
    """Batched views give each view's contributions as rendered alone."""
    p, _ = pkg
    room, pose0 = room_scene(300_000, seed=3, cam_seed=3)
    pose1 = synth.room_camera(room, seed=9)
    r = p.Rasterizer()
    P = dev(room.params)
    outs = r.render_batch([(P, ROOM_CAM, dev(pose0.reshape(12))), (P, ROOM_CAM, dev(pose1.reshape(12)))],
                          contribution=True)
    torch.cuda.synchronize()
    for k, ps in enumerate((pose0, pose1)):
        one = r.render_batch([(P, ROOM_CAM, dev(ps.reshape(12)))], contribution=True)[0]
        torch.cuda.synchronize()
        np.testing.assert_allclose(host(outs[k].contrib), host(one.contrib), rtol=1e-5, atol=1e-6)


def test_covisibility_and_keyframe(pkg):
    _, ms = pkg
    g = np.random.default_rng(5)
    for n in (0, 1, 3, 1000, 1_000_003, 4_194_306):
        ca = g.uniform(0, 1, n).astype(np.float32)
        cb = g.uniform(0, 1, n).astype(np.float32)
        if n > 2:
            ca[:2] = 0.5  # the threshold is strict
            cb[:2] = np.float32(0.5000001)
        cnt = ms.covisibility_counts(dev(ca), dev(cb))
        torch.cuda.synchronize()
        got = tuple(int(v) for v in cnt.cpu().numpy().view(np.uint32))
        assert got == om.covisibility_counts(ca, cb), n
        if n > 1:  # arrays that do not start on a 16-byte boundary take the scalar loads
            cnt = ms.covisibility_counts(dev(ca)[1:], dev(cb)[1:])
            got = tuple(int(v) for v in cnt.cpu().numpy().view(np.uint32))
            assert got == om.covisibility_counts(ca[1:], cb[1:]), n
    I = np.hstack([np.eye(3), np.zeros((3, 1))]).astype(np.float32)
    cases = [((90, 100), [0.1, 0.0, 0.05]), ((89, 100), [0.1, 0.0, 0.05]), ((95, 100), [0.12, 0.1, 0.05]),
             ((95, 100), [0.1, 0.1, 0.0]), ((0, 0), [0.0, 0.0, 0.0]), ((9, 10), [0.0, 0.0, 0.0])]
    for (i, u), t in cases:
        cur = I.copy()
        cur[:, 3] = t
        counts = torch.tensor([i, u], dtype=torch.int32, device="cuda:0")
        k = int(ms.keyframe_test(counts, dev(cur.reshape(12)), dev(I.reshape(12))).item())
        score = i / u if u else 0.0
        assert k == int(om.is_keyframe(score, cur.astype(np.float64), I.astype(np.float64))), ((i, u), t)


def test_prune_and_compact(pkg):
    _, ms = pkg
    g = np.random.default_rng(6)
    for n in (0, 5, 1023, 4096, 1_000_001):
        contrib = g.uniform(0, 1, n).astype(np.float32)
        closest = g.integers(0, 4, n).astype(np.int32)
        rm = ms.prune_mask(dev(contrib), torch.from_numpy(closest).cuda(), 2)
        torch.cuda.synchronize()
        ref = om.prune_mask(contrib, closest, 2)
        np.testing.assert_array_equal(rm.cpu().numpy().astype(bool), ref)
        if n > 1:  # unaligned: scalar path
            rm1 = ms.prune_mask(dev(contrib)[1:], torch.from_numpy(closest).cuda()[1:], 2)
            np.testing.assert_array_equal(rm1.cpu().numpy().astype(bool), ref[1:])
        planes = g.standard_normal((15, n)).astype(np.float32)
        out, n_out = ms.compact(dev(planes), rm)
        torch.cuda.synchronize()
        kept = int(n_out.item())
        (want,) = om.compact([planes], ~ref)
        assert kept == want.shape[1]
        np.testing.assert_array_equal(out.cpu().numpy()[:, :kept], want)
    # no mask keeps everything; a full mask keeps nothing
    planes = g.standard_normal((3, 3000)).astype(np.float32)
    out, n_out = ms.compact(dev(planes), None)
    assert int(n_out.item()) == 3000
    np.testing.assert_array_equal(out.cpu().numpy(), planes)
    _, n_out = ms.compact(dev(planes), torch.ones(3000, dtype=torch.uint8, device="cuda:0"))
    assert int(n_out.item()) == 0


@pytest.mark.parametrize("loop", [None, 40])
def test_state_update(pkg, loop):
    _, ms = pkg
    g = np.random.default_rng(7)
    n = 1_000_000
    params = np.zeros((15, n), dtype=np.float32)
    params[0:3] = g.uniform(-3, 3, (3, n))
    contrib = g.uniform(0, 1, n).astype(np.float32)
    pose = synth.look_at_pose([1.0, -0.5, 0.3], [0.0, 0.0, 0.0]).astype(np.float32)
    t_c = g.integers(0, 60, n).astype(np.int32)
    d_c = g.uniform(0, 6, n).astype(np.float32)
    t_l = g.integers(0, 60, n).astype(np.int32)
    act = (g.random(n) < 0.7).astype(np.int32)
    st = ms.MapState(n, "cuda:0")
    st.t_closest.copy_(torch.from_numpy(t_c))
    st.d_closest.copy_(torch.from_numpy(d_c))
    st.t_last.copy_(torch.from_numpy(t_l))
    st.active.copy_(torch.from_numpy(act))
    st.update(dev(params), dev(contrib), dev(pose.reshape(12)), 60, inactive_after=10, loop_frame=loop)
    torch.cuda.synchronize()
    tc, dc, tl, a = om.state_update(params, contrib, pose, 60, t_c, d_c, t_l, act.astype(bool), 10, loop)
    np.testing.assert_array_equal(st.t_closest.cpu().numpy(), tc)
    np.testing.assert_array_equal(st.t_last.cpu().numpy(), tl)
    np.testing.assert_array_equal(st.active.cpu().numpy().astype(bool), a)
    np.testing.assert_allclose(st.d_closest.cpu().numpy(), dc, rtol=1e-7)
    print("updated closest", int((tc == 60).sum()), "deactivated", int((act.astype(bool) & ~a).sum()))


def test_correction(pkg):
    _, ms = pkg
    g = np.random.default_rng(8)
    n = 500_000
    s = synth.random_surfels(n, seed=11)
    closest = g.integers(-1, 12, n).astype(np.int32)  # -1 and 10, 11: no increment
    from oracle import se3

    D = np.stack([se3.exp(g.normal(size=6) * 0.2)[:3] for _ in range(10)]).astype(np.float32)
    P = dev(s.params)
    ms.correct(P, torch.from_numpy(closest).cuda(), dev(D))
    torch.cuda.synchronize()
    ref = om.correct(s.params, closest, D)
    got = host(P)
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-6 * max(1.0, float(np.abs(ref).max())))
    untouched = (closest < 0) | (closest >= 10)
    np.testing.assert_array_equal(got[:, untouched], s.params[:, untouched].astype(np.float64))
