"""GPU: the normalised and median depth (gs2d_view.depth_norm, .depth_median) and the
relocalisation error e_t (gs2d_tracking_error) against the oracle.

Depths take the depth bar, |d| <= 1e-4 max(|ref|, 1e-3); pixels within the oracle's
decision margin (its render decisions and the median's T > 1/2) are excluded and
counted.  e_t is compared on the oracle's renders rounded to float32.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import loss as oloss
from tests.gpu_common import MARGIN, MAX_EXCLUDED, ROOM_CAM, dev, host, room_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def r():
    from paper_2506_00970_amd import Rasterizer

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return Rasterizer()


def _render(r, params, cam, pose, **kw):
    out = r.render_batch([(dev(params), cam, dev(np.asarray(pose).reshape(12)))], **kw)[0]
    torch.cuda.synchronize()
    return out


def _check_depth(name, got, ref, keep):
    tol = 1e-4 * np.maximum(np.abs(ref), 1e-3)
    err = np.abs(got - ref)
    bad = (err > tol) & keep
    print(f"{name}: worst err/tol {float((err / tol)[keep].max()):.3g}")
    assert not bad.any(), f"{name}: {int(bad.sum())} pixels out of tolerance, worst {err[bad].max():.3g}"


@pytest.mark.parametrize("scene", ["random", "room"])
def test_depth_variants_match_oracle(r, scene):
    if scene == "random":
        s = synth.random_surfels(2000, seed=5)
        params, cam, pose = s.params, s.camera, s.pose
    else:
        room, pose = room_scene(300_000, seed=5, cam_seed=5)
        params, cam = room.params, ROOM_CAM
    out = _render(r, params, cam, pose, depth_variants=True)
    ref = oracle.depth_variants(params, cam, pose)
    keep = ref["margin"] >= MARGIN
    frac = 1.0 - keep.mean()
    print(scene, f"excluded {frac:.4%}")
    assert frac <= MAX_EXCLUDED
    _check_depth("depth_norm", host(out.depth_norm), ref["depth_norm"], keep)
    _check_depth("depth_median", host(out.depth_median), ref["depth_median"], keep)
    # where nothing is composited both are exactly 0
    empty = host(out.alpha) == 0
    assert np.all(host(out.depth_norm)[empty] == 0) and np.all(host(out.depth_median)[empty] == 0)
    # asking for the variants changes nothing else
    plain = _render(r, params, cam, pose)
    for k in ("rgb", "depth", "normal", "alpha"):
        assert torch.equal(getattr(out, k), getattr(plain, k)), k


@pytest.mark.parametrize("obliquity", [0.0, 45.0])
def test_depth_variants_on_planar_carpet(r, obliquity):
    """Coplanar surfels: D/O and the median are the exact ray-plane depth wherever O > 0."""
    s = synth.planar_carpet(obliquity, azimuth_deg=15.0)
    out = _render(r, s.params, s.camera, s.pose, depth_variants=True)
    p = s.params.astype(np.float64)
    T = s.pose.astype(np.float64)
    R, t = T[:, :3], T[:, 3]
    n_c = np.cross(R @ p[3:6, 0], R @ p[6:9, 0])
    h_c = n_c @ (R @ p[0:3, 0] + t)
    cam = s.camera
    ys, xs = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    ray = np.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, np.ones_like(xs, dtype=float)])
    d = h_c / np.einsum("c,chw->hw", n_c, ray)
    m = host(out.alpha) > 1e-6
    assert m.sum() > 1000
    _check_depth("depth_norm", host(out.depth_norm), d, m)
    _check_depth("depth_median", host(out.depth_median), d, m)


@pytest.mark.parametrize("opacity,index", [(0.3, 1), (0.1, 6), (0.7, 0)])
def test_median_of_stacked_surfels(r, opacity, index):
    s = synth.stacked_surfels(count=20, opacity=opacity, z0=2.0, dz=0.1)
    out = _render(r, s.params, s.camera, s.pose, depth_variants=True)
    assert host(out.depth_median)[24, 32] == pytest.approx(float(s.params[2, index]), rel=1e-6)


@pytest.mark.parametrize("scene", ["random", "room"])
def test_tracking_error_matches_oracle(r, scene):
    if scene == "random":
        s, t = synth.random_surfels(2000, seed=6), synth.random_surfels(2000, seed=7)
        img = oracle.render(s.params, s.camera, s.pose)
        tgt = oracle.render(t.params, t.camera, t.pose)
        cam = s.camera
    else:
        room, pose = room_scene(300_000, seed=6, cam_seed=6)
        start = synth.perturb_pose(pose, 0.05, 3.0, seed=7)
        img = oracle.render(room.params, ROOM_CAM, start)
        tgt = oracle.render(room.params, ROOM_CAM, pose)
        cam = ROOM_CAM
    f = {k: np.asarray(img[k], dtype=np.float32) for k in ("depth", "normal", "alpha")}
    td = np.asarray(tgt["depth"], dtype=np.float32)
    e = float(r.tracking_error(cam, dev(f["depth"]), dev(f["normal"]), dev(f["alpha"]), dev(td)))
    want = oloss.tracking_error(f["depth"], f["normal"], f["alpha"], td, cam)
    print(scene, "e_t", e, want)
    assert e == pytest.approx(want, rel=1e-5)
    assert want > 0
