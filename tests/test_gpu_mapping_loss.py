"""GPU: the mapping loss (gs2d_mapping_loss) against the oracle (oracle/mapping_loss.py).

Inputs are the oracle's renders rounded to float32 (the kernel's input precision), and
the oracle evaluates the same float32 images in float64.  Tolerances: the loss terms
to 1e-5 relative; image gradients to the gradient bar, |d| <= 1e-3 |ref| + 1e-5 max|ref|
per image.  The depth normals are a normalised cross product of neighbour differences:
where the two differences are nearly parallel (condition |dx| |dy| / |dx x dy| above
1e3, at depth edges seen edge-on) float32 cannot carry them to the bar, and those pixels
(and, for d_depth, their four neighbours) are excluded and counted.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import mapping_loss as oml
from tests.gpu_common import ROOM_CAM, dev, host, room_scene

pytestmark = pytest.mark.gpu

COND_MAX = 1e3


@pytest.fixture(scope="module")
def ml():
    from paper_2506_00970_amd import maploss

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return maploss


def _f32(d):
    return {k: np.asarray(v, dtype=np.float32) for k, v in d.items()}


def _condition(depth, cam):
    """|dx| |dy| / |dx x dy| of the depth normals per pixel (inf where the cross vanishes,
    0 on the border), in float64 from the float32 depth."""
    W, H, fx, fy, cx, cy = cam.as_tuple()
    D = depth.astype(np.float64)
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    X = np.stack([D * (xs - cx) / fx, D * (ys - cy) / fy, D])
    k = np.zeros((H, W))
    if H >= 3 and W >= 3:
        dx = X[:, 1:-1, 2:] - X[:, 1:-1, :-2]
        dy = X[:, 2:, 1:-1] - X[:, :-2, 1:-1]
        c = np.linalg.norm(np.cross(dx, dy, axis=0), axis=0)
        with np.errstate(divide="ignore", invalid="ignore"):
            k[1:-1, 1:-1] = np.where(c > 0, np.linalg.norm(dx, axis=0) * np.linalg.norm(dy, axis=0) / c, 0.0)
    return k


def _check(name, got, ref, skip=None, rel=1e-3, floor=1e-5):
    assert np.all(np.isfinite(got)) and np.all(np.isfinite(ref)), name
    err = np.abs(got - ref)
    tol = rel * np.abs(ref) + floor * max(np.abs(ref).max(), 1e-30)
    bad = err > tol
    if skip is not None:
        bad &= ~np.broadcast_to(skip, bad.shape)
    worst = float((err / tol)[~np.broadcast_to(skip, err.shape)].max()) if skip is not None else float((err / tol).max())
    print(f"{name}: worst err/tol {worst:.3g}")
    assert not bad.any(), f"{name}: {int(bad.sum())} values out of tolerance, worst {err[bad].max():.3g}"


def _compare(ml, img, tgt, cam, max_excluded=0.02):
    g = {k: dev(v) for k, v in img.items()}
    loss, d_rgb, d_depth, d_normal = ml.mapping_loss(g["rgb"], g["depth"], g["normal"], dev(tgt["rgb"]),
                                                     dev(tgt["depth"]), cam)
    torch.cuda.synchronize()
    ref = oml.mapping_loss(img["rgb"], img["depth"], img["normal"], tgt["rgb"], tgt["depth"], cam)
    got = host(loss)
    want = np.array([ref["loss"], *ref["terms"]])
    print("loss", got, "oracle", want)
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-7)
    bad_n = _condition(img["depth"], cam) > COND_MAX
    near = bad_n.copy()
    near[:, 1:] |= bad_n[:, :-1]
    near[:, :-1] |= bad_n[:, 1:]
    near[1:, :] |= bad_n[:-1, :]
    near[:-1, :] |= bad_n[1:, :]
    frac = near.mean()
    print(f"ill-conditioned depth normals: {int(bad_n.sum())} pixels, {frac:.4%} excluded from d_depth")
    assert frac <= max_excluded
    _check("d_rgb", host(d_rgb), ref["d_rgb"])
    _check("d_normal", host(d_normal), ref["d_normal"], skip=bad_n[None])
    _check("d_depth", host(d_depth), ref["d_depth"], skip=near)
    return loss, d_rgb, d_depth, d_normal


@pytest.mark.parametrize("scene", ["random", "room"])
def test_mapping_loss_matches_oracle(ml, scene):
    if scene == "random":
        s, t = synth.random_surfels(2000, seed=0), synth.random_surfels(2000, seed=1)
        cam = s.camera
        img = _f32(oracle.render(s.params, cam, s.pose))
        tgt = _f32(oracle.render(t.params, cam, t.pose))
    else:
        room, pose = room_scene(300_000, seed=4, cam_seed=4)
        start = synth.perturb_pose(pose, 0.05, 3.0, seed=6)
        cam = ROOM_CAM
        img = _f32(oracle.render(room.params, cam, start))
        tgt = _f32(oracle.render(room.params, cam, pose))
    img = {k: img[k] for k in ("rgb", "depth", "normal")}
    out = _compare(ml, img, tgt, cam)
    # deterministic: fixed-order sums, no atomics
    again = ml.mapping_loss(*(dev(img[k]) for k in ("rgb", "depth", "normal")), dev(tgt["rgb"]), dev(tgt["depth"]),
                            cam)
    for a, b in zip(out, again):
        assert torch.equal(a, b)


@pytest.mark.parametrize("hw", [(1, 1), (2, 5), (17, 3), (33, 18), (16, 16), (47, 61)])
def test_mapping_loss_sizes(ml, hw):
    """Ragged tiles and images too small for any interior depth normal."""
    H, W = hw
    g = np.random.default_rng(H * 100 + W)
    cam = synth.Camera(W, H, 0.9 * W + 5, 0.9 * W + 5, (W - 1) / 2 + 0.3, (H - 1) / 2 - 0.2)
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    img = {"rgb": g.random((3, H, W)).astype(np.float32),
           "depth": (2.0 + 0.01 * xs - 0.02 * ys + 0.05 * g.random((H, W))).astype(np.float32),
           "normal": g.standard_normal((3, H, W)).astype(np.float32)}
    tgt = {"rgb": g.random((3, H, W)).astype(np.float32),
           "depth": (img["depth"] + 0.1 * g.standard_normal((H, W))).astype(np.float32)}
    _compare(ml, img, tgt, cam)


def test_mapping_loss_of_identical_images(ml):
    """Rendered = observed and N = N_D: only the border's normal term remains."""
    H, W = 40, 50
    cam = synth.Camera(W, H, 45.0, 45.0, 24.5, 19.5)
    n = np.array([0.2, -0.1, 1.0])
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    r = np.stack([(xs - 24.5) / 45.0, (ys - 19.5) / 45.0, np.ones_like(xs)])
    D = (2.0 / np.tensordot(n, r, axes=1)).astype(np.float32)
    rgb = np.random.default_rng(7).random((3, H, W)).astype(np.float32)
    N = oml.depth_normals(torch.tensor(D.astype(np.float64)), cam).numpy().astype(np.float32)
    loss, _, _, _ = ml.mapping_loss(dev(rgb), dev(D), dev(N), dev(rgb), dev(D), cam)
    got = host(loss)
    border = (H * W - (H - 2) * (W - 2)) / (H * W)
    assert got[1] == 0.0 and got[3] == 0.0
    assert abs(got[2]) < 1e-6
    assert got[4] == pytest.approx(border, abs=1e-5)
    assert got[0] == pytest.approx(0.02 * border, abs=1e-6)


def test_mapping_gradient_end_to_end(ml):
    """Render, mapping loss and the full backward on the GPU against the oracle's chain
    (its own render, its own mapping loss, its backward) on the single-frame scene."""
    from paper_2506_00970_amd import Rasterizer
    from tests.gpu_common import check_grads, check_pose

    s, t = synth.random_surfels(2000, seed=2), synth.random_surfels(2000, seed=3)
    cam = s.camera
    tgt = _f32(oracle.render(t.params, cam, t.pose))
    r = Rasterizer()
    out = r.render(dev(s.params), cam, dev(s.pose.reshape(12)))
    _, d_rgb, d_depth, d_normal = ml.mapping_loss(out.rgb, out.depth, out.normal, dev(tgt["rgb"]), dev(tgt["depth"]),
                                                  cam)
    dp, dpose = r.backward(out.generation, d_rgb, d_depth, d_normal, None, params_grad=True)
    torch.cuda.synchronize()
    ref = oracle.render(s.params, cam, s.pose)
    oml_out = oml.mapping_loss(ref["rgb"], ref["depth"], ref["normal"], tgt["rgb"], tgt["depth"], cam)
    near = ref["gmargin"] < 1e-5
    og = oracle.backward(s.params, cam, s.pose, d_rgb=oml_out["d_rgb"], d_depth=oml_out["d_depth"],
                         d_normal=oml_out["d_normal"], watch=near, scale=True, scale_mask=near)
    rep = check_grads(host(dp), og["d_params"], skip=og["touched"])
    print("mapping grads", rep, "skipped surfels", int(og["touched"].sum()))
    print("pose", check_pose(host(dpose), og["pose_paper"], scale=og["pose_scale"], flip=og["pose_scale_masked"]))
