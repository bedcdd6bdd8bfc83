"""GPU: the masked L1 image loss (gs2d_image_loss) against the oracle's image_loss, on
the oracle's renders rounded to float32, for the weight and mask settings of the
tracking loss, the single-frame L1 and the mapping window's loss."""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import loss as oloss
from tests.gpu_common import ROOM_CAM, dev, host, room_scene

pytestmark = pytest.mark.gpu

SETTINGS = {
    "tracking": dict(w_rgb=1.0, w_depth=0.7, w_normal=0.0, normal_mask=True, opacity_mask=True),
    "single_frame": dict(w_rgb=1.0, w_depth=1.0, w_normal=1.0, normal_mask=False, opacity_mask=False),
    "mapping_window": dict(w_rgb=1.0, w_depth=0.5, w_normal=0.0, normal_mask=False, opacity_mask=True),
}


@pytest.fixture(scope="module")
def r():
    from paper_2506_00970_amd import Rasterizer

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return Rasterizer()


@pytest.fixture(scope="module")
def frames():
    room, pose = room_scene(300_000, seed=8, cam_seed=8)
    start = synth.perturb_pose(pose, 0.05, 3.0, seed=9)
    f32 = lambda d: {k: np.asarray(d[k], dtype=np.float32) for k in ("rgb", "depth", "normal", "alpha")}
    return f32(oracle.render(room.params, ROOM_CAM, start)), f32(oracle.render(room.params, ROOM_CAM, pose))


@pytest.mark.parametrize("setting", list(SETTINGS))
def test_image_loss_matches_oracle(r, frames, setting):
    img, tgt = frames
    w = SETTINGS[setting]
    g = {k: dev(v) for k, v in img.items()}
    t = {k: dev(v) for k, v in tgt.items()}
    loss, d_rgb, d_depth, d_normal = r.image_loss(ROOM_CAM, g["rgb"], g["depth"], g["normal"], g["alpha"], t["rgb"],
                                                  t["depth"], t["normal"], **w)
    torch.cuda.synchronize()
    L, e_rgb, e_depth, e_normal = oloss.image_loss(img["rgb"], img["depth"], img["normal"], img["alpha"], tgt["rgb"],
                                                   tgt["depth"], tgt["normal"], ROOM_CAM, w_rgb=w["w_rgb"],
                                                   w_d=w["w_depth"], w_n=w["w_normal"],
                                                   normal_mask=w["normal_mask"], opacity_mask=w["opacity_mask"])
    print(setting, float(loss), L)
    assert float(loss) == pytest.approx(L, rel=1e-5)
    np.testing.assert_allclose(host(d_rgb), e_rgb, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(host(d_depth), e_depth, rtol=1e-6, atol=1e-12)
    if w["w_normal"]:
        np.testing.assert_allclose(host(d_normal), e_normal, rtol=1e-6, atol=1e-12)
    else:
        assert d_normal is None


def test_tracking_loss_and_error_are_instances(r, frames):
    """gs2d_tracking_loss and gs2d_tracking_error give exactly the image loss's values."""
    img, tgt = frames
    g = {k: dev(v) for k, v in img.items()}
    t = {k: dev(v) for k, v in tgt.items()}
    a = r.tracking_loss(ROOM_CAM, g["rgb"], g["depth"], g["normal"], g["alpha"], t["rgb"], t["depth"], lambda_d=0.7)
    b = r.image_loss(ROOM_CAM, g["rgb"], g["depth"], g["normal"], g["alpha"], t["rgb"], t["depth"], None,
                     **SETTINGS["tracking"])
    for x, y in zip(a, b[:3]):
        assert torch.equal(x, y)
    e = r.tracking_error(ROOM_CAM, g["depth"], g["normal"], g["alpha"], t["depth"])
    c = r.image_loss(ROOM_CAM, None, g["depth"], g["normal"], g["alpha"], None, t["depth"], None, w_rgb=0.0,
                     w_depth=1.0, normal_mask=True, opacity_mask=True, grads=False)
    assert torch.equal(e, c[0])


def test_image_loss_batch_equals_single_calls(r):
    """gs2d_image_loss_batch over views of two sizes equals one gs2d_image_loss call per
    view, bit for bit (loss and gradients), with and without the masks and the normal term."""
    cams = [synth.Camera(64, 48, 60.0, 60.0, 32.0, 24.0), synth.Camera(70, 45, 55.0, 55.0, 35.0, 22.5)]
    g = np.random.default_rng(3)
    views = []
    for k in range(5):
        c = cams[k % 2]
        H, W = c.height, c.width
        nrm = g.normal(size=(3, H, W))
        nrm /= np.linalg.norm(nrm, axis=0, keepdims=True)
        v = {"camera": c, "rgb": g.random((3, H, W)), "depth": g.random((H, W)) + 1.0, "normal": nrm,
             "alpha": g.random((H, W)), "tgt_rgb": g.random((3, H, W)), "tgt_depth": g.random((H, W)) + 1.0,
             "tgt_normal": nrm[::-1].copy()}
        views.append({kk: (dev(vv) if isinstance(vv, np.ndarray) else vv) for kk, vv in v.items()})
    for kw in (dict(w_rgb=1.0, w_depth=0.5, opacity_mask=True), dict(w_rgb=1.0, w_depth=1.0, w_normal=1.0),
               dict(w_rgb=1.0, w_depth=0.7, normal_mask=True, opacity_mask=True)):
        losses, grads = r.image_loss_batch(views, **kw)
        torch.cuda.synchronize()
        for k, v in enumerate(views):
            loss, d_rgb, d_depth, d_normal = r.image_loss(v["camera"], v["rgb"], v["depth"], v["normal"], v["alpha"],
                                                          v["tgt_rgb"], v["tgt_depth"], v["tgt_normal"], **kw)
            torch.cuda.synchronize()
            assert host(losses)[k] == host(loss), (kw, k)
            for a, b in zip(grads[k], (d_rgb, d_depth, d_normal)):
                assert (a is None) == (b is None)
                if a is not None:
                    np.testing.assert_array_equal(host(a), host(b))
