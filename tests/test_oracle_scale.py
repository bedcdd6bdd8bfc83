"""CPU pins of the oracle's magnitude scales (``oracle.backward(..., scale=True)``).

Each gradient entry is a sum over (pixel, surfel) pairs of the pair's term; its
scale is the sum of |term|.  The GPU parity tests use the scale to bound the
floating-point rounding of entries that cancel (Sec. "Camera Pose Optimization",
eq:derivatives, is a sum over every pair of the image).  These pins fix what the
scale is: the exact sum of |per-pixel contributions| where each pixel holds one
pair, an upper bound of it where pixels hold several, and an additive split over
disjoint pixel masks.
"""

import numpy as np
import pytest

import synth


def _delta_grads(H, W, p, g):
    """Image gradients that are zero except at pixel p (random values on all 8 channels)."""
    y, x = divmod(p, W)
    out = {"d_rgb": np.zeros((3, H, W)), "d_depth": np.zeros((H, W)), "d_normal": np.zeros((3, H, W)),
           "d_alpha": np.zeros((H, W))}
    out["d_rgb"][:, y, x] = g.normal(size=3)
    out["d_depth"][y, x] = g.normal()
    out["d_normal"][:, y, x] = g.normal(size=3)
    out["d_alpha"][y, x] = g.normal()
    return out


def _sum_grads(parts):
    return {k: sum(p[k] for p in parts) for k in parts[0]}


@pytest.mark.parametrize("scene", ["fronto", "tilted"])
def test_scale_single_surfel_per_pixel_brute_force(oracle_mod, scene):
    """One surfel: every pixel holds one pair, so the scale of every entry and of the
    pose equals the sum over pixels of |the pixel's gradient|."""
    s = synth.single_surfel(scale=0.1) if scene == "fronto" else synth.tiny_scene(5, n=1)
    H, W = s.camera.height, s.camera.width
    ref = oracle_mod.render(s.params, s.camera, s.pose)
    pix = np.flatnonzero(ref["alpha"].ravel() > 0)
    g = np.random.default_rng(0)
    parts = [_delta_grads(H, W, p, g) for p in pix]
    absum = np.zeros((15, 1))
    pabs = np.zeros(6)
    for gr in parts:
        o = oracle_mod.backward(s.params, s.camera, s.pose, nthreads=1, **gr)
        absum += np.abs(o["d_params"])
        pabs += np.abs(o["pose_paper"])
    full = oracle_mod.backward(s.params, s.camera, s.pose, scale=True, nthreads=1, **_sum_grads(parts))
    np.testing.assert_allclose(full["d_scale"], absum, rtol=1e-12)
    np.testing.assert_allclose(full["pose_scale"], pabs, rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_scale_bounds_per_pixel_sums(oracle_mod, seed):
    """Several overlapping surfels: the scale bounds the sum over pixels of |the
    pixel's gradient| of every entry and of the pose, and so bounds the result."""
    s = synth.tiny_scene(seed, n=4)
    H, W = s.camera.height, s.camera.width
    g = np.random.default_rng(seed)
    parts = [_delta_grads(H, W, p, g) for p in range(H * W)]
    absum = np.zeros((15, s.n))
    pabs = np.zeros(6)
    for gr in parts:
        o = oracle_mod.backward(s.params, s.camera, s.pose, nthreads=1, **gr)
        absum += np.abs(o["d_params"])
        pabs += np.abs(o["pose_paper"])
    full = oracle_mod.backward(s.params, s.camera, s.pose, scale=True, **_sum_grads(parts))
    assert np.all(full["d_scale"] >= absum * (1 - 1e-12))
    assert np.all(full["pose_scale"] >= pabs * (1 - 1e-12))
    assert np.all(full["d_scale"] >= np.abs(full["d_params"]) * (1 - 1e-12))
    assert np.all(full["pose_scale"] >= np.abs(full["pose_paper"]) * (1 - 1e-12))


def test_scale_mask_is_additive(oracle_mod):
    """The masked pose scale sums the same pair magnitudes over the masked pixels: a
    mask and its complement add up to the full scale; all-ones gives the full scale and
    all-zeros gives zero; the scale does not depend on the threads' split of rows."""
    s = synth.random_surfels(2000, seed=0)
    H, W = s.camera.height, s.camera.width
    g = np.random.default_rng(3)
    gr = {"d_rgb": g.normal(size=(3, H, W)), "d_depth": g.normal(size=(H, W)),
          "d_normal": g.normal(size=(3, H, W)), "d_alpha": g.normal(size=(H, W))}
    m = g.uniform(size=(H, W)) < 0.3
    a = oracle_mod.backward(s.params, s.camera, s.pose, scale=True, scale_mask=m, **gr)
    b = oracle_mod.backward(s.params, s.camera, s.pose, scale=True, scale_mask=~m, nthreads=3, **gr)
    np.testing.assert_allclose(a["pose_scale_masked"] + b["pose_scale_masked"], a["pose_scale"], rtol=1e-12)
    np.testing.assert_allclose(a["pose_scale"], b["pose_scale"], rtol=1e-12)
    np.testing.assert_allclose(a["d_scale"], b["d_scale"], rtol=1e-12)
    ones = oracle_mod.backward(s.params, s.camera, s.pose, scale=True, scale_mask=np.ones((H, W), bool), **gr)
    np.testing.assert_allclose(ones["pose_scale_masked"], ones["pose_scale"], rtol=1e-12)
    zero = oracle_mod.backward(s.params, s.camera, s.pose, scale=True, scale_mask=np.zeros((H, W), bool), **gr)
    assert np.all(zero["pose_scale_masked"] == 0.0)
    # the scale outputs leave the gradients themselves unchanged
    plain = oracle_mod.backward(s.params, s.camera, s.pose, **gr)
    np.testing.assert_array_equal(plain["d_params"], a["d_params"])
    np.testing.assert_array_equal(plain["pose_paper"], a["pose_paper"])
