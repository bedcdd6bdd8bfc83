"""CPU pins of the oracle's depth variants (normalised and median depth) and of the
relocalisation error e_t (eq:tracking_error).

Pins: coplanar surfels, where every composited intersection lies on the plane, so
both D/O and the median depth equal the exact ray-plane depth; stacked surfels on the
optical axis, where the median index is the largest i with (1 - o)^i > 1/2; a single
surfel; and e_t against the tracking loss with a zero colour residual (eq:tracking_error
uses the tracking loss's formulation) and a hand-worked case.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import loss as oloss


def _plane_depth(s):
    p = s.params.astype(np.float64)
    T = s.pose.astype(np.float64)
    R, t = T[:, :3], T[:, 3]
    n_c = np.cross(R @ p[3:6, 0], R @ p[6:9, 0])
    h_c = n_c @ (R @ p[0:3, 0] + t)
    cam = s.camera
    ys, xs = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    r = np.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, np.ones_like(xs, dtype=float)])
    return h_c / np.einsum("c,chw->hw", n_c, r)


@pytest.mark.parametrize("obliquity", [0.0, 30.0, 60.0])
def test_depth_variants_on_planar_carpets(obliquity):
    s = synth.planar_carpet(obliquity, azimuth_deg=10.0 + obliquity)
    dv = oracle.depth_variants(s.params, s.camera, s.pose)
    o = oracle.render(s.params, s.camera, s.pose)
    d = _plane_depth(s)
    m = o["alpha"] > 0
    assert m.sum() > 1000
    np.testing.assert_allclose(dv["depth_norm"][m], d[m], rtol=1e-12)
    np.testing.assert_allclose(dv["depth_median"][m], d[m], rtol=1e-12)
    assert np.all(dv["depth_norm"][~m] == 0) and np.all(dv["depth_median"][~m] == 0)


@pytest.mark.parametrize("opacity,index", [(0.3, 1), (0.1, 6), (0.45, 1), (0.7, 0)])
def test_median_depth_of_stacked_surfels(opacity, index):
    """At the optical axis every surfel has alpha = o, so T_i = (1 - o)^i and the median
    is surfel i* = max{i : (1 - o)^i > 1/2}, at depth z0 + i* dz."""
    assert (1 - opacity) ** index > 0.5 >= (1 - opacity) ** (index + 1)
    s = synth.stacked_surfels(count=20, opacity=opacity, z0=2.0, dz=0.1)
    dv = oracle.depth_variants(s.params, s.camera, s.pose)
    # the surfel parameters are float32: z is float32(z0 + i dz)
    assert dv["depth_median"][24, 32] == pytest.approx(float(s.params[2, index]), abs=1e-12)
    assert float(s.params[2, index]) == pytest.approx(2.0 + 0.1 * index, abs=1e-6)
    assert dv["margin"][24, 32] > 1e-3
    # T = 1/2 exactly is not "above one half": o = 0.5 stops at the first surfel, with
    # a zero margin
    s = synth.stacked_surfels(count=20, opacity=0.5)
    dv = oracle.depth_variants(s.params, s.camera, s.pose)
    assert dv["depth_median"][24, 32] == pytest.approx(2.0, abs=1e-12)
    assert dv["margin"][24, 32] == 0.0


def test_single_surfel_median_is_its_depth():
    s = synth.single_surfel(scale=0.1, opacity=0.8)
    dv = oracle.depth_variants(s.params, s.camera, s.pose)
    o = oracle.render(s.params, s.camera, s.pose)
    m = o["alpha"] > 0
    np.testing.assert_allclose(dv["depth_median"][m], dv["depth_norm"][m], rtol=1e-14)
    np.testing.assert_allclose(dv["depth_norm"][m], 2.0, rtol=1e-12)


def test_tracking_error_is_the_depth_term_of_the_tracking_loss():
    s = synth.random_surfels(2000, seed=0)
    t = synth.random_surfels(2000, seed=1)
    o = oracle.render(s.params, s.camera, s.pose)
    tg = oracle.render(t.params, t.camera, t.pose)
    e = oloss.tracking_error(o["depth"], o["normal"], o["alpha"], tg["depth"], s.camera)
    L = oloss.tracking_loss(o["rgb"], o["depth"], o["normal"], o["alpha"], o["rgb"], tg["depth"], s.camera)[0]
    assert e == pytest.approx(L, rel=1e-14)
    assert e > 0


def test_tracking_error_worked_example():
    """2 x 2 image, camera centre at pixel (0.5, 0.5), rays (+-0.5, +-0.5, 1)/f = 1."""
    cam = synth.Camera(2, 2, 1.0, 1.0, 0.5, 0.5)
    depth = np.array([[1.0, 2.0], [3.0, 4.0]])
    tgt = np.array([[1.5, 1.0], [3.0, 6.0]])
    alpha = np.array([[0.99, 0.99], [0.5, 0.99]])  # pixel (0, 1) fails the opacity mask
    normal = np.zeros((3, 2, 2))
    normal[2] = 1.0  # N . r = 1 > 0: front faces everywhere ...
    normal[:, 0, 1] = [0.0, 0.0, -1.0]  # ... except pixel (x=1, y=0)
    # kept: (x=0,y=0) |1-1.5| = 0.5 and (x=1,y=1) |4-6| = 2; (1,0) fails M_n, (0,1) fails M_o
    assert oloss.tracking_error(depth, normal, alpha, tgt, cam) == pytest.approx((0.5 + 2.0) / 4, rel=1e-15)
