"""Pins of the FP64 oracle against closed forms, invariants, brute force and finite differences.

Each test fixes a part of the oracle by something other than the oracle itself:
closed-form footprints (single surfel, filter branch, stacked surfels), an
independent ray-plane route, exact depth of a coplanar carpet from several
views, brute force without culling rectangles, central finite differences,
rigid-motion equivariance, linearity in colour, and library rotations.
"""

import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")


def _golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            tok = line.split()
            rows.append((tok[0], int(tok[1]), int(tok[2]), tok[3], float(tok[4])))
    return rows


def _scene(tag):
    if tag == "S1":
        return synth.single_surfel(scale=0.1)
    if tag == "S2":
        return synth.single_surfel(scale=0.01)
    if tag == "S3a":
        return synth.stacked_surfels(opacity=0.5)
    if tag == "S3b":
        return synth.stacked_surfels(opacity=0.8)
    raise KeyError(tag)


def test_golden_closed_forms(oracle_mod):
    """Single surfel (3D and filter branches) and stacked-surfel transmittance cutoff."""
    cache = {}
    for tag, x, y, qty, val in _golden():
        if tag not in cache:
            s = _scene(tag)
            cache[tag] = oracle_mod.render(s.params, s.camera, s.pose)
        o = cache[tag]
        if qty == "alpha":
            got = o["alpha"][y, x]
        elif qty == "depth":
            got = o["depth"][y, x]
        elif qty == "depth_over_alpha":
            got = o["depth"][y, x] / o["alpha"][y, x]
        elif qty == "count":
            got = o["count"][y, x]
        elif qty == "t_final":
            got = o["t_final"][y, x]
        else:
            raise KeyError(qty)
        # inputs are float32 (0.8 and 0.1 are not representable): 1e-6 relative
        assert got == pytest.approx(val, rel=1e-6, abs=1e-12), (tag, x, y, qty)


def test_single_surfel_full_image(oracle_mod):
    """Every pixel of the fronto-parallel surfel against u = (x-cx) z/(f s)."""
    s = synth.single_surfel(scale=0.1)
    o = oracle_mod.render(s.params, s.camera, s.pose)
    p = s.params.astype(np.float64)
    z, sc, op = p[2, 0], p[9, 0], p[11, 0]
    H, W = 48, 64
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = (xs - 32.0) * z / (60.0 * sc)
    v = (ys - 24.0) * z / (60.0 * sc)
    rho = u * u + v * v
    a = op * np.exp(-rho / 2)
    a[rho > 9] = 0
    a[a < 1 / 255] = 0
    np.testing.assert_allclose(o["alpha"], a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(o["depth"], a * z, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(o["normal"][2], a, rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(o["normal"][:2], 0.0)
    for c in range(3):
        np.testing.assert_allclose(o["rgb"][c], a * p[12 + c, 0], rtol=1e-12, atol=1e-15)


def test_stacked_depth_and_order(oracle_mod):
    """Transmittance cutoff composites exactly the first 13 (o=0.5); order is by depth, not index."""
    s = synth.stacked_surfels(opacity=0.5)
    p = s.params.astype(np.float64)
    z = p[2]
    expect_d = sum(0.5 * 0.5 ** k * z[k] for k in range(13))
    expect_r = sum(0.5 * 0.5 ** k * p[12, k] for k in range(13))
    perm = np.random.default_rng(3).permutation(s.n)
    for params in (s.params, s.params[:, perm]):
        o = oracle_mod.render(params, s.camera, s.pose)
        assert o["count"][24, 32] == 13
        assert o["depth"][24, 32] == pytest.approx(expect_d, rel=1e-14)
        assert o["rgb"][0, 24, 32] == pytest.approx(expect_r, rel=1e-14)


def test_alpha_min_threshold(oracle_mod):
    """A pair is kept at o G = 1.01/255 and dropped at 0.99/255."""
    for f, kept in ((1.01, True), (0.99, False)):
        s = synth.single_surfel(scale=0.1)
        g = np.exp(-0.5)  # pixel (35, 24) has rho = 1
        s.params[11, 0] = np.float32(f / (255.0 * g))
        o = oracle_mod.render(s.params, s.camera, s.pose)
        if kept:
            assert o["alpha"][24, 35] == pytest.approx(f / 255.0, rel=1e-6)
        else:
            assert o["alpha"][24, 35] == 0.0


def _ray_plane(s, x, y):
    """Independent intersection: X = r (n.mu_c)/(n.r); (u,v) from the tangent frame."""
    p = s.params.astype(np.float64)
    T = s.pose.astype(np.float64)
    R, t = T[:, :3], T[:, 3]
    mu_c = R @ p[0:3, 0] + t
    tuc = R @ p[3:6, 0]
    tvc = R @ p[6:9, 0]
    n = np.cross(tuc, tvc)
    cam = s.camera
    r = np.array([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, 1.0])
    X = r * (n @ mu_c) / (n @ r)
    d = X - mu_c
    # tangents are orthonormal only to float32 precision: solve d = u s_u tuc + v s_v tvc
    A = np.stack([p[9, 0] * tuc, p[10, 0] * tvc], axis=1)
    uv, *_ = np.linalg.lstsq(A, d, rcond=None)
    return uv[0], uv[1], X[2]


@pytest.mark.parametrize("seed", range(4))
def test_tilted_surfel_ray_plane(oracle_mod, seed):
    """The homography intersection equals an explicit ray-plane intersection (odd
    seeds with f_x != f_y and an off-centre principal point, so that the two focal
    lengths and the two principal-point coordinates cannot stand in for each other)."""
    g = np.random.default_rng(100 + seed)
    s = synth.single_surfel(scale=0.25, opacity=0.9)
    if seed % 2:
        s.camera = synth.Camera(64, 48, 56.0, 71.0, 30.5, 25.25)
    rot = Rotation.from_rotvec(g.normal(size=3) * 0.6).as_matrix()
    s.params[3:6, 0] = (rot @ np.array([1.0, 0, 0])).astype(np.float32)
    s.params[6:9, 0] = (rot @ np.array([0, 1.0, 0])).astype(np.float32)
    s.params[0:3, 0] = np.array([g.uniform(-0.2, 0.2), g.uniform(-0.2, 0.2), 2.5], dtype=np.float32)
    o = oracle_mod.render(s.params, s.camera, s.pose, filter=False)
    checked = 0
    for y in range(48):
        for x in range(64):
            a = o["alpha"][y, x]
            if a <= 0:
                continue
            u, v, z = _ray_plane(s, x, y)
            expect = s.params[11, 0].astype(np.float64) * np.exp(-(u * u + v * v) / 2)
            assert a == pytest.approx(expect, rel=1e-10)
            assert o["depth"][y, x] / a == pytest.approx(z, rel=1e-10)
            checked += 1
    assert checked > 50


@pytest.mark.parametrize("obliquity", [0.0, 15.0, 30.0, 45.0, 60.0])
def test_planar_carpet_depth(oracle_mod, obliquity):
    """Coplanar surfels give D/O = exact ray-plane depth and N/O = the plane normal (from any view)."""
    s = synth.planar_carpet(obliquity, azimuth_deg=20.0 + obliquity)
    o = oracle_mod.render(s.params, s.camera, s.pose)
    p = s.params.astype(np.float64)
    T = s.pose.astype(np.float64)
    R, t = T[:, :3], T[:, 3]
    tuc, tvc = R @ p[3:6, 0], R @ p[6:9, 0]
    n_c = np.cross(tuc, tvc)
    h_c = n_c @ (R @ p[0:3, 0] + t)
    cam = s.camera
    ys, xs = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    r = np.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, np.ones_like(xs, dtype=float)])
    d_plane = h_c / np.einsum("c,chw->hw", n_c, r)
    m = o["alpha"] > 1e-9
    assert m.sum() > 1000
    np.testing.assert_allclose(o["depth"][m] / o["alpha"][m], d_plane[m], rtol=1e-12)
    for c in range(3):
        np.testing.assert_allclose(o["normal"][c][m] / o["alpha"][m], n_c[c], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_equals_rect(oracle_mod, seed):
    """The conservative per-surfel rectangle never changes a single bit of the result."""
    s = synth.random_surfels(300, seed=seed)
    a = oracle_mod.render(s.params, s.camera, s.pose)
    b = oracle_mod.render(s.params, s.camera, s.pose, use_rect=False)
    for k in ("rgb", "depth", "normal", "alpha", "t_final", "count"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    ga = oracle_mod.backward(s.params, s.camera, s.pose, d_rgb=np.ones((3, 48, 64)))
    gb = oracle_mod.backward(s.params, s.camera, s.pose, d_rgb=np.ones((3, 48, 64)), use_rect=False)
    np.testing.assert_allclose(ga["d_params"], gb["d_params"], rtol=1e-12, atol=1e-14)


def test_colour_linearity_and_contribution(oracle_mod):
    """Doubling colours doubles rgb exactly and leaves D, N, O alone; sum_k dL/dc_k = sum_p O(p)."""
    s = synth.random_surfels(500, seed=4)
    a = oracle_mod.render(s.params, s.camera, s.pose)
    p2 = s.params.astype(np.float64).copy()
    p2[12:15] *= 2.0
    b = oracle_mod.render(p2, s.camera, s.pose)
    np.testing.assert_array_equal(b["rgb"], 2.0 * a["rgb"])
    for k in ("depth", "normal", "alpha"):
        np.testing.assert_array_equal(a[k], b[k])
    g = np.zeros((3, 48, 64))
    g[1] = 1.0
    gr = oracle_mod.backward(s.params, s.camera, s.pose, d_rgb=g)
    # dL/dc_k(green) = sum_p w_k(p) = the surfel's contribution; summed over k it is sum_p O
    assert gr["d_params"][13].sum() == pytest.approx(a["alpha"].sum(), rel=1e-12)
    assert np.all(gr["d_params"][13] >= 0)
    np.testing.assert_array_equal(gr["d_params"][12], 0.0)


def _rigid(seed):
    g = np.random.default_rng(seed)
    R = Rotation.from_rotvec(g.normal(size=3)).as_matrix()
    return R, g.normal(size=3)


def test_rigid_equivariance(oracle_mod):
    """render(G mu, G t_u, G t_v; T G^-1) = render(mu, t_u, t_v; T)."""
    s = synth.random_surfels(400, seed=5)
    Rg, tg = _rigid(9)
    p = s.params.astype(np.float64).copy()
    q = p.copy()
    q[0:3] = Rg @ p[0:3] + tg[:, None]
    q[3:6] = Rg @ p[3:6]
    q[6:9] = Rg @ p[6:9]
    T = np.eye(4)
    T[:3, :] = s.pose.astype(np.float64)
    G = np.eye(4)
    G[:3, :3], G[:3, 3] = Rg, tg
    TG = (T @ np.linalg.inv(G))[:3]
    a = oracle_mod.render(p, s.camera, T[:3])
    b = oracle_mod.render(q, s.camera, TG)
    for k in ("rgb", "depth", "normal", "alpha"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-9, atol=1e-12, err_msg=k)


def _fd_scene(oracle_mod, seed0):
    for seed in range(seed0, seed0 + 200):
        s = synth.tiny_scene(seed)
        o = oracle_mod.render(s.params, s.camera, s.pose)
        if o["alpha"].max() > 0.3 and o["gmargin"].min() > 1e-3:
            return s, o
    raise RuntimeError("no FD scene with a clean margin")


def _linear_loss(o, w):
    return (np.sum(o["rgb"] * w["rgb"]) + np.sum(o["depth"] * w["depth"])
            + np.sum(o["normal"] * w["normal"]) + np.sum(o["alpha"] * w["alpha"]))


@pytest.mark.parametrize("seed0", [0, 1000, 2000])
def test_finite_differences(oracle_mod, seed0):
    """Analytic gradients to all 15 parameters per surfel and the se(3) pose vs central differences."""
    s, o = _fd_scene(oracle_mod, seed0)
    H, W = s.camera.height, s.camera.width
    g = np.random.default_rng(seed0)
    w = {"rgb": g.normal(size=(3, H, W)), "depth": g.normal(size=(H, W)),
         "normal": g.normal(size=(3, H, W)), "alpha": g.normal(size=(H, W))}
    an = oracle_mod.backward(s.params, s.camera, s.pose, d_rgb=w["rgb"], d_depth=w["depth"],
                             d_normal=w["normal"], d_alpha=w["alpha"])
    p0 = s.params.astype(np.float64)

    def L(p, T=s.pose):
        return _linear_loss(oracle_mod.render(p, s.camera, T, nthreads=1), w)

    fd = np.zeros_like(p0)
    for r in range(15):
        for i in range(s.n):
            h = 1e-6 * max(1.0, abs(p0[r, i]))
            pp, pm = p0.copy(), p0.copy()
            pp[r, i] += h
            pm[r, i] -= h
            fd[r, i] = (L(pp) - L(pm)) / (2 * h)
    scale = np.abs(fd).max()
    np.testing.assert_allclose(an["d_params"], fd, rtol=1e-6, atol=1e-7 * scale)

    from oracle import se3

    fdp = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1e-6
        fdp[k] = (L(p0, se3.left_perturb(e, s.pose)) - L(p0, se3.left_perturb(-e, s.pose))) / 2e-6
    np.testing.assert_allclose(an["pose_paper"], fdp, rtol=1e-6, atol=1e-7 * np.abs(fdp).max())


@pytest.mark.parametrize("seed", [0, 7])
def test_pose_identity(oracle_mod, seed):
    """The paper's per-splat Jacobian form equals the world-gradient form (Jacobi identity)."""
    s = synth.random_surfels(600, seed=seed)
    g = np.random.default_rng(seed)
    an = oracle_mod.backward(s.params, s.camera, s.pose, d_rgb=g.normal(size=(3, 48, 64)),
                             d_depth=g.normal(size=(48, 64)), d_normal=g.normal(size=(3, 48, 64)),
                             d_alpha=g.normal(size=(48, 64)))
    np.testing.assert_allclose(an["pose_paper"], an["pose_identity"], rtol=1e-9,
                               atol=1e-12 * np.abs(an["pose_paper"]).max())


def test_margin_flags_boundary_pixel(oracle_mod):
    """The rho = 9 boundary pixel of the single surfel carries a tiny margin; interior pixels do not."""
    s = synth.single_surfel(scale=0.1)
    o = oracle_mod.render(s.params, s.camera, s.pose)
    assert o["fmargin"][24, 41] < 1e-6
    assert o["fmargin"][24, 35] > 1e-2


def test_preprocess_box_contains_footprint(oracle_mod):
    """Every pixel where a surfel is composited lies inside its exact box (plus nothing else)."""
    s = synth.random_surfels(50, seed=11)
    pre = oracle_mod.preprocess(s.params, s.camera, s.pose)
    for i in range(s.n):
        if pre["culled"][i]:
            continue
        one = s.params[:, i:i + 1]
        o = oracle_mod.render(one, s.camera, s.pose, use_rect=False)
        ys, xs = np.nonzero(o["alpha"] > 0)
        if len(xs) == 0:
            continue
        x0, x1, y0, y1 = pre["aabb"][:, i]
        assert xs.min() >= x0 - 1e-9 and xs.max() <= x1 + 1e-9
        assert ys.min() >= y0 - 1e-9 and ys.max() <= y1 + 1e-9


def test_finite_differences_clamped_opacity(oracle_mod):
    """Near-opaque surfels (o G > 0.99 around their centres): the clamp has zero derivative."""
    for seed in range(300, 500):
        s = synth.tiny_scene(seed, n=3)
        s.params[11, :] = np.float32(1.0)
        o = oracle_mod.render(s.params, s.camera, s.pose)
        if o["gmargin"].min() > 1e-3 and o["alpha"].max() >= 0.99:
            break
    else:
        raise RuntimeError("no clean clamped scene")
    H, W = s.camera.height, s.camera.width
    g = np.random.default_rng(seed)
    w = {"rgb": g.normal(size=(3, H, W)), "depth": g.normal(size=(H, W)),
         "normal": g.normal(size=(3, H, W)), "alpha": g.normal(size=(H, W))}
    an = oracle_mod.backward(s.params, s.camera, s.pose, d_rgb=w["rgb"], d_depth=w["depth"],
                             d_normal=w["normal"], d_alpha=w["alpha"])
    p0 = s.params.astype(np.float64)
    fd = np.zeros((4, s.n))
    for j, r in enumerate((0, 2, 9, 11)):
        for i in range(s.n):
            h = 1e-6 * max(1.0, abs(p0[r, i]))
            pp, pm = p0.copy(), p0.copy()
            pp[r, i] += h
            pm[r, i] -= h
            fd[j, i] = (_linear_loss(oracle_mod.render(pp, s.camera, s.pose), w)
                        - _linear_loss(oracle_mod.render(pm, s.camera, s.pose), w)) / (2 * h)
    got = an["d_params"][[0, 2, 9, 11]]
    np.testing.assert_allclose(got, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())
