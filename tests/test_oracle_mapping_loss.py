"""CPU pins of the oracle's mapping loss (oracle/mapping_loss.py).

Each pin checks the oracle against something other than itself: SSIM's fixed points
and closed forms on constant images (interior and the zero-padded border, which
fixes C1, C2 and the window), a brute-force two-pass evaluation with the 2-D Gaussian
written out, exact plane normals from ray-plane depth, analytic normals where central
differences are exact (quadratic lifted points), the loss terms under constant
offsets, and finite differences of the whole loss.
"""

import math

import numpy as np
import torch

import synth
from oracle import mapping_loss as ml

CAM = synth.Camera(23, 17, 20.0, 22.0, 11.3, 8.1)


def _g1():
    g = np.array([math.exp(-(i * i) / (2 * 1.5 ** 2)) for i in range(-5, 6)])
    return g / g.sum()


def test_ssim_of_identical_images_is_one():
    x = torch.rand((3, 20, 31), dtype=torch.float64, generator=torch.Generator().manual_seed(0))
    np.testing.assert_allclose(ml.ssim_map(x, x).numpy(), 1.0, atol=1e-12)


def test_ssim_is_symmetric():
    g = torch.Generator().manual_seed(1)
    x, y = torch.rand((3, 14, 15), dtype=torch.float64, generator=g), torch.rand((3, 14, 15), dtype=torch.float64,
                                                                               generator=g)
    np.testing.assert_allclose(ml.ssim_map(x, y).numpy(), ml.ssim_map(y, x).numpy(), atol=1e-14)


def test_ssim_of_constant_images():
    """x = a, y = b: with S the window mass inside the image at a pixel, the local
    statistics are mu = a S, var = a^2 S (1 - S), cov = a b S (1 - S); in the interior
    S = 1 and SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b, H, W = 0.7, 0.3, 16, 18
    s = ml.ssim_map(torch.full((1, H, W), a, dtype=torch.float64), torch.full((1, H, W), b, dtype=torch.float64))
    s = s[0].numpy()
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    assert np.allclose(s[5:H - 5, 5:W - 5], (2 * a * b + C1) / (a * a + b * b + C1), atol=1e-14)
    g = _g1()
    for (py, px) in [(0, 0), (0, 7), (3, 1), (H - 1, W - 2), (8, 0)]:
        Sy = sum(g[i + 5] for i in range(-5, 6) if 0 <= py + i < H)
        Sx = sum(g[j + 5] for j in range(-5, 6) if 0 <= px + j < W)
        S = Sy * Sx
        want = ((2 * a * b * S * S + C1) * (2 * a * b * S * (1 - S) + C2)) / (
            ((a * a + b * b) * S * S + C1) * ((a * a + b * b) * S * (1 - S) + C2))
        assert abs(s[py, px] - want) < 1e-13, (py, px, s[py, px], want)


def test_ssim_brute_force_window():
    """The separable zero-padded filtering against the 2-D Gaussian written out, with
    two-pass (centred) local statistics."""
    g = np.random.default_rng(2)
    x, y = g.random((2, 13, 17)), g.random((2, 13, 17))
    s = ml.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    w = np.array([[math.exp(-(i * i + j * j) / (2 * 1.5 ** 2)) for j in range(-5, 6)] for i in range(-5, 6)])
    w /= w.sum()
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    for c in range(2):
        for (py, px) in [(0, 0), (6, 8), (12, 16), (2, 14), (9, 3)]:
            vals = []
            for i in range(-5, 6):
                for j in range(-5, 6):
                    yy, xx = py + i, px + j
                    inside = 0 <= yy < 13 and 0 <= xx < 17
                    vals.append((w[i + 5, j + 5], x[c, yy, xx] if inside else 0.0, y[c, yy, xx] if inside else 0.0))
            mx = sum(wt * a for wt, a, _ in vals)
            my = sum(wt * b for wt, _, b in vals)
            vx = sum(wt * (a - mx) ** 2 for wt, a, _ in vals)
            vy = sum(wt * (b - my) ** 2 for wt, _, b in vals)
            cxy = sum(wt * (a - mx) * (b - my) for wt, a, b in vals)
            want = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
            assert abs(s[c, py, px] - want) < 1e-12


def _plane_depth(n, d, cam):
    W, H, fx, fy, cx, cy = cam.as_tuple()
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    r = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)])
    return d / np.tensordot(n, r, axes=1)


def test_depth_normals_of_planes():
    """Points of a plane n . X = d (d > 0, in front of the camera): every interior N_D is
    the unit normal pointing away from the camera, +n/|n|; the border is 0."""
    for n in ([0.0, 0.0, 1.0], [0.3, -0.2, 1.0], [-0.5, 0.4, 0.8], [0.1, 0.9, 0.6]):
        n = np.asarray(n)
        D = _plane_depth(n, 2.0, CAM)
        assert np.all(D > 0)
        N = ml.depth_normals(torch.tensor(D), CAM).numpy()
        np.testing.assert_allclose(N[:, 1:-1, 1:-1], (n / np.linalg.norm(n))[:, None, None] * np.ones((1, 15, 21)),
                                   atol=1e-12)
        assert np.all(N[:, 0] == 0) and np.all(N[:, -1] == 0) and np.all(N[:, :, 0] == 0) and np.all(N[:, :, -1] == 0)
        # scaling the depth scales the points: the normals do not change
        np.testing.assert_allclose(ml.depth_normals(torch.tensor(3.7 * D), CAM).numpy(), N, atol=1e-12)


def test_loss_of_a_perfect_render():
    """Rendered = observed, N_r = N_D with opacity O: L1 = 0, SSIM = 1, L_D = 0, and
    L_n = 1 - O inside, 1 on the border."""
    n = np.array([0.2, -0.1, 1.0])
    D = _plane_depth(n, 2.5, CAM)
    rgb = np.random.default_rng(3).random((3, 17, 23))
    O = 0.8
    N = O * ml.depth_normals(torch.tensor(D), CAM).numpy()
    out = ml.mapping_loss(rgb, D, N, rgb, D, CAM)
    border = 17 * 23 - 15 * 21
    l1, dssim, ld, ln = out["terms"]
    assert l1 == 0.0 and ld == 0.0 and abs(dssim) < 1e-12
    assert abs(ln - (border + 15 * 21 * (1 - O)) / (17 * 23)) < 1e-12
    assert abs(out["loss"] - ml.W_N * ln) < 1e-12


def test_gradients_match_finite_differences():
    g = np.random.default_rng(4)
    H, W = 17, 23
    rgb, tgt = g.random((3, H, W)), g.random((3, H, W))
    D = _plane_depth(np.array([0.2, -0.1, 1.0]), 2.5, CAM) + 0.05 * g.standard_normal((H, W))
    Dt = D + 0.1 * g.standard_normal((H, W))
    N = g.standard_normal((3, H, W))
    out = ml.mapping_loss(rgb, D, N, tgt, Dt, CAM)
    h = 1e-6

    def fd(arr_name, idx):
        args = {"rgb": rgb.copy(), "depth": D.copy(), "normal": N.copy()}
        args[arr_name][idx] += h
        lp = ml.mapping_loss(args["rgb"], args["depth"], args["normal"], tgt, Dt, CAM)["loss"]
        args[arr_name][idx] -= 2 * h
        lm = ml.mapping_loss(args["rgb"], args["depth"], args["normal"], tgt, Dt, CAM)["loss"]
        return (lp - lm) / (2 * h)

    for idx in [(0, 0, 0), (1, 8, 11), (2, 16, 22), (0, 5, 1), (2, 3, 19)]:
        assert abs(fd("rgb", idx) - out["d_rgb"][idx]) < 1e-8 * max(1.0, abs(out["d_rgb"][idx]) * 1e3)
        assert abs(fd("normal", idx) - out["d_normal"][idx]) < 1e-9
    for idx in [(0, 0), (1, 1), (8, 11), (16, 22), (2, 21), (9, 1)]:
        assert abs(fd("depth", idx) - out["d_depth"][idx]) < 1e-8


def test_depth_normals_exact_on_quadratic_points():
    """D = a + b x + c y makes the lifted points X = D r quadratic in (x, y), so central
    differences are exact: N_D = (dX/dx x dX/dy) / |.| with the analytic derivatives
    dX/dx = b r + D e_x / f_x and dX/dy = c r + D e_y / f_y."""
    W, H, fx, fy, cx, cy = CAM.as_tuple()
    a, b, c = 2.0, 0.03, -0.02
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    D = a + b * xs + c * ys
    N = ml.depth_normals(torch.tensor(D), CAM).numpy()
    r = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)])
    Xx = b * r + D * np.array([1 / fx, 0, 0])[:, None, None]
    Xy = c * r + D * np.array([0, 1 / fy, 0])[:, None, None]
    n = np.cross(Xx, Xy, axis=0)
    n /= np.linalg.norm(n, axis=0)
    np.testing.assert_allclose(N[:, 1:-1, 1:-1], n[:, 1:-1, 1:-1], atol=1e-12)
    assert np.abs(n[:, 1:-1, 1:-1] - n[:, 8:9, 11:12]).max() > 1e-3  # the normal varies over the image


def test_terms_of_constant_offsets():
    """rgb = tgt + (0.1, -0.2, 0.05) and depth = tgt_depth + 0.3: the L1 term is 0.35 per
    pixel (summed over RGB), the depth term 0.3, and the loss is their weighted sum plus
    the SSIM and normal terms."""
    g = np.random.default_rng(5)
    tgt = 0.3 + 0.4 * g.random((3, 17, 23))
    rgb = tgt + np.array([0.1, -0.2, 0.05])[:, None, None]
    Dt = 2.0 + 0.1 * g.random((17, 23))
    N = g.standard_normal((3, 17, 23))
    out = ml.mapping_loss(rgb, Dt + 0.3, N, tgt, Dt, CAM)
    l1, dssim, ld, ln = out["terms"]
    assert abs(l1 - 0.35) < 1e-12 and abs(ld - 0.3) < 1e-12
    assert abs(out["loss"] - (0.875 * 0.35 + 0.125 * dssim + 0.5 * 0.3 + 0.02 * ln)) < 1e-12
    assert 0.0 < dssim < 1.0


def test_gradients_where_the_depth_normal_vanishes():
    """Zero depth (no surface) around some pixels: N_D = 0 there with a zero, finite
    gradient, and finite differences still agree everywhere else."""
    g = np.random.default_rng(6)
    H, W = 17, 23
    D = _plane_depth(np.array([0.2, -0.1, 1.0]), 2.5, CAM)
    D[5:11, 6:14] = 0.0
    rgb, tgt = g.random((3, H, W)), g.random((3, H, W))
    N = g.standard_normal((3, H, W))
    out = ml.mapping_loss(rgb, D, N, tgt, D + 0.1, CAM)
    assert all(np.all(np.isfinite(out[k])) for k in ("d_rgb", "d_depth", "d_normal"))
    nd = ml.depth_normals(torch.tensor(D), CAM).numpy()
    assert np.all(nd[:, 6:10, 7:13] == 0) and np.all(out["d_normal"][:, 6:10, 7:13] == 0)
    h = 1e-6
    for idx in [(4, 6), (8, 9), (11, 14), (2, 20)]:
        Dp, Dm = D.copy(), D.copy()
        Dp[idx] += h
        Dm[idx] -= h
        fd = (ml.mapping_loss(rgb, Dp, N, tgt, D + 0.1, CAM)["loss"] -
              ml.mapping_loss(rgb, Dm, N, tgt, D + 0.1, CAM)["loss"]) / (2 * h)
        assert abs(fd - out["d_depth"][idx]) < 1e-7, (idx, fd, out["d_depth"][idx])
