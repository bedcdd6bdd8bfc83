"""Pins of the oracle's SE(3) maps, tracking loss and AdamW pose step."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from oracle import loss, se3


@pytest.mark.parametrize("seed", range(5))
def test_so3_exp_matches_library(seed):
    phi = np.random.default_rng(seed).normal(size=3) * (0.3 + seed)
    np.testing.assert_allclose(se3.so3_exp(phi), Rotation.from_rotvec(phi).as_matrix(), atol=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_se3_exp_log_roundtrip(seed):
    g = np.random.default_rng(seed)
    tau = np.concatenate([g.normal(size=3), g.normal(size=3) * 0.8])
    T = se3.exp(tau)
    np.testing.assert_allclose(se3.log(T), tau, atol=1e-12)
    np.testing.assert_allclose(se3.exp(se3.log(T)), T, atol=1e-12)
    R = T[:3, :3]
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-13)
    assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-13)


def test_se3_small_angle_continuity():
    rho = np.array([0.3, -0.2, 0.1])
    for th in (1e-9, 1e-7, 1e-5, 1e-3):
        ax = np.array([1.0, 2.0, -0.5]) / np.linalg.norm([1.0, 2.0, -0.5])
        a = se3.exp(np.concatenate([rho, ax * th]))
        b = se3.exp(np.concatenate([rho, ax * th * (1 + 1e-6)]))
        assert np.abs(a - b).max() < 1e-6 * max(th, 1e-9) * 10 + 1e-15


def _mp_hat4(tau):
    import mpmath

    r, p = [mpmath.mpf(float(v)) for v in tau[:3]], [mpmath.mpf(float(v)) for v in tau[3:]]
    return mpmath.matrix([[0, -p[2], p[1], r[0]], [p[2], 0, -p[0], r[1]], [-p[1], p[0], 0, r[2]], [0, 0, 0, 0]])


@pytest.mark.parametrize("th", [0.0, 1e-9, 1e-7, 1e-6, 3e-6, 1e-5, 1e-4, 1e-3, 9.9e-3, 1.01e-2, 0.1, 1.0, 3.0])
def test_se3_exp_log_against_matrix_exponential(th):
    """Exp(tau) against the matrix exponential of the 4x4 twist, evaluated by mpmath at
    50 digits (its definition, independent of the closed forms), and Log(Exp(tau)) =
    tau, at angles from 0 to 3 rad: the closed forms keep FP64 accuracy at small
    angles, where 1 - cos and th - sin th would cancel."""
    import mpmath

    mpmath.mp.dps = 50
    g = np.random.default_rng(int(th * 1e9) % 1000)
    ax = g.normal(size=3)
    ax /= np.linalg.norm(ax)
    tau = np.concatenate([g.normal(size=3) * 0.7, ax * th])
    E = mpmath.expm(_mp_hat4(tau))
    ref = np.array([[float(E[i, j]) for j in range(4)] for i in range(4)])
    np.testing.assert_allclose(se3.exp(tau), ref, rtol=0, atol=4e-16 * max(1.0, np.abs(tau).max()))
    back = se3.log(se3.exp(tau))
    np.testing.assert_allclose(back[3:], tau[3:], rtol=1e-12 if th > 1e-6 else 0, atol=2e-16 + 1e-13 * th)
    np.testing.assert_allclose(back[:3], tau[:3], rtol=0, atol=1e-14)


@pytest.mark.parametrize("th", [1e-8, 1e-6, 1e-4, 5e-3, 2e-2, 0.5, 2.0])
def test_so3_left_jacobian_against_series(th):
    """J(phi) against its defining series sum_n (phi^)^n / (n+1)!, summed by mpmath at 50
    digits to n = 80."""
    import mpmath

    mpmath.mp.dps = 50
    ax = np.array([0.3, -0.8, 0.5])
    ax /= np.linalg.norm(ax)
    phi = ax * th
    K = mpmath.matrix([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    S = mpmath.zeros(3, 3)
    P = mpmath.eye(3)
    for n in range(80):
        S += P / mpmath.factorial(n + 1)
        P = P * K
    ref = np.array([[float(S[i, j]) for j in range(3)] for i in range(3)])
    np.testing.assert_allclose(se3.so3_left_jacobian(phi), ref, rtol=0, atol=3e-16)


def test_se3_translation_only_and_composition():
    T = se3.exp(np.array([0.1, 0.2, 0.3, 0, 0, 0]))
    np.testing.assert_allclose(T[:3, 3], [0.1, 0.2, 0.3])
    np.testing.assert_allclose(T[:3, :3], np.eye(3))
    # rotations about one axis compose additively
    a = se3.exp(np.array([0, 0, 0, 0, 0, 0.3]))
    b = se3.exp(np.array([0, 0, 0, 0, 0, 0.5]))
    np.testing.assert_allclose(a @ b, se3.exp(np.array([0, 0, 0, 0, 0, 0.8])), atol=1e-14)


def test_left_perturbation_moves_camera_frame_points():
    """Exp(tau) T maps a world point to R(phi) (T X) + J(phi) rho: first order rho + phi x X_c."""
    T = synth.look_at_pose([1.0, 2.0, 1.5], [3.0, 2.5, 1.0]).astype(np.float64)
    X = np.array([2.0, 1.0, 0.7])
    Xc = T[:, :3] @ X + T[:, 3]
    tau = np.array([1e-7, -2e-7, 3e-7, 2e-7, 1e-7, -1e-7])
    Tp = se3.left_perturb(tau, T)
    Xp = Tp[:, :3] @ X + Tp[:, 3]
    np.testing.assert_allclose(Xp - Xc, tau[:3] + np.cross(tau[3:], Xc), atol=1e-12)


def _cam():
    return synth.Camera(4, 3, 2.0, 2.0, 2.0, 1.0)


def test_tracking_loss_hand_example():
    """A 4x3 example worked by hand: masks by N.r > 0 and O > 0.95, mean over all 12 pixels."""
    cam = _cam()
    H, W = 3, 4
    rgb = np.zeros((3, H, W))
    tgt = np.zeros((3, H, W))
    depth = np.zeros((H, W))
    tdepth = np.zeros((H, W))
    normal = np.zeros((3, H, W))
    normal[2] = 1.0        # facing away from the camera: N.r = 1 > 0 everywhere
    alpha = np.full((H, W), 0.99)
    rgb[0, 1, 2] = 0.5     # |d rgb| = 0.5 at (x=2, y=1)
    depth[1, 2] = 2.0
    tdepth[1, 2] = 1.5     # |d D| = 0.5
    rgb[1, 0, 0] = 0.25    # pixel (0,0): masked out by opacity
    alpha[0, 0] = 0.95     # not > 0.95
    rgb[2, 2, 3] = 1.0     # pixel (3,2): masked out by the normal
    normal[:, 2, 3] = [-1.0, 0.0, 0.0]  # N.r = -(3-2)/2 < 0
    L, d_rgb, d_depth, m = loss.tracking_loss(rgb, depth, normal, alpha, tgt, tdepth, cam, lambda_d=2.0)
    assert L == pytest.approx((0.5 + 2.0 * 0.5) / 12.0)
    assert not m[0, 0] and not m[2, 3] and m[1, 2]
    assert d_rgb[0, 1, 2] == pytest.approx(1 / 12)
    assert d_depth[1, 2] == pytest.approx(2.0 / 12)
    assert d_rgb[1, 0, 0] == 0 and d_rgb[2, 2, 3] == 0
    assert d_rgb[0, 0, 1] == 0  # sign(0) = 0


def test_tracking_loss_gradient_fd():
    g = np.random.default_rng(0)
    cam = synth.Camera(8, 6, 5.0, 5.0, 4.0, 3.0)
    rgb, tgt = g.uniform(size=(3, 6, 8)), g.uniform(size=(3, 6, 8))
    depth, tdepth = g.uniform(1, 2, size=(6, 8)), g.uniform(1, 2, size=(6, 8))
    normal = g.normal(size=(3, 6, 8))
    alpha = g.uniform(0.9, 1.0, size=(6, 8))
    L, d_rgb, d_depth, _ = loss.tracking_loss(rgb, depth, normal, alpha, tgt, tdepth, cam, lambda_d=0.7)
    for idx in [(0, 1, 2), (2, 5, 7), (1, 3, 3)]:
        e = np.zeros_like(rgb)
        e[idx] = 1e-7
        Lp = loss.tracking_loss(rgb + e, depth, normal, alpha, tgt, tdepth, cam, lambda_d=0.7)[0]
        Lm = loss.tracking_loss(rgb - e, depth, normal, alpha, tgt, tdepth, cam, lambda_d=0.7)[0]
        assert (Lp - Lm) / 2e-7 == pytest.approx(d_rgb[idx], abs=1e-6)
    e = np.zeros_like(depth)
    e[2, 2] = 1e-7
    Lp = loss.tracking_loss(rgb, depth + e, normal, alpha, tgt, tdepth, cam, lambda_d=0.7)[0]
    Lm = loss.tracking_loss(rgb, depth - e, normal, alpha, tgt, tdepth, cam, lambda_d=0.7)[0]
    assert (Lp - Lm) / 2e-7 == pytest.approx(d_depth[2, 2], abs=1e-6)


def test_adamw_first_step_closed_form():
    """First bias-corrected Adam step is -lr g / (|g| + eps) per component."""
    T = synth.look_at_pose([0, 0, 0], [0, 0, 1]).astype(np.float64)
    g = np.array([0.3, -2.0, 1e-3, 0.0, 5.0, -0.1])
    lr = np.array([1e-3, 1e-3, 1e-3, 3e-3, 3e-3, 3e-3])
    st = loss.AdamState()
    T1, tau = loss.adamw_pose_step(T, g, st, lr)
    np.testing.assert_allclose(tau, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(T1, se3.left_perturb(tau, T), atol=1e-15)
    # second step with the same gradient: still -lr sign(g) up to eps
    T2, tau2 = loss.adamw_pose_step(T1, g, st, lr)
    np.testing.assert_allclose(tau2, -lr * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_image_loss_instances():
    """The general masked L1 against the tracking loss (both masks, no normal term), the
    unmasked frame loss (all three terms), and a hand-worked opacity-mask-only case."""
    import oracle

    s = synth.random_surfels(2000, seed=0)
    t = synth.random_surfels(2000, seed=1)
    o = oracle.render(s.params, s.camera, s.pose)
    g = oracle.render(t.params, t.camera, t.pose)
    L, d_rgb, d_depth, _ = loss.tracking_loss(o["rgb"], o["depth"], o["normal"], o["alpha"], g["rgb"], g["depth"],
                                              s.camera, lambda_d=0.7)
    G = loss.image_loss(o["rgb"], o["depth"], o["normal"], o["alpha"], g["rgb"], g["depth"], g["normal"], s.camera,
                        w_rgb=1.0, w_d=0.7, w_n=0.0)
    assert G[0] == pytest.approx(L, rel=1e-14)
    np.testing.assert_array_equal(G[1], d_rgb)
    np.testing.assert_array_equal(G[2], d_depth)
    assert not G[3].any()
    F = loss.frame_loss(o["rgb"], o["depth"], o["normal"], g["rgb"], g["depth"], g["normal"])
    G = loss.image_loss(o["rgb"], o["depth"], o["normal"], o["alpha"], g["rgb"], g["depth"], g["normal"], s.camera,
                        w_rgb=1.0, w_d=1.0, w_n=1.0, normal_mask=False, opacity_mask=False)
    assert G[0] == pytest.approx(F[0], rel=1e-14)
    for a, b in zip(G[1:], F[1:]):
        np.testing.assert_array_equal(a, b)
    # 1 x 2 image: the opacity mask keeps pixel 0 only; the normal mask is not applied
    cam = synth.Camera(2, 1, 1.0, 1.0, 0.5, 0.0)
    rgb = np.array([[[0.5, 0.5]], [[0.2, 0.2]], [[0.9, 0.9]]])
    tgt = np.zeros_like(rgb)
    depth, tdepth = np.array([[2.0, 2.0]]), np.array([[1.0, 1.0]])
    normal = np.zeros((3, 1, 2))
    normal[2] = -1.0  # back faces: the normal mask would reject both pixels
    alpha = np.array([[0.99, 0.9]])
    G = loss.image_loss(rgb, depth, normal, alpha, tgt, tdepth, None, cam, w_rgb=1.0, w_d=0.5, w_n=0.0,
                        normal_mask=False, opacity_mask=True)
    assert G[0] == pytest.approx((0.5 + 0.2 + 0.9 + 0.5 * 1.0) / 2, rel=1e-15)
    np.testing.assert_array_equal(G[2], [[0.5 / 2, 0.0]])
