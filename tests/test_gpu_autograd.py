"""GPU: the torch.autograd.Function over the rasterizer, against the oracle and finite differences."""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import se3
from tests.gpu_common import check_grads, check_pose, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_00970_amd as p

    return p


def _weights(H, W, seed):
    g = np.random.default_rng(seed)
    return {"rgb": g.normal(size=(3, H, W)) / (H * W), "depth": g.normal(size=(H, W)) / (H * W),
            "normal": g.normal(size=(3, H, W)) / (H * W), "alpha": g.normal(size=(H, W)) / (H * W)}


def _torch_loss(outs, w):
    rgb, depth, normal, alpha = outs
    return ((rgb * dev(w["rgb"])).sum() + (depth * dev(w["depth"])).sum() + (normal * dev(w["normal"])).sum()
            + (alpha * dev(w["alpha"])).sum())


def test_autograd_matches_oracle_at_zero_tau(pkg):
    s = synth.random_surfels(2000, seed=2)
    r = pkg.Rasterizer()
    params = dev(s.params).requires_grad_(True)
    tau = torch.zeros(6, device="cuda:0", requires_grad=True)
    w = _weights(48, 64, 0)
    L = _torch_loss(pkg.render(r, params, tau, dev(s.pose.reshape(12)), s.camera), w)
    L.backward()
    ref = oracle.render(s.params, s.camera, s.pose)
    near = ref["gmargin"] < 1e-5
    og = oracle.backward(s.params, s.camera, s.pose, d_rgb=w["rgb"], d_depth=w["depth"], d_normal=w["normal"],
                         d_alpha=w["alpha"], watch=near, scale=True, scale_mask=near)
    check_grads(host(params.grad), og["d_params"], skip=og["touched"])
    check_pose(host(tau.grad), og["pose_paper"], scale=og["pose_scale"], flip=og["pose_scale_masked"])


def test_autograd_tau_finite_differences(pkg):
    """d L / d tau at tau != 0 against FP64 central differences of the oracle through Exp(tau) T."""
    tau0 = np.array([0.01, -0.02, 0.015, 0.02, -0.03, 0.025])
    # a scene with no decision within 1e-3 (relative) at the evaluation pose, so that
    # the central differences do not straddle a discontinuity
    for seed in range(50, 400):
        s = synth.tiny_scene(seed, n=6)
        o = oracle.render(s.params, s.camera, se3.left_perturb(tau0, s.pose))
        if o["gmargin"].min() > 1e-3 and o["alpha"].max() > 0.3:
            break
    else:
        raise RuntimeError("no clean scene")
    r = pkg.Rasterizer()
    tau = dev(tau0).requires_grad_(True)
    w = _weights(s.camera.height, s.camera.width, 1)
    L = _torch_loss(pkg.render(r, dev(s.params), tau, dev(s.pose.reshape(12)), s.camera), w)
    L.backward()
    g = host(tau.grad)

    def Lo(t):
        o = oracle.render(s.params, s.camera, se3.left_perturb(t, s.pose))
        return (np.sum(o["rgb"] * w["rgb"]) + np.sum(o["depth"] * w["depth"]) + np.sum(o["normal"] * w["normal"])
                + np.sum(o["alpha"] * w["alpha"]))

    fd = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1e-6
        fd[k] = (Lo(tau0 + e) - Lo(tau0 - e)) / 2e-6
    # float32 rounding: the pose scale at Exp(tau0) T pulled back through |J_l(tau0)|^T,
    # J_l by central differences of Exp and Log (its definition)
    T1 = se3.left_perturb(tau0, s.pose)
    ob = oracle.backward(s.params, s.camera, T1, d_rgb=w["rgb"], d_depth=w["depth"], d_normal=w["normal"],
                         d_alpha=w["alpha"], scale=True)
    Einv = np.linalg.inv(se3.exp(tau0))
    J = np.zeros((6, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1e-6
        J[:, k] = (se3.log(se3.exp(tau0 + e) @ Einv) - se3.log(se3.exp(tau0 - e) @ Einv)) / 2e-6
    # central differences in FP64 carry about 1e-9 relative error of their own
    check_pose(g, fd, rel=1e-3, floor=1e-6, scale=np.abs(J).T @ ob["pose_scale"])


def test_autograd_pose_only_and_unused_outputs(pkg):
    """Only rgb used, params frozen: the pose-only path gives the pose gradient of the full path."""
    s = synth.random_surfels(2000, seed=6)
    r = pkg.Rasterizer()
    P = dev(s.params)
    pose = dev(s.pose.reshape(12))
    w = _weights(48, 64, 2)
    tau = torch.zeros(6, device="cuda:0", requires_grad=True)
    rgb, _, _, _ = pkg.render(r, P, tau, pose, s.camera)
    (rgb * dev(w["rgb"])).sum().backward()
    ref = oracle.render(s.params, s.camera, s.pose)
    near = ref["gmargin"] < 1e-5
    og = oracle.backward(s.params, s.camera, s.pose, d_rgb=w["rgb"], scale=True, scale_mask=near)
    check_pose(host(tau.grad), og["pose_paper"], scale=og["pose_scale"], flip=og["pose_scale_masked"])
