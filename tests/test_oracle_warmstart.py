"""Pins of the warm-start oracle (oracle/warmstart.py) against things other than itself.

* bfloat16 rounding: hand-worked ties and torch's own float32 -> bfloat16 conversion;
* convolution: scipy.signal.correlate2d on the zero-padded image, subsampled by the stride;
* backward: the adjoint identity <conv(x), y> = <x, conv^T(y)>, and central finite
  differences of the whole network (rounding off) on sampled parameters;
* sizes: the 128 x 4 x 5 code of a 60 x 80 input and the parameter count;
* downsampling: a linear ramp's block means are the ramp at the block centres;
* AdamW: the closed-form first step.
"""

import numpy as np
import pytest
import scipy.signal
import torch

from oracle import warmstart as ws


def test_bf16_round_hand_worked():
    one = 1.0
    ulp = 2.0 ** -7  # bfloat16 spacing in [1, 2)
    cases = {
        one: one,
        one + ulp: one + ulp,
        one + 0.5 * ulp: one,                   # tie -> even (1.0)
        one + 1.5 * ulp: one + 2 * ulp,         # tie -> even (mantissa 2)
        one + 0.49 * ulp: one,
        one + 0.51 * ulp: one + ulp,
        -3.0 - 0.5 * 2 * ulp: -3.0,             # in [2, 4) the spacing is 2 ulp; tie -> even
        0.0: 0.0,
        2.0 ** -100 * (1 + 0.75 * ulp): 2.0 ** -100 * (1 + ulp),
    }
    for x, want in cases.items():
        assert ws.bf16_round(x) == want, (x, ws.bf16_round(x), want)


def test_bf16_round_matches_torch():
    g = np.random.default_rng(0)
    x = (g.normal(size=20000) * 10.0 ** g.uniform(-6, 6, size=20000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ws.bf16_round(x.astype(np.float64)), ref)


@pytest.mark.parametrize("k", [3, 5])
def test_conv_matches_scipy_correlate(k):
    g = np.random.default_rng(k)
    B, ci, co, H, W = 2, 3, 4, 11, 14
    x = g.normal(size=(B, ci, H, W))
    w = g.normal(size=(co, ci, k, k))
    b = g.normal(size=co)
    y = ws.conv2d(x, w, b)
    p = k // 2
    for bi in range(B):
        for o in range(co):
            acc = np.zeros((H, W))
            for c in range(ci):
                xp = np.pad(x[bi, c], p)
                acc += scipy.signal.correlate2d(xp, w[o, c], mode="valid")
            ref = acc[::2, ::2] + b[o]
            np.testing.assert_allclose(y[bi, o], ref, rtol=1e-12, atol=1e-12)


def test_conv_backward_adjoint_and_bias():
    g = np.random.default_rng(3)
    x = g.normal(size=(2, 3, 9, 12))
    w = g.normal(size=(5, 3, 3, 3))
    b = np.zeros(5)
    y = ws.conv2d(x, w, b)
    dy = g.normal(size=y.shape)
    dx, dw, db = ws.conv2d_backward(x, w, dy)
    # <conv(x), dy> is linear in x and in w: its gradients are dx and dw
    assert np.isclose((y * dy).sum(), (x * dx).sum(), rtol=1e-12)
    assert np.isclose((y * dy).sum(), (w * dw).sum(), rtol=1e-12)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 2, 3)), rtol=1e-12)


def test_sizes_and_parameter_count():
    assert ws.param_count() == 900_326
    theta = np.random.default_rng(0).normal(size=ws.param_count()) * 0.01
    out, acts = ws.forward(theta, np.zeros((2, 4, 60, 80)))
    assert out.shape == (2, 6)
    assert acts[4].shape == (2, 128, 4, 5) and acts[5].shape == (2, 256)


def test_downsample_ramp():
    H, W = 48, 64
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    img = np.stack([2.0 * xs + 3.0 * ys, -xs + 0.5, np.full((H, W), 7.0)])
    d = ws.downsample(img)
    cy = np.arange(H // 8)[:, None] * 8 + 3.5
    cx = np.arange(W // 8)[None, :] * 8 + 3.5
    np.testing.assert_allclose(d[0], 2 * cx + 3 * cy, rtol=1e-14)
    np.testing.assert_allclose(d[1], np.broadcast_to(-cx + 0.5, d[1].shape), rtol=1e-14)
    np.testing.assert_allclose(d[2], 7.0, rtol=1e-14)


def _init(seed):
    g = np.random.default_rng(seed)
    layers = []
    for ws_, bs in ws.param_shapes():
        fan_in = int(np.prod(ws_[1:]))
        layers.append((g.uniform(-1, 1, ws_) * np.sqrt(6.0 / fan_in), g.normal(size=bs) * 0.1))
    return ws.flatten(layers)


def test_network_gradient_finite_differences():
    """FP64 central differences of L(theta) on sampled parameters of every layer."""
    theta = _init(1)
    g = np.random.default_rng(2)
    x = g.normal(size=(2, 4, 60, 80)) * 0.3
    target = g.normal(size=(2, 6))
    out, acts = ws.forward(theta, x, rounding=False)
    L, dout = ws.loss_and_grad(out, target)
    grad = ws.backward(theta, acts, dout, rounding=False)
    offs = np.cumsum([0] + [int(np.prod(a)) + int(np.prod(b)) for a, b in ws.param_shapes()])
    h = 1e-6
    checked = 0
    for li in range(6):
        idx = g.integers(offs[li], offs[li + 1], size=6)
        for i in idx:
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            Lp = ws.loss_and_grad(ws.forward(tp, x, rounding=False)[0], target)[0]
            Lm = ws.loss_and_grad(ws.forward(tm, x, rounding=False)[0], target)[0]
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), 1e-3), (li, i, fd, grad[i])
            checked += 1
    assert checked == 36


def test_rounding_points_change_little():
    """The bfloat16 network stays within bfloat16 noise of the exact one."""
    theta = _init(4)
    x = np.random.default_rng(5).normal(size=(3, 4, 60, 80)) * 0.3
    exact = ws.forward(theta, x, rounding=False)[0]
    rounded = ws.forward(theta, x, rounding=True)[0]
    assert np.abs(rounded - exact).max() <= 0.05 * np.abs(exact).max()
    assert not np.array_equal(rounded, exact)


def test_adamw_first_step_closed_form():
    theta = np.array([1.0, -2.0, 0.5])
    grad = np.array([0.3, -1e-3, 0.0])
    st = ws.AdamWState(3)
    lr, wd = 1e-3, 0.01
    new = ws.adamw_step(theta, grad, st, lr=lr, weight_decay=wd, eps=1e-8)
    # first step: m_hat = g, v_hat = g^2, so the update is lr g / (|g| + eps)
    want = theta * (1 - lr * wd) - lr * grad / (np.abs(grad) + 1e-8)
    np.testing.assert_allclose(new, want, rtol=1e-12)


def test_label_is_the_inverse_twist():
    """T_start = Exp(tau) T_gt  =>  Log(T_gt T_start^-1) = -tau."""
    from oracle import se3

    g = np.random.default_rng(6)
    for _ in range(5):
        tau = np.concatenate([g.normal(size=3) * 0.05, g.normal(size=3) * 0.08])
        T = se3.exp(np.concatenate([g.normal(size=3), g.normal(size=3) * 0.5]))
        Ts = se3.exp(tau) @ T
        lab = se3.log(T @ np.linalg.inv(Ts))
        np.testing.assert_allclose(lab, -tau, atol=1e-12)
