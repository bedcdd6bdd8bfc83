"""CPU pins of the oracle's Adam step over surfel parameters (oracle/optim.py):
closed forms of the first step and of a constant gradient, decoupled weight decay
alone, the group learning rates, and the clamps."""

import numpy as np
import pytest

from oracle import optim

LR = (1e-3, 2e-3, 3e-3, 4e-3, 5e-3, 6e-3)


def test_first_step_is_lr_times_sign():
    """m_hat = g and v_hat = g^2 after one step: p -= lr g / (|g| + eps)."""
    g = np.random.default_rng(0).standard_normal((15, 50))
    p0 = np.random.default_rng(1).uniform(0.1, 0.9, (15, 50))
    p, m, v = optim.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, LR, eps=1e-8)
    lr_row = np.array([LR[optim.GROUP_OF_ROW[r]] for r in range(15)])[:, None]
    want = p0 - lr_row * g / (np.abs(g) + 1e-8)
    want[9:11] = np.maximum(want[9:11], 0.0)
    want[11] = np.clip(want[11], 0.0, 1.0)
    np.testing.assert_allclose(p, want, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_constant_gradient_moves_linearly():
    """With the same g every step, m_hat = g and v_hat = g^2 at every t (bias-corrected):
    k steps move every parameter by k lr g / (|g| + eps)."""
    g = np.full((15, 3), 0.25)
    g[:, 1] = -0.5
    p = np.full((15, 3), 10.0)  # far from the clamps
    m = np.zeros_like(g)
    v = np.zeros_like(g)
    for t in range(1, 8):
        p, m, v = optim.adam_step(p, g, m, v, t, LR, eps=0.0)
    lr_row = np.array([LR[optim.GROUP_OF_ROW[r]] for r in range(15)])[:, None]
    want = 10.0 - 7 * lr_row * np.sign(g)
    # the opacity row is clamped to 1 after the first step, then moves from there
    want[11] = np.where(g[11] > 0, 1.0 - 6 * LR[4], 1.0)
    np.testing.assert_allclose(p, want, rtol=1e-12)


def test_weight_decay_alone_and_zero_gradient():
    p0 = np.full((15, 4), 0.5)
    p, _, _ = optim.adam_step(p0, np.zeros((15, 4)), np.zeros((15, 4)), np.zeros((15, 4)), 3, LR)
    np.testing.assert_array_equal(p, p0)
    p, _, _ = optim.adam_step(p0, np.zeros((15, 4)), np.zeros((15, 4)), np.zeros((15, 4)), 3, LR, weight_decay=0.1)
    lr_row = np.array([LR[optim.GROUP_OF_ROW[r]] for r in range(15)])[:, None]
    np.testing.assert_allclose(p, np.broadcast_to(0.5 * (1.0 - 0.1 * lr_row), p.shape), rtol=1e-15)


def test_clamps():
    p0 = np.zeros((15, 2))
    p0[9:11] = 0.001
    p0[11] = [0.999, 0.001]
    g = np.zeros((15, 2))
    g[9:11] = 1.0        # scales pushed down past s_min
    g[11] = [-1.0, 1.0]  # opacity pushed up past o_max, down past o_min
    p, _, _ = optim.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, (0.01,) * 6, s_min=1e-4, o_min=0.005,
                              o_max=0.99)
    np.testing.assert_array_equal(p[9:11], 1e-4)
    assert p[11, 0] == 0.99 and p[11, 1] == 0.005
