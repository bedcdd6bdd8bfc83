"""Losses, their image gradients and the pose update, in plain NumPy (test infrastructure only).

* ``tracking_loss``: the paper's tracking loss (Sec. "Tracking and Keyframe
  Selection", eq:LD, eq:normal_mask, eq:opacity_mask, eq:tracking_loss):
  L_t = (1/|Omega|) sum_p M_n(p) M_o(p) (L_I(p) + lambda_d L_D(p)), with
  L_I the per-pixel L1 distance summed over RGB, L_D the per-pixel depth L1,
  M_n = [N_r . r > 0] (r the pixel's unit ray, camera frame) and
  M_o = [O > 0.95].  |Omega| is every pixel.  Masks are held constant in the
  gradient; the L1 derivative at zero is zero.
* ``image_loss``: the masked, weighted L1 over colour, depth and normal that the
  tracking loss, the single-frame workload's loss and the mapping window's loss are
  instances of.
* ``tracking_error``: the relocalisation check e_t (eq:tracking_error), the masked
  depth L1 of the tracking loss on its own.
* ``frame_loss``: unmasked L1 over colour, depth and normal, averaged over
  pixels (the single-frame random-surfel workload).
* ``adamw_pose_step``: AdamW on the left-perturbation twist, which is reset to
  zero after every step (T <- Exp(tau) T).
"""

from __future__ import annotations

import numpy as np

from . import se3

OPACITY_MASK = 0.95


def _rays(camera):
    t = camera.as_tuple() if hasattr(camera, "as_tuple") else tuple(camera)
    W, H, fx, fy, cx, cy = t
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    return (xs - cx) / fx, (ys - cy) / fy, int(W), int(H)


def masks(normal, alpha, camera, decision_dtype=np.float32):
    """M_n and M_o, both decided in ``decision_dtype``.

    The sign of N . r does not depend on normalising r, so the unnormalised
    ray ((x-cx)/fx, (y-cy)/fy, 1) is used.
    """
    rx, ry, W, H = _rays(camera)
    dt = decision_dtype
    n = np.asarray(normal).astype(dt)
    ndotr = n[0] * rx.astype(dt) + n[1] * ry.astype(dt) + n[2]
    m_n = ndotr > 0
    m_o = np.asarray(alpha).astype(dt) > dt(OPACITY_MASK)
    return m_n, m_o, ndotr


def tracking_loss(rgb, depth, normal, alpha, tgt_rgb, tgt_depth, camera, lambda_d=1.0,
                  use_masks=True, decision_dtype=np.float32):
    """Returns (loss, d_rgb, d_depth, mask) in FP64."""
    rgb = np.asarray(rgb, dtype=np.float64)
    depth = np.asarray(depth, dtype=np.float64)
    _, _, W, H = _rays(camera)
    if use_masks:
        m_n, m_o, _ = masks(normal, alpha, camera, decision_dtype)
        m = (m_n & m_o).astype(np.float64)
    else:
        m = np.ones((H, W))
    dr = rgb - np.asarray(tgt_rgb, dtype=np.float64)
    dd = depth - np.asarray(tgt_depth, dtype=np.float64)
    hw = float(H * W)
    loss = float(np.sum(m * (np.abs(dr).sum(axis=0) + lambda_d * np.abs(dd))) / hw)
    d_rgb = m[None] * np.sign(dr) / hw
    d_depth = lambda_d * m * np.sign(dd) / hw
    return loss, d_rgb, d_depth, m.astype(bool)


def image_loss(rgb, depth, normal, alpha, tgt_rgb, tgt_depth, tgt_normal, camera, w_rgb=1.0, w_d=1.0, w_n=0.0,
               normal_mask=True, opacity_mask=True, decision_dtype=np.float32):
    """(1/|Omega|) sum_p M(p) (w_rgb |d rgb|_1 + w_d |d D| + w_n |d N|_1) with M the
    product of the selected masks (M_n, M_o; none: 1), and its gradients to the three
    rendered images (masks constant, d|x|/dx = 0 at 0).  The tracking loss is
    (1, lambda_d, 0, both masks); the single-frame L1 (1, 1, 1, no masks); the mapping
    window's (1, 0.5, 0, opacity mask only).  Returns (loss, d_rgb, d_depth, d_normal)."""
    _, _, W, H = _rays(camera)
    m = np.ones((H, W), dtype=bool)
    if normal_mask or opacity_mask:
        m_n, m_o, _ = masks(normal, alpha, camera, decision_dtype)
        if normal_mask:
            m &= m_n
        if opacity_mask:
            m &= m_o
    mf = m.astype(np.float64)
    hw = float(H * W)
    dr = np.asarray(rgb, dtype=np.float64) - np.asarray(tgt_rgb, dtype=np.float64)
    dd = np.asarray(depth, dtype=np.float64) - np.asarray(tgt_depth, dtype=np.float64)
    terms = w_rgb * np.abs(dr).sum(axis=0) + w_d * np.abs(dd)
    d_normal = np.zeros((3, H, W))
    if w_n != 0.0:
        dn = np.asarray(normal, dtype=np.float64) - np.asarray(tgt_normal, dtype=np.float64)
        terms = terms + w_n * np.abs(dn).sum(axis=0)
        d_normal = w_n * mf[None] * np.sign(dn) / hw
    loss = float(np.sum(mf * terms) / hw)
    return loss, w_rgb * mf[None] * np.sign(dr) / hw, w_d * mf * np.sign(dd) / hw, d_normal


def tracking_error(depth, normal, alpha, tgt_depth, camera, decision_dtype=np.float32):
    """e_t of eq:tracking_error: (1/|Omega|) sum_p M_n(p) M_o(p) |D_r(p) - D(p)|, the
    masked depth L1 of the rendered depth against the observed one (the relocalisation
    check), with the tracking loss's masks decided in ``decision_dtype``."""
    m_n, m_o, _ = masks(normal, alpha, camera, decision_dtype)
    dd = np.asarray(depth, dtype=np.float64) - np.asarray(tgt_depth, dtype=np.float64)
    return float(np.sum((m_n & m_o) * np.abs(dd)) / dd.size)


def frame_loss(rgb, depth, normal, tgt_rgb, tgt_depth, tgt_normal):
    """Unmasked (1/HW) sum (|d rgb|_1 + |d D| + |d N|_1); returns (loss, d_rgb, d_depth, d_normal)."""
    rgb = np.asarray(rgb, dtype=np.float64)
    H, W = rgb.shape[1:]
    hw = float(H * W)
    dr = rgb - np.asarray(tgt_rgb, dtype=np.float64)
    dd = np.asarray(depth, dtype=np.float64) - np.asarray(tgt_depth, dtype=np.float64)
    dn = np.asarray(normal, dtype=np.float64) - np.asarray(tgt_normal, dtype=np.float64)
    loss = float((np.abs(dr).sum() + np.abs(dd).sum() + np.abs(dn).sum()) / hw)
    return loss, np.sign(dr) / hw, np.sign(dd) / hw, np.sign(dn) / hw


class AdamState:
    def __init__(self):
        self.m = np.zeros(6)
        self.v = np.zeros(6)
        self.t = 0


def adamw_pose_step(pose, grad, state: AdamState, lr, betas=(0.9, 0.999), eps=1e-8,
                    weight_decay=0.0):
    """One AdamW step on tau (which is zero before the step); returns Exp(tau) T (3x4)."""
    g = np.asarray(grad, dtype=np.float64)
    lr = np.broadcast_to(np.asarray(lr, dtype=np.float64), (6,))
    b1, b2 = betas
    state.t += 1
    state.m = b1 * state.m + (1 - b1) * g
    state.v = b2 * state.v + (1 - b2) * g * g
    mhat = state.m / (1 - b1 ** state.t)
    vhat = state.v / (1 - b2 ** state.t)
    tau = -lr * mhat / (np.sqrt(vhat) + eps)  # decoupled decay acts on tau = 0: no effect
    del weight_decay
    return se3.left_perturb(tau, pose), tau
