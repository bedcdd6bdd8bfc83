"""The learned pose warm start, in plain FP64 NumPy (test infrastructure only).

Not a step of the paper: this is the learned extension of the tracking front end
(the paper's tracking, Sec. "Tracking and Keyframe Selection", starts from the
previous pose and iterates).  A small network looks at the residual between
the frame rendered at the start pose and the observed RGB-D frame and proposes
a left-perturbation twist tau_hat (the same se(3) convention as the pose
gradient of eq:derivatives), so that T_0 = Exp(tau_hat) T_start.

Network, as defined for this project (every size fixed):

* input: the residual (rendered - observed) of R, G, B and depth, each the mean
  over 8 x 8 pixel blocks: 4 x 60 x 80 for a 640 x 480 frame;
* conv 4->32 k5, 32->64 k3, 64->128 k3, 128->128 k3, all stride 2 with zero
  padding k // 2, each followed by ReLU: 128 x 4 x 5;
* fully connected 2560 -> 256 (ReLU) -> 6;
* the 6 outputs are the twist normalised component-wise: rho / 0.1 m and
  phi / (8 deg in radians).

Precision, as the network defines it: weights and activations are bfloat16
(the stored copies of FP32 master weights; every layer's output, and every
layer's input gradient, rounded to bfloat16 with round-to-nearest-even), the
sums are exact here (FP64) where the GPU accumulates in FP32, biases are FP32,
and the last layer's output and all weight gradients stay unrounded.
``rounding=False`` turns every bfloat16 rounding off (the exact network, used
to pin the gradients against finite differences).

Tensor layouts: activations [B][C][H][W]; conv weights [Co][Ci][k][k]; linear
weights [O][I]; the flat parameter vector concatenates, layer by layer, the
weight then the bias.
"""

from __future__ import annotations

import numpy as np

IN_C, IN_H, IN_W = 4, 60, 80
CONVS = ((4, 32, 5), (32, 64, 3), (64, 128, 3), (128, 128, 3))  # (ci, co, k), stride 2
FCS = ((2560, 256), (256, 6))
RHO_SCALE = 0.1                  # metres
PHI_SCALE = np.deg2rad(8.0)      # radians
BLOCK = 8                        # residual downsampling block (pixels)


def param_shapes():
    """[(weight shape, bias shape)] per layer, in order."""
    out = [((co, ci, k, k), (co,)) for ci, co, k in CONVS]
    out += [((o, i), (o,)) for i, o in FCS]
    return out


def param_count() -> int:
    return int(sum(np.prod(w) + np.prod(b) for w, b in param_shapes()))


def unflatten(theta):
    """Split the flat parameter vector into [(W, b)] per layer."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb].reshape(bs)))
        o += nw + nb
    assert o == theta.size
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([np.ravel(w), np.ravel(b)]) for w, b in layers])


def bf16_round(x):
    """Round to the nearest bfloat16 value (8 significant bits), ties to even.

    frexp gives x = m 2^e with 0.5 <= |m| < 1, so m 2^8 holds the 8 significant
    bits in its integer part; numpy's round is round-half-to-even.
    """
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.round(m * 256.0), e - 8)


def downsample(res, block: int = BLOCK):
    """[C][H][W] -> [C][H/block][W/block], the mean of each block x block patch."""
    res = np.asarray(res, dtype=np.float64)
    C, H, W = res.shape
    assert H % block == 0 and W % block == 0
    out = np.zeros((C, H // block, W // block))
    for dy in range(block):
        for dx in range(block):
            out += res[:, dy::block, dx::block]
    return out / (block * block)


def residual_input(rgb, depth, tgt_rgb, tgt_depth):
    """Network input for one frame: downsampled (rendered - observed) of R, G, B, D."""
    res = np.concatenate([np.asarray(rgb, np.float64) - np.asarray(tgt_rgb, np.float64),
                          (np.asarray(depth, np.float64) - np.asarray(tgt_depth, np.float64))[None]])
    return downsample(res)


# --- layers (definitions written out) ---------------------------------------------


def _out_size(n, k, stride=2):
    return (n + 2 * (k // 2) - k) // stride + 1


def im2col(x, k, stride=2):
    """[B][C][H][W] -> [B][C k k][OH OW]: column (oy, ox) holds the zero-padded
    k x k patch whose top-left input pixel is (stride oy - k//2, stride ox - k//2)."""
    B, C, H, W = x.shape
    p = k // 2
    OH, OW = _out_size(H, k, stride), _out_size(W, k, stride)
    xp = np.zeros((B, C, H + 2 * p + stride, W + 2 * p + stride))
    xp[:, :, p:p + H, p:p + W] = x
    cols = np.empty((B, C, k, k, OH, OW))
    for ky in range(k):
        for kx in range(k):
            cols[:, :, ky, kx] = xp[:, :, ky:ky + stride * OH:stride, kx:kx + stride * OW:stride]
    return cols.reshape(B, C * k * k, OH * OW), (OH, OW)


def col2im(cols, shape, k, stride=2):
    """Adjoint of im2col: scatter-add the patches back onto a [B][C][H][W] image."""
    B, C, H, W = shape
    p = k // 2
    OH, OW = _out_size(H, k, stride), _out_size(W, k, stride)
    cols = cols.reshape(B, C, k, k, OH, OW)
    xp = np.zeros((B, C, H + 2 * p + stride, W + 2 * p + stride))
    for ky in range(k):
        for kx in range(k):
            xp[:, :, ky:ky + stride * OH:stride, kx:kx + stride * OW:stride] += cols[:, :, ky, kx]
    return xp[:, :, p:p + H, p:p + W]


def conv2d(x, w, b, stride=2):
    """y[b, co, oy, ox] = b[co] + sum_{ci,ky,kx} w[co,ci,ky,kx] x[b, ci, s oy + ky - k//2, s ox + kx - k//2]."""
    co, ci, k, _ = w.shape
    cols, (OH, OW) = im2col(x, k, stride)
    y = np.einsum("ok,bkn->bon", w.reshape(co, ci * k * k), cols) + b[None, :, None]
    return y.reshape(x.shape[0], co, OH, OW)


def conv2d_backward(x, w, dy, stride=2):
    """(dx, dw, db) of conv2d for the output gradient dy."""
    co, ci, k, _ = w.shape
    B = x.shape[0]
    cols, _ = im2col(x, k, stride)
    dyf = dy.reshape(B, co, -1)
    dw = np.einsum("bon,bkn->ok", dyf, cols).reshape(w.shape)
    db = dyf.sum(axis=(0, 2))
    dcols = np.einsum("ok,bon->bkn", w.reshape(co, -1), dyf)
    dx = col2im(dcols, x.shape, k, stride)
    return dx, dw, db


def linear(x, w, b):
    return x @ w.T + b[None]


def linear_backward(x, w, dy):
    return dy @ w, dy.T @ x, dy.sum(axis=0)


# --- the network ------------------------------------------------------------------


def forward(theta, x, rounding: bool = True):
    """Normalised twist [B][6] for inputs x [B][4][60][80]; also the saved activations."""
    r = bf16_round if rounding else (lambda v: np.asarray(v, np.float64))
    layers = unflatten(theta)
    a = r(x)
    acts = [a]
    for (w, b), _ in zip(layers[:4], CONVS):
        a = r(np.maximum(conv2d(a, r(w), b), 0.0))
        acts.append(a)
    h = a.reshape(a.shape[0], -1)
    (w1, b1), (w2, b2) = layers[4], layers[5]
    h1 = r(np.maximum(linear(h, r(w1), b1), 0.0))
    acts.append(h1)
    out = linear(h1, r(w2), b2)
    return out, acts


def loss_and_grad(out, target):
    """Mean squared error over the batch and the 6 normalised components, and dL/dout."""
    d = np.asarray(out, np.float64) - np.asarray(target, np.float64)
    n = d.size
    return float((d * d).sum() / n), 2.0 * d / n


def backward(theta, acts, dout, rounding: bool = True):
    """Flat gradient of the parameters for dL/dout [B][6], through the saved activations."""
    r = bf16_round if rounding else (lambda v: np.asarray(v, np.float64))
    layers = unflatten(theta)
    grads = [None] * 6
    (w1, _), (w2, _) = layers[4], layers[5]
    h1 = acts[5]
    g = r(dout)
    dh1, dw2, db2 = linear_backward(h1, r(w2), g)
    grads[5] = (dw2, db2)
    g = r(dh1 * (h1 > 0))
    h = acts[4].reshape(acts[4].shape[0], -1)
    dh, dw1, db1 = linear_backward(h, r(w1), g)
    grads[4] = (dw1, db1)
    g = r(dh.reshape(acts[4].shape) * (acts[4] > 0))
    for li in range(3, -1, -1):
        w, _ = layers[li]
        dx, dw, db = conv2d_backward(acts[li], r(w), g)
        grads[li] = (dw, db)
        if li > 0:
            g = r(dx * (acts[li] > 0))
    return flatten(grads)


def denormalise(out):
    """Network output -> twist (rho in metres, phi in radians)."""
    out = np.asarray(out, np.float64)
    return np.concatenate([out[..., :3] * RHO_SCALE, out[..., 3:] * PHI_SCALE], axis=-1)


def normalise(tau):
    tau = np.asarray(tau, np.float64)
    return np.concatenate([tau[..., :3] / RHO_SCALE, tau[..., 3:] / PHI_SCALE], axis=-1)


class AdamWState:
    def __init__(self, n):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0


def adamw_step(theta, grad, state: AdamWState, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01):
    """One AdamW step (decoupled weight decay, bias-corrected moments) on the master weights."""
    b1, b2 = betas
    state.t += 1
    state.m = b1 * state.m + (1 - b1) * grad
    state.v = b2 * state.v + (1 - b2) * grad * grad
    mh = state.m / (1 - b1 ** state.t)
    vh = state.v / (1 - b2 ** state.t)
    return theta * (1 - lr * weight_decay) - lr * mh / (np.sqrt(vh) + eps)
