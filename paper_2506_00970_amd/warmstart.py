"""PyTorch-facing binding of the learned pose warm start (include/gs2d_warm.h).

The network, its training step and the warm start itself run in libgs2d.so;
this module only checks and marshals arguments.  Inputs and outputs are CUDA
float32 tensors on the network's device, used on torch's current stream.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .rasterizer import Rasterizer, _camera, _check_tensor, _dev_ptr

PARAMS = 900_326
IN_SHAPE = (4, 60, 80)
RHO_SCALE = 0.1
PHI_SCALE = float(np.deg2rad(8.0))


class WarmStartNet:
    """The BF16 warm-start network with FP32 master weights and AdamW state."""

    def __init__(self, device: int | str | torch.device = 0, max_batch: int = 256):
        lib = _lib.load()
        idx = device if isinstance(device, int) else (torch.device(device).index or 0)
        self.device = torch.device("cuda", idx)
        self.max_batch = int(max_batch)
        net = ctypes.c_void_p()
        _lib.check(lib.gs2d_ws_create(ctypes.byref(net), idx, self.max_batch))
        self._net = net
        self._lib = lib

    def close(self):
        if getattr(self, "_net", None):
            self._lib.gs2d_ws_destroy(self._net)
            self._net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _batch(self, t, name, tail):
        if t.dim() != len(tail) + 1:
            raise ValueError(f"{name} must have shape [B, {', '.join(map(str, tail))}]")
        B = t.shape[0]
        if not 1 <= B <= self.max_batch:
            raise ValueError(f"batch {B} outside 1..{self.max_batch}")
        _check_tensor(t, name, (B,) + tuple(tail), self.device)
        return B

    def set_params(self, theta: torch.Tensor) -> None:
        _check_tensor(theta, "theta", (PARAMS,), self.device)
        _lib.check(self._lib.gs2d_ws_set_params(self._net, _dev_ptr(theta), self._stream()))

    def params(self) -> torch.Tensor:
        out = torch.empty(PARAMS, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.gs2d_ws_get_params(self._net, _dev_ptr(out), self._stream()))
        return out

    def residual(self, rgb, depth, tgt_rgb, tgt_depth) -> torch.Tensor:
        """Network inputs [B, 4, 60, 80] from rendered and observed frames ([B, 3, H, W], [B, H, W])."""
        if rgb.dim() == 3:
            rgb, depth, tgt_rgb, tgt_depth = (x.unsqueeze(0) for x in (rgb, depth, tgt_rgb, tgt_depth))
        B, _, H, W = rgb.shape
        for t, n, sh in ((rgb, "rgb", (B, 3, H, W)), (depth, "depth", (B, H, W)), (tgt_rgb, "tgt_rgb", (B, 3, H, W)),
                         (tgt_depth, "tgt_depth", (B, H, W))):
            _check_tensor(t, n, sh, self.device)
        out = torch.empty((B,) + IN_SHAPE, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.gs2d_ws_residual(_dev_ptr(rgb), _dev_ptr(depth), _dev_ptr(tgt_rgb), _dev_ptr(tgt_depth),
                                              W, H, B, _dev_ptr(out), self._stream()))
        return out

    def forward(self, inp: torch.Tensor) -> torch.Tensor:
        """Normalised twists [B, 6]."""
        B = self._batch(inp, "input", IN_SHAPE)
        out = torch.empty((B, 6), dtype=torch.float32, device=self.device)
        _lib.check(self._lib.gs2d_ws_forward(self._net, _dev_ptr(inp), B, _dev_ptr(out), self._stream()))
        return out

    def gradient(self, inp: torch.Tensor, target: torch.Tensor, want_grad: bool = True):
        """(loss [1], out [B, 6], dL/dtheta [PARAMS] or None) of the mean squared error."""
        B = self._batch(inp, "input", IN_SHAPE)
        _check_tensor(target, "target", (B, 6), self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        out = torch.empty((B, 6), dtype=torch.float32, device=self.device)
        grad = torch.empty(PARAMS, dtype=torch.float32, device=self.device) if want_grad else None
        _lib.check(self._lib.gs2d_ws_gradient(self._net, _dev_ptr(inp), _dev_ptr(target), B, _dev_ptr(loss),
                                              _dev_ptr(out), _dev_ptr(grad), self._stream()))
        return loss, out, grad

    def adamw_step(self, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8, weight_decay: float = 0.01):
        o = _lib.WsAdamW(float(lr), float(betas[0]), float(betas[1]), float(eps), float(weight_decay))
        _lib.check(self._lib.gs2d_ws_adamw_step(self._net, ctypes.byref(o), self._stream()))

    def train_step(self, inp, target, **adamw) -> torch.Tensor:
        loss, _, _ = self.gradient(inp, target, want_grad=False)
        self.adamw_step(**adamw)
        return loss

    def warm_start(self, rast: Rasterizer, params, camera, pose_start, tgt_rgb, tgt_depth, lambda_d: float = 1.0,
                   use_masks: bool = False):
        """(chosen pose [12], info [4] = loss at T_start, loss at T_0, 1 if T_0 kept, 0).

        The fallback compares unmasked tracking losses by default: a proposal that sees
        nothing has a masked loss of 0."""
        if rast.device != self.device:
            raise ValueError("the rasterizer and the network must share a device")
        cam = _camera(camera)
        n = params.shape[1]
        _check_tensor(params, "params", (15, n), self.device)
        _check_tensor(pose_start, "pose_start", (12,), self.device)
        _check_tensor(tgt_rgb, "tgt_rgb", (3, cam.height, cam.width), self.device)
        _check_tensor(tgt_depth, "tgt_depth", (cam.height, cam.width), self.device)
        pose = torch.empty(12, dtype=torch.float32, device=self.device)
        info = torch.empty(4, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.gs2d_warm_start(rast._ctx, self._net, _dev_ptr(params), n, ctypes.byref(cam),
                                             _dev_ptr(pose_start), _dev_ptr(tgt_rgb), _dev_ptr(tgt_depth),
                                             float(lambda_d), 1 if use_masks else 0, _dev_ptr(pose),
                                             _dev_ptr(info), self._stream()), rast._ctx)
        return pose, info

    def propose(self, rast: Rasterizer, params, camera, pose_start, tgt_rgb, tgt_depth, lambda_d: float = 1.0):
        """(T_0 [12], unmasked tracking loss at T_start [1]): the warm start without its
        render at T_0.  Track from T_0 with ``fallback=(pose_start, loss)``; the first
        tracking iteration then falls back to T_start if T_0 is worse."""
        if rast.device != self.device:
            raise ValueError("the rasterizer and the network must share a device")
        cam = _camera(camera)
        n = params.shape[1]
        _check_tensor(params, "params", (15, n), self.device)
        _check_tensor(pose_start, "pose_start", (12,), self.device)
        _check_tensor(tgt_rgb, "tgt_rgb", (3, cam.height, cam.width), self.device)
        _check_tensor(tgt_depth, "tgt_depth", (cam.height, cam.width), self.device)
        pose = torch.empty(12, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.gs2d_warm_start_propose(rast._ctx, self._net, _dev_ptr(params), n, ctypes.byref(cam),
                                                     _dev_ptr(pose_start), _dev_ptr(tgt_rgb), _dev_ptr(tgt_depth),
                                                     float(lambda_d), _dev_ptr(pose), _dev_ptr(loss),
                                                     self._stream()), rast._ctx)
        return pose, loss


def denormalise(out: torch.Tensor) -> torch.Tensor:
    """Network output -> twist (rho in metres, phi in radians)."""
    return torch.cat([out[..., :3] * RHO_SCALE, out[..., 3:] * PHI_SCALE], dim=-1)


def normalise(tau: torch.Tensor) -> torch.Tensor:
    return torch.cat([tau[..., :3] / RHO_SCALE, tau[..., 3:] / PHI_SCALE], dim=-1)
