"""PyTorch-facing binding of the mapping loss (include/gs2d_map.h, gs2d_mapping_loss).

The loss and its image gradients run in libgs2d.so; this module only checks and
marshals arguments.  Tensors are CUDA tensors on one device, used on torch's current
stream.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib
from .mapstate import _check, _stream
from .rasterizer import _camera, _dev_ptr

DEFAULT_WEIGHTS = (0.875, 0.125, 0.5, 0.02)  # w_l1, w_ssim, w_d, w_n


def mapping_loss(rgb, depth, normal, tgt_rgb, tgt_depth, camera, weights=DEFAULT_WEIGHTS):
    """L_m of one view and its gradients to the rendered images.

    Returns (loss [5] = (L_m, mean |d rgb|_1, mean 1 - SSIM, mean |d depth|, mean
    1 - N_D . N), d_rgb [3, H, W], d_depth [H, W], d_normal [3, H, W]), all device tensors.
    """
    cam = _camera(camera)
    H, W = cam.height, cam.width
    dev = rgb.device
    for t, name, shape in ((rgb, "rgb", (3, H, W)), (depth, "depth", (H, W)), (normal, "normal", (3, H, W)),
                           (tgt_rgb, "tgt_rgb", (3, H, W)), (tgt_depth, "tgt_depth", (H, W))):
        _check(t, name, shape, torch.float32, dev)
    lib = _lib.load()
    w = _lib.MappingWeights(*[float(v) for v in weights])
    work = torch.empty(lib.gs2d_mapping_loss_workspace(W, H), dtype=torch.float32, device=dev)
    loss = torch.empty(5, dtype=torch.float32, device=dev)
    d_rgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    d_depth = torch.empty((H, W), dtype=torch.float32, device=dev)
    d_normal = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    _lib.check(lib.gs2d_mapping_loss(ctypes.byref(cam), _dev_ptr(rgb), _dev_ptr(depth), _dev_ptr(normal),
                                     _dev_ptr(tgt_rgb), _dev_ptr(tgt_depth), ctypes.byref(w), _dev_ptr(loss),
                                     _dev_ptr(d_rgb), _dev_ptr(d_depth), _dev_ptr(d_normal), _dev_ptr(work),
                                     _stream(dev)))
    return loss, d_rgb, d_depth, d_normal
