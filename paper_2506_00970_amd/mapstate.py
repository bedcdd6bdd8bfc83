"""PyTorch-facing binding of the map bookkeeping (include/gs2d_map.h).

Covisibility and the keyframe test, contribution pruning with stable compaction, the
per-splat map state update and map correction all run in libgs2d.so; this module
only checks and marshals arguments.  Tensors are CUDA tensors on one device, used on
torch's current stream.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib
from .rasterizer import _check_tensor, _dev_ptr

VISIBLE = 0.5     # visible when the contribution exceeds 0.5
COVIS_KF = 0.9    # c_k
DIST_KF = 0.15    # d_k (metres)
PRUNE = 0.5


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check(t, name, shape, dtype, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _vec(t, name, n, dtype, device):
    _check(t, name, (n,), dtype, device)


def covisibility_counts(contrib_a: torch.Tensor, contrib_b: torch.Tensor, threshold: float = VISIBLE):
    """Device int32 tensor [2] holding the uint32 counts (|G_A & G_B|, |G_A | G_B|)."""
    n = contrib_a.shape[0]
    _vec(contrib_a, "contrib_a", n, torch.float32, contrib_a.device)
    _vec(contrib_b, "contrib_b", n, torch.float32, contrib_a.device)
    lib = _lib.load()
    counts = torch.empty(2, dtype=torch.int32, device=contrib_a.device)
    work = torch.empty(lib.gs2d_covisibility_workspace(n), dtype=torch.int32, device=contrib_a.device)
    _lib.check(lib.gs2d_covisibility(_dev_ptr(contrib_a), _dev_ptr(contrib_b), n, float(threshold),
                                     _dev_ptr(counts), _dev_ptr(work), _stream(contrib_a.device)))
    return counts


def covisibility(contrib_a, contrib_b, threshold: float = VISIBLE) -> float:
    c = covisibility_counts(contrib_a, contrib_b, threshold).cpu().numpy().view("uint32")
    return float(c[0]) / float(c[1]) if c[1] else 0.0


def keyframe_test(counts: torch.Tensor, pose_cur: torch.Tensor, pose_kf: torch.Tensor, c_k: float = COVIS_KF,
                  d_k: float = DIST_KF) -> torch.Tensor:
    """Device int32 [1]: 1 when the current frame is a keyframe."""
    dev = counts.device
    _check(counts, "counts", (2,), torch.int32, dev)
    pose_cur, pose_kf = pose_cur.reshape(12), pose_kf.reshape(12)
    _check_tensor(pose_cur, "pose_cur", (12,), dev)
    _check_tensor(pose_kf, "pose_kf", (12,), dev)
    out = torch.empty(1, dtype=torch.int32, device=dev)
    _lib.check(_lib.load().gs2d_keyframe_test(_dev_ptr(counts), _dev_ptr(pose_cur), _dev_ptr(pose_kf), float(c_k),
                                              float(d_k), _dev_ptr(out), _stream(dev)))
    return out


def prune_mask(contrib: torch.Tensor, closest_frame: torch.Tensor, frame: int, threshold: float = PRUNE):
    """Device uint8 [n]: 1 for the splats to remove."""
    n = contrib.shape[0]
    _vec(contrib, "contrib", n, torch.float32, contrib.device)
    _vec(closest_frame, "closest_frame", n, torch.int32, contrib.device)
    out = torch.empty(n, dtype=torch.uint8, device=contrib.device)
    _lib.check(_lib.load().gs2d_prune_mask(_dev_ptr(contrib), _dev_ptr(closest_frame), int(frame), float(threshold),
                                           n, _dev_ptr(out), _stream(contrib.device)))
    return out


def compact(planes: torch.Tensor, remove: torch.Tensor | None):
    """Keep the columns of planes [k, n] (32-bit) with remove == 0, in order.

    Returns (out [k, n] with the kept columns in front, kept count as a device tensor)."""
    if planes.element_size() != 4 or planes.dim() != 2 or not planes.is_contiguous():
        raise ValueError("planes must be a contiguous [k, n] tensor of 32-bit values")
    k, n = planes.shape
    dev = planes.device
    if remove is not None:
        _vec(remove, "remove", n, torch.uint8, dev)
    lib = _lib.load()
    work = torch.empty(max(1, lib.gs2d_compact_workspace(n)), dtype=torch.int32, device=dev)
    out = torch.empty_like(planes)
    n_out = torch.empty(1, dtype=torch.int32, device=dev)
    _lib.check(lib.gs2d_compact(_dev_ptr(planes), n, k, n, _dev_ptr(remove), _dev_ptr(out), n, _dev_ptr(n_out),
                                _dev_ptr(work), _stream(dev)))
    return out, n_out


class MapState:
    """Per-splat map state of eq:map: closest frame and distance, last frame, active."""

    def __init__(self, n: int, device):
        self.t_closest = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.d_closest = torch.full((n,), float("inf"), dtype=torch.float32, device=device)
        self.t_last = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.active = torch.ones(n, dtype=torch.int32, device=device)

    def update(self, params: torch.Tensor, contrib: torch.Tensor, pose_kf: torch.Tensor, frame: int,
               inactive_after: int, loop_frame: int | None = None) -> None:
        n = params.shape[1]
        dev = params.device
        _check_tensor(params, "params", (15, n), dev)
        _vec(contrib, "contrib", n, torch.float32, dev)
        pose_kf = pose_kf.reshape(12)
        _check_tensor(pose_kf, "pose_kf", (12,), dev)
        for nm in ("t_closest", "t_last", "active"):
            _vec(getattr(self, nm), nm, n, torch.int32, dev)
        _vec(self.d_closest, "d_closest", n, torch.float32, dev)
        _lib.check(_lib.load().gs2d_map_state_update(
            _dev_ptr(params), n, _dev_ptr(contrib), _dev_ptr(pose_kf), int(frame), int(inactive_after),
            -1 if loop_frame is None else int(loop_frame), _dev_ptr(self.t_closest), _dev_ptr(self.d_closest),
            _dev_ptr(self.t_last), _dev_ptr(self.active), _stream(dev)))


def correct(params: torch.Tensor, closest_frame: torch.Tensor, delta: torch.Tensor) -> None:
    """In place: each splat moves with the pose increment of its closest keyframe
    (delta [K, 12] or [K, 3, 4], [R|t] acting on world points)."""
    n = params.shape[1]
    dev = params.device
    _check_tensor(params, "params", (15, n), dev)
    _vec(closest_frame, "closest_frame", n, torch.int32, dev)
    if delta.numel() % 12 or delta.shape[-1] not in (4, 12):
        raise ValueError(f"delta must be [K, 12] or [K, 3, 4], got {tuple(delta.shape)}")
    d = delta.reshape(-1, 12)
    _check(d, "delta", (d.shape[0], 12), torch.float32, dev)
    _lib.check(_lib.load().gs2d_map_correct(_dev_ptr(params), n, _dev_ptr(closest_frame), _dev_ptr(d), d.shape[0],
                                            _stream(dev)))


class ParamAdam:
    """Adam over a surfel parameter tensor [15, n] (gs2d_params_adam): one learning
    rate per group (mu, t_u, t_v, scales, opacity, colour), moments kept here."""

    def __init__(self, params: torch.Tensor, lr=(1.6e-4, 1e-3, 1e-3, 5e-3, 5e-2, 2.5e-3), betas=(0.9, 0.999),
                 eps: float = 1e-15, weight_decay: float = 0.0, s_min: float = 1e-5, o_min: float = 0.0,
                 o_max: float = 0.99):
        n = params.shape[1]
        _check(params, "params", (15, n), torch.float32, params.device)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0
        self.lr, self.betas, self.eps, self.weight_decay = tuple(lr), betas, eps, weight_decay
        self.s_min, self.o_min, self.o_max = s_min, o_min, o_max

    def step(self, params: torch.Tensor, grad: torch.Tensor) -> None:
        n = params.shape[1]
        dev = params.device
        _check(params, "params", (15, n), torch.float32, dev)
        _check(grad, "grad", (15, n), torch.float32, dev)
        if self.m.shape != params.shape:
            raise ValueError("params changed shape; make a new ParamAdam")
        self.t += 1
        a = _lib.AdamArgs((ctypes.c_float * 6)(*self.lr), self.betas[0], self.betas[1], self.eps, self.weight_decay,
                          self.t, self.s_min, self.o_min, self.o_max)
        _lib.check(_lib.load().gs2d_params_adam(_dev_ptr(params), _dev_ptr(grad), _dev_ptr(self.m), _dev_ptr(self.v),
                                                n, ctypes.byref(a), _stream(dev)))
