"""Shared helpers of the GPU parity tests: inputs, tolerances and exclusion masks."""

from __future__ import annotations

import numpy as np
import torch

import synth

ROOM_CAM = synth.Camera(640, 480, 525.0, 525.0, 320.0, 240.0)
MARGIN = 1e-5            # pixels closer than this (relative) to a decision are excluded
MAX_EXCLUDED = 1e-3      # ... and may be at most 0.1 % of the image


def dev(a, device="cuda:0"):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).to(device)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def room_scene(n=300_000, seed=0, cam_seed=0):
    room = synth.make_room(n, seed=seed)
    pose = synth.room_camera(room, seed=cam_seed)
    return room, pose


def check_images(gpu: dict, ref: dict, margin: np.ndarray, what=("rgb", "depth", "normal", "alpha"),
                 max_excluded=MAX_EXCLUDED):
    """Parity of planar images with the tolerances of the method's parity bar.

    colour and opacity: |d| <= 1e-4 absolute per channel; depth: |d| <= 1e-4 max(|ref|, 1e-3);
    normal: a 3-vector, so "1e-4 relative" is read on its norm,
    ||d N||_2 <= 1e-4 max(||N_ref||_2, 1e-3) per pixel, with one allowance: N is a sum of unit
    normals weighted by w_i, and where they cancel (||N|| << sum_i w_i = O) the sum is
    ill-conditioned.  FP32 rounding of a k-term blend is then bounded relative to the scale of
    its terms, not of its result: each weight carries the rounding of the k transmittance
    factors in front of it and the sum that of its own k additions, so
    ||d N|| <= (2 k + 8) 2^-24 O (k = the pixel's composited count).  The bar is the larger of
    the two; wherever ||N|| is not cancelled the first one is the binding one.
    Pixels with a decision margin below MARGIN are excluded and counted (at most
    max_excluded of the image).
    """
    keep = margin >= MARGIN
    frac = 1.0 - keep.mean()
    assert frac <= max_excluded, f"{frac:.4%} of pixels excluded by margin"
    report = {"excluded_frac": float(frac)}
    for k in what:
        g, r = gpu[k], ref[k]
        if k in ("rgb", "alpha"):
            tol = 1e-4 + 0 * r
            err = np.abs(g - r)
        elif k == "depth":
            tol = 1e-4 * np.maximum(np.abs(r), 1e-3)
            err = np.abs(g - r)
        else:
            tol = 1e-4 * np.maximum(np.linalg.norm(r, axis=0), 1e-3)
            tol = np.maximum(tol, (2.0 * ref["count"] + 8.0) * 2.0**-24 * ref["alpha"])
            err = np.linalg.norm(g - r, axis=0)
        bad = (err > tol) & (keep if err.ndim == 2 else keep[None])
        report[k] = float(err[..., keep].max()) if keep.any() else 0.0
        assert not bad.any(), f"{k}: {int(bad.sum())} values out of tolerance, worst {err[bad].max():.3g}"
    return report


GROUPS = {"mu": slice(0, 3), "t_u": slice(3, 6), "t_v": slice(6, 9), "s": slice(9, 11), "o": slice(11, 12),
          "rgb": slice(12, 15)}


def check_grads(gpu: np.ndarray, ref: np.ndarray, skip: np.ndarray | None = None, rel=1e-3, floor=1e-5):
    """|d| <= rel |ref| + floor ||group||_inf per parameter group (surfels in `skip` excluded).

    The floor covers float32 accumulation: a surfel's gradient sums many pixel terms
    of both signs, each carrying ~1e-6 relative rounding, so an entry that cancels to
    a small net value carries an absolute error proportional to the terms, not to itself.
    """
    report = {}
    keep = np.ones(ref.shape[1], dtype=bool) if skip is None else ~skip
    for name, sl in GROUPS.items():
        g, r = gpu[sl][:, keep], ref[sl][:, keep]
        scale = np.abs(r).max() if r.size else 0.0
        tol = rel * np.abs(r) + floor * scale
        err = np.abs(g - r)
        bad = err > tol
        report[name] = float((err / np.maximum(np.abs(r), 1e-30)).max()) if r.size else 0.0
        assert not bad.any(), (f"{name}: {int(bad.sum())}/{bad.size} out of tolerance; "
                               f"worst abs {err[bad].max():.3g} at ref {r[bad][np.argmax(err[bad])]:.3g}, "
                               f"scale {scale:.3g}")
    return report


def check_pose(gpu, ref, rel=1e-3, floor=1e-6):
    gpu = np.asarray(gpu, dtype=np.float64)
    for sl in (slice(0, 3), slice(3, 6)):
        g, r = gpu[sl], ref[sl]
        tol = rel * np.abs(r) + floor * np.abs(r).max()
        assert np.all(np.abs(g - r) <= tol), (g, r)
