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

# Rounding allowance of the pose gradient, relative to its magnitude scale (the
# oracle's pose_scale, the sum over pairs of |the pair's share|; see check_pose).
ROUND = 2.0 ** -17


def check_grads(gpu: np.ndarray, ref: np.ndarray, skip: np.ndarray | None = None, rel=1e-3, floor=1e-6):
    """Gradient parity per parameter group (surfels in `skip` excluded), the method's
    bar: |d| <= rel |ref| + floor ||group||_inf (1e-3 relative, 1e-6 of the group's
    largest entry).  The report gives, per group, the largest relative error and the
    largest error as a fraction of the bar."""
    report = {}
    keep = np.ones(ref.shape[1], dtype=bool) if skip is None else ~skip
    for name, sl in GROUPS.items():
        g, r = gpu[sl][:, keep], ref[sl][:, keep]
        gmax = np.abs(r).max() if r.size else 0.0
        tol = rel * np.abs(r) + floor * gmax
        err = np.abs(g - r)
        bad = err > tol
        report[name] = {"rel": float((err / np.maximum(np.abs(r), 1e-30)).max()) if r.size else 0.0,
                        "of_bar": float((err / np.maximum(tol, 1e-300)).max()) if r.size else 0.0}
        assert not bad.any(), (f"{name}: {int(bad.sum())}/{bad.size} out of tolerance; "
                               f"worst abs {err[bad].max():.3g} at ref {r[bad][np.argmax(err[bad])]:.3g}, "
                               f"group max {gmax:.3g}")
    return report


def check_pose(gpu, ref, rel=1e-3, floor=1e-6, scale=None, flip=None, round_k=ROUND):
    """Pose-gradient parity per group (rho, phi): |d| <= rel |ref| + floor max|ref_group|
    + round_k scale + 2 flip.

    The pose gradient sums one share per (pixel, surfel) pair of the whole image, so
    two allowances are added to the method's bar.  `scale` is the oracle's pose_scale,
    the sum over pairs of |the pair's share|: a float32 sum of such shares carries a
    rounding error proportional to it, not to the (possibly cancelled) total; round_k
    = 2^-17 allows 7 of the 24 significand bits for each share's chain of a few dozen
    operations, the transmittance products in front of it and the summation trees.
    `flip` is the pose scale of the pixels where the two sides may take a different
    discrete decision (a decision margin below 1e-5, or a loss residual or mask within
    the rendering tolerance of its switch): there each side's pixel share is at most
    that pixel's scale, so the two differ by at most twice it."""
    gpu = np.asarray(gpu, dtype=np.float64)
    rep = {}
    for sl in (slice(0, 3), slice(3, 6)):
        g, r = gpu[sl], ref[sl]
        bar = rel * np.abs(r) + floor * np.abs(r).max()
        tol = bar.copy()
        if scale is not None:
            tol = tol + round_k * np.asarray(scale)[sl]
        if flip is not None:
            tol = tol + 2.0 * np.asarray(flip)[sl]
        err = np.abs(g - r)
        rep["rho" if sl.start == 0 else "phi"] = float((err / np.maximum(bar, 1e-300)).max())
        assert np.all(err <= tol), (g, r, err, tol)
    return rep


def tracking_ambiguous(ren: dict, tgt: dict, cam, margin_ren=None, margin_tgt=None, tol=2e-4):
    """Pixels where the GPU and the oracle may take different discrete decisions in the
    tracking loss (eq:tracking_loss with eq:normal_mask and eq:opacity_mask): a residual
    sign within `tol` (twice the colour and relative-depth parity bar: each side renders
    both the frame and, unless shared, the target), the opacity mask within 1e-4 of 0.95,
    the normal mask within 1e-4 of its sign change, or a render decision margin below
    the exclusion threshold."""
    H, W = cam.height, cam.width
    amb = np.zeros((H, W), dtype=bool)
    amb |= (np.abs(ren["rgb"] - tgt["rgb"]) <= tol).any(axis=0)
    amb |= np.abs(ren["depth"] - tgt["depth"]) <= tol * np.maximum(np.abs(tgt["depth"]), 1e-3)
    amb |= np.abs(ren["alpha"] - 0.95) <= 1e-4
    ys, xs = np.mgrid[0:H, 0:W]
    ray = np.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, np.ones((H, W))])
    ndr = (ren["normal"] * ray).sum(axis=0)
    amb |= np.abs(ndr) <= 1e-4 * np.maximum(np.linalg.norm(ren["normal"], axis=0), 1e-3) * np.linalg.norm(ray, axis=0)
    if margin_ren is not None:
        amb |= margin_ren < MARGIN
    if margin_tgt is not None:
        amb |= margin_tgt < MARGIN
    return amb


def flip_scale(params, cam, pose, mask, lambda_d=1.0, filter=True):
    """Pose scale of the largest loss gradient any side may apply at the masked pixels:
    1/HW on each colour channel and lambda_d/HW on depth, one channel at a time, so
    that the channel shares add in magnitude."""
    import oracle

    H, W = cam.height, cam.width
    m = mask.astype(np.float64) / (H * W)
    tot = np.zeros(6)
    for ch in range(4):
        if ch < 3:
            d_rgb = np.zeros((3, H, W))
            d_rgb[ch] = m
            ob = oracle.backward(params, cam, pose, d_rgb=d_rgb, filter=filter, scale=True)
        else:
            ob = oracle.backward(params, cam, pose, d_depth=lambda_d * m, filter=filter, scale=True)
        tot += ob["pose_scale"]
    return tot
