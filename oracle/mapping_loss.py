"""The mapping loss and its image gradients (test infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing in the product path.
Plain PyTorch CPU operations in float64, following Sec. "Mapping":

* colour term L_c(p) = w_l1 |I_r(p) - I(p)|_1 + w_ssim (1 - SSIM(p)), the L1 distance
  summed over RGB, SSIM(p) the mean over the three channels of Wang et al.'s SSIM map
  (an 11 x 11 Gaussian window with sigma 1.5, zero outside the image, C1 = 0.01^2,
  C2 = 0.03^2 for values in [0, 1]);
* depth term L_D(p) = |D_r(p) - D(p)| (eq:LD, unmasked);
* normal consistency L_n(p) = 1 - N_{D_r}(p) . N_r(p), with N_{D_r} from the rendered
  depth by eq:normal_fromD: the pixels are lifted to camera-frame points
  X(x, y) = D(x, y) ((x - c_x)/f_x, (y - c_y)/f_y, 1), the neighbour differences are
  the central ones X(x+1, y) - X(x-1, y) and X(x, y+1) - X(x, y-1) (x the column,
  y the row), and their normalised cross product is N_{D_r}; pixels on the image border,
  and pixels whose cross product vanishes, get N_{D_r} = 0;
* L_m = (1/|Omega|) sum_p (L_c(p) + w_d L_D(p) + w_n L_n(p)) over every pixel.

The weights default to the table of parameters: 0.125 on the SSIM term (so 0.875 on
the L1 term), w_d = 0.5, w_n = 0.02.  The gradients are torch.autograd's of this
float64 definition; |x| has derivative 0 at 0.
"""

from __future__ import annotations

import math

import numpy as np
import torch

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
W_L1, W_SSIM, W_D, W_N = 0.875, 0.125, 0.5, 0.02


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> torch.Tensor:
    """The 2-D window: outer product of the normalised 1-D Gaussian (sums to 1)."""
    r = size // 2
    g = torch.tensor([math.exp(-(i * i) / (2.0 * sigma * sigma)) for i in range(-r, r + 1)], dtype=torch.float64)
    g = g / g.sum()
    return torch.outer(g, g)


def _local_mean(img: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """Window-weighted mean of each channel of img [C, H, W], zero outside the image."""
    c = img.shape[0]
    k = w[None, None].expand(c, 1, *w.shape)
    return torch.nn.functional.conv2d(img[None], k, padding=w.shape[0] // 2, groups=c)[0]


def ssim_map(x: torch.Tensor, y: torch.Tensor, window: int = WINDOW, sigma: float = SIGMA) -> torch.Tensor:
    """Per-channel SSIM map [C, H, W] of images [C, H, W]."""
    w = gaussian_window(window, sigma)
    mx, my = _local_mean(x, w), _local_mean(y, w)
    vx = _local_mean(x * x, w) - mx * mx
    vy = _local_mean(y * y, w) - my * my
    cxy = _local_mean(x * y, w) - mx * my
    return ((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2))


def _camera(camera):
    t = camera.as_tuple() if hasattr(camera, "as_tuple") else tuple(camera)
    W, H, fx, fy, cx, cy = t
    return int(W), int(H), float(fx), float(fy), float(cx), float(cy)


def depth_normals(depth: torch.Tensor, camera) -> torch.Tensor:
    """N_{D}(x, y) of eq:normal_fromD for a depth image [H, W]: [3, H, W]."""
    W, H, fx, fy, cx, cy = _camera(camera)
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(W, dtype=torch.float64),
                            indexing="ij")
    X = torch.stack([depth * (xs - cx) / fx, depth * (ys - cy) / fy, depth])  # [3, H, W]
    n = torch.zeros((3, H, W), dtype=torch.float64)
    if H < 3 or W < 3:
        return n
    dx = X[:, 1:-1, 2:] - X[:, 1:-1, :-2]
    dy = X[:, 2:, 1:-1] - X[:, :-2, 1:-1]
    c = torch.linalg.cross(dx, dy, dim=0)
    # N_D = 0 where the cross product vanishes; the square root is taken of a guarded
    # value so that its derivative stays finite there (the gradient is then 0)
    n2 = (c * c).sum(dim=0)
    norm = torch.sqrt(torch.where(n2 > 0, n2, torch.ones_like(n2)))
    inner = torch.where(n2 > 0, c / norm, torch.zeros_like(c))
    return torch.nn.functional.pad(inner, (1, 1, 1, 1))


def mapping_loss(rgb, depth, normal, tgt_rgb, tgt_depth, camera, w_l1=W_L1, w_ssim=W_SSIM, w_d=W_D, w_n=W_N):
    """L_m and its gradients to the rendered images.

    Returns {"loss", "terms": (mean L1, mean 1 - SSIM, mean |dD|, mean L_n),
    "d_rgb" [3, H, W], "d_depth" [H, W], "d_normal" [3, H, W]} in float64.
    """
    f64 = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))
    I = f64(rgb).requires_grad_(True)
    D = f64(depth).requires_grad_(True)
    N = f64(normal).requires_grad_(True)
    It, Dt = f64(tgt_rgb), f64(tgt_depth)
    hw = float(D.shape[0] * D.shape[1])
    l1 = (I - It).abs().sum(dim=0)
    dssim = 1.0 - ssim_map(I, It).mean(dim=0)
    ld = (D - Dt).abs()
    ln = 1.0 - (depth_normals(D, camera) * N).sum(dim=0)
    per_pixel = w_l1 * l1 + w_ssim * dssim + w_d * ld + w_n * ln
    loss = per_pixel.sum() / hw
    loss.backward()
    terms = tuple(float(t.detach().sum() / hw) for t in (l1, dssim, ld, ln))
    return {"loss": float(loss.detach()), "terms": terms, "d_rgb": I.grad.numpy(), "d_depth": D.grad.numpy(),
            "d_normal": N.grad.numpy()}
