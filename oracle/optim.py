"""Adam (with optional decoupled weight decay) over the surfel parameters (test
infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing in the product path.

The map is optimised with Adam, as 2D Gaussian splatting maps are; the paper names
the losses (Sec. "Mapping") but not the optimiser's constants, so this is the
textbook step written out in float64 NumPy, per parameter:
  m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
  p <- p - lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd p),
with one learning rate per parameter group (rows 0-2 mu, 3-5 t_u, 6-8 t_v, 9-10 the
scales, 11 the opacity, 12-14 the colour), then the post-activation scales clamped to
>= s_min and the opacity to [o_min, o_max].
"""

from __future__ import annotations

import numpy as np

GROUP_OF_ROW = (0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 4, 5, 5, 5)


def adam_step(params, grad, m, v, step: int, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0,
              s_min=0.0, o_min=0.0, o_max=1.0):
    """One step; returns (params, m, v) as new float64 arrays ([15, n] each)."""
    p = np.array(params, dtype=np.float64, copy=True)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    c1, c2 = 1.0 - beta1 ** step, 1.0 - beta2 ** step
    lr_row = np.array([lr[GROUP_OF_ROW[r]] for r in range(15)], dtype=np.float64)[:, None]
    p = p - lr_row * ((m / c1) / (np.sqrt(v / c2) + eps) + weight_decay * p)
    p[9:11] = np.maximum(p[9:11], s_min)
    p[11] = np.clip(p[11], o_min, o_max)
    return p, m, v
