"""Seeded draws for the warm-start network: initial weights, inputs and twists.

Only random numbers: the network's arithmetic, the residual and the Lie-group
maps live in the oracle and in the HIP path.  Layer order and layouts are the
network's flat parameter vector: per layer the weight ([co][ci][k][k] for the
convolutions, [o][i] for the fully connected layers) then the bias.
"""

from __future__ import annotations

import numpy as np

# (weight shape, bias length) per layer of the warm-start network
LAYER_SHAPES = (((32, 4, 5, 5), 32), ((64, 32, 3, 3), 64), ((128, 64, 3, 3), 128), ((128, 128, 3, 3), 128),
                ((256, 2560), 256), ((6, 256), 6))


def init_params(seed: int = 0, bias_std: float = 0.0) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), biases N(0, bias_std); float32, flat."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for wshape, nb in LAYER_SHAPES:
        fan_in = int(np.prod(wshape[1:]))
        bound = np.sqrt(6.0 / fan_in)
        parts.append(g.uniform(-bound, bound, size=int(np.prod(wshape))))
        parts.append(g.normal(size=nb) * bias_std if bias_std > 0 else np.zeros(nb))
    return np.concatenate(parts).astype(np.float32)


def random_inputs(batch: int, seed: int = 0, scale: float = 0.3) -> np.ndarray:
    """Network inputs [batch][4][60][80], N(0, scale^2), float32."""
    g = np.random.Generator(np.random.PCG64(seed))
    return (g.normal(size=(batch, 4, 60, 80)) * scale).astype(np.float32)


def random_twists(count: int, seed: int, max_trans_m: float = 0.10, max_rot_deg: float = 8.0) -> np.ndarray:
    """Twists (rho, phi) [count][6] with |rho| ~ U[0, max_trans_m], |phi| ~ U[0, max_rot_deg]
    (radians), uniformly random directions; float64."""
    g = np.random.Generator(np.random.PCG64(seed))

    def dirs(n):
        v = g.normal(size=(n, 3))
        return v / np.linalg.norm(v, axis=1, keepdims=True)

    rho = dirs(count) * g.uniform(0.0, max_trans_m, size=(count, 1))
    phi = dirs(count) * np.deg2rad(g.uniform(0.0, max_rot_deg, size=(count, 1)))
    return np.concatenate([rho, phi], axis=1)


def exact_params(seed: int = 0, taps=(3, 4, 4, 4, 16, 256)) -> np.ndarray:
    """Sparse weights for exact-arithmetic tests: every output row of layer l (a conv
    filter over ci k k, or an fc row) has taps[l] nonzero entries, each +-1 (the last
    layer dense); biases are multiples of 0.25 in [-0.5, 0.5]; float32, flat."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for (wshape, nb), nt in zip(LAYER_SHAPES, taps):
        rows, cols = wshape[0], int(np.prod(wshape[1:]))
        w = np.zeros((rows, cols))
        for r in range(rows):
            idx = g.choice(cols, size=min(nt, cols), replace=False)
            w[r, idx] = g.choice([-1.0, 1.0], size=idx.size)
        parts.append(w.ravel())
        parts.append(g.integers(-2, 3, size=nb) * 0.25)
    return np.concatenate(parts).astype(np.float32)


def exact_inputs(batch: int, seed: int = 0) -> np.ndarray:
    """Inputs [batch][4][60][80], multiples of 0.25 in [-0.5, 0.5], float32."""
    g = np.random.Generator(np.random.PCG64(seed))
    return (g.integers(-2, 3, size=(batch, 4, 60, 80)) * 0.25).astype(np.float32)


def exact_targets(batch: int, seed: int = 0) -> np.ndarray:
    """Targets [batch][6], multiples of 0.25 in [-2, 2], float32."""
    g = np.random.Generator(np.random.PCG64(seed))
    return (g.integers(-8, 9, size=(batch, 6)) * 0.25).astype(np.float32)
