"""SE(3) / SO(3) exponential and logarithm in FP64 (test infrastructure only).

Closed forms as given in Barfoot, "State Estimation for Robotics", Sec. 7.1
(and Sola et al., "A micro Lie theory for state estimation in robotics",
App. A).  A twist is tau = (rho, phi): rho the translational part, phi the
rotation vector.  Poses are 3x4 [R | t] arrays; the paper's manifold derivative
(Sec. "Camera Pose Optimization") perturbs on the left, T' = Exp(tau) T.
"""

from __future__ import annotations

import numpy as np


def hat(w):
    w = np.asarray(w, dtype=np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def so3_exp(phi):
    """Rodrigues' formula; second-order series below 1e-8 rad."""
    phi = np.asarray(phi, dtype=np.float64)
    th = np.linalg.norm(phi)
    K = hat(phi)
    if th < 1e-8:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th ** 2 * K @ K


def so3_left_jacobian(phi):
    """J(phi) = I + (1-cos th)/th^2 K + (th - sin th)/th^3 K^2."""
    phi = np.asarray(phi, dtype=np.float64)
    th = np.linalg.norm(phi)
    K = hat(phi)
    if th < 1e-6:
        return np.eye(3) + 0.5 * K + K @ K / 6.0
    return np.eye(3) + (1.0 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * K @ K


def so3_log(R):
    R = np.asarray(R, dtype=np.float64)
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = np.arccos(c)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-8:
        return 0.5 * v
    if np.pi - th < 1e-6:
        # near pi: axis from the largest diagonal of (R + I)/2
        B = (R + np.eye(3)) / 2.0
        i = int(np.argmax(np.diag(B)))
        axis = B[:, i] / np.sqrt(B[i, i])
        axis /= np.linalg.norm(axis)
        if np.dot(axis, v) < 0:
            axis = -axis
        return th * axis
    return th / (2.0 * np.sin(th)) * v


def exp(tau):
    """4x4 matrix Exp(tau) for tau = (rho, phi)."""
    tau = np.asarray(tau, dtype=np.float64)
    T = np.eye(4)
    T[:3, :3] = so3_exp(tau[3:])
    T[:3, 3] = so3_left_jacobian(tau[3:]) @ tau[:3]
    return T


def log(T):
    """tau = (rho, phi) with Exp(tau) = T (T given as 3x4 or 4x4)."""
    T = np.asarray(T, dtype=np.float64)
    phi = so3_log(T[:3, :3])
    rho = np.linalg.solve(so3_left_jacobian(phi), T[:3, 3])
    return np.concatenate([rho, phi])


def as4(T):
    T = np.asarray(T, dtype=np.float64)
    if T.shape == (4, 4):
        return T
    out = np.eye(4)
    out[:3, :] = T.reshape(3, 4)
    return out


def left_perturb(tau, T):
    """Exp(tau) T as a 3x4 array."""
    return (exp(tau) @ as4(T))[:3, :]
