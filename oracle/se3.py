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


def _coef_b(th):
    """(1 - cos th)/th^2, written as 2 sin^2(th/2)/th^2 (no cancellation near 0)."""
    if th == 0.0:
        return 0.5
    s = np.sin(0.5 * th)
    return 2.0 * s * s / (th * th)


def _coef_c(th):
    """(th - sin th)/th^3; its Taylor series 1/6 - th^2/120 + th^4/5040 below 1e-2 rad,
    where the difference th - sin th would lose digits (the next term, th^6/362880, is
    below 3e-18 there)."""
    if th < 1e-2:
        t2 = th * th
        return 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0
    return (th - np.sin(th)) / th ** 3


def so3_exp(phi):
    """Rodrigues' formula R = I + sin(th)/th K + (1 - cos th)/th^2 K^2."""
    phi = np.asarray(phi, dtype=np.float64)
    th = np.linalg.norm(phi)
    K = hat(phi)
    a = 1.0 if th == 0.0 else np.sin(th) / th
    return np.eye(3) + a * K + _coef_b(th) * K @ K


def so3_left_jacobian(phi):
    """J(phi) = I + (1-cos th)/th^2 K + (th - sin th)/th^3 K^2."""
    phi = np.asarray(phi, dtype=np.float64)
    th = np.linalg.norm(phi)
    K = hat(phi)
    return np.eye(3) + _coef_b(th) * K + _coef_c(th) * K @ K


def so3_log(R):
    """The rotation vector of R: angle atan2(|v|/2, (tr R - 1)/2) with v the
    antisymmetric part (|v| = 2 sin th), which keeps its digits at small angles."""
    R = np.asarray(R, dtype=np.float64)
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    th = np.arctan2(0.5 * np.linalg.norm(v), c)
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
