"""SO(3)/SE(3) helpers of the oracle (test infrastructure, FP64).

The paper states the pose as an SE(3) transform (Sec. 2.2, Eq. 2: T^bw_i is
base-from-world) and refers to Barfoot's "State Estimation for Robotics" for the
Lie-group machinery (Sec. 2.2.2).  The update used here is the left perturbation
T <- Exp(xi) T with xi = (rho, phi), translation first.

Exp_SO3(phi) = I + A [phi]x + B [phi]x^2,   A = sin(th)/th,  B = (1 - cos th)/th^2
J_l(phi)     = I + B [phi]x + C [phi]x^2,   C = (th - sin th)/th^3
Exp_SE3(rho, phi) = (Exp_SO3(phi), J_l(phi) rho)
Below th = 1e-4 the coefficients use their Taylor series (to th^4).
"""
import math

import numpy as np

TAYLOR_THRESHOLD = 1e-4


def skew(v):
    v = np.asarray(v, float)
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def _coeffs(th):
    if th < TAYLOR_THRESHOLD:
        t2 = th * th
        A = 1.0 - t2 / 6.0 + t2 * t2 / 120.0
        B = 0.5 - t2 / 24.0 + t2 * t2 / 720.0
        C = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0
    else:
        A = math.sin(th) / th
        s = math.sin(0.5 * th)
        B = 2.0 * s * s / (th * th)
        C = (th - math.sin(th)) / (th * th * th)
    return A, B, C


def exp_so3(phi):
    phi = np.asarray(phi, float)
    th = float(np.linalg.norm(phi))
    A, B, _ = _coeffs(th)
    K = skew(phi)
    return np.eye(3) + A * K + B * (K @ K)


def left_jacobian_so3(phi):
    phi = np.asarray(phi, float)
    th = float(np.linalg.norm(phi))
    _, B, C = _coeffs(th)
    K = skew(phi)
    return np.eye(3) + B * K + C * (K @ K)


def exp_se3(xi):
    """xi = (rho, phi) -> 3x4 [R | t]."""
    xi = np.asarray(xi, float)
    rho, phi = xi[:3], xi[3:]
    return np.concatenate([exp_so3(phi), (left_jacobian_so3(phi) @ rho)[:, None]], axis=1)


def retract_pose(pose, xi):
    """Left update Exp(xi) * T of a 3x4 [R | t] pose."""
    D = exp_se3(xi)
    R = D[:, :3] @ pose[:, :3]
    t = D[:, :3] @ pose[:, 3] + D[:, 3]
    return np.concatenate([R, t[:, None]], axis=1)


def rotation_angle(Ra, Rb):
    """Angle between two rotations, 2 asin(||Ra - Rb||_F / (2 sqrt 2))."""
    d = np.linalg.norm(np.asarray(Ra) - np.asarray(Rb))
    return 2.0 * math.asin(min(1.0, d / (2.0 * math.sqrt(2.0))))
