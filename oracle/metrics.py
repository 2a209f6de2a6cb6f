"""Result metrics of the oracle (test infrastructure, FP64)."""
import math

import numpy as np

from .model import residuals


def rms(poses, points, prob, mask=None):
    """sqrt(sum_o ||r_o||^2 / n_obs): the RMS reprojection error per 2-D observation."""
    r = residuals(poses, points, prob)
    if mask is not None:
        r = r[np.asarray(mask, bool)]
    return math.sqrt(float(np.sum(r * r)) / max(1, r.shape[0]))


def centres(poses):
    """Camera (base) centres c_i = -R_i^T t_i."""
    return -np.einsum("nba,nb->na", poses[:, :, :3], poses[:, :, 3])


def align_scale(poses, points, poses_ref, anchor=0):
    """Scale a mono solution about the anchor pose's centre to best match poses_ref.

    s = sum_i (c_i - c_0).(c_i^ref - c_0) / sum_i ||c_i - c_0||^2; centres and
    points move as c0 + s (x - c0); rotations are unchanged."""
    c = centres(poses)
    cr = centres(poses_ref)
    c0 = c[anchor]
    d = c - c0
    den = float(np.sum(d * d))
    s = float(np.sum(d * (cr - c0))) / den if den > 0 else 1.0
    new_c = c0 + s * d
    out = poses.copy()
    out[:, :, 3] = -np.einsum("nab,nb->na", poses[:, :, :3], new_c)
    return out, c0 + s * (points - c0), s


def rotation_errors(poses_a, poses_b):
    """Per-pose rotation angle 2 asin(||Ra - Rb||_F / (2 sqrt 2)) and translation error."""
    dR = np.linalg.norm(poses_a[:, :, :3] - poses_b[:, :, :3], axis=(1, 2))
    ang = 2.0 * np.arcsin(np.minimum(1.0, dR / (2.0 * math.sqrt(2.0))))
    dt = np.linalg.norm(poses_a[:, :, 3] - poses_b[:, :, 3], axis=1)
    return ang, dt
