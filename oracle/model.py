"""Per-observation model of the oracle (test infrastructure, FP64).

Paper Sec. 2.2, Eq. 2: the reprojection residual of landmark j seen by camera k
of the rig at keyframe pose i is  r = pi(T^cb_k T^bw_i p^w_j) - o.
Eq. 3 sums the squared residual norm over the observed (i, j, k).  Here every
observation carries its own (i, j, k), a pixel o = (u, v) and a weight w, and the
norm is made robust with a Huber kernel on the pixel residual:

  x_b = R_i p_j + t_i,  x_c = R^cb_k x_b + t^cb_k = (X, Y, Z)
  pi(x_c) = (fx X / Z + cx, fy Y / Z + cy)          (pinhole, no distortion)
  s = ||r||^2,  rho(s) = s (s <= d^2),  2 d sqrt(s) - d^2 (s > d^2)
  F = 1/2 sum_o w_o rho(s_o)

Jacobians with respect to the left pose perturbation xi = (rho, phi) and the
point (App. of the textbook treatment cited in the paper):
  A   = d pi / d x_c = [[fx/Z, 0, -fx X/Z^2], [0, fy/Z, -fy Y/Z^2]]
  J_p = A R^cb [I, -[x_b]x]      (2 x 6)
  J_l = A R^cb R_i              (2 x 3)
"""
import dataclasses

import numpy as np


@dataclasses.dataclass
class Problem:
    """Structure and measurements of one window (arrays in user order)."""

    intrinsics: np.ndarray   # (C, 4) fx, fy, cx, cy
    extrinsics: np.ndarray   # (C, 3, 4) camera-from-base
    obs_pose: np.ndarray     # (n,) int
    obs_point: np.ndarray    # (n,) int
    obs_cam: np.ndarray      # (n,) int
    obs_uv: np.ndarray       # (n, 2)
    obs_w: np.ndarray        # (n,)
    pose_fixed: np.ndarray   # (N,) bool
    n_poses: int
    n_points: int

    @classmethod
    def from_window(cls, w, obs_uv=None, obs_w=None):
        return cls(intrinsics=np.asarray(w.intrinsics, float),
                   extrinsics=np.asarray(w.extrinsics, float),
                   obs_pose=np.asarray(w.obs_pose, np.int64),
                   obs_point=np.asarray(w.obs_point, np.int64),
                   obs_cam=np.asarray(w.obs_cam, np.int64),
                   obs_uv=np.asarray(w.obs_uv if obs_uv is None else obs_uv, float),
                   obs_w=np.asarray(w.obs_w if obs_w is None else obs_w, float),
                   pose_fixed=np.asarray(w.pose_fixed).astype(bool),
                   n_poses=int(w.poses_gt.shape[0]), n_points=int(w.points_gt.shape[0]))

    @property
    def n_obs(self):
        return int(self.obs_pose.shape[0])

    def free_index(self):
        """Free-pose slot of every pose (-1 when fixed), in pose order."""
        idx = -np.ones(self.n_poses, np.int64)
        free = np.nonzero(~self.pose_fixed)[0]
        idx[free] = np.arange(free.size)
        return idx

    @property
    def n_free(self):
        return int((~self.pose_fixed).sum())


def transform(poses, points, prob):
    """x_b and x_c of every observation, (n, 3) each."""
    R = poses[prob.obs_pose, :, :3]
    t = poses[prob.obs_pose, :, 3]
    p = points[prob.obs_point]
    xb = np.einsum("nab,nb->na", R, p) + t
    Rc = prob.extrinsics[prob.obs_cam, :, :3]
    tc = prob.extrinsics[prob.obs_cam, :, 3]
    xc = np.einsum("nab,nb->na", Rc, xb) + tc
    return xb, xc


def project(xc, K):
    """Pinhole projection of (n, 3) camera points with (n, 4) intrinsics."""
    return np.stack([K[:, 0] * xc[:, 0] / xc[:, 2] + K[:, 2],
                     K[:, 1] * xc[:, 1] / xc[:, 2] + K[:, 3]], axis=1)


def residuals(poses, points, prob):
    """r = pi(x_c) - o, shape (n, 2)."""
    _, xc = transform(poses, points, prob)
    return project(xc, prob.intrinsics[prob.obs_cam]) - prob.obs_uv


def huber(s, delta):
    """rho(s), rho'(s), rho''(s) of the Huber kernel on s = ||r||^2.

    delta <= 0 (or inf) selects plain least squares.  At s == delta^2 the inlier
    branch is taken."""
    s = np.asarray(s, float)
    if not (delta > 0) or not np.isfinite(delta):
        return s.copy(), np.ones_like(s), np.zeros_like(s)
    d2 = delta * delta
    out = s > d2
    sq = np.sqrt(np.where(out, s, 1.0))
    rho = np.where(out, 2.0 * delta * sq - d2, s)
    d1 = np.where(out, delta / sq, 1.0)
    d2r = np.where(out, -0.5 * delta / (sq * sq * sq), 0.0)
    return rho, d1, d2r


def cost(poses, points, prob, delta):
    """F = 1/2 sum_o w_o rho(||r_o||^2)."""
    r = residuals(poses, points, prob)
    rho, _, _ = huber(np.sum(r * r, axis=1), delta)
    return 0.5 * float(np.sum(prob.obs_w * rho))


def projection_jacobian(xc, K):
    """A = d pi / d x_c, shape (n, 2, 3)."""
    X, Y, Z = xc[:, 0], xc[:, 1], xc[:, 2]
    iz = 1.0 / Z
    A = np.zeros((xc.shape[0], 2, 3))
    A[:, 0, 0] = K[:, 0] * iz
    A[:, 0, 2] = -K[:, 0] * X * iz * iz
    A[:, 1, 1] = K[:, 1] * iz
    A[:, 1, 2] = -K[:, 1] * Y * iz * iz
    return A


def skew_batch(v):
    S = np.zeros(v.shape[:-1] + (3, 3))
    S[..., 0, 1] = -v[..., 2]
    S[..., 0, 2] = v[..., 1]
    S[..., 1, 0] = v[..., 2]
    S[..., 1, 2] = -v[..., 0]
    S[..., 2, 0] = -v[..., 1]
    S[..., 2, 1] = v[..., 0]
    return S


def jacobians(poses, points, prob):
    """J_p (n, 2, 6) w.r.t. the left perturbation (rho, phi) and J_l (n, 2, 3)."""
    xb, xc = transform(poses, points, prob)
    A = projection_jacobian(xc, prob.intrinsics[prob.obs_cam])
    Rc = prob.extrinsics[prob.obs_cam, :, :3]
    ARc = np.einsum("nab,nbc->nac", A, Rc)
    dxb = np.concatenate([np.broadcast_to(np.eye(3), xb.shape[:1] + (3, 3)), -skew_batch(xb)],
                         axis=2)                                         # (n, 3, 6)
    Jp = np.einsum("nab,nbc->nac", ARc, dxb)
    Jl = np.einsum("nab,nbc->nac", ARc, poses[prob.obs_pose, :, :3])
    return Jp, Jl
