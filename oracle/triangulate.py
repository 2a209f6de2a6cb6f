"""Multi-view triangulation of landmarks from fixed poses (test infrastructure, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper Sec. 2.2 (3D module): when a keyframe is created, the multi-view
observations collected by the 2D module are triangulated into new landmarks,
which then enter the local map and the bundle adjustment.  The paper names the
step only.  Reading taken here, per landmark j with observations o = (i, k, u,
v, w) and the poses T^bw_i held fixed:

  1. linear start: the weighted least-squares intersection of the viewing rays,
       p0 = argmin_p sum_o w_o |(I - d_o d_o^T)(p - c_o)|^2,
     i.e. (sum_o w_o P_o) p0 = sum_o w_o P_o c_o with P_o = I - d_o d_o^T, where
     c_o is the centre of camera k at pose i and d_o the unit direction of the
     ray through the observed pixel, both in the world frame.  The landmark is
     degenerate (status 3, no estimate) when it has fewer than two
     observations or a Cholesky pivot of the 3x3 matrix is <= 1e-10 times its
     trace (parallel rays).  When p0 lies at depth <= min_depth in any of its
     views the start is kept unrefined (status 4).
  2. refinement of the robust reprojection cost of Eq. 2-3 over p alone, by the
     Levenberg-Marquardt schedule of ``oracle.lm`` on the 3x3 point block:
       V = sum_o w_o rho'(s_o) J_o^T J_o,  g = sum_o w_o rho'(s_o) J_o^T r_o
     (J_o the 2x3 point Jacobian), V + lam diag(max(V_kk, 1e-9)), Cholesky
     solve, candidate p + d, depth guard, accept iff the cost strictly drops,
     exactly max_iters attempts.
"""
import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg

from .lm import DIAG_FLOOR, LMSettings
from .model import Problem, cost, huber, jacobians, residuals, transform

DEGENERATE_TOL = 1e-10
STATUS_OK, STATUS_DEGENERATE, STATUS_BEHIND = 0, 3, 4


@dataclasses.dataclass
class TriObs:
    """The observations of one landmark and the fixed rig and poses they use."""

    intrinsics: np.ndarray   # (C, 4)
    extrinsics: np.ndarray   # (C, 3, 4) camera-from-base
    poses: np.ndarray        # (N, 3, 4) base-from-world, fixed
    obs_pose: np.ndarray     # (n,)
    obs_cam: np.ndarray      # (n,)
    obs_uv: np.ndarray       # (n, 2)
    obs_w: np.ndarray        # (n,)

    def problem(self) -> Problem:
        n = int(np.asarray(self.obs_pose).shape[0])
        return Problem(intrinsics=np.asarray(self.intrinsics, float),
                       extrinsics=np.asarray(self.extrinsics, float),
                       obs_pose=np.asarray(self.obs_pose, np.int64),
                       obs_point=np.zeros(n, np.int64),
                       obs_cam=np.asarray(self.obs_cam, np.int64),
                       obs_uv=np.asarray(self.obs_uv, float),
                       obs_w=np.asarray(self.obs_w, float),
                       pose_fixed=np.ones(self.poses.shape[0], bool),
                       n_poses=int(self.poses.shape[0]), n_points=1)


def rays(ob: TriObs):
    """Centres c_o (n, 3) and unit directions d_o (n, 3) in the world frame."""
    n = int(np.asarray(ob.obs_pose).shape[0])
    c = np.zeros((n, 3))
    d = np.zeros((n, 3))
    for o in range(n):
        T = ob.poses[ob.obs_pose[o]]
        E = ob.extrinsics[ob.obs_cam[o]]
        R_cw = E[:, :3] @ T[:, :3]                 # camera-from-world rotation
        t_cw = E[:, :3] @ T[:, 3] + E[:, 3]
        c[o] = -R_cw.T @ t_cw
        fx, fy, cx, cy = ob.intrinsics[ob.obs_cam[o]]
        v = np.array([(ob.obs_uv[o, 0] - cx) / fx, (ob.obs_uv[o, 1] - cy) / fy, 1.0])
        dw = R_cw.T @ v
        d[o] = dw / np.linalg.norm(dw)
    return c, d


def ray_system(ob: TriObs):
    """M = sum_o w_o (I - d d^T) and b = sum_o w_o (I - d d^T) c."""
    c, d = rays(ob)
    M = np.zeros((3, 3))
    b = np.zeros(3)
    for o in range(c.shape[0]):
        P = np.eye(3) - np.outer(d[o], d[o])
        M += ob.obs_w[o] * P
        b += ob.obs_w[o] * (P @ c[o])
    return M, b


def cholesky_pivots(M):
    """Pivots of the unpivoted Cholesky of a 3x3 matrix, in order (the
    factorisation stops at the first non-positive one)."""
    L = np.zeros((3, 3))
    piv = []
    for a in range(3):
        p = M[a, a] - sum(L[a, m] ** 2 for m in range(a))
        piv.append(p)
        if not p > 0:
            break
        L[a, a] = math.sqrt(p)
        for r in range(a + 1, 3):
            L[r, a] = (M[r, a] - sum(L[r, m] * L[a, m] for m in range(a))) / L[a, a]
    return piv


def linear_point(ob: TriObs):
    """(p0, status) of step 1."""
    n = int(np.asarray(ob.obs_pose).shape[0])
    if n < 2:
        return None, STATUS_DEGENERATE
    M, b = ray_system(ob)
    piv = cholesky_pivots(M)
    tol = DEGENERATE_TOL * np.trace(M)
    if len(piv) < 3 or min(piv) <= tol:
        return None, STATUS_DEGENERATE
    return np.linalg.solve(M, b), STATUS_OK


def point_cost(p, ob: TriObs, delta):
    return cost(ob.poses, np.asarray(p, float)[None], ob.problem(), delta)


def point_normal_equations(p, ob: TriObs, delta):
    """V (3x3) and g (3) of the point block."""
    prob = ob.problem()
    pts = np.asarray(p, float)[None]
    r = residuals(ob.poses, pts, prob)
    _, d1, _ = huber(np.sum(r * r, axis=1), delta)
    wt = prob.obs_w * d1
    _, Jl = jacobians(ob.poses, pts, prob)
    V = np.einsum("n,nab,nac->bc", wt, Jl, Jl)
    g = np.einsum("n,nab,na->b", wt, Jl, r)
    return V, g


@dataclasses.dataclass
class TriResult:
    point: Optional[np.ndarray]
    status: int
    initial_cost: float
    final_cost: float
    final_lambda: float
    accepted: int
    chol_failures: int
    depth_rejects: int
    trace: List[dict]


def triangulate(ob: TriObs, settings: LMSettings = None,
                decisions: Optional[List[bool]] = None) -> TriResult:
    """Steps 1 and 2 for one landmark.  ``decisions`` replays an accept/reject
    sequence (for comparing with a solver whose rounding may flip a near-tie)."""
    st = settings or LMSettings()
    delta = st.huber_delta
    p0, status = linear_point(ob)
    if status != STATUS_OK:
        return TriResult(None, status, math.nan, math.nan, st.lambda_init, 0, 0, 0, [])
    prob = ob.problem()
    _, xc = transform(ob.poses, p0[None], prob)
    if np.any(~(xc[:, 2] > st.min_depth)):
        return TriResult(p0, STATUS_BEHIND, math.nan, math.nan, st.lambda_init, 0, 0, 0, [])
    p = p0.copy()
    F = point_cost(p, ob, delta)
    F0 = F
    lam = st.lambda_init
    system = None
    trace = []
    n_acc = n_chol = n_depth = 0
    for it in range(st.max_iters):
        if system is None:
            system = point_normal_equations(p, ob, delta)
        V, g = system
        A = V.copy()
        idx = np.arange(3)
        A[idx, idx] = V[idx, idx] + lam * np.maximum(V[idx, idx], DIAG_FLOOR)
        rec = dict(iter=it, cost=F, lam=lam, cand_cost=math.nan, status="ok")
        step = None
        if np.all(np.isfinite(A)) and np.all(np.isfinite(g)):
            try:
                c = scipy.linalg.cho_factor(A, lower=False, check_finite=False)
                step = scipy.linalg.cho_solve(c, -g, check_finite=False)
                if not np.all(np.isfinite(step)):
                    step = None
            except np.linalg.LinAlgError:
                step = None
        valid = step is not None
        if not valid:
            rec["status"] = "chol_fail"
            n_chol += 1
        else:
            cand = p + step
            _, xcc = transform(ob.poses, cand[None], prob)
            if np.any(~(xcc[:, 2] > st.min_depth)):
                valid = False
                rec["status"] = "depth"
                n_depth += 1
            else:
                rec["cand_cost"] = point_cost(cand, ob, delta)
        accept = valid and rec["cand_cost"] < F
        if decisions is not None:
            forced = bool(decisions[it])
            if forced and not valid:
                raise ValueError(f"replayed acceptance of an invalid candidate at attempt {it}")
            rec["own_decision"] = accept
            accept = forced
        if accept:
            p, F = cand, rec["cand_cost"]
            lam = max(lam / st.lambda_down, st.lambda_min)
            system = None
            n_acc += 1
        else:
            lam = min(lam * st.lambda_up, st.lambda_max)
        rec["accepted"] = accept
        rec["lam_after"] = lam
        trace.append(rec)
    return TriResult(p, STATUS_OK, F0, F, lam, n_acc, n_chol, n_depth, trace)


def landmark_obs(intrinsics, extrinsics, poses, point_obs_begin, obs_pose, obs_cam, obs_uv, obs_w,
                 j) -> TriObs:
    """The TriObs of landmark j from landmark-major (CSR) arrays."""
    sl = slice(int(point_obs_begin[j]), int(point_obs_begin[j + 1]))
    return TriObs(intrinsics=np.asarray(intrinsics, float), extrinsics=np.asarray(extrinsics, float),
                  poses=np.asarray(poses, float), obs_pose=np.asarray(obs_pose[sl]),
                  obs_cam=np.asarray(obs_cam[sl]), obs_uv=np.asarray(obs_uv[sl], float),
                  obs_w=np.asarray(obs_w[sl], float))
