"""Motion-only bundle adjustment of single frames (test infrastructure, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper Sec. 2.2: in stereo mode the frame pose is estimated from 2D observations
of landmarks taken from the local map (Eq. 4: the robust sum of reprojection
errors over the landmarks and the two cameras, minimised over T^bw alone); the
multi-camera mode sums over every camera of the rig (Eq. 6); loop closing
estimates a relative pose T^bm against landmarks shifted into a map frame by a
known T^mw (Eq. 14).  The landmarks are fixed in all three: only the six pose
parameters move.

The oracle reuses the window model (``oracle.model``: residual, Huber kernel,
pose Jacobian for the left perturbation) on a one-pose problem whose points are
held fixed, and runs the same Levenberg-Marquardt schedule as ``oracle.lm``:

  1. linearise at T (after an accepted step or at the start):
       U = sum_o w_o rho'(s_o) J_o^T J_o,  g = sum_o w_o rho'(s_o) J_o^T r_o
     with J_o the 2x6 pose Jacobian (the plain J^T W J of the 2n x 6 Jacobian);
  2. U_lam = U + lam * diag(max(U_kk, 1e-9));
  3. solve U_lam d = -g by Cholesky; a non-positive or non-finite pivot rejects
     the attempt;
  4. candidate T' = Exp(d) T; a candidate with any camera depth <= min_depth is
     rejected;
  5. accept iff F(T') < F(T); lam / 10 on acceptance, x 10 on rejection.

A frame without observations keeps its pose (every attempt is rejected: the
candidate cost equals the current one).
"""
import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg

from .lm import DIAG_FLOOR, LMSettings
from .model import Problem, cost, huber, jacobians, residuals, transform
from .se3 import retract_pose


@dataclasses.dataclass
class PnPFrame:
    """One frame: the rig, the fixed landmarks it observes and its observations."""

    intrinsics: np.ndarray        # (C, 4)
    extrinsics: np.ndarray        # (C, 3, 4) camera-from-base
    points: np.ndarray            # (M, 3) landmarks in the world frame
    obs_point: np.ndarray         # (n,)
    obs_cam: np.ndarray           # (n,)
    obs_uv: np.ndarray            # (n, 2)
    obs_w: np.ndarray             # (n,)
    map_from_world: Optional[np.ndarray] = None   # (3, 4) T^mw of Eq. 14, or None

    def problem(self) -> Problem:
        n = int(np.asarray(self.obs_point).shape[0])
        return Problem(intrinsics=np.asarray(self.intrinsics, float),
                       extrinsics=np.asarray(self.extrinsics, float),
                       obs_pose=np.zeros(n, np.int64),
                       obs_point=np.asarray(self.obs_point, np.int64),
                       obs_cam=np.asarray(self.obs_cam, np.int64),
                       obs_uv=np.asarray(self.obs_uv, float),
                       obs_w=np.asarray(self.obs_w, float),
                       pose_fixed=np.zeros(1, bool), n_poses=1,
                       n_points=int(np.asarray(self.points).shape[0]))

    def frame_points(self) -> np.ndarray:
        """The landmarks in the frame the pose is estimated against (Eq. 14:
        T^mw p^w; otherwise the world points themselves)."""
        p = np.asarray(self.points, float)
        if self.map_from_world is None:
            return p.copy()
        T = np.asarray(self.map_from_world, float)
        return p @ T[:, :3].T + T[:, 3]


def pnp_cost(pose, fr: PnPFrame, delta):
    return cost(np.asarray(pose, float)[None], fr.frame_points(), fr.problem(), delta)


def pnp_normal_equations(pose, fr: PnPFrame, delta):
    """U (6x6) and g (6) of the pose block: the plain J^T W J over the 2n rows."""
    prob = fr.problem()
    P = np.asarray(pose, float)[None]
    pts = fr.frame_points()
    r = residuals(P, pts, prob)
    _, d1, _ = huber(np.sum(r * r, axis=1), delta)
    wt = np.repeat(prob.obs_w * d1, 2)
    Jp, _ = jacobians(P, pts, prob)
    J = Jp.reshape(-1, 6)
    U = J.T @ (wt[:, None] * J)
    g = J.T @ (wt * r.reshape(-1))
    return U, g


@dataclasses.dataclass
class PnPResult:
    pose: np.ndarray
    initial_cost: float
    final_cost: float
    final_lambda: float
    accepted: int
    chol_failures: int
    trace: List[dict]


def pnp_solve(pose0, fr: PnPFrame, settings: LMSettings = None,
              decisions: Optional[List[bool]] = None) -> PnPResult:
    """Exactly ``settings.max_iters`` LM attempts on one frame's pose.

    ``decisions`` replays a given accept/reject sequence (for comparing with a
    solver whose rounding may flip a near-tie)."""
    st = settings or LMSettings()
    delta = st.huber_delta
    pose = np.array(pose0, float, copy=True)
    prob = fr.problem()
    pts = fr.frame_points()
    F = pnp_cost(pose, fr, delta)
    F0 = F
    lam = st.lambda_init
    system = None
    trace = []
    n_acc = n_chol = 0
    for it in range(st.max_iters):
        if system is None:
            system = pnp_normal_equations(pose, fr, delta)
        U, g = system
        A = U.copy()
        idx = np.arange(6)
        A[idx, idx] = U[idx, idx] + lam * np.maximum(U[idx, idx], DIAG_FLOOR)
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
            cand = retract_pose(pose, step)
            _, xc = transform(cand[None], pts, prob)
            if np.any(~(xc[:, 2] > st.min_depth)):
                valid = False
                rec["status"] = "depth"
            else:
                rec["cand_cost"] = pnp_cost(cand, fr, delta)
        accept = valid and rec["cand_cost"] < F
        if decisions is not None:
            forced = bool(decisions[it])
            if forced and not valid:
                raise ValueError(f"replayed acceptance of an invalid candidate at attempt {it}")
            rec["own_decision"] = accept
            accept = forced
        if accept:
            pose, F = cand, rec["cand_cost"]
            lam = max(lam / st.lambda_down, st.lambda_min)
            system = None
            n_acc += 1
        else:
            lam = min(lam * st.lambda_up, st.lambda_max)
        rec["accepted"] = accept
        rec["cost_after"] = F
        rec["lam_after"] = lam
        trace.append(rec)
    return PnPResult(pose=pose, initial_cost=F0, final_cost=F, final_lambda=lam, accepted=n_acc,
                     chol_failures=n_chol, trace=trace)
