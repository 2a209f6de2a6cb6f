"""Pose-graph optimisation (test infrastructure, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper Sec. 2.3 (loop closing and global map refinement), Eq. 15: given pose
deltas D_ij between poses (from the frontend's integrated predictions or from
loop closures), the keyframe poses minimise the sum over the graph's edges of
|Log(D_ij^-1 T_i^-1 T_j)|^2.  Readings taken here:

  * T_i is the world-from-base pose (so that T_i^-1 T_j is the pose of base j
    in base i, the quantity D_ij measures); Log is the SE(3) logarithm with
    xi = (rho, phi), translation first;
  * F = 1/2 sum_e w_e |r_e|^2, r_e = Log(D_ij^-1 T_i^-1 T_j), with an optional
    weight per edge (default 1; the factor 1/2 does not move the minimum);
  * poses flagged fixed are held (default: pose 0, the gauge);
  * LM with the schedule of ``oracle.lm``: the left perturbation T <- Exp(xi) T,
    H = sum_e w_e J_e^T J_e and g = sum_e w_e J_e^T r_e over the free poses,
    H + lam diag(max(H_kk, 1e-9)), Cholesky (a non-positive pivot rejects the
    attempt), candidate Exp(d_i) T_i, accept iff F strictly drops, exactly
    max_iters attempts.

The Jacobians follow from Exp(a) X = X Exp(Ad(X^-1) a): perturbing T_j by
Exp(xi) left-multiplies E = D^-1 T_i^-1 T_j by Exp(Ad(D^-1 T_i^-1) xi), and
perturbing T_i does the same with -xi, so with B = J_l(r)^-1 Ad(D^-1 T_i^-1)
(J_l the left Jacobian of SE(3)):  dr/dxi_j = B,  dr/dxi_i = -B.
J_l is evaluated from its definition, J_l(xi) = sum_n ad(xi)^n / (n+1)!.
"""
import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg
from scipy.spatial.transform import Rotation

from .lm import DIAG_FLOOR, LMSettings
from .se3 import exp_se3, left_jacobian_so3, retract_pose, skew


def inverse(T):
    R, t = T[:, :3], T[:, 3]
    return np.concatenate([R.T, (-R.T @ t)[:, None]], axis=1)


def compose(A, B):
    return np.concatenate([A[:, :3] @ B[:, :3], (A[:, :3] @ B[:, 3] + A[:, 3])[:, None]], axis=1)


def log_so3(R):
    return Rotation.from_matrix(np.asarray(R, float)).as_rotvec()


def log_se3(T):
    """xi = (rho, phi) with Exp(xi) = T: phi = Log_SO3(R), rho = J_l(phi)^-1 t."""
    phi = log_so3(T[:, :3])
    rho = np.linalg.solve(left_jacobian_so3(phi), T[:, 3])
    return np.concatenate([rho, phi])


def ad_se3(xi):
    """ad(xi) = [[phi^, rho^], [0, phi^]] (6x6)."""
    xi = np.asarray(xi, float)
    A = np.zeros((6, 6))
    A[:3, :3] = skew(xi[3:])
    A[:3, 3:] = skew(xi[:3])
    A[3:, 3:] = skew(xi[3:])
    return A


def left_jacobian_se3(xi, terms=60):
    """J_l(xi) = sum_{n >= 0} ad(xi)^n / (n+1)!  (6x6)."""
    A = ad_se3(xi)
    J = np.zeros((6, 6))
    P = np.eye(6)
    for n in range(terms):
        J += P / math.factorial(n + 1)
        P = P @ A
    return J


def adjoint(T):
    """Ad(T) = [[R, t^ R], [0, R]] for xi = (rho, phi): Exp(Ad(T) xi) = T Exp(xi) T^-1."""
    R, t = T[:, :3], T[:, 3]
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[:3, 3:] = skew(t) @ R
    A[3:, 3:] = R
    return A


@dataclasses.dataclass
class PoseGraph:
    n_poses: int
    edge_i: np.ndarray        # (E,)
    edge_j: np.ndarray        # (E,)
    deltas: np.ndarray        # (E, 3, 4) D_ij
    edge_w: np.ndarray        # (E,)
    pose_fixed: np.ndarray    # (N,) bool

    @property
    def n_edges(self):
        return int(self.edge_i.shape[0])


def residual(Ti, Tj, D):
    """r = Log(D^-1 T_i^-1 T_j)."""
    return log_se3(compose(inverse(D), compose(inverse(Ti), Tj)))


def edge_jacobian(Ti, Tj, D):
    """(r, B) with dr/dxi_j = B and dr/dxi_i = -B."""
    r = residual(Ti, Tj, D)
    X = compose(inverse(D), inverse(Ti))
    B = np.linalg.solve(left_jacobian_se3(r), adjoint(X))
    return r, B


def graph_cost(poses, g: PoseGraph):
    F = 0.0
    for e in range(g.n_edges):
        r = residual(poses[g.edge_i[e]], poses[g.edge_j[e]], g.deltas[e])
        F += g.edge_w[e] * float(r @ r)
    return 0.5 * F


def normal_equations(poses, g: PoseGraph):
    """Dense H (6 n_free square) and g over the free poses (free slots in pose
    order), plus the cost."""
    free = np.nonzero(~g.pose_fixed)[0]
    slot = -np.ones(g.n_poses, np.int64)
    slot[free] = np.arange(free.size)
    n = 6 * free.size
    H = np.zeros((n, n))
    gv = np.zeros(n)
    F = 0.0
    for e in range(g.n_edges):
        i, j = g.edge_i[e], g.edge_j[e]
        r, B = edge_jacobian(poses[i], poses[j], g.deltas[e])
        w = g.edge_w[e]
        F += w * float(r @ r)
        blocks = [(slot[i], -B), (slot[j], B)]
        for (a, Ja) in blocks:
            if a < 0:
                continue
            gv[6 * a:6 * a + 6] += w * Ja.T @ r
            for (b, Jb) in blocks:
                if b < 0:
                    continue
                H[6 * a:6 * a + 6, 6 * b:6 * b + 6] += w * Ja.T @ Jb
    return H, gv, 0.5 * F


@dataclasses.dataclass
class PGOResult:
    poses: np.ndarray
    initial_cost: float
    final_cost: float
    final_lambda: float
    accepted: int
    chol_failures: int
    trace: List[dict]


def pgo_solve(poses0, g: PoseGraph, settings: LMSettings = None, backend: str = "dense",
              decisions: Optional[List[bool]] = None) -> PGOResult:
    """Exactly ``settings.max_iters`` LM attempts.  ``backend`` 'dense' factors
    the damped H by LAPACK Cholesky; 'sparse' solves it with SuperLU (no
    pivot-failure detection; for large graphs).  ``decisions`` replays an
    accept/reject sequence."""
    st = settings or LMSettings()
    poses = np.array(poses0, float, copy=True)
    free = np.nonzero(~g.pose_fixed)[0]
    H, gv, F = normal_equations(poses, g)
    F0 = F
    lam = st.lambda_init
    trace = []
    n_acc = n_chol = 0
    for it in range(st.max_iters):
        A = H.copy()
        idx = np.arange(A.shape[0])
        A[idx, idx] = H[idx, idx] + lam * np.maximum(H[idx, idx], DIAG_FLOOR)
        rec = dict(iter=it, cost=F, lam=lam, cand_cost=math.nan, status="ok")
        step = None
        if np.all(np.isfinite(A)) and np.all(np.isfinite(gv)):
            try:
                if backend == "dense":
                    c = scipy.linalg.cho_factor(A, lower=False, check_finite=False)
                    step = scipy.linalg.cho_solve(c, -gv, check_finite=False)
                else:
                    step = scipy.sparse.linalg.splu(scipy.sparse.csc_matrix(A)).solve(-gv)
                if not np.all(np.isfinite(step)):
                    step = None
            except (np.linalg.LinAlgError, RuntimeError):
                step = None
        valid = step is not None
        if not valid:
            rec["status"] = "chol_fail"
            n_chol += 1
        else:
            cand = poses.copy()
            for a, i in enumerate(free):
                cand[i] = retract_pose(poses[i], step[6 * a:6 * a + 6])
            Hc, gc, Fc = normal_equations(cand, g)
            rec["cand_cost"] = Fc
        accept = valid and rec["cand_cost"] < F
        if decisions is not None:
            forced = bool(decisions[it])
            if forced and not valid:
                raise ValueError(f"replayed acceptance of an invalid candidate at attempt {it}")
            rec["own_decision"] = accept
            accept = forced
        if accept:
            poses, H, gv, F = cand, Hc, gc, Fc
            lam = max(lam / st.lambda_down, st.lambda_min)
            n_acc += 1
        else:
            lam = min(lam * st.lambda_up, st.lambda_max)
        rec["accepted"] = accept
        rec["lam_after"] = lam
        trace.append(rec)
    return PGOResult(poses=poses, initial_cost=F0, final_cost=F, final_lambda=lam, accepted=n_acc,
                     chol_failures=n_chol, trace=trace)
