"""Visual-inertial bundle adjustment (test infrastructure, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper Sec. 2.2, "Visual-Inertial", Eq. 9: the robot state of keyframe i is
S_i = [T_i in SE(3), v_i, b^a_i, b^w_i] (15 DoF: pose, linear velocity,
accelerometer and gyroscope biases), and the local map is refined by
minimising the IMU factors between consecutive states plus the visual
(reprojection) factors of Eq. 3.  The paper defers the IMU factor to
Forster et al. 2017 (on-manifold preintegration); it is restated here from
that model.  Readings taken (the paper gives none of these):

  * the IMU frame is the base frame; T_i is base-from-world as in the visual
    model, so the world-from-base rotation is R_i^T and the base position is
    p_i = -R_i^T t_i; v_i is the world-frame velocity of the base origin;
  * gravity g is a known world-frame vector (the paper estimates it before
    VI-SBA runs); specific force a~ = R_i (a_w - g) + b^a + noise, angular
    rate w~ = w + b^w + noise, sampled at a fixed rate, piecewise constant
    over a sample interval;
  * preintegration between keyframes i and j at the bias estimate b_bar
    (kept fixed during a solve, no re-preintegration; a bias change enters
    to first order through the bias Jacobians), with w^ = w~ - b_bar^w,
    a^ = a~ - b_bar^a, per sample:
        dR <- dR Exp(w^ dt)
        dv <- dv + dR a^ dt
        dp <- dp + dv dt + 1/2 dR a^ dt^2        (dp and dv before the update)
  * residual of the factor (i, j), dT = t_j - t_i, db = b_i - b_bar:
        r_R = Log( (dR Exp(J_Rg db^w))^T R_i R_j^T )
        r_v = R_i (v_j - v_i - g dT) - (dv + J_vg db^w + J_va db^a)
        r_p = R_i (p_j - p_i - v_i dT - 1/2 g dT^2) - (dp + J_pg db^w + J_pa db^a)
        r_ba = b^a_j - b^a_i,   r_bg = b^w_j - b^w_i
    with information Sigma^-1: the propagated 9x9 covariance of (r_R, r_v,
    r_p) from white gyro / accelerometer noise of densities sigma_g,
    sigma_a, and a bias random walk of densities sigma_bg, sigma_ba
    (variance sigma^2 dT);
  * cost F = 1/2 sum_o w_o rho(|r_o|^2) (Eq. 3) + 1/2 sum r^T Sigma^-1 r;
  * variables: the left perturbation of each free pose (as in the visual
    model), additive updates of velocities, biases and points; the first
    pose is fixed by default (gravity fixes roll and pitch; yaw and position
    are the gauge), velocities and biases of every state are free;
  * LM with the schedule of ``oracle.lm`` (Marquardt damping, x10 / /10,
    strict decrease, depth guard, exactly max_iters attempts).

Jacobians of the factor (derived from the perturbations: R_k <- Exp(phi_k)
R_k, so R_k^T <- R_k^T Exp(-phi_k), and p_k <- p_k - R_k^T rho_k to first
order, p_k independent of phi_k), with E = (dR Exp(J_Rg db^w))^T R_i R_j^T
and J_r the right Jacobian of SO(3):
    dr_R/dphi_i = J_r(r_R)^-1 R_j R_i^T     dr_R/dphi_j = -J_r(r_R)^-1
    dr_R/db^w_i = -J_r(r_R)^-1 E^T J_r(J_Rg db^w) J_Rg
    dr_v/dphi_i = -[R_i (v_j - v_i - g dT)]x,  dr_v/dv_i = -R_i,  dr_v/dv_j = R_i
    dr_v/db^w_i = -J_vg,  dr_v/db^a_i = -J_va
    dr_p/dphi_i = -[R_i (p_j - p_i - v_i dT - 1/2 g dT^2)]x
    dr_p/drho_i = I,  dr_p/drho_j = -R_i R_j^T,  dr_p/dv_i = -R_i dT
    dr_p/db^w_i = -J_pg,  dr_p/db^a_i = -J_pa
    dr_ba/db^a_{i,j} = -I, I;  dr_bg/db^w_{i,j} = -I, I
"""
import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy.spatial.transform import Rotation

from .lm import LMSettings, _chol_solve, _damp, normal_equations_dense
from .model import cost as visual_cost, transform
from .se3 import exp_so3, left_jacobian_so3, retract_pose, skew

GRAVITY = 9.81


def log_so3(R):
    return Rotation.from_matrix(np.asarray(R, float)).as_rotvec()


def right_jacobian_so3(phi):
    """J_r(phi) = J_l(-phi)."""
    return left_jacobian_so3(-np.asarray(phi, float))


@dataclasses.dataclass
class ImuNoise:
    sigma_g: float = 1.7e-4     # gyro white noise, rad / s / sqrt(Hz)
    sigma_a: float = 2.0e-3     # accelerometer white noise, m / s^2 / sqrt(Hz)
    sigma_bg: float = 2.0e-5    # gyro bias random walk, rad / s^2 / sqrt(Hz)
    sigma_ba: float = 3.0e-3    # accelerometer bias random walk, m / s^3 / sqrt(Hz)


@dataclasses.dataclass
class Preintegration:
    dR: np.ndarray      # (3, 3)
    dv: np.ndarray      # (3,)
    dp: np.ndarray      # (3,)
    dT: float
    J_Rg: np.ndarray    # (3, 3) d dR / d b^w (right perturbation of dR)
    J_vg: np.ndarray
    J_va: np.ndarray
    J_pg: np.ndarray
    J_pa: np.ndarray
    cov: np.ndarray     # (9, 9) of (r_R, r_v, r_p)
    bg_bar: np.ndarray  # bias estimates the samples were integrated with
    ba_bar: np.ndarray


def preintegrate(gyro, accel, dt, bg_bar, ba_bar, noise: ImuNoise = None) -> Preintegration:
    """Preintegrate samples (n, 3) of angular rate and specific force taken
    every dt seconds, at the bias estimates bg_bar, ba_bar."""
    noise = noise or ImuNoise()
    gyro = np.asarray(gyro, float)
    accel = np.asarray(accel, float)
    bg_bar = np.asarray(bg_bar, float)
    ba_bar = np.asarray(ba_bar, float)
    dR, dv, dp = np.eye(3), np.zeros(3), np.zeros(3)
    J_Rg = np.zeros((3, 3))
    J_vg, J_va, J_pg, J_pa = (np.zeros((3, 3)) for _ in range(4))
    cov = np.zeros((9, 9))
    Qg = (noise.sigma_g ** 2 / dt) * np.eye(3)
    Qa = (noise.sigma_a ** 2 / dt) * np.eye(3)
    for k in range(gyro.shape[0]):
        w = gyro[k] - bg_bar
        a = accel[k] - ba_bar
        Ek = exp_so3(w * dt)
        Jr = right_jacobian_so3(w * dt)
        Ax = skew(a)
        # covariance of the errors (dphi, dv, dp) before this sample's update
        A = np.zeros((9, 9))
        A[0:3, 0:3] = Ek.T
        A[3:6, 0:3] = -dR @ Ax * dt
        A[3:6, 3:6] = np.eye(3)
        A[6:9, 0:3] = -0.5 * dR @ Ax * dt * dt
        A[6:9, 3:6] = np.eye(3) * dt
        A[6:9, 6:9] = np.eye(3)
        Bg = np.zeros((9, 3))
        Bg[0:3] = Jr * dt
        Ba = np.zeros((9, 3))
        Ba[3:6] = dR * dt
        Ba[6:9] = 0.5 * dR * dt * dt
        cov = A @ cov @ A.T + Bg @ Qg @ Bg.T + Ba @ Qa @ Ba.T
        # bias Jacobians (use dR, dv and J_Rg before the update)
        J_pa = J_pa + J_va * dt - 0.5 * dR * dt * dt
        J_pg = J_pg + J_vg * dt - 0.5 * dR @ Ax @ J_Rg * dt * dt
        J_va = J_va - dR * dt
        J_vg = J_vg - dR @ Ax @ J_Rg * dt
        J_Rg = Ek.T @ J_Rg - Jr * dt
        # the preintegrated measurement
        dp = dp + dv * dt + 0.5 * dR @ a * dt * dt
        dv = dv + dR @ a * dt
        dR = dR @ Ek
    return Preintegration(dR=dR, dv=dv, dp=dp, dT=dt * gyro.shape[0], J_Rg=J_Rg, J_vg=J_vg, J_va=J_va,
                          J_pg=J_pg, J_pa=J_pa, cov=cov, bg_bar=bg_bar.copy(), ba_bar=ba_bar.copy())


def base_position(pose):
    """p = -R^T t of a base-from-world pose."""
    return -pose[:, :3].T @ pose[:, 3]


def imu_residual(pose_i, v_i, ba_i, bg_i, pose_j, v_j, ba_j, bg_j, pre: Preintegration, g):
    """The 15-vector (r_R, r_v, r_p, r_ba, r_bg) of the factor between states i and j."""
    Ri, Rj = pose_i[:, :3], pose_j[:, :3]
    pi, pj = base_position(pose_i), base_position(pose_j)
    dbg = bg_i - pre.bg_bar
    dba = ba_i - pre.ba_bar
    dRc = pre.dR @ exp_so3(pre.J_Rg @ dbg)
    rR = log_so3(dRc.T @ Ri @ Rj.T)
    dT = pre.dT
    rv = Ri @ (v_j - v_i - g * dT) - (pre.dv + pre.J_vg @ dbg + pre.J_va @ dba)
    rp = Ri @ (pj - pi - v_i * dT - 0.5 * g * dT * dT) - (pre.dp + pre.J_pg @ dbg + pre.J_pa @ dba)
    return np.concatenate([rR, rv, rp, ba_j - ba_i, bg_j - bg_i])


def imu_jacobians(pose_i, v_i, ba_i, bg_i, pose_j, v_j, ba_j, bg_j, pre: Preintegration, g):
    """(15, 15) Jacobians of the residual w.r.t. state i and state j, each in
    the order (rho, phi, v, b^a, b^w)."""
    Ri, Rj = pose_i[:, :3], pose_j[:, :3]
    pi, pj = base_position(pose_i), base_position(pose_j)
    dbg = bg_i - pre.bg_bar
    dRc = pre.dR @ exp_so3(pre.J_Rg @ dbg)
    E = dRc.T @ Ri @ Rj.T
    rR = log_so3(E)
    Jr_inv = np.linalg.inv(right_jacobian_so3(rR))
    dT = pre.dT
    wv = Ri @ (v_j - v_i - g * dT)
    wp = Ri @ (pj - pi - v_i * dT - 0.5 * g * dT * dT)
    I3 = np.eye(3)
    Ji = np.zeros((15, 15))
    Jj = np.zeros((15, 15))
    # rows 0-2: r_R
    Ji[0:3, 3:6] = Jr_inv @ Rj @ Ri.T
    Ji[0:3, 12:15] = -Jr_inv @ E.T @ right_jacobian_so3(pre.J_Rg @ dbg) @ pre.J_Rg
    Jj[0:3, 3:6] = -Jr_inv
    # rows 3-5: r_v
    Ji[3:6, 3:6] = -skew(wv)
    Ji[3:6, 6:9] = -Ri
    Ji[3:6, 9:12] = -pre.J_va
    Ji[3:6, 12:15] = -pre.J_vg
    Jj[3:6, 6:9] = Ri
    # rows 6-8: r_p
    Ji[6:9, 0:3] = I3
    Ji[6:9, 3:6] = -skew(wp)
    Ji[6:9, 6:9] = -Ri * dT
    Ji[6:9, 9:12] = -pre.J_pa
    Ji[6:9, 12:15] = -pre.J_pg
    Jj[6:9, 0:3] = -Ri @ Rj.T
    # rows 9-14: bias random walk
    Ji[9:12, 9:12] = -I3
    Jj[9:12, 9:12] = I3
    Ji[12:15, 12:15] = -I3
    Jj[12:15, 12:15] = I3
    return Ji, Jj


def imu_information(pre: Preintegration, noise: ImuNoise = None):
    """Sigma^-1 (15, 15): inverse of the preintegrated 9x9 covariance and of the
    bias random walk over the factor's interval."""
    noise = noise or ImuNoise()
    Info = np.zeros((15, 15))
    Info[0:9, 0:9] = np.linalg.inv(pre.cov)
    Info[9:12, 9:12] = np.eye(3) / (noise.sigma_ba ** 2 * pre.dT)
    Info[12:15, 12:15] = np.eye(3) / (noise.sigma_bg ** 2 * pre.dT)
    return Info


@dataclasses.dataclass
class ViProblem:
    """A visual window (``oracle.Problem``) plus IMU factors between states."""
    visual: object                  # oracle.Problem
    factors: List[tuple]            # (i, j, Preintegration, information (15, 15))
    gravity: np.ndarray             # (3,)


@dataclasses.dataclass
class ViState:
    poses: np.ndarray               # (N, 3, 4) base-from-world
    vel: np.ndarray                 # (N, 3) world frame
    ba: np.ndarray                  # (N, 3)
    bg: np.ndarray                  # (N, 3)
    points: np.ndarray              # (M, 3)

    def copy(self):
        return ViState(self.poses.copy(), self.vel.copy(), self.ba.copy(), self.bg.copy(), self.points.copy())


def imu_cost(x: ViState, vp: ViProblem):
    F = 0.0
    for i, j, pre, Info in vp.factors:
        r = imu_residual(x.poses[i], x.vel[i], x.ba[i], x.bg[i], x.poses[j], x.vel[j], x.ba[j], x.bg[j],
                         pre, vp.gravity)
        F += 0.5 * float(r @ Info @ r)
    return F


def vi_cost(x: ViState, vp: ViProblem, delta):
    return visual_cost(x.poses, x.points, vp.visual, delta) + imu_cost(x, vp)


def state_columns(vp: ViProblem):
    """Column of each state's block in the VI system: per state its pose
    tangent (6, when the pose is free) then v, b^a, b^w (9); then the points.
    Returns (pose_col (N,), vel_col (N,), n_state_cols)."""
    fixed = vp.visual.pose_fixed
    N = fixed.shape[0]
    pose_col = np.full(N, -1, np.int64)
    vel_col = np.zeros(N, np.int64)
    c = 0
    for k in range(N):
        if not fixed[k]:
            pose_col[k] = c
            c += 6
        vel_col[k] = c
        c += 9
    return pose_col, vel_col, c


def vi_normal_equations(x: ViState, vp: ViProblem, delta):
    """H and g of the damped-free Gauss-Newton system over all VI variables."""
    prob = vp.visual
    pose_col, vel_col, ns = state_columns(vp)
    M = prob.n_points
    n = ns + 3 * M
    H = np.zeros((n, n))
    g = np.zeros(n)
    # visual part, from the visual normal equations (free poses, then points)
    Hv, gv = normal_equations_dense(x.poses, x.points, prob, delta)
    free_poses = np.flatnonzero(~prob.pose_fixed)
    vis_cols = np.concatenate([pose_col[k] + np.arange(6) for k in free_poses] + [ns + np.arange(3 * M)])
    H[np.ix_(vis_cols, vis_cols)] += Hv
    g[vis_cols] += gv
    # IMU factors
    for i, j, pre, Info in vp.factors:
        r = imu_residual(x.poses[i], x.vel[i], x.ba[i], x.bg[i], x.poses[j], x.vel[j], x.ba[j], x.bg[j],
                         pre, vp.gravity)
        Ji, Jj = imu_jacobians(x.poses[i], x.vel[i], x.ba[i], x.bg[i], x.poses[j], x.vel[j], x.ba[j],
                               x.bg[j], pre, vp.gravity)
        cols, blocks = [], []
        for k, J in ((i, Ji), (j, Jj)):
            if pose_col[k] >= 0:
                cols.append(pose_col[k] + np.arange(6))
                blocks.append(J[:, 0:6])
            cols.append(vel_col[k] + np.arange(9))
            blocks.append(J[:, 6:15])
        c = np.concatenate(cols)
        Jf = np.concatenate(blocks, axis=1)
        H[np.ix_(c, c)] += Jf.T @ Info @ Jf
        g[c] += Jf.T @ Info @ r
    return H, g


def vi_apply_step(x: ViState, vp: ViProblem, d):
    pose_col, vel_col, ns = state_columns(vp)
    y = x.copy()
    for k in range(x.poses.shape[0]):
        if pose_col[k] >= 0:
            y.poses[k] = retract_pose(x.poses[k], d[pose_col[k]:pose_col[k] + 6])
        c = vel_col[k]
        y.vel[k] = x.vel[k] + d[c:c + 3]
        y.ba[k] = x.ba[k] + d[c + 3:c + 6]
        y.bg[k] = x.bg[k] + d[c + 6:c + 9]
    y.points = x.points + d[ns:].reshape(-1, 3)
    return y


@dataclasses.dataclass
class ViResult:
    state: ViState
    initial_cost: float
    final_cost: float
    final_lambda: float
    accepted: int
    chol_failures: int
    trace: List[dict]


def vi_lm_solve(x0: ViState, vp: ViProblem, settings: LMSettings = None,
                decisions: Optional[List[bool]] = None) -> ViResult:
    """Exactly ``settings.max_iters`` LM attempts on the VI cost (Eq. 9), with
    the schedule of ``oracle.lm.lm_solve``; ``decisions`` replays a given
    accept / reject sequence."""
    st = settings or LMSettings()
    x = x0.copy()
    delta = st.huber_delta
    F = vi_cost(x, vp, delta)
    F0 = F
    lam = st.lambda_init
    system = None
    trace = []
    n_acc = n_chol = 0
    for it in range(st.max_iters):
        if system is None:
            system = vi_normal_equations(x, vp, delta)
        H, g = system
        step = _chol_solve(_damp(H, lam), -g)
        rec = dict(iter=it, cost=F, lam=lam, cand_cost=math.nan, status="ok")
        valid = step is not None
        if not valid:
            rec["status"] = "chol_fail"
            n_chol += 1
        else:
            cand = vi_apply_step(x, vp, step)
            _, xc = transform(cand.poses, cand.points, vp.visual)
            if np.any(~(xc[:, 2] > st.min_depth)):
                valid = False
                rec["status"] = "depth"
            else:
                rec["cand_cost"] = vi_cost(cand, vp, delta)
        accept = valid and rec["cand_cost"] < F
        if decisions is not None:
            forced = bool(decisions[it])
            if forced and not valid:
                raise ValueError(f"replayed acceptance of an invalid candidate at attempt {it}")
            rec["own_decision"] = accept
            accept = forced
        if accept:
            x, F = cand, rec["cand_cost"]
            lam = max(lam / st.lambda_down, st.lambda_min)
            system = None
            n_acc += 1
        else:
            lam = min(lam * st.lambda_up, st.lambda_max)
        rec["accepted"] = accept
        rec["cost_after"] = F
        rec["lam_after"] = lam
        trace.append(rec)
    return ViResult(state=x, initial_cost=F0, final_cost=F, final_lambda=lam, accepted=n_acc,
                    chol_failures=n_chol, trace=trace)


def vi_gradient(x: ViState, vp: ViProblem, delta):
    """g of the VI system (the exact gradient of the cost over the variables)."""
    return vi_normal_equations(x, vp, delta)[1]


__all__ = ["ImuNoise", "Preintegration", "preintegrate", "imu_residual", "imu_jacobians",
           "imu_information", "ViProblem", "ViState", "vi_cost", "imu_cost", "vi_normal_equations",
           "vi_apply_step", "vi_lm_solve", "vi_gradient", "state_columns", "base_position", "GRAVITY"]
