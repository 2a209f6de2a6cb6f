"""Pins of the visual-inertial oracle (Sec. 2.2, "Visual-Inertial", Eq. 9):
IMU preintegration, the IMU factor and its Jacobians, and the VI-SBA solve.

Each pin is fixed by something other than the oracle's own formulas:
closed-form integrals of constant rates, finite differences, a Monte-Carlo
estimate of the preintegrated noise, the exact consistency of noiseless
samples with the motion that produced them, and recovery of the ground truth
from noiseless data."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import bagen
import oracle
from oracle import imu


def _rotvec(R):
    return Rotation.from_matrix(R).as_rotvec()


def _states(vw, P, vel, ba, bg, L):
    return imu.ViState(poses=np.array(P, float), vel=np.array(vel, float), ba=np.array(ba, float),
                       bg=np.array(bg, float), points=np.array(L, float))


def _vi_problem(vw, bias_bar=None, prob=None):
    w = vw.window
    prob = prob or oracle.Problem.from_window(w)
    n = imu.ImuNoise(*vw.noise)
    factors = []
    for i in range(w.n_poses - 1):
        bg_bar = vw.bg_init[i] if bias_bar is None else bias_bar[1]
        ba_bar = vw.ba_init[i] if bias_bar is None else bias_bar[0]
        pre = imu.preintegrate(vw.gyro[i], vw.accel[i], vw.dt, bg_bar, ba_bar, n)
        factors.append((i, i + 1, pre, imu.imu_information(pre, n)))
    return imu.ViProblem(visual=prob, factors=factors, gravity=vw.gravity)


# ---------------------------------------------------------------- preintegration

def test_constant_rate_rotation_is_the_exponential():
    w = np.array([0.3, -0.2, 0.5])
    n, dt = 80, 0.005
    pre = imu.preintegrate(np.tile(w, (n, 1)), np.zeros((n, 3)), dt, np.zeros(3), np.zeros(3))
    R = Rotation.from_rotvec(w * n * dt).as_matrix()
    assert np.abs(pre.dR - R).max() < 1e-13
    assert np.abs(pre.dv).max() == 0.0 and np.abs(pre.dp).max() == 0.0
    assert pre.dT == pytest.approx(n * dt)


def test_constant_force_without_rotation_is_uniform_acceleration():
    a = np.array([0.7, -1.1, 9.5])
    ba = np.array([0.1, 0.2, -0.3])
    n, dt = 60, 0.005
    T = n * dt
    pre = imu.preintegrate(np.zeros((n, 3)), np.tile(a + ba, (n, 1)), dt, np.zeros(3), ba)
    assert np.abs(pre.dR - np.eye(3)).max() == 0.0
    assert np.abs(pre.dv - a * T).max() < 1e-13
    assert np.abs(pre.dp - 0.5 * a * T * T).max() < 1e-13


def test_bias_jacobians_match_finite_differences():
    vw = bagen.make_vi_window(seed=9001, n_kf=3, n_lm=60)
    gy, ac, dt = vw.gyro[0], vw.accel[0], vw.dt
    bg0, ba0 = np.array([0.01, -0.02, 0.015]), np.array([0.05, -0.03, 0.02])
    pre = imu.preintegrate(gy, ac, dt, bg0, ba0)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        gp, gm = (imu.preintegrate(gy, ac, dt, bg0 + s * e, ba0) for s in (1, -1))
        ap, am = (imu.preintegrate(gy, ac, dt, bg0, ba0 + s * e) for s in (1, -1))
        dphi = (_rotvec(pre.dR.T @ gp.dR) - _rotvec(pre.dR.T @ gm.dR)) / (2 * h)
        assert np.abs(dphi - pre.J_Rg[:, k]).max() < 1e-7 * max(1.0, np.abs(pre.J_Rg).max())
        assert np.abs((gp.dv - gm.dv) / (2 * h) - pre.J_vg[:, k]).max() < 1e-7
        assert np.abs((gp.dp - gm.dp) / (2 * h) - pre.J_pg[:, k]).max() < 1e-7
        assert np.abs((ap.dv - am.dv) / (2 * h) - pre.J_va[:, k]).max() < 1e-7
        assert np.abs((ap.dp - am.dp) / (2 * h) - pre.J_pa[:, k]).max() < 1e-7


def test_preintegrated_covariance_matches_monte_carlo():
    # noiseless samples of one keyframe interval, then many noisy copies
    # integrated trial-parallel (Rotation compositions), against the
    # propagated covariance of (dphi, dv, dp)
    vw = bagen.make_vi_window(seed=9002, n_kf=2, n_lm=40, imu_noise=False)
    gy, ac, dt = vw.gyro[0], vw.accel[0], vw.dt
    noise = imu.ImuNoise(sigma_g=2e-3, sigma_a=2e-2)
    pre = imu.preintegrate(gy, ac, dt, np.zeros(3), np.zeros(3), noise)
    rng = np.random.default_rng(5)
    T = 20000
    R = Rotation.identity(T)
    dv = np.zeros((T, 3))
    dp = np.zeros((T, 3))
    for k in range(gy.shape[0]):
        w = gy[k] + rng.normal(scale=noise.sigma_g / math.sqrt(dt), size=(T, 3))
        a = ac[k] + rng.normal(scale=noise.sigma_a / math.sqrt(dt), size=(T, 3))
        Ra = R.apply(a)
        dp = dp + dv * dt + 0.5 * Ra * dt * dt
        dv = dv + Ra * dt
        R = R * Rotation.from_rotvec(w * dt)
    err = np.concatenate([(Rotation.from_matrix(np.broadcast_to(pre.dR.T, (T, 3, 3))) * R).as_rotvec(),
                          dv - pre.dv, dp - pre.dp], axis=1)
    C = np.cov(err.T)
    Wh = np.linalg.inv(np.linalg.cholesky(pre.cov))
    M = Wh @ C @ Wh.T
    assert np.abs(M - np.eye(9)).max() < 0.06, np.abs(M - np.eye(9)).max()


# ---------------------------------------------------------------- the factor

def test_noiseless_samples_give_a_zero_residual():
    vw = bagen.make_vi_window(seed=9003, n_kf=5, n_lm=80, imu_noise=False)
    w = vw.window
    for i in range(w.n_poses - 1):
        pre = imu.preintegrate(vw.gyro[i], vw.accel[i], vw.dt, vw.bg_gt, vw.ba_gt)
        r = imu.imu_residual(w.poses_gt[i], vw.vel_gt[i], vw.ba_gt, vw.bg_gt, w.poses_gt[i + 1],
                             vw.vel_gt[i + 1], vw.ba_gt, vw.bg_gt, pre, vw.gravity)
        assert np.abs(r).max() < 1e-11, r
    # a wrong gravity or a shifted velocity does not
    pre = imu.preintegrate(vw.gyro[0], vw.accel[0], vw.dt, vw.bg_gt, vw.ba_gt)
    r = imu.imu_residual(w.poses_gt[0], vw.vel_gt[0] + 0.01, vw.ba_gt, vw.bg_gt, w.poses_gt[1],
                         vw.vel_gt[1], vw.ba_gt, vw.bg_gt, pre, vw.gravity)
    assert np.abs(r[3:9]).max() > 1e-3


def test_factor_jacobians_match_finite_differences():
    vw = bagen.make_vi_window(seed=9004, n_kf=3, n_lm=60)
    w = vw.window
    rng = np.random.default_rng(3)
    pre = imu.preintegrate(vw.gyro[0], vw.accel[0], vw.dt, np.zeros(3), np.zeros(3))
    # a state away from the minimum, with a bias change from the linearisation point
    st = [w.poses_init[0], vw.vel_init[0], rng.normal(scale=0.05, size=3), rng.normal(scale=0.01, size=3),
          w.poses_init[1], vw.vel_init[1], rng.normal(scale=0.05, size=3), rng.normal(scale=0.01, size=3)]
    Ji, Jj = imu.imu_jacobians(*st, pre, vw.gravity)
    h = 1e-6
    for side, J in ((0, Ji), (4, Jj)):
        for c in range(15):
            vals = []
            for s in (1, -1):
                x = [a.copy() for a in st]
                if c < 6:
                    e = np.zeros(6)
                    e[c] = s * h
                    x[side] = oracle.retract_pose(st[side], e)
                else:
                    blk = side + 1 + (c - 6) // 3
                    x[blk][(c - 6) % 3] += s * h
                vals.append(imu.imu_residual(*x, pre, vw.gravity))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert np.abs(fd - J[:, c]).max() < 1e-6 * max(1.0, np.abs(J[:, c]).max()), (side, c)


# ---------------------------------------------------------------- the VI solve

def test_vi_gradient_matches_finite_differences():
    vw = bagen.make_vi_window(seed=9005, n_kf=4, n_lm=30)
    w = vw.window
    vp = _vi_problem(vw)
    x = _states(vw, w.poses_init, vw.vel_init, vw.ba_init + 0.01, vw.bg_init - 0.002, w.points_init)
    g = imu.vi_gradient(x, vp, 1.0)
    r = oracle.residuals(x.poses, x.points, vp.visual)
    assert np.any(np.sum(r * r, 1) > 1.0)          # Huber's outer branch is exercised
    h = 1e-6
    rng = np.random.default_rng(1)
    for c in rng.choice(g.size, size=60, replace=False):
        d = np.zeros(g.size)
        d[c] = h
        Fp = imu.vi_cost(imu.vi_apply_step(x, vp, d), vp, 1.0)
        Fm = imu.vi_cost(imu.vi_apply_step(x, vp, -d), vp, 1.0)
        fd = (Fp - Fm) / (2 * h)
        assert abs(fd - g[c]) < 1e-6 * max(1.0, abs(g[c])) + 1e-5 * np.abs(g).max() * 1e-3, (c, fd, g[c])


def test_noiseless_vi_window_recovers_ground_truth():
    # noiseless pixels and IMU, preintegrated at the true biases; start
    # perturbed (poses, velocities, points) with zero bias estimates
    vw = bagen.make_vi_window(seed=9006, n_kf=6, n_lm=120, sigma_px=0.0, imu_noise=False)
    w = vw.window
    vp = _vi_problem(vw, bias_bar=(vw.ba_gt, vw.bg_gt))
    x0 = _states(vw, w.poses_init, vw.vel_init, vw.ba_init, vw.bg_init, w.points_init)
    res = imu.vi_lm_solve(x0, vp, oracle.LMSettings(max_iters=40, lambda_init=1e-3))
    x = res.state
    assert res.final_cost < 1e-14 * res.initial_cost
    costs = [t["cost"] for t in res.trace if t["accepted"]]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    assert np.abs(x.poses - w.poses_gt).max() < 1e-7
    assert np.abs(x.points - w.points_gt).max() < 1e-6
    assert np.abs(x.vel - vw.vel_gt).max() < 1e-7
    assert np.abs(x.ba - vw.ba_gt).max() < 1e-6 and np.abs(x.bg - vw.bg_gt).max() < 1e-7


def test_noisy_vi_window_improves_on_vision_alone_for_scale():
    # with IMU the mono window has metric scale: the VI solve's camera track
    # length is close to the truth without any scale alignment
    vw = bagen.make_vi_window(seed=9007, n_kf=8, n_lm=200)
    w = vw.window
    vp = _vi_problem(vw)
    x0 = _states(vw, w.poses_init, vw.vel_init, vw.ba_init, vw.bg_init, w.points_init)
    res = imu.vi_lm_solve(x0, vp, oracle.LMSettings(max_iters=20))
    c = np.stack([imu.base_position(P) for P in res.state.poses])
    cg = np.stack([imu.base_position(P) for P in w.poses_gt])
    L, Lg = np.linalg.norm(c[-1] - c[0]), np.linalg.norm(cg[-1] - cg[0])
    assert abs(L / Lg - 1.0) < 0.02, (L, Lg)
    assert res.final_cost < 0.1 * res.initial_cost
