"""Pins of the motion-only oracle (oracle/pnp.py) against things other than itself.

* noiseless frames: the ground-truth pose is recovered (stereo, rig, mono and the
  map-frame form of Eq. 14), and the generator's pixels give zero residual there;
* the gradient g equals central differences of the cost along Exp(e) T;
* plain least squares: the converged pose equals scipy.optimize.least_squares
  over the same 6 tangent parameters;
* robust (Huber) cost: the converged cost is not above a Nelder-Mead minimum of
  the same cost and the poses agree;
* Eq. 14: the pose found against the map frame, composed with T^mw, equals the
  pose found against the world points directly;
* every accepted step lowers the cost and lambda follows the schedule;
* degenerate frames: no observations (pose kept), a depth guard that rejects
  every candidate (pose kept).
"""
import numpy as np
import pytest
import scipy.optimize

import bagen
import oracle
from oracle import pnp
from oracle.lm import LMSettings


def _frame(b, f, mfw=True):
    sl = b.frame_slice(f)
    return pnp.PnPFrame(intrinsics=b.intrinsics, extrinsics=b.extrinsics, points=b.points,
                        obs_point=b.obs_point[sl], obs_cam=b.obs_cam[sl], obs_uv=b.obs_uv[sl],
                        obs_w=b.obs_w[sl],
                        map_from_world=(b.map_from_world[f] if (mfw and b.map_from_world is not None)
                                        else None))


def _pose_err(A, B):
    ang = oracle.rotation_angle(A[:, :3], B[:, :3])
    return float(ang), float(np.linalg.norm(A[:, 3] - B[:, 3]))


@pytest.mark.parametrize("kind,map_frame,mono", [("stereo", False, False), ("stereo", True, False),
                                                 ("rig", False, False), ("stereo", False, True)])
def test_noiseless_frames_recover_ground_truth(kind, map_frame, mono):
    b = bagen.make_pnp_batch(3, kind, 40, seed=11, sigma=0.0, outlier_frac=0.0, map_frame=map_frame)
    for f in range(b.n_frames):
        fr = _frame(b, f)
        if mono:
            keep = fr.obs_cam == 0
            fr = pnp.PnPFrame(fr.intrinsics, fr.extrinsics, fr.points, fr.obs_point[keep],
                              fr.obs_cam[keep], fr.obs_uv[keep], fr.obs_w[keep], fr.map_from_world)
        prob = fr.problem()
        r = oracle.residuals(b.poses_gt[f][None], fr.frame_points(), prob)
        assert np.abs(r).max() < 1e-9
        res = pnp.pnp_solve(b.poses_init[f], fr, LMSettings(max_iters=20))
        ang, dt = _pose_err(res.pose, b.poses_gt[f])
        assert ang < 1e-9 and dt < 1e-8, (ang, dt)


def test_gradient_matches_central_differences():
    b = bagen.make_pnp_batch(1, "stereo", 30, seed=12, outlier_frac=0.1)
    fr = _frame(b, 0)
    T = b.poses_init[0]
    for delta in (1.0, np.inf):
        _, g = pnp.pnp_normal_equations(T, fr, delta)
        h = 1e-6
        fd = np.zeros(6)
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            fd[k] = (pnp.pnp_cost(oracle.retract_pose(T, e), fr, delta)
                     - pnp.pnp_cost(oracle.retract_pose(T, -e), fr, delta)) / (2 * h)
        assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(g).max())


def test_least_squares_minimum_matches_scipy():
    b = bagen.make_pnp_batch(1, "rig", 50, seed=13, outlier_frac=0.0)
    fr = _frame(b, 0)
    prob = fr.problem()
    pts = fr.frame_points()
    T0 = b.poses_init[0]
    res = pnp.pnp_solve(T0, fr, LMSettings(max_iters=40, huber_delta=np.inf))

    def fun(xi):
        return oracle.residuals(oracle.retract_pose(T0, xi)[None], pts, prob).reshape(-1)

    ls = scipy.optimize.least_squares(fun, np.zeros(6), xtol=1e-15, ftol=1e-15, gtol=1e-15)
    T_ls = oracle.retract_pose(T0, ls.x)
    ang, dt = _pose_err(res.pose, T_ls)
    assert ang < 1e-9 and dt < 1e-8, (ang, dt)


def test_robust_minimum_not_above_nelder_mead():
    b = bagen.make_pnp_batch(1, "stereo", 20, seed=14, outlier_frac=0.15)
    fr = _frame(b, 0)
    T0 = b.poses_init[0]
    res = pnp.pnp_solve(T0, fr, LMSettings(max_iters=60, huber_delta=1.0))

    def f(xi):
        return pnp.pnp_cost(oracle.retract_pose(res.pose, xi), fr, 1.0)

    nm = scipy.optimize.minimize(f, np.zeros(6), method="Nelder-Mead",
                                 options=dict(xatol=1e-12, fatol=1e-14, maxiter=40000, maxfev=40000,
                                              initial_simplex=np.vstack([np.zeros(6), 1e-3 * np.eye(6)])))
    assert res.final_cost <= nm.fun + 1e-9 * max(1.0, nm.fun)
    ang, dt = _pose_err(res.pose, oracle.retract_pose(res.pose, nm.x))
    assert ang < 1e-5 and dt < 1e-4, (ang, dt)


def test_map_frame_pose_composes_with_the_world_pose():
    b = bagen.make_pnp_batch(2, "stereo", 40, seed=15, map_frame=True)
    st = LMSettings(max_iters=30)
    for f in range(b.n_frames):
        fr_m = _frame(b, f, mfw=True)
        fr_w = _frame(b, f, mfw=False)
        T_mw = b.map_from_world[f]
        res_m = pnp.pnp_solve(b.poses_init[f], fr_m, st)
        init_w = bagen._compose(b.poses_init[f], T_mw)
        res_w = pnp.pnp_solve(init_w, fr_w, st)
        ang, dt = _pose_err(bagen._compose(res_m.pose, T_mw), res_w.pose)
        assert ang < 1e-9 and dt < 1e-8, (ang, dt)
        assert abs(res_m.final_cost - res_w.final_cost) <= 1e-9 * res_w.final_cost


def test_accepted_steps_lower_the_cost_and_lambda_follows_the_schedule():
    b = bagen.make_pnp_batch(2, "rig", 60, seed=16, outlier_frac=0.05)
    for f in range(b.n_frames):
        res = pnp.pnp_solve(b.poses_init[f], _frame(b, f), LMSettings(max_iters=15))
        for t in res.trace:
            if t["accepted"]:
                assert t["cand_cost"] < t["cost"]
                assert np.isclose(t["lam_after"], max(t["lam"] / 10, 1e-10))
            else:
                assert np.isclose(t["lam_after"], min(t["lam"] * 10, 1e10))
        assert res.final_cost < res.initial_cost


def test_frame_without_observations_keeps_its_pose():
    b = bagen.make_pnp_batch(1, "stereo", 10, seed=17)
    fr = pnp.PnPFrame(b.intrinsics, b.extrinsics, b.points, np.zeros(0, np.int64), np.zeros(0, np.int64),
                      np.zeros((0, 2)), np.zeros(0))
    res = pnp.pnp_solve(b.poses_init[0], fr, LMSettings(max_iters=5))
    assert np.array_equal(res.pose, b.poses_init[0])
    assert res.accepted == 0 and res.final_cost == 0.0


def test_depth_guard_rejects_every_candidate():
    b = bagen.make_pnp_batch(1, "stereo", 20, seed=18)
    res = pnp.pnp_solve(b.poses_init[0], _frame(b, 0), LMSettings(max_iters=4, min_depth=1e6))
    assert res.accepted == 0
    assert all(t["status"] == "depth" for t in res.trace)
    assert np.array_equal(res.pose, b.poses_init[0])
