"""Pins of the triangulation oracle (oracle/triangulate.py) against things
other than itself.

* noiseless observations: the linear start is the true landmark and the
  refinement keeps it (cost 0);
* the 3x3 ray system equals the stacked least-squares problem solved by
  numpy.linalg.lstsq;
* a rectified stereo pair: the textbook depth Z = f b / disparity;
* plain least squares: the refined point equals scipy.optimize.least_squares;
* robust cost: the refined cost is not above a Nelder-Mead minimum;
* the gradient g equals central differences of the cost;
* degenerate landmarks (one view, identical rays) and a start behind a camera;
* accepted steps lower the cost and lambda follows the schedule.
"""
import numpy as np
import pytest
import scipy.optimize

import bagen
import oracle
from oracle import triangulate as tri
from oracle.lm import LMSettings


def _batch(noiseless=False, windows=2, cfg=1):
    ws = [bagen.make_window(cfg, i) for i in range(windows)]
    b = bagen.make_tri_batch(ws)
    if noiseless:
        for j in range(b.n_points):
            ob = _obs(b, j)
            r = oracle.residuals(ob.poses, b.points_gt[j][None], ob.problem())
            b.obs_uv[b.point_slice(j)] = ob.obs_uv + r
    return b


def _obs(b, j):
    return tri.landmark_obs(b.intrinsics, b.extrinsics, b.poses, b.point_obs_begin, b.obs_pose, b.obs_cam,
                            b.obs_uv, b.obs_w, j)


def test_noiseless_linear_start_is_the_landmark():
    b = _batch(noiseless=True)
    for j in range(0, b.n_points, 7):
        ob = _obs(b, j)
        p0, st = tri.linear_point(ob)
        assert st == tri.STATUS_OK
        assert np.abs(p0 - b.points_gt[j]).max() <= 1e-9 * max(1.0, np.abs(b.points_gt[j]).max())
        res = tri.triangulate(ob, LMSettings(max_iters=5))
        assert res.status == tri.STATUS_OK and res.final_cost < 1e-18


def test_ray_system_equals_stacked_least_squares():
    b = _batch()
    for j in range(0, b.n_points, 11):
        ob = _obs(b, j)
        p0, st = tri.linear_point(ob)
        c, d = tri.rays(ob)
        rows, rhs = [], []
        for o in range(c.shape[0]):
            P = np.sqrt(ob.obs_w[o]) * (np.eye(3) - np.outer(d[o], d[o]))
            rows.append(P)
            rhs.append(P @ c[o])
        ref = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)[0]
        assert np.abs(p0 - ref).max() <= 1e-8 * max(1.0, np.abs(ref).max())


def _stereo_pair():
    K = np.array([[718.0, 718.0, 607.0, 185.0]] * 2)
    E = np.zeros((2, 3, 4))
    E[:, :, :3] = np.eye(3)
    E[1, 0, 3] = -0.54
    T = np.zeros((1, 3, 4))
    T[0, :, :3] = np.eye(3)
    return K, E, T


def test_rectified_stereo_depth_from_disparity():
    K, E, T = _stereo_pair()
    f, cx, cy, base = 718.0, 607.0, 185.0, 0.54
    for ul, disp, v in ((700.0, 12.5, 150.0), (300.0, 40.0, 250.0), (1000.0, 3.2, 100.0)):
        ob = tri.TriObs(K, E, T, np.array([0, 0]), np.array([0, 1]),
                        np.array([[ul, v], [ul - disp, v]]), np.ones(2))
        Z = f * base / disp
        ref = np.array([(ul - cx) * Z / f, (v - cy) * Z / f, Z])
        p0, st = tri.linear_point(ob)
        assert st == tri.STATUS_OK and np.abs(p0 - ref).max() <= 1e-9 * Z
        res = tri.triangulate(ob, LMSettings(max_iters=5))
        assert np.abs(res.point - ref).max() <= 1e-9 * Z and res.final_cost < 1e-18


def test_least_squares_minimum_matches_scipy():
    b = _batch(cfg=1, windows=1)
    st = LMSettings(max_iters=40, huber_delta=np.inf)
    for j in range(0, b.n_points, 17):
        ob = _obs(b, j)
        res = tri.triangulate(ob, st)
        p0, _ = tri.linear_point(ob)

        def fun(p):
            return oracle.residuals(ob.poses, p[None], ob.problem()).reshape(-1)

        ls = scipy.optimize.least_squares(fun, p0, xtol=1e-15, ftol=1e-15, gtol=1e-15)
        assert np.abs(res.point - ls.x).max() <= 1e-8 * max(1.0, np.abs(ls.x).max()), j


def test_robust_minimum_not_above_nelder_mead():
    b = _batch(cfg=1, windows=1)
    for j in range(0, b.n_points, 29):
        ob = _obs(b, j)
        res = tri.triangulate(ob, LMSettings(max_iters=60, huber_delta=1.0))
        nm = scipy.optimize.minimize(lambda p: tri.point_cost(p, ob, 1.0), res.point, method="Nelder-Mead",
                                     options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000, maxfev=20000,
                                                  initial_simplex=res.point + np.vstack([np.zeros(3),
                                                                                         1e-3 * np.eye(3)])))
        assert res.final_cost <= nm.fun + 1e-9 * max(1.0, nm.fun)
        assert np.abs(res.point - nm.x).max() < 1e-4 * max(1.0, np.abs(nm.x).max())


def test_gradient_matches_central_differences():
    b = _batch(cfg=2, windows=1)
    for j in range(0, b.n_points, 500):
        ob = _obs(b, j)
        p0, _ = tri.linear_point(ob)
        p = p0 + np.array([0.02, -0.01, 0.03])
        for delta in (1.0, np.inf):
            _, g = tri.point_normal_equations(p, ob, delta)
            h = 1e-6
            fd = np.array([(tri.point_cost(p + h * e, ob, delta) - tri.point_cost(p - h * e, ob, delta)) / (2 * h)
                           for e in np.eye(3)])
            assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(g).max())


def test_degenerate_landmarks():
    K, E, T = _stereo_pair()
    one = tri.TriObs(K, E, T, np.array([0]), np.array([0]), np.array([[600.0, 180.0]]), np.ones(1))
    assert tri.triangulate(one).status == tri.STATUS_DEGENERATE
    same = tri.TriObs(K, E, T, np.array([0, 0]), np.array([0, 0]), np.array([[600.0, 180.0]] * 2), np.ones(2))
    assert tri.triangulate(same).status == tri.STATUS_DEGENERATE


def test_start_behind_a_camera_is_kept_unrefined():
    K, E, T = _stereo_pair()
    # rays from the two centres diverge forward: they meet behind the rig
    ob = tri.TriObs(K, E, T, np.array([0, 0]), np.array([0, 1]),
                    np.array([[600.0, 185.0], [620.0, 185.0]]), np.ones(2))
    p0, _ = tri.linear_point(ob)
    assert p0[2] < 0
    res = tri.triangulate(ob)
    assert res.status == tri.STATUS_BEHIND and np.array_equal(res.point, p0) and res.accepted == 0


def test_accepted_steps_lower_the_cost_and_lambda_follows_the_schedule():
    b = _batch(cfg=2, windows=1)
    n_ok = 0
    for j in range(0, b.n_points, 125):
        res = tri.triangulate(_obs(b, j), LMSettings(max_iters=12))
        if res.status != tri.STATUS_OK:   # an outlier can pull the start behind a camera
            assert res.status == tri.STATUS_BEHIND
            continue
        n_ok += 1
        assert res.final_cost <= res.initial_cost
        for t in res.trace:
            if t["accepted"]:
                assert t["cand_cost"] < t["cost"]
                assert np.isclose(t["lam_after"], max(t["lam"] / 10, 1e-10))
            else:
                assert np.isclose(t["lam_after"], min(t["lam"] * 10, 1e10))
    assert n_ok >= 35
