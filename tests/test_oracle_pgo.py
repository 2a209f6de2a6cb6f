"""Pins of the pose-graph oracle (oracle/pgo.py) against things other than
itself.

* Log_SE3 inverts Exp_SE3; the rotation block of the series J_l equals the
  closed-form SO(3) left Jacobian; J_l satisfies Exp(xi + h d) ~ Exp(h J_l d) Exp(xi);
* Ad(T) satisfies Exp(Ad(T) xi) = T Exp(xi) T^-1;
* the edge Jacobians equal central differences of the residual under the left
  perturbation of either pose;
* dead reckoning along a tree of edges has zero cost (the residual's order and
  signs); a global transform of every pose leaves the cost unchanged;
* noiseless measurements: LM recovers the ground truth;
* plain least squares: the LM minimum equals scipy.optimize.least_squares over
  every free pose's tangent parameters; the dense and sparse backends agree;
* accepted steps lower the cost and lambda follows the schedule.
"""
import numpy as np
import pytest
import scipy.optimize

import bagen
from oracle import pgo
from oracle.lm import LMSettings
from oracle.se3 import exp_se3, left_jacobian_so3, retract_pose


def _graph(d):
    return pgo.PoseGraph(d.n_poses, d.edge_i, d.edge_j, d.deltas, d.edge_w, d.pose_fixed.astype(bool))


def _rand_xi(rng, scale=1.0):
    return np.concatenate([rng.normal(0, 1, 3), rng.normal(0, scale, 3)])


def test_log_inverts_exp_and_left_jacobian():
    rng = np.random.default_rng(1)
    for _ in range(20):
        xi = _rand_xi(rng, 0.8)
        assert np.abs(pgo.log_se3(exp_se3(xi)) - xi).max() < 1e-12
        J = pgo.left_jacobian_se3(xi)
        assert np.abs(J[3:, 3:] - left_jacobian_so3(xi[3:])).max() < 1e-13
        assert np.abs(J[:3, :3] - left_jacobian_so3(xi[3:])).max() < 1e-13
        d = rng.normal(0, 1, 6)
        h = 1e-6
        E0 = exp_se3(xi)
        lhs = [pgo.log_se3(pgo.compose(exp_se3(xi + s * h * d), pgo.inverse(E0))) for s in (1, -1)]
        fd = (lhs[0] - lhs[1]) / (2 * h)
        assert np.abs(fd - J @ d).max() < 1e-7 * max(1.0, np.abs(J @ d).max())


def test_adjoint_moves_a_perturbation_through_a_pose():
    rng = np.random.default_rng(2)
    for _ in range(10):
        T = exp_se3(_rand_xi(rng))
        xi = 0.3 * _rand_xi(rng)
        lhs = exp_se3(pgo.adjoint(T) @ xi)
        rhs = pgo.compose(pgo.compose(T, exp_se3(xi)), pgo.inverse(T))
        assert np.abs(lhs - rhs).max() < 1e-12


def test_edge_jacobians_match_central_differences():
    rng = np.random.default_rng(3)
    for _ in range(10):
        Ti, Tj = exp_se3(_rand_xi(rng)), exp_se3(_rand_xi(rng))
        D = pgo.compose(exp_se3(0.2 * _rand_xi(rng)), pgo.compose(pgo.inverse(Ti), Tj))
        r, B = pgo.edge_jacobian(Ti, Tj, D)
        h = 1e-6
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            fj = (pgo.residual(Ti, retract_pose(Tj, e), D) - pgo.residual(Ti, retract_pose(Tj, -e), D)) / (2 * h)
            fi = (pgo.residual(retract_pose(Ti, e), Tj, D) - pgo.residual(retract_pose(Ti, -e), Tj, D)) / (2 * h)
            assert np.abs(fj - B[:, k]).max() < 1e-7
            assert np.abs(fi + B[:, k]).max() < 1e-7


def test_dead_reckoning_along_a_tree_has_zero_cost_and_the_cost_is_gauge_invariant():
    d = bagen.make_pose_graph(laps=1, per_lap=40, seed=4)
    g = _graph(d)
    assert g.n_edges == d.n_poses - 1            # one lap: odometry only (a chain)
    assert pgo.graph_cost(d.poses_init, g) < 1e-24
    d2 = bagen.make_pose_graph(laps=2, per_lap=20, seed=5)
    g2 = _graph(d2)
    G = exp_se3(np.array([1.0, -2.0, 0.5, 0.3, -0.2, 0.9]))
    moved = np.stack([pgo.compose(G, T) for T in d2.poses_init])
    assert abs(pgo.graph_cost(moved, g2) - pgo.graph_cost(d2.poses_init, g2)) < 1e-12


def test_noiseless_graph_recovers_ground_truth():
    d = bagen.make_pose_graph(laps=2, per_lap=20, sigma_rot=0.0, sigma_trans=0.0, seed=6)
    g = _graph(d)
    rng = np.random.default_rng(7)
    init = d.poses_gt.copy()
    for k in range(1, d.n_poses):
        init[k] = retract_pose(init[k], 0.05 * _rand_xi(rng))
    res = pgo.pgo_solve(init, g, LMSettings(max_iters=20))
    assert res.final_cost < 1e-20
    assert np.abs(res.poses - d.poses_gt).max() < 1e-9


def test_least_squares_minimum_matches_scipy_and_backends_agree():
    d = bagen.make_pose_graph(laps=2, per_lap=6, seed=8, sigma_rot=0.02, sigma_trans=0.05, loop_prob=1.0)
    g = _graph(d)
    res = pgo.pgo_solve(d.poses_init, g, LMSettings(max_iters=30))
    res_s = pgo.pgo_solve(d.poses_init, g, LMSettings(max_iters=30), backend="sparse")
    # at the minimum a pose change of 1e-8 moves the cost by about 1e-16, so
    # the two solvers' rounding decides steps of that size: poses agree to
    # 1e-7, costs to 1e-12
    assert np.abs(res.poses - res_s.poses).max() < 1e-7
    assert abs(res.final_cost - res_s.final_cost) <= 1e-12 * res.final_cost
    free = np.nonzero(~g.pose_fixed)[0]

    def fun(x):
        P = d.poses_init.copy()
        for a, i in enumerate(free):
            P[i] = retract_pose(d.poses_init[i], x[6 * a:6 * a + 6])
        return np.concatenate([pgo.residual(P[g.edge_i[e]], P[g.edge_j[e]], g.deltas[e])
                               for e in range(g.n_edges)])

    ls = scipy.optimize.least_squares(fun, np.zeros(6 * free.size), xtol=1e-15, ftol=1e-15, gtol=1e-15)
    # same minimum: the oracle's cost is not above scipy's, its gradient
    # vanishes, and the poses agree within the flat valley's width (smallest
    # Hessian eigenvalue about 3e-3 here)
    assert res.final_cost <= 0.5 * float(ls.fun @ ls.fun) + 1e-12
    H, gv, _ = pgo.normal_equations(res.poses, g)
    assert np.abs(gv).max() < 1e-7
    ref = d.poses_init.copy()
    for a, i in enumerate(free):
        ref[i] = retract_pose(d.poses_init[i], ls.x[6 * a:6 * a + 6])
    assert np.abs(res.poses - ref).max() < 2e-5


def test_accepted_steps_lower_the_cost_and_lambda_follows_the_schedule():
    d = bagen.make_pose_graph(laps=2, per_lap=25, seed=9)
    res = pgo.pgo_solve(d.poses_init, _graph(d), LMSettings(max_iters=12))
    assert res.final_cost < res.initial_cost
    for t in res.trace:
        if t["accepted"]:
            assert t["cand_cost"] < t["cost"]
            assert np.isclose(t["lam_after"], max(t["lam"] / 10, 1e-10))
        else:
            assert np.isclose(t["lam_after"], min(t["lam"] * 10, 1e10))
