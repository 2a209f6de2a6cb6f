"""Pins of the FP64 oracle against things other than itself.

Each test fixes a part of the oracle by a hand-worked value, a closed form, a
library routine, brute force, finite differences or an invariant, chosen so that
a dropped term, a wrong sign or index, or a transposed operand fails one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.optimize
from scipy.spatial.transform import Rotation

import bagen
import oracle
from oracle import adjoint as oadj
from oracle import lm as olm
from oracle import model as om

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _prob(w):
    return oracle.Problem.from_window(w)


# ---------------------------------------------------------------------------
# projection / residual (Eq. 2)
# ---------------------------------------------------------------------------

def test_projection_hand_examples():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "projection_example.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = np.array([float(x) for x in row])
        K, Rbw, tbw, Rcb, tcb, p, o, r_ref = (v[0:4], v[4:13].reshape(3, 3), v[13:16],
                                               v[16:25].reshape(3, 3), v[25:28], v[28:31],
                                               v[31:33], v[33:35])
        prob = oracle.Problem(intrinsics=K[None], extrinsics=np.concatenate([Rcb, tcb[:, None]], 1)[None],
                              obs_pose=np.array([0]), obs_point=np.array([0]), obs_cam=np.array([0]),
                              obs_uv=o[None], obs_w=np.ones(1), pose_fixed=np.array([True]),
                              n_poses=1, n_points=1)
        pose = np.concatenate([Rbw, tbw[:, None]], 1)[None]
        r = oracle.residuals(pose, p[None], prob)[0]
        np.testing.assert_allclose(r, r_ref, rtol=0, atol=1e-9)


@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_noiseless_ground_truth_has_zero_residual(cfg):
    w = bagen.make_window(cfg)
    prob = _prob(w)
    # regenerate the exact pixels with the generator's own (independent) projection
    uv = np.empty_like(w.obs_uv)
    for o in range(w.n_obs):
        xc = bagen._to_cam(w.poses_gt[w.obs_pose[o]], w.extrinsics[w.obs_cam[o]],
                           w.points_gt[w.obs_point[o]][None])
        uv[o] = bagen._project(w.intrinsics[w.obs_cam[o]], xc)[0]
    prob.obs_uv = uv
    r = oracle.residuals(w.poses_gt, w.points_gt, prob)
    assert np.max(np.abs(r)) < 1e-9


# ---------------------------------------------------------------------------
# SO(3) / SE(3)
# ---------------------------------------------------------------------------

def test_exp_so3_matches_scipy_rotvec():
    rng = np.random.default_rng(1)
    for scale in (1e-7, 1e-5, 3e-4, 0.1, 1.0, 3.0):
        for _ in range(5):
            phi = rng.normal(size=3)
            phi *= scale / np.linalg.norm(phi)
            np.testing.assert_allclose(oracle.exp_so3(phi), Rotation.from_rotvec(phi).as_matrix(),
                                       rtol=0, atol=1e-14)


def test_left_jacobian_is_integral_of_exp():
    # J_l(phi) = int_0^1 Exp(s phi) ds (closed form of the left Jacobian)
    rng = np.random.default_rng(2)
    for scale in (1e-6, 0.3, 2.0):
        phi = rng.normal(size=3)
        phi *= scale / np.linalg.norm(phi)
        ref = np.array([[scipy.integrate.quad(lambda s: Rotation.from_rotvec(s * phi).as_matrix()[a, b],
                                              0, 1, epsabs=1e-14)[0] for b in range(3)] for a in range(3)])
        np.testing.assert_allclose(oracle.left_jacobian_so3(phi), ref, atol=1e-12)


def test_exp_se3_is_matrix_exponential():
    import scipy.linalg
    rng = np.random.default_rng(3)
    xi = rng.normal(size=6) * 0.7
    T = np.zeros((4, 4))
    T[:3, :3] = oracle.skew(xi[3:])
    T[:3, 3] = xi[:3]
    ref = scipy.linalg.expm(T)[:3]
    np.testing.assert_allclose(oracle.exp_se3(xi), ref, atol=1e-13)


def test_retract_is_left_multiplication():
    rng = np.random.default_rng(4)
    R = Rotation.random(random_state=5).as_matrix()
    T = np.concatenate([R, rng.normal(size=(3, 1))], 1)
    xi = rng.normal(size=6) * 0.2
    D = np.vstack([oracle.exp_se3(xi), [0, 0, 0, 1]])
    ref = (D @ np.vstack([T, [0, 0, 0, 1]]))[:3]
    np.testing.assert_allclose(oracle.retract_pose(T, xi), ref, atol=1e-14)


# ---------------------------------------------------------------------------
# Huber kernel
# ---------------------------------------------------------------------------

def test_huber_closed_form_and_continuity():
    d = 1.0
    s = np.array([0.0, 0.25, 1.0, 4.0, 9.0])
    rho, d1, d2 = oracle.huber(s, d)
    np.testing.assert_allclose(rho, [0.0, 0.25, 1.0, 3.0, 5.0], atol=0)
    np.testing.assert_allclose(d1, [1, 1, 1, 0.5, 1 / 3], atol=1e-15)
    np.testing.assert_allclose(d2, [0, 0, 0, -0.5 / 8, -0.5 / 27], atol=1e-15)
    # continuity of rho and rho' at the kink
    e = 1e-12
    r_lo, p_lo, _ = oracle.huber(np.array([1.0 - e]), d)
    r_hi, p_hi, _ = oracle.huber(np.array([1.0 + e]), d)
    assert abs(r_lo[0] - r_hi[0]) < 1e-11 and abs(p_lo[0] - p_hi[0]) < 1e-11
    # derivatives by central differences (away from the kink)
    for s0 in (0.3, 2.5, 40.0):
        h = 1e-5 * max(1.0, s0)
        rp, _, _ = oracle.huber(np.array([s0 + h]), 1.3)
        rm, _, _ = oracle.huber(np.array([s0 - h]), 1.3)
        _, dp, _ = oracle.huber(np.array([s0 + h]), 1.3)
        _, dm, _ = oracle.huber(np.array([s0 - h]), 1.3)
        _, d1a, d2a = oracle.huber(np.array([s0]), 1.3)
        assert abs((rp[0] - rm[0]) / (2 * h) - d1a[0]) < 1e-8
        assert abs((dp[0] - dm[0]) / (2 * h) - d2a[0]) < 1e-7
    # no kernel -> least squares
    rho, d1, d2 = oracle.huber(s, 0.0)
    np.testing.assert_array_equal(rho, s)
    rho, _, _ = oracle.huber(s, 1e9)
    np.testing.assert_array_equal(rho, s)


# ---------------------------------------------------------------------------
# Jacobians and gradient by finite differences on the manifold
# ---------------------------------------------------------------------------

def _perturbed(w, i, xi):
    p = w.copy()
    p.poses_init[i] = oracle.retract_pose(w.poses_init[i], xi)
    return p


@pytest.mark.parametrize("stereo", [False, True])
def test_jacobians_match_central_differences(stereo):
    w = bagen.tiny_window(seed=7, n_kf=3, n_lm=6, stereo=stereo)
    prob = _prob(w)
    Jp, Jl = oracle.jacobians(w.poses_init, w.points_init, prob)
    h = 1e-6
    for o in range(0, prob.n_obs, 3):
        i, j = prob.obs_pose[o], prob.obs_point[o]
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            Pp = w.poses_init.copy()
            Pm = w.poses_init.copy()
            Pp[i] = oracle.retract_pose(w.poses_init[i], e)
            Pm[i] = oracle.retract_pose(w.poses_init[i], -e)
            fd = (oracle.residuals(Pp, w.points_init, prob)[o] - oracle.residuals(Pm, w.points_init, prob)[o]) / (2 * h)
            np.testing.assert_allclose(Jp[o, :, c], fd, rtol=1e-6, atol=1e-6 * np.abs(Jp[o]).max())
        for c in range(3):
            Lp = w.points_init.copy()
            Lm = w.points_init.copy()
            Lp[j, c] += h
            Lm[j, c] -= h
            fd = (oracle.residuals(w.poses_init, Lp, prob)[o] - oracle.residuals(w.poses_init, Lm, prob)[o]) / (2 * h)
            np.testing.assert_allclose(Jl[o, :, c], fd, rtol=1e-6, atol=1e-6 * np.abs(Jl[o]).max())


def _fd_gradient(w, prob, delta, h=1e-6):
    nf = prob.n_free
    fi = prob.free_index()
    g = np.zeros(6 * nf + 3 * prob.n_points)
    for i in range(prob.n_poses):
        if fi[i] < 0:
            continue
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            Pp = w.poses_init.copy()
            Pm = w.poses_init.copy()
            Pp[i] = oracle.retract_pose(w.poses_init[i], e)
            Pm[i] = oracle.retract_pose(w.poses_init[i], -e)
            g[6 * fi[i] + c] = (oracle.cost(Pp, w.points_init, prob, delta)
                                - oracle.cost(Pm, w.points_init, prob, delta)) / (2 * h)
    for j in range(prob.n_points):
        for c in range(3):
            Lp = w.points_init.copy()
            Lm = w.points_init.copy()
            Lp[j, c] += h
            Lm[j, c] -= h
            g[6 * nf + 3 * j + c] = (oracle.cost(w.poses_init, Lp, prob, delta)
                                     - oracle.cost(w.poses_init, Lm, prob, delta)) / (2 * h)
    return g


def test_gradient_matches_fd_of_cost():
    w = bagen.tiny_window(seed=8, n_kf=3, n_lm=8, noise=2.0)     # many obs beyond the kink
    prob = _prob(w)
    delta = 1.0
    r = oracle.residuals(w.poses_init, w.points_init, prob)
    s = np.sum(r * r, 1)
    assert np.all(np.abs(s - delta ** 2) > 1e-3) and np.any(s > delta ** 2)
    H, g = olm.normal_equations_dense(w.poses_init, w.points_init, prob, delta)
    g_fd = _fd_gradient(w, prob, delta)
    np.testing.assert_allclose(g, g_fd, rtol=1e-6, atol=1e-7 * np.abs(g).max())


def test_gauss_newton_matrix_from_fd_jacobian():
    # H = J^T W J with J built column by column from central differences of the
    # stacked residual vector; W from the closed-form Huber weights.
    w = bagen.tiny_window(seed=9, n_kf=3, n_lm=5, stereo=True, noise=1.5)
    prob = _prob(w)
    delta = 1.0
    H, _ = olm.normal_equations_dense(w.poses_init, w.points_init, prob, delta)
    nf = prob.n_free
    fi = prob.free_index()
    h = 1e-6
    cols = []
    for i in range(prob.n_poses):
        if fi[i] < 0:
            continue
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            Pp = w.poses_init.copy()
            Pm = w.poses_init.copy()
            Pp[i] = oracle.retract_pose(w.poses_init[i], e)
            Pm[i] = oracle.retract_pose(w.poses_init[i], -e)
            cols.append(((oracle.residuals(Pp, w.points_init, prob)
                          - oracle.residuals(Pm, w.points_init, prob)) / (2 * h)).reshape(-1))
    for j in range(prob.n_points):
        for c in range(3):
            Lp = w.points_init.copy()
            Lm = w.points_init.copy()
            Lp[j, c] += h
            Lm[j, c] -= h
            cols.append(((oracle.residuals(w.poses_init, Lp, prob)
                          - oracle.residuals(w.poses_init, Lm, prob)) / (2 * h)).reshape(-1))
    J = np.stack(cols, 1)
    r = oracle.residuals(w.poses_init, w.points_init, prob)
    _, d1, _ = oracle.huber(np.sum(r * r, 1), delta)
    wt = np.repeat(prob.obs_w * d1, 2)
    H_ref = J.T @ (wt[:, None] * J)
    np.testing.assert_allclose(H, H_ref, rtol=1e-6, atol=1e-6 * np.abs(H_ref).max())


def test_block_assembly_equals_dense():
    w = bagen.tiny_window(seed=10, n_kf=4, n_lm=10, stereo=True, noise=1.0, fixed=(0, 2))
    prob = _prob(w)
    H, g = olm.normal_equations_dense(w.poses_init, w.points_init, prob, 1.0)
    b = olm.normal_equations_blocks(w.poses_init, w.points_init, prob, 1.0)
    nf = prob.n_free
    Hb = np.zeros_like(H)
    for f in range(nf):
        Hb[6 * f:6 * f + 6, 6 * f:6 * f + 6] = b.U[f]
    for j in range(prob.n_points):
        o = 6 * nf + 3 * j
        Hb[o:o + 3, o:o + 3] = b.V[j]
    for q in range(b.W.shape[0]):
        f, j = b.pair_pose[q], b.pair_point[q]
        o = 6 * nf + 3 * j
        Hb[6 * f:6 * f + 6, o:o + 3] = b.W[q]
        Hb[o:o + 3, 6 * f:6 * f + 6] = b.W[q].T
    np.testing.assert_allclose(Hb, H, rtol=1e-13, atol=1e-13 * np.abs(H).max())
    np.testing.assert_allclose(np.concatenate([b.gp.reshape(-1), b.gl.reshape(-1)]), g,
                               rtol=1e-13, atol=1e-13 * np.abs(g).max())


@pytest.mark.parametrize("lam", [1e-8, 1e-3, 10.0])
def test_schur_solve_equals_dense_solve(lam):
    w = bagen.tiny_window(seed=11, n_kf=4, n_lm=12, stereo=True, noise=1.0)
    prob = _prob(w)
    H, g = olm.normal_equations_dense(w.poses_init, w.points_init, prob, 1.0)
    b = olm.normal_equations_blocks(w.poses_init, w.points_init, prob, 1.0)
    dx_d = olm.solve_dense(H, g, lam)
    dx_s = olm.solve_schur(b, lam)
    # and against numpy's general solver on the damped system
    Hd = H + lam * np.diag(np.maximum(np.diag(H), 1e-9))
    dx_np = np.linalg.solve(Hd, -g)
    np.testing.assert_allclose(dx_s, dx_d, rtol=1e-10, atol=1e-12 * np.abs(dx_d).max())
    np.testing.assert_allclose(dx_d, dx_np, rtol=1e-10, atol=1e-12 * np.abs(dx_d).max())


# ---------------------------------------------------------------------------
# LM control
# ---------------------------------------------------------------------------

def test_lm_monotone_and_lambda_schedule():
    w = bagen.make_window(1)
    prob = _prob(w)
    st = oracle.LMSettings(max_iters=12, lambda_init=1e-3)
    res = oracle.lm_solve(w.poses_init, w.points_init, prob, st)
    costs = [res.initial_cost] + [t["cost_after"] for t in res.trace]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    lam = st.lambda_init
    for t in res.trace:
        assert t["lam"] == lam
        lam = max(lam / 10, 1e-10) if t["accepted"] else min(lam * 10, 1e10)
        assert t["lam_after"] == lam
        if t["accepted"]:
            assert t["cand_cost"] < t["cost"]
    assert res.final_cost < 0.01 * res.initial_cost


def test_lm_rejects_and_raises_lambda():
    # a huge initial error with a tiny lambda makes the first steps overshoot
    w = bagen.tiny_window(seed=12, n_kf=3, n_lm=10, noise=0.5)
    prob = _prob(w)
    p0 = w.poses_init.copy()
    for i in range(1, p0.shape[0]):
        p0[i] = oracle.retract_pose(p0[i], np.array([0.4, -0.3, 0.2, 0.2, -0.15, 0.1]))
    res = oracle.lm_solve(p0, w.points_init + 0.5, prob,
                          oracle.LMSettings(max_iters=25, lambda_init=1e-9))
    assert any(not t["accepted"] for t in res.trace)
    for t in res.trace:
        if not t["accepted"]:
            assert t["lam_after"] == min(t["lam"] * 10, 1e10)


def test_decision_replay_reproduces_own_run():
    w = bagen.make_window(1)
    prob = _prob(w)
    st = oracle.LMSettings(max_iters=10)
    a = oracle.lm_solve(w.poses_init, w.points_init, prob, st)
    b = oracle.lm_solve(w.poses_init, w.points_init, prob, st,
                        decisions=[t["accepted"] for t in a.trace])
    np.testing.assert_array_equal(a.poses, b.poses)
    np.testing.assert_array_equal(a.points, b.points)


def test_depth_guard_rejects_candidates_behind_camera():
    w = bagen.tiny_window(seed=13, n_kf=2, n_lm=4, noise=0.0)
    prob = _prob(w)
    pts = w.points_gt.copy()
    res = oracle.lm_solve(w.poses_gt, pts, prob,
                          oracle.LMSettings(max_iters=3, min_depth=1e6))   # every candidate too shallow
    assert all(t["status"] == "depth" and not t["accepted"] for t in res.trace)


# ---------------------------------------------------------------------------
# the converged minimum
# ---------------------------------------------------------------------------

def test_least_squares_minimum_matches_scipy():
    # plain least squares (no robust kernel) on a small stereo window, run to
    # convergence, against scipy.optimize.least_squares on the same residuals
    w = bagen.tiny_window(seed=14, n_kf=3, n_lm=10, stereo=True, noise=0.7)
    prob = _prob(w)
    st = oracle.LMSettings(max_iters=60, huber_delta=0.0)
    res = oracle.lm_solve(w.poses_init, w.points_init, prob, st)
    nf = prob.n_free
    fi = prob.free_index()

    def unpack(x):
        P = w.poses_init.copy()
        for i in range(prob.n_poses):
            if fi[i] >= 0:
                P[i, :, :3] = Rotation.from_rotvec(x[6 * fi[i] + 3:6 * fi[i] + 6]).as_matrix() @ w.poses_init[i, :, :3]
                P[i, :, 3] = w.poses_init[i, :, 3] + x[6 * fi[i]:6 * fi[i] + 3]
        return P, x[6 * nf:].reshape(-1, 3)

    def fun(x):
        P, L = unpack(x)
        return oracle.residuals(P, L, prob).reshape(-1)

    x0 = np.concatenate([np.zeros(6 * nf), w.points_init.reshape(-1)])
    ls = scipy.optimize.least_squares(fun, x0, xtol=1e-15, ftol=1e-15, gtol=1e-15, method="trf")
    F_ls = 0.5 * float(np.sum(ls.fun ** 2))
    assert abs(res.final_cost - F_ls) <= 1e-8 * F_ls
    P, L = unpack(ls.x)
    np.testing.assert_allclose(res.points, L, atol=1e-6)
    np.testing.assert_allclose(res.poses, P, atol=1e-7)


def test_huber_point_minimum_matches_brute_force():
    # all poses fixed: each landmark is an independent robust 3-parameter problem;
    # one observation is an outlier.  Nelder-Mead on the Huber cost is the reference.
    w = bagen.tiny_window(seed=15, n_kf=4, n_lm=1, noise=0.8, fixed=(0, 1, 2, 3))
    w.obs_uv[0] += np.array([25.0, -10.0])
    prob = _prob(w)
    # IRLS (Gauss-Newton weights without the rho'' term) converges linearly on
    # the outlier, hence the long run
    res = oracle.lm_solve(w.poses_gt, w.points_init, prob, oracle.LMSettings(max_iters=300))

    def f(p):
        return oracle.cost(w.poses_gt, p.reshape(1, 3), prob, 1.0)

    nm = scipy.optimize.minimize(f, w.points_init[0], method="Nelder-Mead",
                                 options=dict(xatol=1e-11, fatol=1e-14, maxiter=20000, maxfev=40000))
    np.testing.assert_allclose(res.points[0], nm.x, atol=1e-6)
    assert abs(res.final_cost - nm.fun) < 1e-9


@pytest.mark.parametrize("stereo", [False, True])
def test_noiseless_recovery(stereo):
    w = bagen.tiny_window(seed=16, n_kf=4, n_lm=25, stereo=stereo, noise=0.0)
    prob = _prob(w)
    res = oracle.lm_solve(w.poses_init, w.points_init, prob, oracle.LMSettings(max_iters=40))
    assert res.final_cost < 1e-14
    P, L = res.poses, res.points
    if not stereo:                       # mono: up to the scale gauge about pose 0
        P, L, s = oracle.align_scale(P, L, w.poses_gt)
    np.testing.assert_allclose(P, w.poses_gt, atol=1e-7)
    np.testing.assert_allclose(L, w.points_gt, atol=1e-6)


def test_noiseless_triangulation_special_case():
    # every pose fixed at ground truth: the problem is independent triangulations
    w = bagen.tiny_window(seed=17, n_kf=3, n_lm=8, noise=0.0, fixed=(0, 1, 2))
    prob = _prob(w)
    res = oracle.lm_solve(w.poses_gt, w.points_init, prob, oracle.LMSettings(max_iters=30))
    np.testing.assert_allclose(res.points, w.points_gt, atol=1e-9)


@pytest.mark.parametrize("delta,iters,tol", [(0.0, 60, 1e-9), (1.0, 400, 1e-8)])
def test_gradient_vanishes_at_convergence(delta, iters, tol):
    # Gauss-Newton converges quadratically for plain least squares; with Huber
    # weights (IRLS) it converges linearly, hence the longer run
    w = bagen.tiny_window(seed=18, n_kf=3, n_lm=12, stereo=True, noise=0.7)
    prob = _prob(w)
    res = oracle.lm_solve(w.poses_init, w.points_init, prob,
                          oracle.LMSettings(max_iters=iters, huber_delta=delta))
    g0 = oadj.gradient_dense(w.poses_init, w.points_init, prob, delta)
    g = oadj.gradient_dense(res.poses, res.points, prob, delta)
    assert np.abs(g).max() < tol * np.abs(g0).max()


def test_gauge_invariance_under_rigid_motion():
    w = bagen.tiny_window(seed=19, n_kf=3, n_lm=12, stereo=True, noise=0.7)
    prob = _prob(w)
    # Marquardt's diagonal damping is not frame-invariant, so only the converged
    # minimum (reached quadratically without the robust kernel) is compared
    st = oracle.LMSettings(max_iters=60, huber_delta=0.0)
    a = oracle.lm_solve(w.poses_init, w.points_init, prob, st)
    G = np.concatenate([Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix(), [[1.0], [-2.0], [0.5]]], 1)
    Ginv_R = G[:, :3].T
    Ginv_t = -Ginv_R @ G[:, 3]
    # world' = G world: poses T' = T G^-1, points p' = G p
    P2 = w.poses_init.copy()
    P2[:, :, :3] = w.poses_init[:, :, :3] @ Ginv_R
    P2[:, :, 3] = np.einsum("nab,b->na", w.poses_init[:, :, :3], Ginv_t) + w.poses_init[:, :, 3]
    L2 = w.points_init @ G[:, :3].T + G[:, 3]
    b = oracle.lm_solve(P2, L2, prob, st)
    ra = oracle.residuals(a.poses, a.points, prob)
    rb = oracle.residuals(b.poses, b.points, prob)
    np.testing.assert_allclose(rb, ra, atol=1e-9)


def test_scale_alignment_recovers_similarity():
    w = bagen.tiny_window(seed=20, n_kf=4, n_lm=5)
    s_true = 1.7
    P = w.poses_gt.copy()
    c = -np.einsum("nba,nb->na", P[:, :, :3], P[:, :, 3])
    c0 = c[0]
    c_new = c0 + (c - c0) / s_true
    P[:, :, 3] = -np.einsum("nab,nb->na", P[:, :, :3], c_new)
    L = c0 + (w.points_gt - c0) / s_true
    P2, L2, s = oracle.align_scale(P, L, w.poses_gt)
    assert abs(s - s_true) < 1e-12
    np.testing.assert_allclose(P2, w.poses_gt, atol=1e-12)
    np.testing.assert_allclose(L2, w.points_gt, atol=1e-12)


# ---------------------------------------------------------------------------
# exact Hessian and adjoint
# ---------------------------------------------------------------------------

def test_exact_hessian_matches_fd_of_gradient():
    w = bagen.tiny_window(seed=21, n_kf=3, n_lm=6, stereo=True, noise=1.5, fixed=(0,))
    # include an extrinsic rotation so that R_c enters every term
    w.extrinsics[1, :, :3] = Rotation.from_rotvec([0.05, -0.1, 0.02]).as_matrix()
    prob = _prob(w)
    r = oracle.residuals(w.poses_init, w.points_init, prob)
    s = np.sum(r * r, 1)
    assert np.all(np.abs(s - 1.0) > 1e-2) and np.any(s > 1.0)
    H = oadj.exact_hessian_dense(w.poses_init, w.points_init, prob, 1.0)
    nf = prob.n_free
    fi = prob.free_index()
    h = 1e-5
    Hfd = np.zeros_like(H)
    col = 0
    for i in range(prob.n_poses):
        if fi[i] < 0:
            continue
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            Pp = w.poses_init.copy()
            Pm = w.poses_init.copy()
            Pp[i] = oracle.retract_pose(w.poses_init[i], e)
            Pm[i] = oracle.retract_pose(w.poses_init[i], -e)
            Hfd[:, 6 * fi[i] + c] = (oadj.gradient_dense(Pp, w.points_init, prob, 1.0)
                                     - oadj.gradient_dense(Pm, w.points_init, prob, 1.0)) / (2 * h)
    for j in range(prob.n_points):
        for c in range(3):
            Lp = w.points_init.copy()
            Lm = w.points_init.copy()
            Lp[j, c] += h
            Lm[j, c] -= h
            Hfd[:, 6 * nf + 3 * j + c] = (oadj.gradient_dense(w.poses_init, Lp, prob, 1.0)
                                          - oadj.gradient_dense(w.poses_init, Lm, prob, 1.0)) / (2 * h)
    # the FD Hessian of the gradient in this chart is exact only where the gradient
    # vanishes (Exp(e)Exp(x) != Exp(e + x)); compare its symmetric part and check the
    # pose-pose difference is explained by the gradient, at a point chosen away from
    # convergence.  The point blocks are chart-free and must match directly.
    np.testing.assert_allclose(H[6 * nf:, :], Hfd[6 * nf:, :], rtol=1e-5, atol=1e-5 * np.abs(H).max())


def test_exact_hessian_at_minimum_is_symmetric_fd():
    # at a stationary point the chart's second-order correction vanishes and the
    # whole FD Hessian (poses included) matches the analytic one
    w = bagen.tiny_window(seed=22, n_kf=3, n_lm=8, stereo=True, noise=1.2)
    prob = _prob(w)
    res = oracle.lm_solve(w.poses_init, w.points_init, prob, oracle.LMSettings(max_iters=80))
    P, L = res.poses, res.points
    r = oracle.residuals(P, L, prob)
    s = np.sum(r * r, 1)
    assert np.all(np.abs(s - 1.0) > 1e-3)
    H = oadj.exact_hessian_dense(P, L, prob, 1.0)
    nf = prob.n_free
    fi = prob.free_index()
    h = 1e-5
    Hfd = np.zeros_like(H)
    for i in range(prob.n_poses):
        if fi[i] < 0:
            continue
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            Pp = P.copy()
            Pm = P.copy()
            Pp[i] = oracle.retract_pose(P[i], e)
            Pm[i] = oracle.retract_pose(P[i], -e)
            Hfd[:, 6 * fi[i] + c] = (oadj.gradient_dense(Pp, L, prob, 1.0)
                                     - oadj.gradient_dense(Pm, L, prob, 1.0)) / (2 * h)
    for j in range(prob.n_points):
        for c in range(3):
            Lp = L.copy()
            Lm = L.copy()
            Lp[j, c] += h
            Lm[j, c] -= h
            Hfd[:, 6 * nf + 3 * j + c] = (oadj.gradient_dense(P, Lp, prob, 1.0)
                                          - oadj.gradient_dense(P, Lm, prob, 1.0)) / (2 * h)
    np.testing.assert_allclose(H, Hfd, rtol=1e-5, atol=2e-6 * np.abs(H).max())
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())


def _solve_tight(poses0, points0, prob, delta=1.0):
    """LM followed by Newton polishing to the stationary point.  Whatever the
    Hessian used by the polish, its fixed point is where the (FD-pinned)
    gradient vanishes, which the caller asserts."""
    res = oracle.lm_solve(poses0, points0, prob,
                          oracle.LMSettings(max_iters=30, lambda_init=1e-6, huber_delta=delta))
    return oadj.newton_polish(res.poses, res.points, prob, delta)


@pytest.mark.parametrize("delta", [0.0, 1.0])
def test_adjoint_matches_fd_of_solution_map(delta):
    # brute force over every keypoint coordinate and weight of a tiny window with
    # the gauge fully fixed (two fixed keyframes), loss = chordal pose error
    w = bagen.tiny_window(seed=23, n_kf=4, n_lm=10, noise=0.8, fixed=(0, 1))
    prob = _prob(w)
    free = ~prob.pose_fixed
    P, L = _solve_tight(w.poses_init, w.points_init, prob, delta)
    g0 = oadj.gradient_dense(w.poses_init, w.points_init, prob, delta)
    assert np.abs(oadj.gradient_dense(P, L, prob, delta)).max() < 1e-12 * np.abs(g0).max()
    r = oracle.residuals(P, L, prob)
    s = np.sum(r * r, 1)
    if delta > 0:
        assert np.any(s > delta ** 2)          # the Huber branch is exercised
    Lval, G = oracle.chordal_loss(P, w.poses_gt, free)
    gx = np.concatenate([oracle.ambient_to_tangent(P, G)[free].reshape(-1), np.zeros(3 * prob.n_points)])
    g_uv, g_w = oracle.adjoint_dense(P, L, prob, delta, gx)
    h = 1e-4
    scale_uv = np.abs(g_uv).max()
    scale_w = np.abs(g_w).max()
    checked = 0
    for o in range(prob.n_obs):
        if delta > 0 and abs(math.sqrt(s[o]) - delta) < 1e-3:
            continue                           # too close to the kink for a central difference
        for c in range(3):
            vals = []
            for sign in (1, -1):
                uv, ww = prob.obs_uv.copy(), prob.obs_w.copy()
                if c < 2:
                    uv[o, c] += sign * h
                else:
                    ww[o] += sign * h
                pr = oracle.Problem(**{**prob.__dict__, "obs_uv": uv, "obs_w": ww})
                P2, L2 = oadj.newton_polish(P, L, pr, delta)
                vals.append(oracle.chordal_loss(P2, w.poses_gt, free)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            ref, sc = (g_uv[o, c], scale_uv) if c < 2 else (g_w[o], scale_w)
            assert abs(fd - ref) <= 1e-6 * sc, (o, c, fd, ref)
            checked += 1
    assert checked >= 2 * prob.n_obs


def test_ambient_to_tangent_matches_fd_of_loss():
    rng = np.random.default_rng(24)
    P = np.stack([np.concatenate([Rotation.random(random_state=k).as_matrix(), rng.normal(size=(3, 1))], 1)
                  for k in range(3)])
    Pref = P + 0.1 * rng.normal(size=P.shape)
    free = np.ones(3, bool)
    _, G = oracle.chordal_loss(P, Pref, free)
    g = oracle.ambient_to_tangent(P, G)
    h = 1e-6
    for i in range(3):
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            Pp = P.copy()
            Pm = P.copy()
            Pp[i] = oracle.retract_pose(P[i], e)
            Pm[i] = oracle.retract_pose(P[i], -e)
            fd = (oracle.chordal_loss(Pp, Pref, free)[0] - oracle.chordal_loss(Pm, Pref, free)[0]) / (2 * h)
            assert abs(fd - g[i, c]) < 1e-7
