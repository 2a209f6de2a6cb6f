"""Pins of the oracle's per-window freeze tests (grad_tol, step_tol; the
paper gives no stopping rule, the reading is stated in oracle/lm.py): the
reduced-gradient norm equals the Schur complement of the damped normal
equations written out with dense inverses, vanishes at the minimum (and only
there), and the two tests freeze a window exactly where they should, leaving
its state untouched afterwards."""
import math

import numpy as np
import pytest

import bagen
import oracle
from oracle import adjoint as oadj
from oracle import lm as olm


def _prob(w):
    return oracle.Problem.from_window(w)


@pytest.mark.parametrize("lam", [0.0, 1e-3, 10.0])
def test_reduced_gradient_is_the_dense_schur_rhs(lam):
    # b~ = -(g_p - H_pl (H_ll + lam D_ll)^-1 g_l) with the whole landmark block
    # inverted at once (no per-landmark blocks), both backends
    w = bagen.tiny_window(seed=21, n_kf=4, n_lm=10, stereo=True, noise=1.0)
    prob = _prob(w)
    H, g = olm.normal_equations_dense(w.poses_init, w.points_init, prob, 1.0)
    n = 6 * prob.n_free
    Hll = H[n:, n:].copy()
    d = np.diag(Hll).copy()
    Hll[np.diag_indices_from(Hll)] = d + lam * np.maximum(d, 1e-9)
    bt = -(g[:n] - H[:n, n:] @ np.linalg.inv(Hll) @ g[n:])
    want = max(np.abs(bt).max(), np.abs(g[n:]).max())
    got_d = olm.reduced_gradient_norm((H, g), "dense", lam, prob.n_free)
    blocks = olm.normal_equations_blocks(w.poses_init, w.points_init, prob, 1.0)
    got_s = olm.reduced_gradient_norm(blocks, "schur", lam, prob.n_free)
    assert abs(got_d - want) <= 1e-10 * want and abs(got_s - want) <= 1e-10 * want


def test_reduced_gradient_vanishes_only_at_the_minimum():
    w = bagen.tiny_window(seed=22, n_kf=3, n_lm=12, stereo=True, noise=0.0)
    prob = _prob(w)
    H, g = olm.normal_equations_dense(w.poses_gt, w.points_gt, prob, 1.0)
    assert olm.reduced_gradient_norm((H, g), "dense", 1e-3, prob.n_free) < 1e-9
    # away from it the landmark gradient alone is already large
    H, g = olm.normal_equations_dense(w.poses_init, w.points_init, prob, 1.0)
    gl = oadj.gradient_dense(w.poses_init, w.points_init, prob, 1.0)[6 * prob.n_free:]
    gn = olm.reduced_gradient_norm((H, g), "dense", 1e-3, prob.n_free)
    assert gn >= np.abs(gl).max() > 1.0


def _run(w, **kw):
    prob = _prob(w)
    return oracle.lm_solve(w.poses_init, w.points_init, prob, oracle.LMSettings(max_iters=25, **kw))


def test_zero_tolerances_change_nothing():
    w = bagen.make_window(1)
    a = _run(w)
    b = _run(w, grad_tol=0.0, step_tol=0.0)
    assert [t["status"] for t in b.trace].count("frozen") == 0 and b.iters == 25
    np.testing.assert_array_equal(a.poses, b.poses)
    np.testing.assert_array_equal(a.points, b.points)


def test_gradient_freeze_happens_at_the_first_small_gradient():
    w = bagen.tiny_window(seed=23, n_kf=4, n_lm=20, stereo=True, noise=0.0)
    prob = _prob(w)
    free = _run(w)
    # the reduced-gradient norm of every attempt of the unfrozen run
    norms = []
    P, L = w.poses_init.copy(), w.points_init.copy()
    lam = 1e-3
    for t in free.trace:
        H, g = olm.normal_equations_dense(P, L, prob, 1.0)
        norms.append(olm.reduced_gradient_norm((H, g), "dense", t["lam"], prob.n_free))
        if t["accepted"]:
            P, L = olm.apply_step(P, L, prob, olm.solve_dense(H, g, t["lam"]))
    # a threshold between two consecutive norms that differ by 10x or more
    k = next(i for i in range(1, len(norms)) if norms[i] < 0.1 * norms[i - 1] and norms[i] < 1.0)
    tol = math.sqrt(norms[k] * norms[k - 1])
    res = _run(w, grad_tol=tol)
    st = [t["status"] for t in res.trace]
    assert st[:k] == [t["status"] for t in free.trace[:k]] and all(s == "frozen" for s in st[k:])
    assert res.iters == k
    np.testing.assert_array_equal(res.poses, P if k == len(norms) else _state_after(w, prob, free, k)[0])
    for t in res.trace[k:]:
        assert not t["accepted"] and math.isnan(t["cand_cost"]) and t["cost"] == res.final_cost
        assert t["lam"] == res.trace[k]["lam"]


def _state_after(w, prob, run, k):
    P, L = w.poses_init.copy(), w.points_init.copy()
    for t in run.trace[:k]:
        if t["accepted"]:
            H, g = olm.normal_equations_dense(P, L, prob, 1.0)
            P, L = olm.apply_step(P, L, prob, olm.solve_dense(H, g, t["lam"]))
    return P, L


def test_step_freeze_after_the_first_small_accepted_step():
    w = bagen.tiny_window(seed=24, n_kf=4, n_lm=20, stereo=True, noise=0.3)
    prob = _prob(w)
    free = _run(w)
    steps = [(i, t["step_norm"]) for i, t in enumerate(free.trace) if t["accepted"]]
    # the first accepted step 10x or more below the accepted step before it
    j = next(n for n in range(1, len(steps)) if steps[n][1] < 0.1 * steps[n - 1][1])
    k, tol = steps[j][0], math.sqrt(steps[j][1] * steps[j - 1][1])
    res = _run(w, step_tol=tol)
    assert [t["status"] for t in res.trace[k + 1:]] == ["frozen"] * (25 - k - 1)
    assert res.trace[k]["accepted"] and res.iters == k + 1
    P, L = _state_after(w, prob, free, k + 1)
    np.testing.assert_array_equal(res.poses, P)
    np.testing.assert_array_equal(res.points, L)


def test_a_window_at_its_minimum_freezes_at_once():
    w = bagen.tiny_window(seed=25, n_kf=3, n_lm=12, stereo=True, noise=0.0)
    prob = _prob(w)
    res = oracle.lm_solve(w.poses_gt, w.points_gt, prob, oracle.LMSettings(max_iters=5, grad_tol=1e-6))
    assert res.iters == 0 and all(t["status"] == "frozen" for t in res.trace)
    np.testing.assert_array_equal(res.poses, w.poses_gt)
