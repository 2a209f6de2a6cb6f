"""GPU implicit-function adjoint against the dense FP64 oracle adjoint.

At the same converged state x*, the library's d(loss)/d(keypoints) and
d(loss)/d(weights) must equal the oracle's dense exact-Hessian adjoint: to
1e-9 relative in FP64 mode, to 1e-3 (relative 2-norm) in mixed mode.
"""
import numpy as np
import pytest

import bagen
import oracle
from oracle import adjoint as oadj

pytestmark = pytest.mark.gpu


def _gpu_adjoint(w, s, P, L, obs_w=None, grad_points=None):
    import torch
    import paper_2506_04359_amd as ba
    dev = torch.device("cuda:0")
    W = ba.Window.from_problem(w)
    Pt = torch.tensor(P, dtype=torch.float64, device=dev)
    Lt = torch.tensor(L, dtype=torch.float64, device=dev)
    uv = torch.tensor(w.obs_uv, dtype=torch.float64, device=dev)
    wt = None if obs_w is None else torch.tensor(obs_w, dtype=torch.float64, device=dev)
    free = ~w.pose_fixed.astype(bool)
    _, G = oracle.chordal_loss(P, w.poses_gt, free)
    gP = torch.tensor(G, dtype=torch.float64, device=dev)
    gL = None if grad_points is None else torch.tensor(grad_points, dtype=torch.float64, device=dev)
    guv = torch.zeros_like(uv)
    gw = torch.zeros(w.n_obs, dtype=torch.float64, device=dev)
    rep, _ = ba.adjoint(W, s, Pt, Lt, uv, wt, gP, gL, guv, gw)
    torch.cuda.synchronize()
    return guv.cpu().numpy(), gw.cpu().numpy(), ba.parse_reports(rep)[0], G


def _oracle_adjoint(w, P, L, G, obs_w=None, grad_points=None, delta=1.0):
    prob = oracle.Problem.from_window(w, obs_w=obs_w)
    free = ~prob.pose_fixed
    gx = np.concatenate([oracle.ambient_to_tangent(P, G)[free].reshape(-1),
                         np.zeros(3 * prob.n_points) if grad_points is None else grad_points.reshape(-1)])
    return oracle.adjoint_dense(P, L, prob, delta, gx)


@pytest.mark.parametrize("stereo,with_points", [(False, False), (True, True)])
def test_fp64_adjoint_matches_dense_oracle(stereo, with_points):
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=51, n_kf=5, n_lm=30, noise=0.8, stereo=stereo, fixed=(0, 1))
    prob = oracle.Problem.from_window(w)
    res = oracle.lm_solve(w.poses_init, w.points_init, prob, oracle.LMSettings(max_iters=30))
    P, L = oadj.newton_polish(res.poses, res.points, prob, 1.0)
    gl = np.random.default_rng(3).normal(size=L.shape) * 0.1 if with_points else None
    s = ba.Settings(max_iters=1, precision=ba.BA_FP64)
    guv, gw, rep, G = _gpu_adjoint(w, s, P, L, grad_points=gl)
    ruv, rw = _oracle_adjoint(w, P, L, G, grad_points=gl)
    assert rep["chol_failures"] == 0
    assert np.abs(guv - ruv).max() <= 1e-9 * np.abs(ruv).max()
    assert np.abs(gw - rw).max() <= 1e-9 * np.abs(rw).max()


def test_fp64_adjoint_with_weights():
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=52, n_kf=4, n_lm=25, noise=1.0, fixed=(0, 1))
    ow = np.random.default_rng(2).uniform(0.3, 2.0, w.n_obs)
    prob = oracle.Problem.from_window(w, obs_w=ow)
    res = oracle.lm_solve(w.poses_init, w.points_init, prob, oracle.LMSettings(max_iters=30))
    P, L = oadj.newton_polish(res.poses, res.points, prob, 1.0)
    s = ba.Settings(max_iters=1, precision=ba.BA_FP64)
    guv, gw, rep, G = _gpu_adjoint(w, s, P, L, obs_w=ow)
    ruv, rw = _oracle_adjoint(w, P, L, G, obs_w=ow)
    assert np.abs(guv - ruv).max() <= 1e-9 * np.abs(ruv).max()
    assert np.abs(gw - rw).max() <= 1e-9 * np.abs(rw).max()


def test_mixed_adjoint_on_adjoint_workload_window():
    # a window of the 64-window adjoint workload: mixed forward solve to x*, then
    # the mixed adjoint against the dense FP64 adjoint at the same x*
    import torch
    import paper_2506_04359_amd as ba
    w = bagen.make_window(5, 0)
    s = ba.Settings(max_iters=50, precision=ba.BA_MIXED)
    from helpers import gpu_solve
    g = gpu_solve(w, s, with_trace=False)
    P, L = g["poses"], g["points"]
    guv, gw, rep, G = _gpu_adjoint(w, s, P, L)
    ruv, rw = _oracle_adjoint(w, P, L, G)
    e_uv = np.linalg.norm(guv - ruv) / np.linalg.norm(ruv)
    e_w = np.linalg.norm(gw - rw) / np.linalg.norm(rw)
    print("mixed adjoint rel err", e_uv, e_w)
    assert e_uv <= 1e-3 and e_w <= 1e-3


def test_autograd_function_matches_direct_adjoint():
    import torch
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=53, n_kf=4, n_lm=20, noise=0.6, fixed=(0, 1))
    dev = torch.device("cuda:0")
    W = ba.Window.from_problem(w)
    s = ba.Settings(max_iters=40, precision=ba.BA_FP64)
    P0 = torch.tensor(w.poses_init, dtype=torch.float64, device=dev)
    L0 = torch.tensor(w.points_init, dtype=torch.float64, device=dev)
    uv = torch.tensor(w.obs_uv, dtype=torch.float64, device=dev, requires_grad=True)
    ow = torch.ones(w.n_obs, dtype=torch.float64, device=dev, requires_grad=True)
    Pgt = torch.tensor(w.poses_gt, dtype=torch.float64, device=dev)
    free = torch.tensor(1.0 - w.pose_fixed, dtype=torch.float64, device=dev)
    Ps, Ls = ba.BASolve.apply(P0, L0, uv, ow, W, s)
    loss = (((Ps - Pgt) ** 2) * free[:, None, None]).sum() + 0.01 * (Ls ** 2).sum()
    loss.backward()
    Pn, Ln = Ps.detach().cpu().numpy(), Ls.detach().cpu().numpy()
    prob = oracle.Problem.from_window(w)
    freeb = ~prob.pose_fixed
    _, G = oracle.chordal_loss(Pn, w.poses_gt, freeb)
    gx = np.concatenate([oracle.ambient_to_tangent(Pn, G)[freeb].reshape(-1), (0.02 * Ln).reshape(-1)])
    ruv, rw = oracle.adjoint_dense(Pn, Ln, prob, 1.0, gx)
    assert np.abs(uv.grad.cpu().numpy() - ruv).max() <= 1e-8 * np.abs(ruv).max()
    assert np.abs(ow.grad.cpu().numpy() - rw).max() <= 1e-8 * np.abs(rw).max()


def test_fp64_batched_adjoint_of_four_classes_matches_single_windows():
    """A batch whose windows fall into all four size classes (pass A forks the
    two largest classes onto side streams): every window's adjoint equals the
    single-window call's, and the single-window calls follow the dense oracle."""
    import torch
    import paper_2506_04359_amd as ba
    ws = [bagen.tiny_window(seed=80 + k, n_kf=n, n_lm=25, noise=0.6, fixed=(0, 1))
          for k, n in enumerate((6, 15, 22, 28))]
    assert [int((w.pose_fixed == 0).sum()) for w in ws] == [4, 13, 20, 26]
    dev = torch.device("cuda:0")
    s = ba.Settings(max_iters=1, precision=ba.BA_FP64)
    single = []
    for k, w in enumerate(ws):
        P0, L0 = np.ascontiguousarray(w.poses_gt), np.ascontiguousarray(w.points_gt)
        guv, gw, rep, G = _gpu_adjoint(w, s, P0, L0)
        assert rep["chol_failures"] == 0
        if k == 0:
            ruv, rw = _oracle_adjoint(w, P0, L0, G)
            assert np.abs(guv - ruv).max() <= 1e-9 * np.abs(ruv).max()
            assert np.abs(gw - rw).max() <= 1e-9 * np.abs(rw).max()
        single.append((guv, gw, G))
    B = ba.Batch([ba.Window.from_problem(w, host_only=True) for w in ws])
    cat = lambda xs: torch.tensor(np.ascontiguousarray(np.concatenate(xs)), dtype=torch.float64, device=dev)
    P, L = cat([w.poses_gt for w in ws]), cat([w.points_gt for w in ws])
    uv = cat([w.obs_uv for w in ws])
    gP = cat([g[2] for g in single])
    guv = torch.zeros_like(uv)
    gw = torch.zeros(uv.shape[0], dtype=torch.float64, device=dev)
    for _ in range(2):   # the first call makes the side streams, the second forks onto them
        guv.zero_()
        gw.zero_()
        rep, _ = ba.adjoint(B, s, P, L, uv, None, gP, None, guv, gw)
        torch.cuda.synchronize()
        assert np.all(ba.parse_reports(rep)[: len(ws)]["chol_failures"] == 0)
        o = 0
        for w, (suv, sw, _) in zip(ws, single):
            buv, bw = guv[o:o + w.n_obs].cpu().numpy(), gw[o:o + w.n_obs].cpu().numpy()
            assert np.abs(buv - suv).max() <= 1e-9 * np.abs(suv).max()
            assert np.abs(bw - sw).max() <= 1e-9 * np.abs(sw).max()
            o += w.n_obs


def test_adjoint_workload_window_against_finite_differences():
    """A full window of the adjoint workload (about 19k observations): the FP64
    adjoint at the oracle's converged state equals the dense oracle adjoint to
    1e-9; the mixed adjoint at the GPU's own mixed solution (50 attempts) meets
    the stored central differences of the solution map (100 coordinates,
    written by tests/golden/make_adjoint_fd.py from the oracle) to 1e-3 of the
    coordinate, with a floor of 1e-2 times the adjoint's RMS."""
    import json
    import os
    import paper_2506_04359_amd as ba
    from helpers import gpu_solve
    import adjoint_fd as F
    doc = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "adjoint_cfg5_fd.json")))
    w = bagen.make_window(5, 0)
    prob = oracle.Problem.from_window(w)
    P, L = F.tight_solution(w, prob)
    s64 = ba.Settings(max_iters=1, precision=ba.BA_FP64)
    guv, gw, rep, G = _gpu_adjoint(w, s64, P, L)
    ruv, rw = _oracle_adjoint(w, P, L, G)
    assert rep["chol_failures"] == 0
    assert np.abs(guv - ruv).max() <= 1e-9 * np.abs(ruv).max()
    assert np.abs(gw - rw).max() <= 1e-9 * np.abs(rw).max()

    sm = ba.Settings(max_iters=50, precision=ba.BA_MIXED)
    g = gpu_solve(w, sm, with_trace=False)
    muv, mw, rep, _ = _gpu_adjoint(w, sm, g["poses"], g["points"])
    assert rep["chol_failures"] == 0
    floor = 1e-2 * doc["adjoint_rms"]
    worst = 0.0
    for row in doc["coordinates"]:
        a = F.adjoint_value(muv, mw, row["obs"], row["comp"])
        worst = max(worst, abs(a - row["fd_h"]) / max(abs(row["fd_h"]), floor))
    print("mixed adjoint vs finite differences: worst relative error", worst)
    assert worst <= 1e-3, worst
