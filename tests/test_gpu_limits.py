"""GPU parity at the library's size limits, at the benchmark's full launch
shape, and on degenerate windows.

* the largest reduced systems: 29 free poses in FP64 mode and 32 in mixed
  mode, in windows of up to 64 poses, every landmark seen by every keyframe
  that sees it (long tracks: up to 32 free pairs per landmark);
* the full 256-window batch at 2048 observations per work item (the launch
  shape the benchmark times): every report, and sampled windows against the
  FP64 oracle;
* the 64-window adjoint batch: sampled windows against the dense oracle adjoint;
* an empty window (no landmarks) inside a batch.
"""
import numpy as np
import pytest

import bagen
import oracle
from oracle import adjoint as oadj
from helpers import (check_decisions, gpu_solve, gpu_solve_batched, mixed_check, oracle_replay,
                     rel_err)

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


def _fp64_replay_parity(w, s, g):
    prob, ref = oracle_replay(w, s, g["trace"])
    check_decisions(ref, g["trace"])
    for t, gt in zip(ref.trace, g["trace"]):
        assert abs(t["cost"] - gt["cost"]) <= TOL64 * abs(t["cost"]), (t, gt)
    assert abs(g["report"]["final_cost"] - ref.final_cost) <= TOL64 * ref.final_cost
    P, L, _ = oracle.align_scale(g["poses"], g["points"], ref.poses)
    assert rel_err(P, ref.poses) <= TOL64 and rel_err(L, ref.points) <= TOL64
    return ref


@pytest.mark.parametrize("n_kf,fixed,n_free", [(30, (0,), 29), (64, tuple(range(35)), 29),
                                               (64, tuple(range(36)), 28)])
def test_fp64_largest_reduced_system(n_kf, fixed, n_free):
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=61, n_kf=n_kf, n_lm=150, noise=0.5, fixed=fixed)
    W = ba.Window.from_problem(w)
    info = W.info()
    assert info["n_free"] == n_free and info["n_poses"] == n_kf
    s = ba.Settings(max_iters=6, precision=ba.BA_FP64)
    g = gpu_solve(w, s)
    ref = _fp64_replay_parity(w, s, g)
    assert ref.final_cost < 0.1 * ref.trace[0]["cost"]


def test_fp64_beyond_29_free_poses_is_unsupported_and_mixed_is_not():
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=63, n_kf=64, n_lm=60, fixed=tuple(range(34)))
    W = ba.Window.from_problem(w)
    with pytest.raises(ba.BAError) as e:
        W.workspace_size(ba.Settings(max_iters=1, precision=ba.BA_FP64))
    assert e.value.status == ba.BA_ERR_UNSUPPORTED
    assert W.workspace_size(ba.Settings(max_iters=1, precision=ba.BA_MIXED)) > 0


@pytest.mark.parametrize("n_kf,fixed,gauge_fixed", [(34, (0, 1), True), (64, tuple(range(32)), True),
                                                    (33, (0,), False)])
def test_mixed_largest_reduced_system(n_kf, fixed, gauge_fixed):
    # With one fixed keyframe a mono window keeps its scale gauge: S is singular
    # along it (smallest eigenvalue ~1e-11 of ~3e6) and once lambda has been
    # divided down, FP32 rounding of S exceeds the damping there; such attempts
    # fail their pivot and are rejected (lambda raised), which the LM schedule
    # allows.  Two fixed keyframes remove the gauge: then no pivot may fail.
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=62, n_kf=n_kf, n_lm=250, noise=0.5, fixed=fixed)
    assert int((w.pose_fixed == 0).sum()) == 32
    s = ba.Settings(max_iters=10, precision=ba.BA_MIXED)
    g = gpu_solve(w, s)
    if gauge_fixed:
        assert g["report"]["chol_failures"] == 0
    mixed_check(w, g, backend="dense", align=True, s=s)


def test_full_batch_at_benchmark_launch_shape():
    import paper_2506_04359_amd as ba
    ws = [bagen.make_window(3, i) for i in range(256)]
    s = ba.Settings(max_iters=15, precision=ba.BA_MIXED, lambda_init=1e-3, huber_delta=1.0)
    out = gpu_solve_batched(ws, s, chunk_obs=2048)
    for w, o in zip(ws, out):
        r = o["report"]
        assert r["iters"] == 15 and r["status"] == 0, (w.name, r)
        assert np.isfinite(r["final_cost"]) and r["final_cost"] < 0.5 * r["initial_cost"], (w.name, r)
        assert np.all(np.isfinite(o["poses"])) and np.all(np.isfinite(o["points"]))
    n_free = [int((w.pose_fixed == 0).sum()) for w in ws]
    n_obs = [w.n_obs for w in ws]
    sample = sorted({0, 255, int(np.argmax(n_free)), int(np.argmin(n_free)), int(np.argmax(n_obs)),
                     int(np.argmin(n_obs))})
    for k in sample:
        print("window", k, ws[k].name, "free", n_free[k], "obs", n_obs[k], flush=True)
        mixed_check(ws[k], out[k], align=True, s=s)


def test_adjoint_batch_sampled_windows():
    import torch
    import paper_2506_04359_amd as ba
    dev = torch.device("cuda:0")
    wa = [bagen.make_window(5, i) for i in range(64)]
    B = ba.Batch([ba.Window.from_problem(w, host_only=True) for w in wa])
    s = ba.Settings(max_iters=50, precision=ba.BA_MIXED, lambda_init=1e-3, huber_delta=1.0)
    P = torch.tensor(np.concatenate([w.poses_init for w in wa]), dtype=torch.float64, device=dev)
    L = torch.tensor(np.concatenate([w.points_init for w in wa]), dtype=torch.float64, device=dev)
    uv = torch.tensor(np.concatenate([w.obs_uv for w in wa]), dtype=torch.float64, device=dev)
    ba.solve_batched(B, s, P, L, uv, None)
    torch.cuda.synchronize()
    Pn, Ln = P.cpu().numpy(), L.cpu().numpy()
    po = np.cumsum([0] + [w.n_poses for w in wa])
    lo = np.cumsum([0] + [w.n_points for w in wa])
    oo = np.cumsum([0] + [w.n_obs for w in wa])
    G = np.zeros_like(Pn)
    for k, w in enumerate(wa):
        free = ~w.pose_fixed.astype(bool)
        _, G[po[k]:po[k + 1]] = oracle.chordal_loss(Pn[po[k]:po[k + 1]], w.poses_gt, free)
    gP = torch.tensor(G, dtype=torch.float64, device=dev)
    guv = torch.zeros_like(uv)
    gw = torch.zeros(uv.shape[0], dtype=torch.float64, device=dev)
    rep, _ = ba.adjoint(B, s, P, L, uv, None, gP, None, guv, gw)
    torch.cuda.synchronize()
    assert np.all(ba.parse_reports(rep)["chol_failures"] == 0)
    guv, gw = guv.cpu().numpy(), gw.cpu().numpy()
    assert np.all(np.isfinite(guv)) and np.all(np.isfinite(gw))
    for k in (0, 37, 63):
        w = wa[k]
        prob = oracle.Problem.from_window(w)
        Pk, Lk = Pn[po[k]:po[k + 1]], Ln[lo[k]:lo[k + 1]]
        free = ~prob.pose_fixed
        gx = np.concatenate([oracle.ambient_to_tangent(Pk, G[po[k]:po[k + 1]])[free].reshape(-1),
                             np.zeros(3 * prob.n_points)])
        ruv, rw = oracle.adjoint_dense(Pk, Lk, prob, 1.0, gx)
        e_uv = np.linalg.norm(guv[oo[k]:oo[k + 1]] - ruv) / np.linalg.norm(ruv)
        e_w = np.linalg.norm(gw[oo[k]:oo[k + 1]] - rw) / np.linalg.norm(rw)
        print("adjoint window", k, e_uv, e_w, flush=True)
        assert e_uv <= 1e-3 and e_w <= 1e-3


def _empty_like(w, n_poses=3):
    e = w.copy()
    e.poses_gt = w.poses_gt[:n_poses].copy()
    e.poses_init = w.poses_init[:n_poses].copy()
    e.pose_fixed = w.pose_fixed[:n_poses].copy()
    e.points_gt = np.zeros((0, 3))
    e.points_init = np.zeros((0, 3))
    for f in ("obs_pose", "obs_point", "obs_cam"):
        setattr(e, f, np.zeros(0, np.int32))
    e.obs_uv = np.zeros((0, 2))
    e.obs_w = np.zeros(0)
    e.outlier = np.zeros(0, bool)
    return e


def test_batch_with_an_empty_window():
    import paper_2506_04359_amd as ba
    a = bagen.tiny_window(seed=71, n_kf=4, n_lm=15)
    b = bagen.tiny_window(seed=72, n_kf=5, n_lm=12)
    e = _empty_like(a)
    s = ba.Settings(max_iters=6, precision=ba.BA_FP64)
    out = gpu_solve_batched([a, e, b], s)
    for w, o in ((a, out[0]), (b, out[2])):
        _fp64_replay_parity(w, s, o)
    r = out[1]["report"]
    assert r["initial_cost"] == 0.0 and r["final_cost"] == 0.0 and r["accepted"] == 0
    assert r["iters"] == 6
    assert np.array_equal(out[1]["poses"], e.poses_init)


def test_four_class_batch_with_an_empty_largest_class():
    """Windows of four size classes, so that each class runs its LM loop as its
    own chain: the largest class holds only a window without landmarks (its
    chain has no pass-A or pass-B work), the others follow the oracle."""
    import paper_2506_04359_amd as ba
    a = bagen.tiny_window(seed=74, n_kf=4, n_lm=15)
    b = bagen.tiny_window(seed=75, n_kf=12, n_lm=30)
    c = bagen.tiny_window(seed=76, n_kf=20, n_lm=40)
    e = _empty_like(bagen.tiny_window(seed=77, n_kf=27, n_lm=4), n_poses=27)
    assert [int((w.pose_fixed == 0).sum()) for w in (a, b, c, e)] == [3, 11, 19, 26]
    s = ba.Settings(max_iters=6, precision=ba.BA_FP64)
    out = gpu_solve_batched([c, e, a, b], s)
    for w, o in ((c, out[0]), (a, out[2]), (b, out[3])):
        _fp64_replay_parity(w, s, o)
    r = out[1]["report"]
    assert r["initial_cost"] == 0.0 and r["final_cost"] == 0.0 and r["accepted"] == 0
    assert r["iters"] == 6
    assert np.array_equal(out[1]["poses"], e.poses_init)
