"""The sliding-window local map on the GPU (Sec. 2.1 local odometry map, Sec.
2.2 keyframe insertion and SBA): the device values of every window equal the
oracle map's (the gather kernels copy, bit for bit), the refined values a solve
leaves are carried into the next windows, and a solve of the map's window
equals ba_solve of the same window built directly (bit for bit) and the FP64
oracle (decision replay, 1e-9)."""
import numpy as np
import pytest

import bagen
import oracle
from oracle.window_map import WindowMap
from helpers import check_decisions, oracle_settings, rel_err

TOL64 = 1e-9

pytestmark = pytest.mark.gpu


def _kf_args(o, N, kf):
    k_after = min(o.n_keyframes() + 1, N)
    return (kf.pose_init, kf.new_ids, kf.new_points, np.full(kf.obs_lm.shape[0], k_after - 1, np.int32),
            kf.obs_lm, kf.obs_cam, kf.obs_uv)


def _check_values(m, o):
    P, L, uv, w = m.read()
    ow = o.window()
    assert np.array_equal(P, ow["poses"]) and np.array_equal(L, ow["points"])
    assert np.array_equal(uv, ow["obs_uv"]) and np.array_equal(w, ow["obs_w"])


def test_values_follow_the_oracle_through_solves():
    import torch
    import paper_2506_04359_amd as ba
    seq = bagen.make_stereo_sequence(n_keyframes=12, births=80, seed=11010)
    N = 5
    m = ba.Map(N, seq.intrinsics, seq.extrinsics.reshape(-1, 12))
    o = WindowMap(N, 2)
    s = ba.Settings(max_iters=4, precision=ba.BA_MIXED)
    for i, kf in enumerate(seq.keyframes):
        args = _kf_args(o, N, kf)
        assert m.add_keyframe(*args) == len(o.add_keyframe(*args))
        _check_values(m, o)
        if i >= 1:
            rep, _, _ = m.solve(s)
            torch.cuda.synchronize()
            r = ba.parse_reports(rep)[0]
            assert r["status"] == 0 and r["final_cost"] <= r["initial_cost"]
            P, L, _, _ = m.read()
            o.set_state(P, L)      # the oracle map carries the GPU's refined values
    assert m.info()[0] == N


def test_map_solve_equals_direct_solve_and_oracle():
    import torch
    import paper_2506_04359_amd as ba
    seq = bagen.make_stereo_sequence(n_keyframes=9, births=60, seed=11011)
    N = 6
    m = ba.Map(N, seq.intrinsics, seq.extrinsics.reshape(-1, 12))
    o = WindowMap(N, 2)
    for kf in seq.keyframes:
        args = _kf_args(o, N, kf)
        m.add_keyframe(*args)
        o.add_keyframe(*args)
    w = o.window()
    s = ba.Settings(max_iters=8, precision=ba.BA_FP64)
    dev = torch.device("cuda:0")
    # direct window of the same arrays
    Wd = ba.Window(w["poses"].shape[0], w["points"].shape[0], w["obs_pose"], w["obs_point"], seq.intrinsics,
                   obs_cam=w["obs_cam"], pose_fixed=w["pose_fixed"], extrinsics=seq.extrinsics.reshape(-1, 12))
    P = torch.tensor(w["poses"], dtype=torch.float64, device=dev)
    L = torch.tensor(w["points"], dtype=torch.float64, device=dev)
    uv = torch.tensor(w["obs_uv"], dtype=torch.float64, device=dev)
    tr_d = torch.zeros(32 * s.max_iters, dtype=torch.uint8, device=dev)
    rep_d, _, _ = ba.solve(Wd, s, P, L, uv, None, trace=tr_d)
    tr_m = torch.zeros(32 * s.max_iters, dtype=torch.uint8, device=dev)
    rep_m, _, _ = m.solve(s, trace=tr_m)
    torch.cuda.synchronize()
    Pm, Lm, _, _ = m.read()
    assert np.array_equal(Pm, P.cpu().numpy()) and np.array_equal(Lm, L.cpu().numpy())
    assert rep_m.cpu().numpy().tobytes() == rep_d.cpu().numpy().tobytes()
    trace = ba.parse_traces(tr_m, 1, s.max_iters)[0]
    # the FP64 oracle on the oracle map's window, following the GPU's decisions
    prob = oracle.Problem(intrinsics=seq.intrinsics, extrinsics=seq.extrinsics, obs_pose=w["obs_pose"].astype(np.int64),
                          obs_point=w["obs_point"].astype(np.int64), obs_cam=w["obs_cam"].astype(np.int64),
                          obs_uv=w["obs_uv"], obs_w=w["obs_w"], pose_fixed=w["pose_fixed"].astype(bool),
                          n_poses=w["poses"].shape[0], n_points=w["points"].shape[0])
    ref = oracle.lm_solve(w["poses"], w["points"], prob, oracle_settings(s), backend="schur",
                          decisions=[bool(a) for a in trace["accepted"]])
    check_decisions(ref, trace)
    r = ba.parse_reports(rep_m)[0]
    assert abs(r["final_cost"] - ref.final_cost) <= TOL64 * ref.final_cost
    assert rel_err(Pm, ref.poses) <= TOL64 and rel_err(Lm, ref.points) <= TOL64


def test_map_arrays_are_the_solve_arrays():
    import torch
    import paper_2506_04359_amd as ba
    seq = bagen.make_stereo_sequence(n_keyframes=3, births=30, seed=11012)
    m = ba.Map(4, seq.intrinsics, seq.extrinsics.reshape(-1, 12))
    o = WindowMap(4, 2)
    for kf in seq.keyframes:
        args = _kf_args(o, 4, kf)
        m.add_keyframe(*args)
        o.add_keyframe(*args)
    ptrs = m.arrays()
    assert all(p for p in ptrs)
    K, M, n = m.info()
    W = m.window()
    assert (W.n_poses, W.n_points, W.n_obs) == (K, M, n)
    torch.cuda.synchronize()
