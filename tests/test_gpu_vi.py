"""Visual-inertial window solve on the GPU (Sec. 2.2, "Visual-Inertial", Eq. 9)
against the FP64 visual-inertial oracle: the preintegrated factors, the FP64
solve with decision replay (1e-9), a noiseless window recovered exactly, and
the mixed-precision bar."""
import math

import numpy as np
import pytest

import bagen
import oracle
from oracle import imu
from helpers import check_decisions, rel_err

pytestmark = pytest.mark.gpu
TOL64 = 1e-9


def _gpu_inputs(vw, bias_bar):
    import torch
    dev = torch.device("cuda:0")
    n = len(vw.gyro)
    sb = np.concatenate([[0], np.cumsum([g.shape[0] for g in vw.gyro])]).astype(np.int32)
    t = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    bb = np.tile(np.concatenate([bias_bar[0], bias_bar[1]]), (n, 1))
    return t(sb, torch.int32), t(np.concatenate(vw.gyro)), t(np.concatenate(vw.accel)), t(bb)


def _oracle_problem(vw, bias_bar):
    w = vw.window
    noise = imu.ImuNoise(*vw.noise)
    factors = []
    for i in range(w.n_poses - 1):
        pre = imu.preintegrate(vw.gyro[i], vw.accel[i], vw.dt, bias_bar[1], bias_bar[0], noise)
        factors.append((i, i + 1, pre, imu.imu_information(pre, noise)))
    return imu.ViProblem(visual=oracle.Problem.from_window(w), factors=factors, gravity=vw.gravity)


def _gpu_solve(vw, s, preint, states0=None, poses0=None, points0=None):
    import torch
    import paper_2506_04359_amd as ba
    dev = torch.device("cuda:0")
    w = vw.window
    W = ba.Window.from_problem(w)
    P = torch.tensor(w.poses_init if poses0 is None else poses0, dtype=torch.float64, device=dev)
    L = torch.tensor(w.points_init if points0 is None else points0, dtype=torch.float64, device=dev)
    st0 = np.concatenate([vw.vel_init, vw.ba_init, vw.bg_init], axis=1) if states0 is None else states0
    X = torch.tensor(st0, dtype=torch.float64, device=dev)
    uv = torch.tensor(w.obs_uv, dtype=torch.float64, device=dev)
    tr = torch.zeros(32 * s.max_iters, dtype=torch.uint8, device=dev)
    rep, tr, _ = ba.vi_solve(W, s, preint, vw.gravity, P, L, X, uv, None, trace=tr)
    torch.cuda.synchronize()
    return dict(poses=P.cpu().numpy(), points=L.cpu().numpy(), states=X.cpu().numpy(),
                report=ba.parse_reports(rep)[0], trace=ba.parse_traces(tr, 1, s.max_iters)[0])


def test_preintegration_matches_oracle():
    import paper_2506_04359_amd as ba
    vw = bagen.make_vi_window(seed=9101, n_kf=6, n_lm=60)
    bias_bar = (np.array([0.02, -0.01, 0.03]), np.array([0.004, -0.002, 0.003]))
    sb, gy, ac, bb = _gpu_inputs(vw, bias_bar)
    pre = ba.vi_preintegrate(sb, gy, ac, vw.dt, bb, vw.noise).cpu().numpy()
    noise = imu.ImuNoise(*vw.noise)
    for f in range(len(vw.gyro)):
        o = imu.preintegrate(vw.gyro[f], vw.accel[f], vw.dt, bias_bar[1], bias_bar[0], noise)
        Info = imu.imu_information(o, noise)
        g = pre[f]
        for arr, off, n in ((o.dR.reshape(-1), 0, 9), (o.dv, 9, 3), (o.dp, 12, 3), (np.array([o.dT]), 15, 1),
                            (o.J_Rg.reshape(-1), 16, 9), (o.J_vg.reshape(-1), 25, 9), (o.J_va.reshape(-1), 34, 9),
                            (o.J_pg.reshape(-1), 43, 9), (o.J_pa.reshape(-1), 52, 9), (bias_bar[0], 61, 3),
                            (bias_bar[1], 64, 3)):
            assert np.abs(g[off:off + n] - arr).max() <= 1e-12 * max(1.0, np.abs(arr).max()), (f, off)
        gi = g[67:67 + 225].reshape(15, 15)
        assert np.abs(gi - Info).max() <= 1e-9 * np.abs(Info).max(), f


def test_fp64_vi_solve_matches_oracle():
    import paper_2506_04359_amd as ba
    vw = bagen.make_vi_window(seed=9102, n_kf=7, n_lm=150)
    bias_bar = (vw.ba_init[0], vw.bg_init[0])
    sb, gy, ac, bb = _gpu_inputs(vw, bias_bar)
    preint = ba.vi_preintegrate(sb, gy, ac, vw.dt, bb, vw.noise)
    s = ba.Settings(max_iters=10, precision=ba.BA_FP64)
    g = _gpu_solve(vw, s, preint)
    vp = _oracle_problem(vw, bias_bar)
    w = vw.window
    x0 = imu.ViState(poses=w.poses_init.copy(), vel=vw.vel_init.copy(), ba=vw.ba_init.copy(), bg=vw.bg_init.copy(),
                     points=w.points_init.copy())
    ref = imu.vi_lm_solve(x0, vp, oracle.LMSettings(max_iters=10),
                          decisions=[bool(a) for a in g["trace"]["accepted"]])
    check_decisions(ref, g["trace"])
    r = g["report"]
    assert r["status"] == 0 and r["accepted"] >= 5
    assert abs(r["initial_cost"] - ref.initial_cost) <= TOL64 * ref.initial_cost
    assert abs(r["final_cost"] - ref.final_cost) <= TOL64 * ref.final_cost
    for t, gt in zip(ref.trace, g["trace"]):
        assert abs(t["cost"] - gt["cost"]) <= TOL64 * abs(t["cost"])
    X = ref.state
    assert rel_err(g["poses"], X.poses) <= TOL64 and rel_err(g["points"], X.points) <= TOL64
    st = np.concatenate([X.vel, X.ba, X.bg], axis=1)
    assert np.abs(g["states"] - st).max() <= TOL64 * max(1.0, np.abs(st).max())


def test_noiseless_vi_window_is_recovered():
    import paper_2506_04359_amd as ba
    vw = bagen.make_vi_window(seed=9103, n_kf=6, n_lm=120, sigma_px=0.0, imu_noise=False)
    bias_bar = (vw.ba_gt, vw.bg_gt)
    sb, gy, ac, bb = _gpu_inputs(vw, bias_bar)
    preint = ba.vi_preintegrate(sb, gy, ac, vw.dt, bb, vw.noise)
    s = ba.Settings(max_iters=30, precision=ba.BA_FP64, lambda_init=1e-3)
    g = _gpu_solve(vw, s, preint)
    w = vw.window
    assert g["report"]["final_cost"] < 1e-14 * g["report"]["initial_cost"]
    assert np.abs(g["poses"] - w.poses_gt).max() < 1e-7
    assert np.abs(g["points"] - w.points_gt).max() < 1e-6
    st = np.concatenate([vw.vel_gt, np.tile(vw.ba_gt, (6, 1)), np.tile(vw.bg_gt, (6, 1))], axis=1)
    assert np.abs(g["states"] - st).max() < 1e-6


def test_mixed_vi_solve_meets_the_bar():
    import paper_2506_04359_amd as ba
    vw = bagen.make_vi_window(seed=9104, n_kf=8, n_lm=200)
    bias_bar = (vw.ba_init[0], vw.bg_init[0])
    sb, gy, ac, bb = _gpu_inputs(vw, bias_bar)
    preint = ba.vi_preintegrate(sb, gy, ac, vw.dt, bb, vw.noise)
    s = ba.Settings(max_iters=10, precision=ba.BA_MIXED)
    g = _gpu_solve(vw, s, preint)
    vp = _oracle_problem(vw, bias_bar)
    w = vw.window
    x0 = imu.ViState(poses=w.poses_init.copy(), vel=vw.vel_init.copy(), ba=vw.ba_init.copy(), bg=vw.bg_init.copy(),
                     points=w.points_init.copy())
    try:
        ref = imu.vi_lm_solve(x0, vp, oracle.LMSettings(max_iters=10),
                              decisions=[bool(a) for a in g["trace"]["accepted"]])
    except ValueError:
        ref = imu.vi_lm_solve(x0, vp, oracle.LMSettings(max_iters=10))
    prob = vp.visual
    assert abs(oracle.rms(g["poses"], g["points"], prob) - oracle.rms(ref.state.poses, ref.state.points, prob)) <= 1e-3
    ang, dt = oracle.rotation_errors(g["poses"], ref.state.poses)
    tn = np.maximum(np.linalg.norm(ref.state.poses[:, :, 3], axis=1), 1.0)
    assert ang.max() <= 1e-4 and (dt / tn).max() <= 1e-4
    assert np.abs(g["states"][:, :3] - ref.state.vel).max() <= 1e-4 * max(1.0, np.abs(ref.state.vel).max())


def test_preintegration_ragged_intervals():
    # intervals of 2 to 64 samples, each integrated at its own bias estimate,
    # and intervals of one and no sample, whose covariance is singular
    import torch
    import paper_2506_04359_amd as ba
    dev = torch.device("cuda:0")
    vw = bagen.make_vi_window(seed=9105, n_kf=9, n_lm=30)
    gy_all, ac_all = np.concatenate(vw.gyro), np.concatenate(vw.accel)
    counts = np.array([2, 3, 61, 7, 33, 2, 50, 12, 64, 4, 1, 0])
    sb = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    assert sb[-1] <= gy_all.shape[0]
    rng = np.random.default_rng(9105)
    bb = np.concatenate([rng.normal(scale=0.05, size=(counts.size, 3)), rng.normal(scale=0.01, size=(counts.size, 3))],
                        axis=1)
    t = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    pre = ba.vi_preintegrate(t(sb, torch.int32), t(gy_all), t(ac_all), vw.dt, t(bb), vw.noise).cpu().numpy()
    noise = imu.ImuNoise(*vw.noise)
    for f in range(counts.size):
        s0, s1 = sb[f], sb[f + 1]
        g = pre[f]
        assert abs(g[15] - counts[f] * vw.dt) <= 1e-15
        if counts[f] < 2:
            assert np.isnan(g[67:67 + 225].reshape(15, 15)[:9, :9]).all()
            if counts[f] == 1:
                o = imu.preintegrate(gy_all[s0:s1], ac_all[s0:s1], vw.dt, bb[f, 3:], bb[f, :3], noise)
                assert np.linalg.matrix_rank(o.cov) == 6
            continue
        o = imu.preintegrate(gy_all[s0:s1], ac_all[s0:s1], vw.dt, bb[f, 3:], bb[f, :3], noise)
        for arr, off in ((o.dR.reshape(-1), 0), (o.dv, 9), (o.dp, 12), (o.J_Rg.reshape(-1), 16),
                         (o.J_vg.reshape(-1), 25), (o.J_va.reshape(-1), 34), (o.J_pg.reshape(-1), 43),
                         (o.J_pa.reshape(-1), 52)):
            assert np.abs(g[off:off + arr.size] - arr).max() <= 1e-12 * max(1.0, np.abs(arr).max()), (f, off)
        Info = imu.imu_information(o, noise)
        assert np.abs(g[67:67 + 225].reshape(15, 15) - Info).max() <= 1e-9 * np.abs(Info).max(), f


@pytest.mark.parametrize("n_kf,n_lm", [(2, 80), (24, 300)])
def test_fp64_vi_solve_at_the_pose_count_limits(n_kf, n_lm):
    # the smallest window (one factor) and the largest (24 states)
    import paper_2506_04359_amd as ba
    vw = bagen.make_vi_window(seed=9106 + n_kf, n_kf=n_kf, n_lm=n_lm)
    bias_bar = (vw.ba_init[0], vw.bg_init[0])
    sb, gy, ac, bb = _gpu_inputs(vw, bias_bar)
    preint = ba.vi_preintegrate(sb, gy, ac, vw.dt, bb, vw.noise)
    s = ba.Settings(max_iters=8, precision=ba.BA_FP64)
    g = _gpu_solve(vw, s, preint)
    vp = _oracle_problem(vw, bias_bar)
    w = vw.window
    x0 = imu.ViState(poses=w.poses_init.copy(), vel=vw.vel_init.copy(), ba=vw.ba_init.copy(), bg=vw.bg_init.copy(),
                     points=w.points_init.copy())
    ref = imu.vi_lm_solve(x0, vp, oracle.LMSettings(max_iters=8),
                          decisions=[bool(a) for a in g["trace"]["accepted"]])
    check_decisions(ref, g["trace"])
    r = g["report"]
    assert r["status"] == 0 and r["accepted"] >= 3
    assert abs(r["final_cost"] - ref.final_cost) <= TOL64 * ref.final_cost
    X = ref.state
    assert rel_err(g["poses"], X.poses) <= TOL64 and rel_err(g["points"], X.points) <= TOL64
    st = np.concatenate([X.vel, X.ba, X.bg], axis=1)
    assert np.abs(g["states"] - st).max() <= TOL64 * max(1.0, np.abs(st).max())


def test_vi_solve_is_deterministic():
    import paper_2506_04359_amd as ba
    vw = bagen.make_vi_window(seed=9108, n_kf=10, n_lm=250)
    bias_bar = (vw.ba_init[0], vw.bg_init[0])
    sb, gy, ac, bb = _gpu_inputs(vw, bias_bar)
    preint = ba.vi_preintegrate(sb, gy, ac, vw.dt, bb, vw.noise)
    s = ba.Settings(max_iters=10, precision=ba.BA_MIXED)
    a, b = _gpu_solve(vw, s, preint), _gpu_solve(vw, s, preint)
    for k in ("poses", "points", "states"):
        assert a[k].tobytes() == b[k].tobytes()
    assert a["report"].tobytes() == b["report"].tobytes()


def test_vi_refusals():
    import ctypes
    import torch
    import paper_2506_04359_amd as ba
    dev = torch.device("cuda:0")
    # 25 keyframes: beyond the 24 states a window may hold
    vw = bagen.make_vi_window(seed=9109, n_kf=25, n_lm=100)
    W = ba.Window.from_problem(vw.window)
    s = ba.Settings(max_iters=2, precision=ba.BA_FP64)
    with pytest.raises(ba.BAError) as e:
        ba.vi_workspace_size(W, s)
    assert e.value.status == ba.BA_ERR_UNSUPPORTED
    # a workspace too small for the IMU records after the solve's own
    vw = bagen.make_vi_window(seed=9110, n_kf=5, n_lm=60)
    W = ba.Window.from_problem(vw.window)
    need = ba.vi_workspace_size(W, s)
    assert need > W.workspace_size(s)
    w = vw.window
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    P, L, uv = t(w.poses_init), t(w.points_init), t(w.obs_uv)
    X = t(np.zeros((5, 9)))
    pre = torch.zeros((4, ba.VI_PREINT_DOUBLES), dtype=torch.float64, device=dev)
    ws = torch.empty(need - 256, dtype=torch.uint8, device=dev)
    rep = torch.zeros(ba.REPORT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    g = np.array(vw.gravity, dtype=np.float64)
    P0 = P.clone()
    st = ba.lib().ba_vi_solve(W.handle, ctypes.byref(s.c()), pre.data_ptr(), g.ctypes.data_as(ctypes.c_void_p),
                              P.data_ptr(), L.data_ptr(), X.data_ptr(), uv.data_ptr(), None, ws.data_ptr(),
                              ws.numel(), rep.data_ptr(), None, None)
    assert st == ba.BA_ERR_WORKSPACE_TOO_SMALL
    torch.cuda.synchronize()
    assert torch.equal(P, P0)
