"""C ABI on the host: the library loads, exports what include/ba.h declares,
validates structure before any device work, and builds a consistent plan.
No compute call is made here (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import bagen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_04359_amd", "libba.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libba.so not built")


def _declared():
    src = open(os.path.join(ROOT, "include", "ba.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert "ba_solve" in names and "ba_adjoint" in names and "ba_solve_batched" in names
    L = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    import paper_2506_04359_amd as ba
    L = ba.lib()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert L.ba_status_string(s).decode() not in ("", "unknown status")


def _mk(w, **kw):
    import paper_2506_04359_amd as ba
    args = dict(n_poses=w.n_poses, n_points=w.n_points, obs_pose=w.obs_pose, obs_point=w.obs_point,
                intrinsics=w.intrinsics, obs_cam=w.obs_cam, pose_fixed=w.pose_fixed,
                extrinsics=w.extrinsics, host_only=True)
    args.update(kw)
    return ba.Window(**args)


@pytest.mark.parametrize("case,frag", [
    ("pose_range", "obs_pose"),
    ("point_range", "obs_point"),
    ("cam_range", "obs_cam"),
    ("single_view", "fewer than 2"),
    ("nan_intr", "non-finite intrinsics"),
    ("neg_focal", "focal"),
    ("bad_rot", "rotation"),
    ("too_many_poses", "64 poses"),
])
def test_validation_errors(case, frag):
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=3, n_kf=3, n_lm=6, stereo=True)
    kw = {}
    if case == "pose_range":
        op = w.obs_pose.copy()
        op[2] = 7
        kw["obs_pose"] = op
    elif case == "point_range":
        oj = w.obs_point.copy()
        oj[0] = -1
        kw["obs_point"] = oj
    elif case == "cam_range":
        oc = w.obs_cam.copy()
        oc[1] = 2
        kw["obs_cam"] = oc
    elif case == "single_view":
        # landmark 0 keeps one observation only
        keep = np.ones(w.n_obs, bool)
        idx = np.nonzero(w.obs_point == 0)[0]
        keep[idx[1:]] = False
        kw.update(obs_pose=w.obs_pose[keep], obs_point=w.obs_point[keep], obs_cam=w.obs_cam[keep])
    elif case == "nan_intr":
        K = w.intrinsics.copy()
        K[0, 2] = np.nan
        kw["intrinsics"] = K
    elif case == "neg_focal":
        K = w.intrinsics.copy()
        K[1, 0] = -1.0
        kw["intrinsics"] = K
    elif case == "bad_rot":
        E = w.extrinsics.copy()
        E[1, 0, 0] = 2.0
        kw["extrinsics"] = E
    elif case == "too_many_poses":
        kw["n_poses"] = 65
        kw["pose_fixed"] = None
    with pytest.raises(ba.BAError) as e:
        _mk(w, **kw)
    assert frag in str(e.value)


def test_plan_is_landmark_major_permutation():
    w = bagen.make_window(2)
    W = _mk(w)
    perm = W.order()
    assert np.array_equal(np.sort(perm), np.arange(w.n_obs))
    lm = w.obs_point[perm]
    assert np.all(np.diff(lm) >= 0)
    # inside a landmark: free poses (by slot) first, then cameras ascending
    pose = w.obs_pose[perm]
    cam = w.obs_cam[perm]
    same = np.diff(lm) == 0
    key = pose.astype(np.int64) * 64 + cam      # pose 0 is the only fixed pose and sorts last
    key[w.pose_fixed[pose] == 1] += 1 << 20
    assert np.all(np.diff(key)[same] >= 0)
    info = W.info()
    pairs = len({(i, j) for i, j in zip(w.obs_pose, w.obs_point)})
    assert info["n_pairs"] == pairs and info["n_obs"] == w.n_obs
    nfree = np.zeros(w.n_points, np.int64)
    for i, j in {(i, j) for i, j in zip(w.obs_pose, w.obs_point)}:
        nfree[j] += 0 if w.pose_fixed[i] else 1
    assert info["schur_blocks"] == int(np.sum(nfree * (nfree + 1) // 2))


def test_single_window_plans_spread_work_items():
    # a plan of one window has nothing to run beside it: its work items aim at
    # n_obs / 256 observations (at least 128, at most 8192), whole tiles each
    for cfg in (1, 2, 4):
        w = bagen.make_window(cfg)
        i = _mk(w).info()
        co = max(128, min(8192, w.n_obs // 256))
        want = max(1, (w.n_obs + co // 2) // co)
        assert i["n_chunks"] == min(want, i["n_tiles"]), (cfg, i)
        assert i["n_chunks"] > 1


def test_host_only_window_cannot_be_solved():
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=4)
    W = _mk(w)
    with pytest.raises(ba.BAError) as e:
        W.workspace_size(ba.Settings())
    assert e.value.status == -6


def test_free_pose_limit_reported_as_unsupported():
    import paper_2506_04359_amd as ba
    n = 40
    rng = np.random.default_rng(0)
    op = np.repeat(np.arange(n), 2)
    oj = np.tile([0, 1], n)
    with pytest.raises(ba.BAError) as e:
        ba.Window(n, 2, op, oj, [[400.0, 400.0, 320.0, 240.0]], pose_fixed=np.zeros(n, np.uint8),
                  host_only=True)
    assert e.value.status == -5


def test_window_without_landmarks_plans_to_nothing():
    import paper_2506_04359_amd as ba
    w = bagen.tiny_window(seed=71, n_kf=4, n_lm=15)
    W = ba.Window(3, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), w.intrinsics,
                  obs_cam=np.zeros(0, np.int32), pose_fixed=w.pose_fixed[:3], extrinsics=w.extrinsics,
                  host_only=True)
    i = W.info()
    assert i["n_obs"] == 0 and i["n_pairs"] == 0 and i["n_points"] == 0 and i["n_free"] == 2


@pytest.mark.parametrize("n_cams,K,frag", [
    (0, [[400.0, 400.0, 320.0, 240.0]], "n_cams"),
    (33, [[400.0, 400.0, 320.0, 240.0]] * 33, "32 cameras"),
    (1, [[400.0, np.nan, 320.0, 240.0]], "non-finite"),
    (1, [[-400.0, 400.0, 320.0, 240.0]], "focal"),
])
def test_rig_validation_errors(n_cams, K, frag):
    import ctypes
    import paper_2506_04359_amd as ba
    L = ba.lib()
    Kh = np.ascontiguousarray(np.asarray(K, float))
    h = ctypes.c_void_p()
    st = L.ba_rig_create(n_cams, Kh.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(h))
    assert st in (-1, -5)
    assert frag in L.ba_last_error().decode()


def test_rig_extrinsic_must_be_a_rotation():
    import ctypes
    import paper_2506_04359_amd as ba
    L = ba.lib()
    K = np.array([[400.0, 400.0, 320.0, 240.0]])
    E = np.array([[2.0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]])
    h = ctypes.c_void_p()
    st = L.ba_rig_create(1, K.ctypes.data_as(ctypes.c_void_p), E.ctypes.data_as(ctypes.c_void_p),
                         ctypes.byref(h))
    assert st == -1 and "rotation" in L.ba_last_error().decode()


def test_pnp_solve_argument_errors():
    import ctypes
    import paper_2506_04359_amd as ba
    L = ba.lib()
    s = ba.Settings().c()
    assert L.ba_pnp_solve(None, ctypes.byref(s), 1, 0, 0, None, None, None, None, None, None, None,
                          None, None, None, None) == -1
    assert "rig" in L.ba_last_error().decode()


def test_rig_waves_per_frame_needs_a_rig():
    import paper_2506_04359_amd as ba
    L = ba.lib()
    assert L.ba_rig_set_waves_per_frame(None, 1) == -1
    assert "rig" in L.ba_last_error().decode()


def test_triangulate_argument_errors():
    import ctypes
    import paper_2506_04359_amd as ba
    L = ba.lib()
    s = ba.Settings().c()
    assert L.ba_triangulate(None, ctypes.byref(s), 1, 0, 0, None, None, None, None, None, None, None,
                            None, None, None) == -1
    assert "rig" in L.ba_last_error().decode()
