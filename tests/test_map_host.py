"""The sliding-window local map's index work (host-only map, no GPU) against
the plain oracle of the same rules (Sec. 2.1 local odometry map, Sec. 2.2
keyframe insertion): after every insertion of a keyframe sequence the window's
index lists, landmark ids and drop counts are equal; invalid insertions are
refused and leave the map as it was."""
import numpy as np
import pytest

import bagen
from oracle.window_map import WindowMap


def _insert_all(seq, N, n_kf=None):
    import paper_2506_04359_amd as ba
    m = ba.Map(N, seq.intrinsics, seq.extrinsics.reshape(-1, 12), host_only=True)
    o = WindowMap(N, seq.intrinsics.shape[0])
    for i, kf in enumerate(seq.keyframes[:n_kf]):
        k_after = min(o.n_keyframes() + 1, N)
        kfi = np.full(kf.obs_lm.shape[0], k_after - 1, np.int32)
        d_o = o.add_keyframe(kf.pose_init, kf.new_ids, kf.new_points, kfi, kf.obs_lm, kf.obs_cam, kf.obs_uv)
        d_m = m.add_keyframe(kf.pose_init, kf.new_ids, kf.new_points, kfi, kf.obs_lm, kf.obs_cam, kf.obs_uv)
        yield i, m, o, d_m, len(d_o)


def _same_window(m, o):
    w = o.window()
    L = m.lists()
    K, M, n = m.info()
    assert (K, M, n) == (w["poses"].shape[0], w["points"].shape[0], w["obs_pose"].shape[0])
    assert np.array_equal(L["landmark_ids"], w["landmark_ids"])
    assert np.array_equal(L["obs_pose"], w["obs_pose"])
    assert np.array_equal(L["obs_point"], w["obs_point"])
    assert np.array_equal(L["obs_cam"], w["obs_cam"])


def test_sequence_windows_equal_oracle():
    seq = bagen.make_stereo_sequence(n_keyframes=14, births=60, seed=11001)
    drops = 0
    for i, m, o, d_m, d_o in _insert_all(seq, 6):
        assert d_m == d_o
        drops += d_m
        _same_window(m, o)
        # every landmark of the window has two distinct views; the oldest is fixed
        w = o.window()
        views = {}
        for p, j, c in zip(w["obs_pose"], w["obs_point"], w["obs_cam"]):
            views.setdefault(j, set()).add((p, c))
        assert all(len(v) >= 2 for v in views.values()) and len(views) == w["points"].shape[0]
        assert w["poses"].shape[0] == min(i + 1, 6)
    assert drops > 0          # the slide did drop landmarks


def test_windows_plan_like_direct_windows():
    # the map's plan of a window equals the plan of the same window created
    # directly (the plan's observation order is a permutation of the map's)
    import paper_2506_04359_amd as ba
    seq = bagen.make_stereo_sequence(n_keyframes=9, births=40, seed=11002)
    for i, m, o, _, _ in _insert_all(seq, 5):
        if i < 1:
            continue
        w = o.window()
        Wd = ba.Window(w["poses"].shape[0], w["points"].shape[0], w["obs_pose"], w["obs_point"], seq.intrinsics,
                       obs_cam=w["obs_cam"], pose_fixed=w["pose_fixed"], extrinsics=seq.extrinsics.reshape(-1, 12),
                       host_only=True)
        Wm = m.window()
        assert np.array_equal(Wm.order(), Wd.order())
        assert Wm.info() == Wd.info()


def test_mono_landmark_seen_in_an_earlier_keyframe():
    # a new landmark observed in the new keyframe and in an earlier one
    import paper_2506_04359_amd as ba
    K = np.array([[458.0, 458.0, 367.0, 248.0]])
    m = ba.Map(3, K, host_only=True)
    o = WindowMap(3, 1)
    P = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    uv = np.array([[100.0, 100.0], [110.0, 100.0]])
    for mm in (m, o):
        mm.add_keyframe(P)
        mm.add_keyframe(P, [7], [[0.0, 0.0, 5.0]], [0, 1], [7, 7], [0, 0], uv)
        mm.add_keyframe(P, [], None, [2, 2], [7, 7], [0, 0], uv)   # two observations of one view
    _same_window(m, o)
    # the slide drops keyframe 0: landmark 7 keeps views (1, 0) and (2, 0)
    for mm in (m, o):
        mm.add_keyframe(P)
    _same_window(m, o)
    assert m.info()[1] == 1
    # and again: only keyframe 2's view is left, so landmark 7 goes
    assert m.add_keyframe(P) == 1 and len(o.add_keyframe(P)) == 1
    _same_window(m, o)
    assert m.info() == (3, 0, 0)


@pytest.mark.parametrize("case", ["dup_new", "existing_id", "unknown_lm", "kf_range", "cam_range", "one_view"])
def test_invalid_insertions_leave_the_map_unchanged(case):
    import paper_2506_04359_amd as ba
    seq = bagen.make_stereo_sequence(n_keyframes=4, births=20, seed=11003)
    m = ba.Map(3, seq.intrinsics, seq.extrinsics.reshape(-1, 12), host_only=True)
    o = WindowMap(3, 2)
    for kf in seq.keyframes[:3]:
        k_after = min(o.n_keyframes() + 1, 3)
        kfi = np.full(kf.obs_lm.shape[0], k_after - 1, np.int32)
        for mm in (m, o):
            mm.add_keyframe(kf.pose_init, kf.new_ids, kf.new_points, kfi, kf.obs_lm, kf.obs_cam, kf.obs_uv)
    before = (m.info(), {k: v.copy() for k, v in m.lists().items()})
    kf = seq.keyframes[3]
    ids, pts = kf.new_ids.copy(), kf.new_points.copy()
    kfi = np.full(kf.obs_lm.shape[0], 2, np.int32)
    lm, cam, uv = kf.obs_lm.copy(), kf.obs_cam.copy(), kf.obs_uv.copy()
    if case == "dup_new":
        ids[1] = ids[0]
    elif case == "existing_id":
        ids[0] = m.lists()["landmark_ids"][-1]
    elif case == "unknown_lm":
        lm[0] = 10 ** 9
    elif case == "kf_range":
        kfi[0] = 3
    elif case == "cam_range":
        cam[0] = 2
    elif case == "one_view":
        keep = ~((lm == ids[0]) & (cam == 1))
        kfi, lm, cam, uv = kfi[keep], lm[keep], cam[keep], uv[keep]
    with pytest.raises(ba.BAError) as e:
        m.add_keyframe(kf.pose_init, ids, pts, kfi, lm, cam, uv)
    assert e.value.status == ba.BA_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        o.add_keyframe(kf.pose_init, ids, pts, kfi, lm, cam, uv)
    after = (m.info(), m.lists())
    assert before[0] == after[0]
    for k in before[1]:
        assert np.array_equal(before[1][k], after[1][k])
    _same_window(m, o)
