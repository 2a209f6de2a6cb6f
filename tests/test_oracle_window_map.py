"""Pins of the window-map oracle (Sec. 2.1 local odometry map, Sec. 2.2
keyframe insertion): a hand-worked four-keyframe sequence in a three-keyframe
window, and the invariants the rules guarantee on a long generated sequence."""
import numpy as np
import pytest

import bagen
from oracle.window_map import WindowMap


def _P(x):
    return np.concatenate([np.eye(3), np.array([[x], [0.0], [0.0]])], axis=1)


def test_hand_worked_sequence():
    # N = 3, one camera.  A: no observations.  B: landmarks 1 and 2, each seen in
    # A and B.  C: landmark 3 seen in B and C, landmark 1 seen again in C.
    # D: the window is full, so A leaves with its observations; landmark 1
    # keeps views B, C; landmark 2 keeps only B and is dropped with (2, B);
    # landmark 3 keeps B, C; D sees landmark 3.  Observation order is the
    # order of insertion: (1,B) (3,B) (3,C) (1,C) (3,D).
    m = WindowMap(3, 1)
    uv = lambda n: np.arange(2 * n, dtype=float).reshape(n, 2)
    assert m.add_keyframe(_P(0.0)) == []
    assert m.add_keyframe(_P(1.0), [1, 2], [[0, 0, 5.0], [1, 0, 6.0]], [0, 1, 0, 1], [1, 1, 2, 2],
                          [0, 0, 0, 0], uv(4)) == []
    assert m.add_keyframe(_P(2.0), [3], [[2, 0, 7.0]], [1, 2, 2], [3, 3, 1], [0, 0, 0], uv(3)) == []
    w = m.window()
    assert w["landmark_ids"].tolist() == [1, 2, 3]
    assert w["obs_pose"].tolist() == [0, 1, 0, 1, 1, 2, 2]
    assert w["obs_point"].tolist() == [0, 0, 1, 1, 2, 2, 0]
    assert m.add_keyframe(_P(3.0), [], None, [2], [3], [0], uv(1)) == [2]
    w = m.window()
    assert w["poses"][:, 0, 3].tolist() == [1.0, 2.0, 3.0]
    assert w["pose_fixed"].tolist() == [1, 0, 0]
    assert w["landmark_ids"].tolist() == [1, 3]
    assert w["obs_pose"].tolist() == [0, 0, 1, 1, 2]
    assert w["obs_point"].tolist() == [0, 1, 1, 0, 1]
    assert w["points"].tolist() == [[0, 0, 5.0], [2, 0, 7.0]]
    # the pixels travel with their observations: (1,B) was the 2nd of B's
    # insertion, (3,B) the 1st of C's, (3,C) the 2nd, (1,C) the 3rd, (3,D) D's
    assert w["obs_uv"].tolist() == [[2, 3], [0, 1], [2, 3], [4, 5], [0, 1]]
    # landmark 2 is gone: observing it is an error, and so is reusing a live id
    with pytest.raises(ValueError):
        m.add_keyframe(_P(4.0), [], None, [2], [2], [0], uv(1))
    with pytest.raises(ValueError):
        m.add_keyframe(_P(4.0), [3], [[0, 0, 1.0]], [1, 2], [3, 3], [0, 0], uv(2))
    assert m.window()["landmark_ids"].tolist() == [1, 3]      # unchanged
    # E: B leaves; landmark 1 keeps only view C and is dropped, landmark 3
    # keeps C, D; the dropped id 2 is created again, seen in D and E
    assert m.add_keyframe(_P(4.0), [2], [[0, 0, 9.0]], [1, 2], [2, 2], [0, 0], uv(2)) == [1]
    w = m.window()
    assert w["landmark_ids"].tolist() == [3, 2]
    assert w["obs_pose"].tolist() == [0, 1, 1, 2] and w["obs_point"].tolist() == [0, 0, 1, 1]


def test_invariants_on_a_long_sequence():
    seq = bagen.make_stereo_sequence(n_keyframes=30, births=50, seed=11004)
    N = 8
    m = WindowMap(N, 2)
    seen = set()
    for i, kf in enumerate(seq.keyframes):
        k_after = min(m.n_keyframes() + 1, N)
        dropped = m.add_keyframe(kf.pose_init, kf.new_ids, kf.new_points, np.full(kf.obs_lm.size, k_after - 1),
                                 kf.obs_lm, kf.obs_cam, kf.obs_uv)
        w = m.window()
        K = w["poses"].shape[0]
        assert K == min(i + 1, N) and w["pose_fixed"].sum() == 1 and w["pose_fixed"][0] == 1
        views = {}
        for p, j, c in zip(w["obs_pose"], w["obs_point"], w["obs_cam"]):
            views.setdefault(int(j), set()).add((int(p), int(c)))
        assert sorted(views) == list(range(w["points"].shape[0]))
        assert all(len(v) >= 2 for v in views.values())
        ids = set(w["landmark_ids"].tolist())
        assert not ids & set(dropped)
        assert seen.isdisjoint(kf.new_ids.tolist())
        seen |= set(kf.new_ids.tolist())
        # the newest keyframe's observations are all there, with their pixels
        newest = w["obs_pose"] == K - 1
        assert newest.sum() == kf.obs_lm.size
        assert np.array_equal(w["obs_uv"][newest], kf.obs_uv)
