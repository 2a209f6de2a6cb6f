"""Synthetic workload generator: determinism, sizes and visibility."""
import numpy as np
import pytest

import bagen


def test_deterministic_per_seed():
    a = bagen.make_window(1)
    b = bagen.make_window(1)
    for f in ("obs_uv", "poses_init", "points_init", "obs_pose", "obs_point"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    c = bagen.make_window(3, 0)
    d = bagen.make_window(3, 1)
    assert c.n_obs != d.n_obs or not np.array_equal(c.obs_uv, d.obs_uv)


@pytest.mark.parametrize("cfg,n_lm,obs_lo,obs_hi", [(1, 200, 600, 1000), (2, 5000, 54000, 66000),
                                                     (4, 20000, 255000, 345000)])
def test_sizes(cfg, n_lm, obs_lo, obs_hi):
    w = bagen.make_window(cfg)
    assert w.n_points == n_lm
    assert obs_lo <= w.n_obs <= obs_hi
    # every landmark has at least two distinct views
    views = {}
    for i, j, k in zip(w.obs_pose, w.obs_point, w.obs_cam):
        views.setdefault(j, set()).add((i, k))
    assert min(len(v) for v in views.values()) >= 2


def test_outlier_fraction_stereo():
    w = bagen.make_window(2)
    assert 0.017 <= w.outlier.mean() <= 0.023


def test_batch_windows_within_ranges():
    for i in range(6):
        w = bagen.make_window(3, i)
        assert 5 <= w.n_poses <= 30 and 500 <= w.n_points <= 8000
        counts = np.bincount(w.obs_point, minlength=w.n_points)
        assert counts.min() >= 2 and counts.max() <= 10


def test_ground_truth_in_front_and_inside_image():
    for cfg in (1, 2, 4):
        w = bagen.make_window(cfg)
        inl = ~w.outlier
        for o in np.nonzero(inl)[0][:2000]:
            xc = bagen._to_cam(w.poses_gt[w.obs_pose[o]], w.extrinsics[w.obs_cam[o]],
                               w.points_gt[w.obs_point[o]][None])[0]
            assert xc[2] > 0.1
            uv = bagen._project(w.intrinsics[w.obs_cam[o]], xc[None])[0]
            assert 0 <= uv[0] < w.image_size[w.obs_cam[o], 0] and 0 <= uv[1] < w.image_size[w.obs_cam[o], 1]
