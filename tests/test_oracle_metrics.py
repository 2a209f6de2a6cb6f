"""Pins of the oracle's result metrics (the figures the mixed-precision bar is
stated in): the RMS reprojection error per 2-D observation, over all
observations or a mask of them, and the rotation angle / translation error of
poses, against hand-worked values (tests/golden/metrics_example.txt)."""
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "metrics_example.txt")


def _rows(tag):
    out = []
    for line in open(GOLDEN):
        f = line.split()
        if f and f[0] == tag:
            out.append([float(x) for x in f[1:]])
    return out


def _axis_rot(axis, theta):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(theta) * K + (1 - math.cos(theta)) * K @ K


def _rms_problem():
    rows = _rows("rms")
    n = len(rows)
    pts = np.array([r[:3] for r in rows])
    uv = np.array([r[3:5] for r in rows])
    prob = oracle.Problem(intrinsics=np.array([[100.0, 100.0, 0.0, 0.0]]),
                          extrinsics=np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None],
                          obs_pose=np.zeros(n, np.int64), obs_point=np.arange(n), obs_cam=np.zeros(n, np.int64),
                          obs_uv=uv, obs_w=np.ones(n), pose_fixed=np.array([True]), n_poses=1, n_points=n)
    poses = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None]
    return prob, poses, pts


def test_rms_is_per_two_d_observation():
    prob, poses, pts = _rms_problem()
    want = _rows("rms_value")[0][0]
    got = oracle.rms(poses, pts, prob)
    assert abs(got - want) <= 1e-15 * want
    # the per-coordinate normalisation differs by sqrt(2): the pin tells them apart
    assert abs(got - want / math.sqrt(2.0)) > 0.1


def test_rms_over_a_mask():
    prob, poses, pts = _rms_problem()
    mask = np.array(_rows("rms_inlier_mask")[0], bool)
    want = _rows("rms_inlier_value")[0][0]
    assert abs(oracle.rms(poses, pts, prob, mask=mask) - want) <= 1e-15


def test_rotation_and_translation_errors():
    rows = _rows("rot")
    Pa, Pb, ang_want, dt_want = [], [], [], []
    for r in rows:
        axis, ta_, tb_ = r[0:3], r[3], r[4]
        Pa.append(np.concatenate([_axis_rot(axis, ta_), np.array(r[5:8])[:, None]], 1))
        Pb.append(np.concatenate([_axis_rot(axis, tb_), np.array(r[8:11])[:, None]], 1))
        ang_want.append(r[11])
        dt_want.append(r[12])
    ang, dt = oracle.rotation_errors(np.array(Pa), np.array(Pb))
    assert np.allclose(ang, ang_want, rtol=0, atol=1e-12), (ang, ang_want)
    assert np.allclose(dt, dt_want, rtol=0, atol=1e-15), (dt, dt_want)
    # symmetric in its arguments
    ang2, dt2 = oracle.rotation_errors(np.array(Pb), np.array(Pa))
    assert np.allclose(ang2, ang, atol=1e-15) and np.allclose(dt2, dt, atol=0)
