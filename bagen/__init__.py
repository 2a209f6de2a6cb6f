"""Seeded synthetic bundle-adjustment windows.

This module only *synthesises inputs*: keyframe poses, camera rigs, landmarks and
noisy pixel observations shaped like the sliding-window local map of the paper's
3D module (Sec. 2.2: the last N keyframe poses, the landmarks they see and the 2D
observations o of landmark j by camera k at pose i).  It holds none of the
solver's arithmetic.  To synthesise pixels it needs a pinhole projection; that
is written here independently (``_project``) so that the oracle's own projection
can be checked against it (noiseless ground truth must give zero residual).

Conventions
-----------
* Camera frame: x right, y down, z forward.  Pinhole without distortion.
* A pose is stored as a 3x4 ``[R | t]`` base-from-world transform (x_b = R x_w + t).
* Extrinsics are 3x4 camera-from-base transforms (x_c = R_cb x_b + t_cb).
* Every random draw comes from ``numpy.random.default_rng(seed)``; the default
  seed of window ``w`` of workload ``cfg`` is ``1000 * cfg + w``.
* Observations are emitted in a random order (not landmark-major), so that the
  solver's own ordering is exercised.

Workloads (sizes as stated for each):
  1  mono, 5 keyframes 0.5 m apart along x, 200 landmarks tracked 3-5 frames
  2  stereo, 20 keyframes, 5000 landmarks, ~60k observations, 2 % outliers
  3  256 mono windows of uneven size (5-30 keyframes, 500-8000 landmarks)
  4  32-camera rig, 10 rig poses on a circle, 20000 landmarks, ~300k observations
  5  64 mono windows, 10 keyframes, 2000 landmarks, every visible frame observed

Motion-only frames (``make_pnp_batch``): many independent frames, each a pose
observing fixed map landmarks with a stereo pair or the 32-camera rig,
optionally against a map frame shifted by a known transform.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = ["Window", "make_window", "make_workload", "tiny_window", "WORKLOAD_NAMES"]

WORKLOAD_NAMES = {
    1: "mono-5kf-200lm",
    2: "stereo-20kf-5000lm",
    3: "batch-256-mono-uneven",
    4: "rig-32cam-10pose-20000lm",
    5: "adjoint-64x-mono-10kf-2000lm",
}


@dataclasses.dataclass
class Window:
    """One sliding-window bundle-adjustment problem (all arrays float64/int32)."""

    intrinsics: np.ndarray      # (C, 4) fx, fy, cx, cy
    extrinsics: np.ndarray      # (C, 3, 4) camera-from-base
    image_size: np.ndarray      # (C, 2) width, height
    poses_gt: np.ndarray        # (N, 3, 4) base-from-world
    points_gt: np.ndarray       # (M, 3) world
    poses_init: np.ndarray      # (N, 3, 4)
    points_init: np.ndarray     # (M, 3)
    obs_pose: np.ndarray        # (n_obs,) int32
    obs_point: np.ndarray       # (n_obs,) int32
    obs_cam: np.ndarray         # (n_obs,) int32
    obs_uv: np.ndarray          # (n_obs, 2) pixels (noisy)
    obs_w: np.ndarray           # (n_obs,) observation weights
    outlier: np.ndarray         # (n_obs,) bool, True where the pixel was replaced
    pose_fixed: np.ndarray      # (N,) uint8
    max_iters: int = 10
    huber_delta: float = 1.0
    lambda_init: float = 1e-3
    mixed: bool = False
    name: str = ""

    @property
    def n_poses(self) -> int:
        return int(self.poses_gt.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.points_gt.shape[0])

    @property
    def n_cams(self) -> int:
        return int(self.intrinsics.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_pose.shape[0])

    def copy(self) -> "Window":
        return dataclasses.replace(self, **{f.name: (getattr(self, f.name).copy()
                                                    if isinstance(getattr(self, f.name), np.ndarray)
                                                    else getattr(self, f.name))
                                           for f in dataclasses.fields(self)})


# ---------------------------------------------------------------------------
# generator-local geometry (independent of the solver and of the oracle)
# ---------------------------------------------------------------------------

def _rot_axis(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rotation about a unit axis (Rodrigues' formula, generator-local)."""
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def _rot_y(angle: float) -> np.ndarray:
    c, s = math.cos(angle), math.sin(angle)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def _pose_from_cam_to_world(R_wc: np.ndarray, centre: np.ndarray) -> np.ndarray:
    R = R_wc.T
    t = -R @ centre
    return np.concatenate([R, t[:, None]], axis=1)


def _to_cam(pose: np.ndarray, ext: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """World points (..., 3) to camera coordinates through base pose and extrinsic."""
    xb = pts @ pose[:, :3].T + pose[:, 3]
    return xb @ ext[:, :3].T + ext[:, 3]


def _project(K: np.ndarray, xc: np.ndarray) -> np.ndarray:
    z = xc[..., 2]
    return np.stack([K[0] * xc[..., 0] / z + K[2], K[1] * xc[..., 1] / z + K[3]], axis=-1)


def _visible(K, size, xc, min_z=0.1):
    uv = _project(K, np.where(xc[..., 2:3] > min_z, xc, 1.0))
    return ((xc[..., 2] > min_z) & (uv[..., 0] >= 0) & (uv[..., 0] < size[0])
            & (uv[..., 1] >= 0) & (uv[..., 1] < size[1]))


def _random_unit(rng, n=None):
    v = rng.normal(size=(3,) if n is None else (n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _perturb_poses(rng, poses, fixed, rot=0.05, trans=0.05):
    """Rotate each free pose by `rot` rad about a random axis and shift its
    translation by `trans` m along a random direction."""
    out = poses.copy()
    for i in range(poses.shape[0]):
        if fixed[i]:
            continue
        Rd = _rot_axis(_random_unit(rng), rot)
        out[i, :, :3] = Rd @ poses[i, :, :3]
        out[i, :, 3] = Rd @ poses[i, :, 3] + trans * _random_unit(rng)
    return out


def _assemble(rng, *, intr, ext, size, poses, points, tracks, sigma, outlier_frac,
              fixed, max_iters, mixed, name, point_sigma=0.1, pose_rot=0.05,
              pose_trans=0.05) -> Window:
    """tracks: list of (point index, pose index, cam index) int arrays."""
    op, oj, ok = (np.asarray(a, np.int32) for a in tracks)
    uv = np.empty((op.shape[0], 2))
    for k in range(intr.shape[0]):
        for i in range(poses.shape[0]):
            m = (ok == k) & (op == i)
            if m.any():
                uv[m] = _project(intr[k], _to_cam(poses[i], ext[k], points[oj[m]]))
    uv += rng.normal(scale=sigma, size=uv.shape)
    outl = np.zeros(op.shape[0], bool)
    if outlier_frac > 0:
        outl = rng.random(op.shape[0]) < outlier_frac
        w = size[ok[outl], 0]
        h = size[ok[outl], 1]
        uv[outl, 0] = rng.random(outl.sum()) * w
        uv[outl, 1] = rng.random(outl.sum()) * h
    order = rng.permutation(op.shape[0])
    fixed_arr = np.zeros(poses.shape[0], np.uint8)
    fixed_arr[list(fixed)] = 1
    return Window(
        intrinsics=np.asarray(intr, float), extrinsics=np.asarray(ext, float),
        image_size=np.asarray(size, float), poses_gt=poses, points_gt=points,
        poses_init=_perturb_poses(rng, poses, fixed_arr, pose_rot, pose_trans),
        points_init=points + rng.normal(scale=point_sigma, size=points.shape),
        obs_pose=op[order], obs_point=oj[order], obs_cam=ok[order], obs_uv=uv[order],
        obs_w=np.ones(op.shape[0]), outlier=outl[order], pose_fixed=fixed_arr,
        max_iters=max_iters, mixed=mixed, name=name)


# ---------------------------------------------------------------------------
# mono windows (workloads 1, 3, 5)
# ---------------------------------------------------------------------------

_MONO_K = np.array([458.0, 458.0, 367.0, 248.0])
_MONO_SIZE = np.array([752.0, 480.0])


def _mono_window(rng, n_kf, n_lm, *, track, x_hi, min_vis, fixed, max_iters, mixed,
                 name, sigma=0.5) -> Window:
    """Keyframes 0.5 m apart along x with U(-5, 5) deg yaw; landmarks uniform in the
    box x in [-4, x_hi], y in [-3, 3], z in [2, 20] m.

    track: ("subset", lo, hi) -> random subset of U{lo..min(hi, #visible)} visible
           frames; ("all",) -> every visible frame.
    """
    yaw = rng.uniform(-5.0, 5.0, n_kf) * math.pi / 180.0
    poses = np.stack([_pose_from_cam_to_world(_rot_y(yaw[i]), np.array([0.5 * i, 0.0, 0.0]))
                      for i in range(n_kf)])
    ext = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)[None]
    intr, size = _MONO_K[None], _MONO_SIZE[None]
    pts, trk_p, trk_j = [], [], []
    n_have = 0
    while n_have < n_lm:
        n_c = max(256, 2 * (n_lm - n_have))
        cand = np.stack([rng.uniform(-4.0, x_hi, n_c), rng.uniform(-3.0, 3.0, n_c),
                         rng.uniform(2.0, 20.0, n_c)], axis=1)
        vis = np.stack([_visible(intr[0], size[0], _to_cam(poses[i], ext[0], cand))
                        for i in range(n_kf)], axis=1)                     # (n_c, K)
        nvis = vis.sum(1)
        keep = np.nonzero(nvis >= min_vis)[0][: n_lm - n_have]
        for c in keep:
            frames = np.nonzero(vis[c])[0]
            if track[0] == "subset":
                L = int(rng.integers(track[1], min(track[2], frames.size) + 1))
                frames = np.sort(rng.choice(frames, size=L, replace=False))
            j = n_have
            pts.append(cand[c])
            trk_p.append(frames)
            trk_j.append(np.full(frames.size, j))
            n_have += 1
    points = np.asarray(pts)
    op = np.concatenate(trk_p)
    oj = np.concatenate(trk_j)
    ok = np.zeros_like(op)
    return _assemble(rng, intr=intr, ext=ext, size=size, poses=poses, points=points,
                     tracks=(op, oj, ok), sigma=sigma, outlier_frac=0.0, fixed=fixed,
                     max_iters=max_iters, mixed=mixed, name=name)


def _workload1(rng, w):
    return _mono_window(rng, 5, 200, track=("subset", 3, 5), x_hi=6.0, min_vis=3,
                        fixed=[0], max_iters=10, mixed=False, name=f"{WORKLOAD_NAMES[1]}")


def _workload3(rng, w):
    n_kf = int(rng.integers(5, 31))
    n_lm = int(rng.integers(500, 8001))
    return _mono_window(rng, n_kf, n_lm, track=("subset", 2, 10),
                        x_hi=0.5 * (n_kf - 1) + 4.0, min_vis=2, fixed=[0], max_iters=15,
                        mixed=True, name=f"{WORKLOAD_NAMES[3]}[{w}]")


def _workload5(rng, w):
    return _mono_window(rng, 10, 2000, track=("all",), x_hi=8.5, min_vis=3, fixed=[0, 1],
                        max_iters=50, mixed=True, name=f"{WORKLOAD_NAMES[5]}[{w}]")


# ---------------------------------------------------------------------------
# stereo window (workload 2)
# ---------------------------------------------------------------------------

def _workload2(rng, w, n_kf=20, n_lm=5000, geom_p=0.14):
    K = np.array([718.0, 718.0, 607.0, 185.0])
    size = np.array([1241.0, 376.0])
    intr = np.stack([K, K])
    sizes = np.stack([size, size])
    ext = np.zeros((2, 3, 4))
    ext[0, :, :3] = np.eye(3)
    ext[1, :, :3] = np.eye(3)
    ext[1, :, 3] = [-0.54, 0.0, 0.0]
    yaw = np.zeros(n_kf)
    centres = np.zeros((n_kf, 3))
    for i in range(1, n_kf):
        yaw[i] = yaw[i - 1] + rng.uniform(-1.0, 1.0) * math.pi / 180.0
        centres[i] = centres[i - 1] + _rot_y(yaw[i - 1]) @ np.array([0.0, 0.0, 1.0])
    poses = np.stack([_pose_from_cam_to_world(_rot_y(yaw[i]), centres[i]) for i in range(n_kf)])
    pts, op, oj, ok = [], [], [], []
    while len(pts) < n_lm:
        # track length 2 + Geom(p) (failures before the first success), at most 15
        # frames; the anchor pixel and log-uniform depth are drawn in the track's
        # last frame e, and the track runs back from e while both views see it.
        L_want = min(2 + int(rng.geometric(geom_p)) - 1, 15, n_kf)
        e = int(rng.integers(1, n_kf))
        u = rng.uniform(0, size[0])
        v = rng.uniform(0, size[1])
        depth = math.exp(rng.uniform(math.log(3.0), math.log(60.0)))
        xc = np.array([(u - K[2]) / K[0] * depth, (v - K[3]) / K[1] * depth, depth])
        R = poses[e, :, :3]
        p = R.T @ (xc - poses[e, :, 3])
        L = 0
        while L < L_want and e - L >= 0 and all(
                _visible(K, size, _to_cam(poses[e - L], ext[k], p[None]))[0] for k in range(2)):
            L += 1
        if L < 2:
            continue
        j = len(pts)
        pts.append(p)
        for i in range(e - L + 1, e + 1):
            for k in range(2):
                op.append(i)
                oj.append(j)
                ok.append(k)
    return _assemble(rng, intr=intr, ext=ext, size=sizes, poses=poses, points=np.asarray(pts),
                     tracks=(op, oj, ok), sigma=0.7, outlier_frac=0.02, fixed=[0],
                     max_iters=10, mixed=True, name=WORKLOAD_NAMES[2])


# ---------------------------------------------------------------------------
# 32-camera rig (workload 4)
# ---------------------------------------------------------------------------

def _workload4(rng, w, n_cam=32, n_pose=10, n_lm=20000, target_obs=300_000):
    K = np.array([400.0, 400.0, 320.0, 240.0])
    size = np.array([640.0, 480.0])
    intr = np.tile(K, (n_cam, 1))
    sizes = np.tile(size, (n_cam, 1))
    ext = np.zeros((n_cam, 3, 4))
    for k in range(n_cam):
        z = _random_unit(rng)
        a = _random_unit(rng)
        x = np.cross(a, z)
        x /= np.linalg.norm(x)
        y = np.cross(z, x)
        roll = rng.uniform(0, 2 * math.pi)
        R_bc = np.stack([x, y, z], axis=1) @ _rot_axis(np.array([0.0, 0.0, 1.0]), roll)
        R_cb = R_bc.T
        ext[k, :, :3] = R_cb
        ext[k, :, 3] = -R_cb @ (0.3 * z)
    radius, step = 2.0, 0.4
    poses = []
    for i in range(n_pose):
        th = i * step / radius
        centre = np.array([radius * math.sin(th), 0.0, radius * math.cos(th)])
        fwd = np.array([math.cos(th), 0.0, -math.sin(th)])       # tangent
        down = np.array([0.0, 1.0, 0.0])
        right = np.cross(down, fwd)
        R_wb = np.stack([right, down, fwd], axis=1)
        poses.append(_pose_from_cam_to_world(R_wb, centre))
    poses = np.stack(poses)

    def sample(n):
        d = _random_unit(rng, n)
        r = rng.uniform(12.0, 15.0, n)
        p = d * r[:, None]
        vis = np.zeros((n, n_pose, n_cam), bool)
        for i in range(n_pose):
            for k in range(n_cam):
                vis[:, i, k] = _visible(K, size, _to_cam(poses[i], ext[k], p))
        return p, vis

    p0, v0 = sample(n_lm)
    q = min(1.0, target_obs / max(1, int(v0.sum())))
    pts, op, oj, ok = [], [], [], []
    p, vis = p0, v0
    while len(pts) < n_lm:
        keep = vis & (rng.random(vis.shape) < q)
        npose = keep.any(axis=2).sum(axis=1)
        good = np.nonzero(npose >= 2)[0][: n_lm - len(pts)]
        for c in good:
            j = len(pts)
            pts.append(p[c])
            ii, kk = np.nonzero(keep[c])
            op.extend(ii.tolist())
            ok.extend(kk.tolist())
            oj.extend([j] * ii.size)
        if len(pts) < n_lm:
            p, vis = sample(max(64, 2 * (n_lm - len(pts))))
    return _assemble(rng, intr=intr, ext=ext, size=sizes, poses=poses, points=np.asarray(pts),
                     tracks=(op, oj, ok), sigma=0.5, outlier_frac=0.0, fixed=[0],
                     max_iters=10, mixed=True, name=WORKLOAD_NAMES[4])


_MAKERS = {1: _workload1, 2: _workload2, 3: _workload3, 4: _workload4, 5: _workload5}
_COUNTS = {1: 1, 2: 1, 3: 256, 4: 1, 5: 64}


def make_window(cfg: int, index: int = 0, seed: Optional[int] = None) -> Window:
    """Window `index` of workload `cfg` (seed defaults to 1000*cfg + index)."""
    rng = np.random.default_rng(1000 * cfg + index if seed is None else seed)
    return _MAKERS[cfg](rng, index)


def make_workload(cfg: int, count: Optional[int] = None) -> List[Window]:
    n = _COUNTS[cfg] if count is None else count
    return [make_window(cfg, w) for w in range(n)]


def tiny_window(seed: int = 0, n_kf: int = 3, n_lm: int = 12, stereo: bool = False,
                noise: float = 0.5, fixed=(0,), outlier_frac: float = 0.0,
                max_iters: int = 10) -> Window:
    """A small window for brute-force checks: mono (or stereo, 0.3 m baseline)
    keyframes 0.5 m apart, landmarks in a 3-8 m box, every visible frame observed."""
    rng = np.random.default_rng(seed)
    yaw = rng.uniform(-5.0, 5.0, n_kf) * math.pi / 180.0
    poses = np.stack([_pose_from_cam_to_world(_rot_y(yaw[i]), np.array([0.5 * i, 0.0, 0.0]))
                      for i in range(n_kf)])
    n_cam = 2 if stereo else 1
    ext = np.zeros((n_cam, 3, 4))
    ext[:, :, :3] = np.eye(3)
    if stereo:
        ext[1, :, 3] = [-0.3, 0.0, 0.0]
    intr = np.tile(_MONO_K, (n_cam, 1))
    size = np.tile(_MONO_SIZE, (n_cam, 1))
    pts, op, oj, ok = [], [], [], []
    while len(pts) < n_lm:
        p = np.array([rng.uniform(-1.0, 0.5 * n_kf + 1.0), rng.uniform(-1.5, 1.5),
                      rng.uniform(3.0, 8.0)])
        views = [(i, k) for i in range(n_kf) for k in range(n_cam)
                 if _visible(intr[k], size[k], _to_cam(poses[i], ext[k], p[None]))[0]]
        if len({v[0] for v in views}) < 2:
            continue
        j = len(pts)
        pts.append(p)
        for i, k in views:
            op.append(i)
            oj.append(j)
            ok.append(k)
    return _assemble(rng, intr=intr, ext=ext, size=size, poses=poses, points=np.asarray(pts),
                     tracks=(op, oj, ok), sigma=noise, outlier_frac=outlier_frac,
                     fixed=list(fixed), max_iters=max_iters, mixed=False,
                     name=f"tiny-{n_kf}kf-{n_lm}lm{'-stereo' if stereo else ''}")


# ---------------------------------------------------------------------------
# motion-only frames (pose refinement against fixed landmarks)
# ---------------------------------------------------------------------------

PNP_WORKLOADS = {
    "pnp-4096x-stereo-300lm": dict(n_frames=4096, kind="stereo", n_lm=300),
    "pnp-512x-rig32-400lm": dict(n_frames=512, kind="rig", n_lm=400),
}


@dataclasses.dataclass
class PnPBatch:
    """Independent frames sharing one camera rig; each frame's observations are
    a contiguous range [frame_obs_begin[f], frame_obs_begin[f + 1])."""

    intrinsics: np.ndarray        # (C, 4)
    extrinsics: np.ndarray        # (C, 3, 4)
    image_size: np.ndarray        # (C, 2)
    points: np.ndarray            # (M, 3) fixed landmarks, world frame
    poses_gt: np.ndarray          # (F, 3, 4) base-from-world (or base-from-map)
    poses_init: np.ndarray        # (F, 3, 4)
    frame_obs_begin: np.ndarray   # (F + 1,) int32
    obs_point: np.ndarray         # (n,) int32
    obs_cam: np.ndarray           # (n,) int32
    obs_uv: np.ndarray            # (n, 2)
    obs_w: np.ndarray             # (n,)
    outlier: np.ndarray           # (n,) bool
    map_from_world: Optional[np.ndarray] = None   # (F, 3, 4) or None
    max_iters: int = 10
    huber_delta: float = 1.0
    lambda_init: float = 1e-3
    name: str = ""

    @property
    def n_frames(self) -> int:
        return int(self.poses_gt.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_point.shape[0])

    def frame_slice(self, f: int) -> slice:
        return slice(int(self.frame_obs_begin[f]), int(self.frame_obs_begin[f + 1]))


def _compose(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """3x4 transforms: A * B."""
    return np.concatenate([A[:, :3] @ B[:, :3], (A[:, :3] @ B[:, 3] + A[:, 3])[:, None]], axis=1)


def _inverse(A: np.ndarray) -> np.ndarray:
    R = A[:, :3].T
    return np.concatenate([R, (-R @ A[:, 3])[:, None]], axis=1)


def _stereo_rig():
    K = np.array([718.0, 718.0, 607.0, 185.0])
    size = np.array([1241.0, 376.0])
    ext = np.zeros((2, 3, 4))
    ext[:, :, :3] = np.eye(3)
    ext[1, :, 3] = [-0.54, 0.0, 0.0]
    return np.stack([K, K]), ext, np.stack([size, size])


def _ring_rig(rng, n_cam=32):
    """Cameras on a 0.3 m sphere facing outward with random roll (the rig of
    workload 4)."""
    K = np.array([400.0, 400.0, 320.0, 240.0])
    size = np.array([640.0, 480.0])
    ext = np.zeros((n_cam, 3, 4))
    for k in range(n_cam):
        z = _random_unit(rng)
        a = _random_unit(rng)
        x = np.cross(a, z)
        x /= np.linalg.norm(x)
        y = np.cross(z, x)
        R_bc = np.stack([x, y, z], axis=1) @ _rot_axis(np.array([0.0, 0.0, 1.0]), rng.uniform(0, 2 * math.pi))
        ext[k, :, :3] = R_bc.T
        ext[k, :, 3] = -R_bc.T @ (0.3 * z)
    return np.tile(K, (n_cam, 1)), ext, np.tile(size, (n_cam, 1))


def make_pnp_batch(n_frames: int, kind: str = "stereo", n_lm: int = 300, seed: int = 7000,
                   sigma: float = 0.7, outlier_frac: float = 0.02, map_frame: bool = False,
                   pose_rot: float = 0.02, pose_trans: float = 0.05, max_iters: int = 10,
                   name: str = "") -> PnPBatch:
    """Frames with random poses; each sees ``n_lm`` landmarks of its own.

    stereo: the KITTI-like pair; every landmark is seen by both cameras (anchor
    pixel uniform in the left image, depth log-uniform in 3-60 m).  rig: the
    32-camera sphere rig; landmarks in a 12-15 m shell, observed by every camera
    that sees them (at least one).  Pixel noise N(0, sigma^2), a fraction of
    observations replaced by uniform pixels, initial pose = ground truth rotated
    by ``pose_rot`` rad and shifted by ``pose_trans`` m.  With ``map_frame`` each
    frame gets a random T^mw and its ground truth is T^bm = T^bw (T^mw)^-1."""
    rng = np.random.default_rng(seed)
    if kind == "stereo":
        intr, ext, size = _stereo_rig()
    else:
        intr, ext, size = _ring_rig(rng)
    n_cam = intr.shape[0]
    pts_all, poses, begin, op, ok = [], [], [0], [], []
    for f in range(n_frames):
        yaw = rng.uniform(-math.pi, math.pi)
        R_wb = _rot_y(yaw) @ _rot_axis(_random_unit(rng), rng.uniform(0.0, 0.1))
        centre = rng.uniform(-50.0, 50.0, 3) * np.array([1.0, 0.1, 1.0])
        pose = _pose_from_cam_to_world(R_wb, centre)
        pts = np.zeros((0, 3))
        vis = np.zeros((0, n_cam), bool)
        while pts.shape[0] < n_lm:
            m = 2 * (n_lm - pts.shape[0]) + 16
            if kind == "stereo":
                K = intr[0]
                u = rng.uniform(0, size[0, 0], m)
                v = rng.uniform(0, size[0, 1], m)
                d = np.exp(rng.uniform(math.log(3.0), math.log(60.0), m))
                xc = np.stack([(u - K[2]) / K[0] * d, (v - K[3]) / K[1] * d, d], axis=1)
                cand = (xc - pose[:, 3]) @ pose[:, :3]
            else:
                cand = (_random_unit(rng, m) * rng.uniform(12.0, 15.0, m)[:, None] - pose[:, 3]) @ pose[:, :3]
            cv = np.stack([_visible(intr[k], size[k], _to_cam(pose, ext[k], cand)) for k in range(n_cam)],
                          axis=1)
            keep = cv.all(axis=1) if kind == "stereo" else cv.any(axis=1)
            pts = np.concatenate([pts, cand[keep]])[:n_lm]
            vis = np.concatenate([vis, cv[keep]])[:n_lm]
        obs = [(j, np.nonzero(vis[j])[0].tolist()) for j in range(n_lm)]
        pts = list(pts)
        base = len(pts_all)
        pts_all.extend(pts)
        for j, cams in obs:
            for k in cams:
                op.append(base + j)
                ok.append(k)
        begin.append(len(op))
        poses.append(pose)
    points = np.asarray(pts_all)
    poses = np.stack(poses)
    op = np.asarray(op, np.int32)
    ok = np.asarray(ok, np.int32)
    begin = np.asarray(begin, np.int32)
    uv = np.empty((op.shape[0], 2))
    for f in range(n_frames):
        sl = slice(begin[f], begin[f + 1])
        xb = points[op[sl]] @ poses[f, :, :3].T + poses[f, :, 3]
        xc = np.einsum("nab,nb->na", ext[ok[sl], :, :3], xb) + ext[ok[sl], :, 3]
        K = intr[ok[sl]]
        uv[sl] = np.stack([K[:, 0] * xc[:, 0] / xc[:, 2] + K[:, 2], K[:, 1] * xc[:, 1] / xc[:, 2] + K[:, 3]],
                          axis=1)
    uv += rng.normal(scale=sigma, size=uv.shape)
    outl = rng.random(op.shape[0]) < outlier_frac
    uv[outl, 0] = rng.random(int(outl.sum())) * size[ok[outl], 0]
    uv[outl, 1] = rng.random(int(outl.sum())) * size[ok[outl], 1]
    mfw = None
    gt = poses
    if map_frame:
        mfw = np.stack([_pose_from_cam_to_world(_rot_axis(_random_unit(rng), rng.uniform(0, 0.5)),
                                                rng.uniform(-5, 5, 3)) for _ in range(n_frames)])
        gt = np.stack([_compose(poses[f], _inverse(mfw[f])) for f in range(n_frames)])
    init = _perturb_poses(rng, gt, np.zeros(n_frames, np.uint8), pose_rot, pose_trans)
    # observations of each frame in a random order
    for f in range(n_frames):
        sl = slice(begin[f], begin[f + 1])
        order = begin[f] + rng.permutation(begin[f + 1] - begin[f])
        op[sl], ok[sl], uv[sl], outl[sl] = op[order], ok[order], uv[order], outl[order]
    return PnPBatch(intrinsics=intr, extrinsics=ext, image_size=size, points=points, poses_gt=gt,
                    poses_init=init, frame_obs_begin=begin, obs_point=op, obs_cam=ok, obs_uv=uv,
                    obs_w=np.ones(op.shape[0]), outlier=outl, map_from_world=mfw,
                    max_iters=max_iters, name=name or f"pnp-{n_frames}x-{kind}-{n_lm}lm")


def make_pnp_workload(name: str, seed: int = 7000) -> PnPBatch:
    return make_pnp_batch(seed=seed, name=name, **PNP_WORKLOADS[name])



# ---------------------------------------------------------------------------
# triangulation batches: the landmarks of windows, re-estimated from their
# observations with every pose held at its ground truth
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class TriBatch:
    """Landmarks with landmark-major (CSR) observations; poses fixed.  All
    windows share one rig (same intrinsics and extrinsics)."""

    intrinsics: np.ndarray        # (C, 4)
    extrinsics: np.ndarray        # (C, 3, 4)
    poses: np.ndarray             # (N, 3, 4) base-from-world (ground truth)
    points_gt: np.ndarray         # (M, 3)
    point_obs_begin: np.ndarray   # (M + 1,) int32
    obs_pose: np.ndarray          # (n,) int32
    obs_cam: np.ndarray           # (n,) int32
    obs_uv: np.ndarray            # (n, 2)
    obs_w: np.ndarray             # (n,)
    max_iters: int = 10
    huber_delta: float = 1.0
    lambda_init: float = 1e-3
    name: str = ""

    @property
    def n_points(self):
        return int(self.points_gt.shape[0])

    @property
    def n_obs(self):
        return int(self.obs_pose.shape[0])

    @property
    def n_poses(self):
        return int(self.poses.shape[0])

    def point_slice(self, j):
        return slice(int(self.point_obs_begin[j]), int(self.point_obs_begin[j + 1]))


def make_tri_batch(windows: List[Window], max_iters: int = 10, name: str = "") -> TriBatch:
    """Every landmark of the given windows (one rig), observations grouped by
    landmark in window order, poses at ground truth."""
    K, E = windows[0].intrinsics, windows[0].extrinsics
    for w in windows:
        if not (np.array_equal(w.intrinsics, K) and np.array_equal(w.extrinsics, E)):
            raise ValueError("windows of a triangulation batch share one rig")
    poses, pts, begin, op, oc, uv, ow = [], [], [0], [], [], [], []
    pose_base = 0
    for w in windows:
        order = np.argsort(w.obs_point, kind="stable")
        counts = np.bincount(w.obs_point, minlength=w.points_gt.shape[0])
        op.append(w.obs_pose[order] + pose_base)
        oc.append(w.obs_cam[order])
        uv.append(w.obs_uv[order])
        ow.append(w.obs_w[order])
        begin.extend((begin[-1] + np.cumsum(counts)).tolist())
        poses.append(w.poses_gt)
        pts.append(w.points_gt)
        pose_base += w.poses_gt.shape[0]
    return TriBatch(intrinsics=K, extrinsics=E, poses=np.concatenate(poses), points_gt=np.concatenate(pts),
                    point_obs_begin=np.asarray(begin, np.int32),
                    obs_pose=np.concatenate(op).astype(np.int32), obs_cam=np.concatenate(oc).astype(np.int32),
                    obs_uv=np.concatenate(uv), obs_w=np.concatenate(ow), max_iters=max_iters,
                    huber_delta=windows[0].huber_delta, lambda_init=windows[0].lambda_init, name=name)


# ---------------------------------------------------------------------------
# pose graphs: a helical multi-lap trajectory with odometry and loop-closure
# edges
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PoseGraphData:
    poses_gt: np.ndarray      # (N, 3, 4) world-from-base
    poses_init: np.ndarray    # (N, 3, 4) dead reckoning from the noisy odometry
    edge_i: np.ndarray        # (E,) int32
    edge_j: np.ndarray        # (E,) int32
    deltas: np.ndarray        # (E, 3, 4) measured T_i^-1 T_j
    edge_w: np.ndarray        # (E,)
    pose_fixed: np.ndarray    # (N,) uint8
    loop: np.ndarray          # (E,) bool, True for loop-closure edges
    max_iters: int = 10
    lambda_init: float = 1e-3
    name: str = ""

    @property
    def n_poses(self):
        return int(self.poses_gt.shape[0])

    @property
    def n_edges(self):
        return int(self.edge_i.shape[0])


def _se3_exp_small(xi):
    """Exp of (rho, phi) (generator only; uses the rotation-vector formula)."""
    phi = np.asarray(xi[3:], float)
    th = float(np.linalg.norm(phi))
    K = np.array([[0.0, -phi[2], phi[1]], [phi[2], 0.0, -phi[0]], [-phi[1], phi[0], 0.0]])
    if th < 1e-8:
        R, V = np.eye(3) + K, np.eye(3) + 0.5 * K
    else:
        R = np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K
        V = np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * K @ K
    return np.concatenate([R, (V @ np.asarray(xi[:3], float))[:, None]], axis=1)


def make_pose_graph(laps: int = 3, per_lap: int = 500, radius: float = 10.0, rise: float = 0.5,
                    sigma_rot: float = 0.002, sigma_trans: float = 0.01, loop_prob: float = 0.5,
                    seed: int = 9000, max_iters: int = 10, name: str = "") -> PoseGraphData:
    """A helix of ``laps`` turns (radius ``radius`` m, ``rise`` m per turn) with
    ``per_lap`` keyframes per turn, heading along the track.  Odometry edges join
    consecutive keyframes; each keyframe after the first turn gets loop
    closures to the keyframes at the same place one turn earlier (offsets -1, 0,
    +1, each kept with probability ``loop_prob``).  Every measured delta is the
    true one times Exp of N(0, sigma^2) noise (per component, rotation and
    translation); the initial poses are dead reckoning from pose 0 along the
    noisy odometry.  Pose 0 is fixed."""
    rng = np.random.default_rng(seed)
    n = laps * per_lap
    gt = np.zeros((n, 3, 4))
    for k in range(n):
        a = 2 * math.pi * k / per_lap
        c = np.array([radius * math.cos(a), rise * k / per_lap, radius * math.sin(a)])
        # base x along the track, y up
        fwd = np.array([-math.sin(a), 0.0, math.cos(a)])
        up = np.array([0.0, 1.0, 0.0])
        side = np.cross(fwd, up)
        R = np.stack([fwd, up, side], axis=1)
        gt[k, :, :3] = R
        gt[k, :, 3] = c
    inv = lambda T: np.concatenate([T[:, :3].T, (-T[:, :3].T @ T[:, 3])[:, None]], axis=1)
    comp = lambda A, B: np.concatenate([A[:, :3] @ B[:, :3], (A[:, :3] @ B[:, 3] + A[:, 3])[:, None]], axis=1)

    def measure(i, j):
        D = comp(inv(gt[i]), gt[j])
        xi = np.concatenate([rng.normal(0, sigma_trans, 3), rng.normal(0, sigma_rot, 3)])
        return comp(_se3_exp_small(xi), D)

    ei, ej, ds, lp = [], [], [], []
    for k in range(n - 1):
        ei.append(k)
        ej.append(k + 1)
        ds.append(measure(k, k + 1))
        lp.append(False)
    for k in range(per_lap, n):
        for off in (-1, 0, 1):
            j0 = k - per_lap + off
            if 0 <= j0 < k - 1 and rng.uniform() < loop_prob:
                ei.append(j0)
                ej.append(k)
                ds.append(measure(j0, k))
                lp.append(True)
    init = np.zeros_like(gt)
    init[0] = gt[0]
    for k in range(n - 1):
        init[k + 1] = comp(init[k], ds[k])
    fixed = np.zeros(n, np.uint8)
    fixed[0] = 1
    return PoseGraphData(poses_gt=gt, poses_init=init, edge_i=np.asarray(ei, np.int32),
                         edge_j=np.asarray(ej, np.int32), deltas=np.asarray(ds), edge_w=np.ones(len(ei)),
                         pose_fixed=fixed, loop=np.asarray(lp), max_iters=max_iters, name=name)


PGO_WORKLOADS = {
    "pgo-helix-3x500": dict(laps=3, per_lap=500),
}


def make_pgo_workload(name: str, seed: int = 9000) -> PoseGraphData:
    return make_pose_graph(seed=seed, name=name, **PGO_WORKLOADS[name])


# ---------------------------------------------------------------------------
# visual-inertial windows: a mono camera on a base that carries the IMU
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class ViWindow:
    """A mono window plus IMU samples between consecutive keyframes.

    The ground-truth motion is integrated from piecewise-constant body rates and
    specific forces (one value per sample interval), so the samples are exactly
    consistent with the discrete motion: R <- R Exp(w dt) (world-from-base),
    v <- v + (g + R f) dt, p <- p + v dt + (g + R f) dt^2 / 2."""
    window: Window
    gravity: np.ndarray         # (3,) world frame, m / s^2 (y down)
    dt: float                   # IMU sample interval, s
    gyro: List[np.ndarray]      # per keyframe interval: (n, 3) measured rates
    accel: List[np.ndarray]     # per keyframe interval: (n, 3) measured specific forces
    vel_gt: np.ndarray          # (N, 3) world-frame velocity at each keyframe
    ba_gt: np.ndarray           # (3,) constant accelerometer bias
    bg_gt: np.ndarray           # (3,) constant gyro bias
    vel_init: np.ndarray        # (N, 3)
    ba_init: np.ndarray         # (N, 3)
    bg_init: np.ndarray         # (N, 3)
    noise: Tuple[float, float, float, float]   # sigma_g, sigma_a, sigma_bg, sigma_ba (densities)


def _exp_so3_gen(phi):
    th = float(np.linalg.norm(phi))
    if th < 1e-12:
        return np.eye(3)
    return _rot_axis(phi / th, th)


def make_vi_window(seed: int = 9000, n_kf: int = 10, n_lm: int = 400, kf_dt: float = 0.25,
                   rate: float = 200.0, sigma_px: float = 0.5, imu_noise: bool = True,
                   init_noise: bool = True, max_iters: int = 15) -> ViWindow:
    """A camera moving forward (+z, about 1 m/s) with smooth rotation and
    acceleration; keyframes every kf_dt s, IMU at `rate` Hz; landmarks in a box
    ahead seen in >= min(3, n_kf) keyframes (tracks of up to 6 visible
    keyframes).  Biases
    are constant; the state estimates start at zero bias, perturbed velocity,
    pose and points (pose 0 fixed at its ground truth)."""
    rng = np.random.default_rng(seed)
    g = np.array([0.0, 9.81, 0.0])
    dt = 1.0 / rate
    n_per = int(round(kf_dt * rate))
    noise = (1.7e-4, 2.0e-3, 2.0e-5, 3.0e-3)
    ba = rng.normal(scale=0.05, size=3)
    bg = rng.normal(scale=0.01, size=3)
    ph = rng.uniform(0, 2 * math.pi, 6)
    Rw = _rot_y(rng.uniform(-0.1, 0.1))        # world-from-base at t = 0
    p = np.zeros(3)
    v = np.array([0.1, 0.0, 1.0])
    poses, vels, gyros, accels = [], [], [], []
    t = 0.0
    for i in range(n_kf):
        poses.append(np.concatenate([Rw.T, (-Rw.T @ p)[:, None]], axis=1))
        vels.append(v.copy())
        if i == n_kf - 1:
            break
        gy, ac = [], []
        for _ in range(n_per):
            w = np.array([0.15 * math.sin(0.9 * t + ph[0]), 0.3 * math.sin(0.6 * t + ph[1]),
                          0.1 * math.sin(1.1 * t + ph[2])])
            aw = np.array([0.4 * math.sin(0.8 * t + ph[3]), 0.2 * math.sin(0.7 * t + ph[4]),
                           0.3 * math.sin(0.5 * t + ph[5])])
            f = Rw.T @ (aw - g)                   # specific force in the base frame
            acc = g + Rw @ f
            p = p + v * dt + 0.5 * acc * dt * dt
            v = v + acc * dt
            Rw = Rw @ _exp_so3_gen(w * dt)
            gy.append(w + bg)
            ac.append(f + ba)
            t += dt
        gy, ac = np.asarray(gy), np.asarray(ac)
        if imu_noise:
            gy = gy + rng.normal(scale=noise[0] / math.sqrt(dt), size=gy.shape)
            ac = ac + rng.normal(scale=noise[1] / math.sqrt(dt), size=ac.shape)
        gyros.append(gy)
        accels.append(ac)
    poses = np.stack(poses)
    ext = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)[None]
    intr, size = _MONO_K[None], _MONO_SIZE[None]
    z_end = float(-(poses[-1, :, :3].T @ poses[-1, :, 3])[2])
    pts, trk_p, trk_j = [], [], []
    min_vis = min(3, n_kf)
    for _ in range(1000):
        if len(pts) >= n_lm:
            break
        n_c = 4 * (n_lm - len(pts)) + 64
        cand = np.stack([rng.uniform(-5.0, 5.0, n_c), rng.uniform(-3.0, 3.0, n_c),
                         rng.uniform(z_end + 3.0, z_end + 20.0, n_c)], axis=1)
        vis = np.stack([_visible(intr[0], size[0], _to_cam(poses[i], ext[0], cand)) for i in range(n_kf)], axis=1)
        for c in np.nonzero(vis.sum(1) >= min_vis)[0]:
            if len(pts) >= n_lm:
                break
            frames = np.nonzero(vis[c])[0]
            L = int(rng.integers(min_vis, min(6, frames.size) + 1))
            frames = np.sort(rng.choice(frames, size=L, replace=False))
            trk_p.append(frames)
            trk_j.append(np.full(frames.size, len(pts)))
            pts.append(cand[c])
    if len(pts) < n_lm:
        raise ValueError("could not place the landmarks in view")
    points = np.asarray(pts)
    op, oj = np.concatenate(trk_p), np.concatenate(trk_j)
    w = _assemble(rng, intr=intr, ext=ext, size=size, poses=poses, points=points,
                  tracks=(op, oj, np.zeros_like(op)), sigma=sigma_px, outlier_frac=0.0, fixed=[0],
                  max_iters=max_iters, mixed=False, name=f"vi-mono-{n_kf}kf-{n_lm}lm",
                  point_sigma=0.1 if init_noise else 0.0, pose_rot=0.03 if init_noise else 0.0,
                  pose_trans=0.03 if init_noise else 0.0)
    vels = np.stack(vels)
    vel_init = vels + (rng.normal(scale=0.05, size=vels.shape) if init_noise else 0.0)
    return ViWindow(window=w, gravity=g, dt=dt, gyro=gyros, accel=accels, vel_gt=vels, ba_gt=ba, bg_gt=bg,
                    vel_init=vel_init, ba_init=np.zeros((n_kf, 3)), bg_init=np.zeros((n_kf, 3)), noise=noise)


# ---------------------------------------------------------------------------
# keyframe sequences for the sliding-window local map
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Keyframe:
    """What the frontend hands the local map at one keyframe: the pose estimate,
    the landmarks created there (ids and triangulated positions) and the
    keyframe's observations (all in the newest keyframe of the window)."""
    pose_gt: np.ndarray         # (3, 4) base-from-world
    pose_init: np.ndarray       # (3, 4) the frontend's estimate
    new_ids: np.ndarray         # (n_new,) int64
    new_points: np.ndarray      # (n_new, 3) triangulated estimates
    obs_lm: np.ndarray          # (n_obs,) int64 landmark ids
    obs_cam: np.ndarray         # (n_obs,) int32
    obs_uv: np.ndarray          # (n_obs, 2) pixels


@dataclasses.dataclass
class Sequence:
    intrinsics: np.ndarray      # (2, 4)
    extrinsics: np.ndarray      # (2, 3, 4)
    points_gt: Dict[int, np.ndarray]
    keyframes: List[Keyframe]


def make_stereo_sequence(n_keyframes: int = 40, births: int = 250, seed: int = 11000,
                         geom_p: float = 0.14, sigma_px: float = 0.7) -> Sequence:
    """The stereo rig of the stereo window (1241x376, f = 718, 0.54 m baseline)
    driving 1 m per keyframe with a small random yaw.  At each keyframe about
    `births` landmarks are created (depth log-uniform in [3, 60] m along a
    random pixel of the left image) and tracked forward for 2 + Geom(p) - 1
    keyframes, at most 15, while both cameras see them; every keyframe observes
    each of its live landmarks in both cameras (pixel noise sigma_px).  The
    pose estimate is the truth perturbed by 0.01 rad / 0.05 m (pose 0 exact),
    a new landmark's estimate the truth plus N(0, (0.02 depth)^2) per axis."""
    rng = np.random.default_rng(seed)
    K = np.array([718.0, 718.0, 607.0, 185.0])
    size = np.array([1241.0, 376.0])
    ext = np.zeros((2, 3, 4))
    ext[0, :, :3] = np.eye(3)
    ext[1, :, :3] = np.eye(3)
    ext[1, :, 3] = [-0.54, 0.0, 0.0]
    yaw, c = 0.0, np.zeros(3)
    poses = []
    for i in range(n_keyframes):
        poses.append(_pose_from_cam_to_world(_rot_y(yaw), c.copy()))
        c = c + _rot_y(yaw) @ np.array([0.0, 0.0, 1.0])
        yaw += rng.uniform(-1.0, 1.0) * math.pi / 180.0
    pts: Dict[int, np.ndarray] = {}
    live: Dict[int, int] = {}   # id -> last keyframe of its track
    kfs = []
    next_id = 0
    for i in range(n_keyframes):
        new_ids, new_pts = [], []
        for _ in range(births):
            for _try in range(50):
                u, v = rng.uniform(0, size[0]), rng.uniform(0, size[1])
                depth = math.exp(rng.uniform(math.log(3.0), math.log(60.0)))
                xc = np.array([(u - K[2]) / K[0] * depth, (v - K[3]) / K[1] * depth, depth])
                p = poses[i][:, :3].T @ (xc - poses[i][:, 3])
                if _visible(K, size, _to_cam(poses[i], ext[1], p[None]))[0]:
                    break
            else:
                continue
            L = min(2 + int(rng.geometric(geom_p)) - 1, 15)
            lid = next_id
            next_id += 1
            pts[lid] = p
            live[lid] = i + L - 1
            new_ids.append(lid)
            new_pts.append(p + rng.normal(scale=0.02 * depth, size=3))
        o_lm, o_cam, o_uv = [], [], []
        for lid in list(live):
            if live[lid] < i:
                del live[lid]
                continue
            p = pts[lid]
            vis = [_visible(K, size, _to_cam(poses[i], ext[k], p[None]))[0] for k in range(2)]
            if not all(vis):
                if lid in new_ids:   # cannot happen for a fresh landmark: both checked
                    raise AssertionError("new landmark not in view")
                del live[lid]
                continue
            for k in range(2):
                o_lm.append(lid)
                o_cam.append(k)
                o_uv.append(_project(K, _to_cam(poses[i], ext[k], p[None]))[0])
        o_uv = np.asarray(o_uv).reshape(-1, 2) + rng.normal(scale=sigma_px, size=(len(o_lm), 2))
        P = poses[i]
        if i == 0:
            Pi = P.copy()
        else:
            Rd = _rot_axis(_random_unit(rng), 0.01)
            Pi = np.concatenate([Rd @ P[:, :3], (Rd @ P[:, 3] + 0.05 * _random_unit(rng))[:, None]], axis=1)
        kfs.append(Keyframe(pose_gt=P, pose_init=Pi, new_ids=np.asarray(new_ids, np.int64),
                            new_points=np.asarray(new_pts).reshape(-1, 3),
                            obs_lm=np.asarray(o_lm, np.int64), obs_cam=np.asarray(o_cam, np.int32),
                            obs_uv=o_uv))
    return Sequence(intrinsics=np.stack([K, K]), extrinsics=ext, points_gt=pts, keyframes=kfs)
