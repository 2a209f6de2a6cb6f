"""Sliding-window local map (test infrastructure; plain Python lists).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper Sec. 2.1: the frontend keeps a local odometry map of the last N
keyframe poses with the landmarks visible from them and their observations;
Sec. 2.2: when a keyframe is created, landmarks triangulated from its
multi-view observations enter the map with those observations, and the
sparse bundle adjustment refines the map.  The paper gives no rules for
leaving the window; the readings taken here:

  * the map holds at most N keyframes; inserting one into a full map first
    drops the oldest keyframe with all its observations, then every landmark
    left with fewer than two distinct (keyframe, camera) views, with its
    remaining observations (no marginalisation: dropped information is gone);
  * an insertion brings the keyframe's pose estimate, the landmarks created at
    it (new ids with their triangulated positions) and observations, each
    naming a keyframe of the window after the insertion (so a new landmark
    may also be observed in earlier keyframes) and a landmark of the map
    after the drop or a new one;
  * an insertion is checked before anything changes: unknown or duplicate
    ids, indices out of range, or a new landmark with fewer than two distinct
    views leave the map untouched and raise ValueError;
  * the window handed to the solver: keyframes oldest first, the oldest held
    fixed; landmarks in order of creation; observations in order of
    insertion (those of one insertion in the order given).
"""
import dataclasses
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class _Obs:
    kf: int          # keyframe serial number
    lm: int          # landmark id
    cam: int
    uv: np.ndarray   # (2,)
    w: float


class WindowMap:
    def __init__(self, max_keyframes: int, n_cams: int):
        if max_keyframes < 2:
            raise ValueError("a window needs at least two keyframes")
        self.N = max_keyframes
        self.n_cams = n_cams
        self.kf_serial: List[int] = []          # serials of the window's keyframes, oldest first
        self.kf_pose: Dict[int, np.ndarray] = {}
        self.lm_order: List[int] = []           # landmark ids in order of creation
        self.lm_point: Dict[int, np.ndarray] = {}
        self.obs: List[_Obs] = []               # in order of insertion
        self.next_serial = 0

    # ---- queries
    def n_keyframes(self):
        return len(self.kf_serial)

    # ---- insertion
    def add_keyframe(self, pose, new_ids=(), new_points=None, obs_kf=(), obs_lm=(), obs_cam=None,
                     obs_uv=None, obs_w=None):
        """Insert a keyframe; returns the ids of the landmarks dropped by the slide."""
        new_ids = [int(x) for x in new_ids]
        new_points = np.zeros((0, 3)) if new_points is None else np.asarray(new_points, float).reshape(-1, 3)
        obs_kf = [int(x) for x in obs_kf]
        obs_lm = [int(x) for x in obs_lm]
        n = len(obs_kf)
        obs_cam = [0] * n if obs_cam is None else [int(x) for x in obs_cam]
        obs_uv = np.zeros((0, 2)) if obs_uv is None else np.asarray(obs_uv, float).reshape(-1, 2)
        obs_w = [1.0] * n if obs_w is None else [float(x) for x in obs_w]
        if len(obs_lm) != n or len(obs_cam) != n or obs_uv.shape[0] != n or len(obs_w) != n:
            raise ValueError("observation arrays differ in length")
        if len(new_ids) != new_points.shape[0]:
            raise ValueError("new landmark arrays differ in length")
        # the slide, computed on copies
        serials = list(self.kf_serial)
        obs = list(self.obs)
        order = list(self.lm_order)
        dropped = []
        if len(serials) == self.N:
            old = serials.pop(0)
            obs = [o for o in obs if o.kf != old]
            views = {}
            for o in obs:
                views.setdefault(o.lm, set()).add((o.kf, o.cam))
            keep = []
            for lm in order:
                if len(views.get(lm, ())) >= 2:
                    keep.append(lm)
                else:
                    dropped.append(lm)
            dset = set(dropped)
            obs = [o for o in obs if o.lm not in dset]
            order = keep
        serial = self.next_serial
        serials.append(serial)
        # checks
        have = set(order)
        if len(set(new_ids)) != len(new_ids) or any(i in have for i in new_ids):
            raise ValueError("new landmark id repeated or already in the map")
        known = have | set(new_ids)
        for k in range(n):
            if not 0 <= obs_kf[k] < len(serials):
                raise ValueError(f"observation {k}: keyframe index out of range")
            if obs_lm[k] not in known:
                raise ValueError(f"observation {k}: landmark {obs_lm[k]} not in the map")
            if not 0 <= obs_cam[k] < self.n_cams:
                raise ValueError(f"observation {k}: camera out of range")
        added = [_Obs(serials[obs_kf[k]], obs_lm[k], obs_cam[k], obs_uv[k].copy(), obs_w[k]) for k in range(n)]
        new_views = {i: set() for i in new_ids}
        for o in added:
            if o.lm in new_views:
                new_views[o.lm].add((o.kf, o.cam))
        for i in new_ids:
            if len(new_views[i]) < 2:
                raise ValueError(f"new landmark {i} has fewer than two distinct views")
        # apply
        if len(self.kf_serial) == self.N:
            del self.kf_pose[self.kf_serial[0]]
            for lm in dropped:
                del self.lm_point[lm]
        self.kf_serial = serials
        self.kf_pose[serial] = np.asarray(pose, float).reshape(3, 4).copy()
        self.next_serial += 1
        for i, p in zip(new_ids, new_points):
            self.lm_point[i] = p.copy()
        self.lm_order = order + new_ids
        self.obs = obs + added
        return dropped

    # ---- the window
    def window(self):
        """dict of the solver's window: poses (K, 3, 4), points (M, 3),
        landmark_ids (M,), obs_pose / obs_point / obs_cam (n,), obs_uv (n, 2),
        obs_w (n,), pose_fixed (K,)."""
        kpos = {s: i for i, s in enumerate(self.kf_serial)}
        lpos = {l: j for j, l in enumerate(self.lm_order)}
        K = len(self.kf_serial)
        fixed = np.zeros(K, np.uint8)
        if K:
            fixed[0] = 1
        return dict(
            poses=np.stack([self.kf_pose[s] for s in self.kf_serial]) if K else np.zeros((0, 3, 4)),
            points=np.stack([self.lm_point[l] for l in self.lm_order]) if self.lm_order else np.zeros((0, 3)),
            landmark_ids=np.array(self.lm_order, np.int64),
            obs_pose=np.array([kpos[o.kf] for o in self.obs], np.int32),
            obs_point=np.array([lpos[o.lm] for o in self.obs], np.int32),
            obs_cam=np.array([o.cam for o in self.obs], np.int32),
            obs_uv=np.array([o.uv for o in self.obs]).reshape(-1, 2),
            obs_w=np.array([o.w for o in self.obs], float),
            pose_fixed=fixed)

    def set_state(self, poses, points):
        """Write refined poses (window order) and points (map order) back."""
        for s, P in zip(self.kf_serial, np.asarray(poses, float)):
            self.kf_pose[s] = P.copy()
        for l, p in zip(self.lm_order, np.asarray(points, float)):
            self.lm_point[l] = p.copy()
