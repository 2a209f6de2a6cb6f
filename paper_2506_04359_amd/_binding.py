"""ctypes binding of libba.so (argument marshalling only)."""
import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libba.so")

BA_FP64 = 0
BA_MIXED = 1
BA_CREATE_HOST_ONLY = 1
# ba_status
BA_OK = 0
BA_ERR_INVALID_ARG = -1
BA_ERR_OOM = -2
BA_ERR_HIP = -3
BA_ERR_WORKSPACE_TOO_SMALL = -4
BA_ERR_UNSUPPORTED = -5
BA_ERR_STATE = -6


# include/ba.h BA_VI_PREINT_DOUBLES
VI_PREINT_DOUBLES = 320
# include/ba.h BA_NOALLOC_SCRATCH_BYTES
NOALLOC_SCRATCH_BYTES = 64 << 20


class BAError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"ba status {status}: {message}")
        self.status = status


class _Settings(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("lambda_init", ctypes.c_double), ("lambda_up", ctypes.c_double),
                ("lambda_down", ctypes.c_double), ("lambda_min", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("huber_delta", ctypes.c_double),
                ("min_depth", ctypes.c_double), ("grad_tol", ctypes.c_double), ("step_tol", ctypes.c_double)]


class _LaunchConfig(ctypes.Structure):   # include/ba.h ba_launch_config
    _fields_ = [("chunk_obs", ctypes.c_int32), ("tile_pairs", ctypes.c_int32),
                ("class_chunk_mult", ctypes.c_int32 * 4), ("class_streams", ctypes.c_int32)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n_poses", ctypes.c_int32), ("n_points", ctypes.c_int32),
                ("n_cams", ctypes.c_int32), ("n_free", ctypes.c_int32),
                ("n_obs", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_tiles", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
                ("schur_blocks", ctypes.c_int64), ("n_free_pairs", ctypes.c_int64)]


REPORT_DTYPE = np.dtype([("initial_cost", "<f8"), ("final_cost", "<f8"), ("final_lambda", "<f8"),
                         ("iters", "<i4"), ("accepted", "<i4"), ("chol_failures", "<i4"),
                         ("depth_rejects", "<i4"), ("status", "<i4"), ("reserved", "<i4")])
TRACE_DTYPE = np.dtype([("cost", "<f8"), ("cand_cost", "<f8"), ("lambda", "<f8"),
                        ("accepted", "<i4"), ("status", "<i4")])
assert REPORT_DTYPE.itemsize == 48 and TRACE_DTYPE.itemsize == 32

_lib = None


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with "
                              "`python -m paper_2506_04359_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.ba_window_create.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp, vp, vp, i32,
                                       ctypes.POINTER(vp)]
        L.ba_window_destroy.argtypes = [vp]
        L.ba_window_info.argtypes = [vp, ctypes.POINTER(_PlanInfo)]
        L.ba_window_order.argtypes = [vp, vp]
        L.ba_batch_create.argtypes = [i32, vp, ctypes.POINTER(vp)]
        L.ba_batch_destroy.argtypes = [vp]
        L.ba_batch_info.argtypes = [vp, i32, ctypes.POINTER(_PlanInfo)]
        L.ba_workspace_size.argtypes = [vp, vp, ctypes.POINTER(_Settings), ctypes.POINTER(sz)]
        L.ba_solve.argtypes = [vp, ctypes.POINTER(_Settings), vp, vp, vp, vp, vp, sz, vp, vp, vp]
        L.ba_solve_noalloc.argtypes = [vp, ctypes.POINTER(_Settings), vp, vp, vp, vp, vp, vp, vp]
        L.ba_solve_batched.argtypes = [vp, ctypes.POINTER(_Settings), vp, vp, vp, vp, vp, sz, vp,
                                       vp, vp]
        L.ba_adjoint.argtypes = [vp, vp, ctypes.POINTER(_Settings), vp, vp, vp, vp, vp, vp, vp,
                                 vp, vp, sz, vp, vp]
        L.ba_autotune.argtypes = [vp, ctypes.POINTER(_Settings), vp, vp, vp, vp, vp, sz, vp,
                                  ctypes.POINTER(i32)]
        L.ba_set_launch.argtypes = [vp, i32]
        L.ba_set_launch_config.argtypes = [vp, ctypes.POINTER(_LaunchConfig)]
        L.ba_get_launch.argtypes = [vp, ctypes.POINTER(_LaunchConfig)]
        L.ba_profile_stages.argtypes = [vp, ctypes.POINTER(_Settings), vp, vp, vp, vp, vp, sz, vp,
                                        vp, ctypes.POINTER(ctypes.c_double)]
        L.ba_rig_create.argtypes = [i32, vp, vp, ctypes.POINTER(vp)]
        L.ba_rig_destroy.argtypes = [vp]
        L.ba_rig_set_waves_per_frame.argtypes = [vp, i32]
        L.ba_graph_create.argtypes = [i32, i32, vp, vp, vp, i32, ctypes.POINTER(vp)]
        L.ba_graph_destroy.argtypes = [vp]
        L.ba_graph_info.argtypes = [vp, vp, vp, vp]
        L.ba_graph_plan_array.argtypes = [vp, i32, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                          ctypes.POINTER(i64)]
        L.ba_graph_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.ba_pgo_solve.argtypes = [vp, ctypes.POINTER(_Settings), vp, vp, vp, vp, ctypes.c_size_t, vp, vp, vp]
        L.ba_triangulate.argtypes = [vp, ctypes.POINTER(_Settings), i32, i64, i32, vp, vp, vp, vp, vp, vp,
                                     vp, vp, vp, vp]
        L.ba_pnp_solve.argtypes = [vp, ctypes.POINTER(_Settings), i32, i64, i64, vp, vp, vp, vp, vp,
                                   vp, vp, vp, vp, vp, vp]
        L.ba_map_create.argtypes = [i32, i32, vp, vp, i32, ctypes.POINTER(vp)]
        L.ba_map_destroy.argtypes = [vp]
        L.ba_map_add_keyframe.argtypes = [vp, vp, i32, vp, vp, i64, vp, vp, vp, vp, vp,
                                          ctypes.POINTER(i32), vp]
        L.ba_map_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.ba_map_lists.argtypes = [vp, vp, vp, vp, vp]
        L.ba_map_arrays.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(vp)]
        L.ba_map_window.argtypes = [vp, ctypes.POINTER(vp)]
        L.ba_map_read.argtypes = [vp, vp, vp, vp, vp]
        L.ba_map_solve.argtypes = [vp, ctypes.POINTER(_Settings), vp, sz, vp, vp, vp]
        L.ba_vi_preintegrate.argtypes = [i32, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp]
        L.ba_vi_workspace_size.argtypes = [vp, ctypes.POINTER(_Settings), ctypes.POINTER(sz)]
        L.ba_vi_solve.argtypes = [vp, ctypes.POINTER(_Settings), vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, vp, vp]
        L.ba_status_string.argtypes = [i32]
        L.ba_status_string.restype = ctypes.c_char_p
        L.ba_last_error.restype = ctypes.c_char_p
        for f in ("ba_window_create", "ba_window_info", "ba_window_order", "ba_batch_create",
                  "ba_batch_info", "ba_workspace_size", "ba_solve", "ba_solve_noalloc", "ba_solve_batched",
                  "ba_adjoint", "ba_autotune", "ba_set_launch", "ba_set_launch_config", "ba_get_launch",
                  "ba_profile_stages",
                  "ba_rig_create", "ba_rig_set_waves_per_frame", "ba_pnp_solve", "ba_triangulate", "ba_graph_create", "ba_graph_info",
                  "ba_graph_plan_array", "ba_graph_workspace_size", "ba_pgo_solve", "ba_map_create",
                  "ba_map_add_keyframe", "ba_map_info", "ba_map_lists", "ba_map_arrays", "ba_map_window", "ba_map_read",
                  "ba_map_solve", "ba_vi_preintegrate", "ba_vi_workspace_size", "ba_vi_solve"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise BAError(status, lib().ba_last_error().decode())


@dataclasses.dataclass
class Settings:
    max_iters: int = 10
    precision: int = BA_FP64
    lambda_init: float = 1e-3
    lambda_up: float = 10.0
    lambda_down: float = 10.0
    lambda_min: float = 1e-10
    lambda_max: float = 1e10
    huber_delta: float = 1.0
    min_depth: float = 1e-3
    grad_tol: float = 0.0
    step_tol: float = 0.0

    def c(self) -> _Settings:
        return _Settings(self.max_iters, self.precision, self.lambda_init, self.lambda_up,
                         self.lambda_down, self.lambda_min, self.lambda_max, self.huber_delta,
                         self.min_depth, self.grad_tol, self.step_tol)


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Window:
    """Plan of one window's structure (index lists are host arrays)."""

    def __init__(self, n_poses, n_points, obs_pose, obs_point, intrinsics, obs_cam=None,
                 pose_fixed=None, extrinsics=None, host_only=False):
        L = lib()
        self._keep = [_host(obs_pose, np.int32), _host(obs_point, np.int32)]
        op, oj = self._keep
        oc = None if obs_cam is None else _host(obs_cam, np.int32)
        pf = None if pose_fixed is None else _host(pose_fixed, np.uint8)
        K = _host(intrinsics, np.float64).reshape(-1, 4)
        E = None if extrinsics is None else _host(extrinsics, np.float64).reshape(-1, 12)
        h = ctypes.c_void_p()
        _check(L.ba_window_create(int(n_poses), int(n_points), int(K.shape[0]), int(op.shape[0]),
                                  op.ctypes.data_as(ctypes.c_void_p), oj.ctypes.data_as(ctypes.c_void_p),
                                  None if oc is None else oc.ctypes.data_as(ctypes.c_void_p),
                                  None if pf is None else pf.ctypes.data_as(ctypes.c_void_p),
                                  K.ctypes.data_as(ctypes.c_void_p),
                                  None if E is None else E.ctypes.data_as(ctypes.c_void_p),
                                  BA_CREATE_HOST_ONLY if host_only else 0, ctypes.byref(h)))
        self._h = h
        self.n_poses, self.n_points, self.n_obs = int(n_poses), int(n_points), int(op.shape[0])
        self._keep = None

    @classmethod
    def from_problem(cls, w, host_only=False):
        """From any object with the fields of a bagen.Window."""
        return cls(w.poses_gt.shape[0] if hasattr(w, "poses_gt") else w.n_poses,
                   w.points_gt.shape[0] if hasattr(w, "points_gt") else w.n_points,
                   w.obs_pose, w.obs_point, w.intrinsics, obs_cam=w.obs_cam,
                   pose_fixed=w.pose_fixed, extrinsics=w.extrinsics, host_only=host_only)

    @property
    def handle(self):
        return self._h

    def info(self):
        i = _PlanInfo()
        _check(lib().ba_window_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _PlanInfo._fields_}

    def order(self):
        p = np.empty(self.n_obs, np.int64)
        _check(lib().ba_window_order(self._h, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    def workspace_size(self, settings: Settings) -> int:
        n = ctypes.c_size_t()
        _check(lib().ba_workspace_size(self._h, None, ctypes.byref(settings.c()), ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ba_window_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many windows packed window-major into one plan."""

    def __init__(self, windows: Sequence[Window]):
        arr = (ctypes.c_void_p * len(windows))(*[w.handle.value for w in windows])
        h = ctypes.c_void_p()
        _check(lib().ba_batch_create(len(windows), arr, ctypes.byref(h)))
        self._h = h
        self.n_windows = len(windows)
        self.n_poses = [w.n_poses for w in windows]
        self.n_points = [w.n_points for w in windows]
        self.n_obs = [w.n_obs for w in windows]

    @property
    def handle(self):
        return self._h

    def workspace_size(self, settings: Settings) -> int:
        n = ctypes.c_size_t()
        _check(lib().ba_workspace_size(None, self._h, ctypes.byref(settings.c()), ctypes.byref(n)))
        return n.value

    def info(self, w):
        i = _PlanInfo()
        _check(lib().ba_batch_info(self._h, int(w), ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _PlanInfo._fields_}

    def set_launch(self, chunk_obs: int):
        _check(lib().ba_set_launch(self._h, int(chunk_obs)))

    def get_launch(self) -> dict:
        """The plan's launch shape (include/ba.h ba_launch_config) as a dict."""
        c = _LaunchConfig()
        _check(lib().ba_get_launch(self._h, ctypes.byref(c)))
        return dict(chunk_obs=c.chunk_obs, tile_pairs=c.tile_pairs, class_chunk_mult=list(c.class_chunk_mult),
                    class_streams=c.class_streams)

    def set_launch_config(self, chunk_obs: int, tile_pairs: int = 0, class_chunk_mult=(1, 1, 1, 1),
                          class_streams: int = 1):
        c = _LaunchConfig(int(chunk_obs), int(tile_pairs), (ctypes.c_int32 * 4)(*[int(m) for m in class_chunk_mult]),
                          int(class_streams))
        _check(lib().ba_set_launch_config(self._h, ctypes.byref(c)))

    def autotune(self, settings, poses, points, obs_uv, obs_w, workspace, stream=None) -> int:
        c = ctypes.c_int32()
        _check(lib().ba_autotune(self._h, ctypes.byref(settings.c()), _ptr(poses), _ptr(points),
                                 _ptr(obs_uv), _ptr(obs_w), _ptr(workspace), workspace.numel(),
                                 _stream(stream), ctypes.byref(c)))
        return c.value

    def profile_stages(self, settings, poses, points, obs_uv, obs_w, workspace, reports,
                       stream=None):
        """Per-stage device time (ms, summed over attempts) of one solve."""
        ms = (ctypes.c_double * 4)()
        _check(lib().ba_profile_stages(self._h, ctypes.byref(settings.c()), _ptr(poses),
                                       _ptr(points), _ptr(obs_uv), _ptr(obs_w), _ptr(workspace),
                                       workspace.numel(), _ptr(reports), _stream(stream), ms))
        return dict(pass_a=ms[0], reduce=ms[1], pass_b=ms[2], accept=ms[3])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ba_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _workspace(plan, settings, workspace, device):
    import torch
    need = plan.workspace_size(settings)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
    return workspace


def solve(window: Window, settings: Settings, poses, points, obs_uv, obs_w=None, workspace=None,
          report=None, trace=None, stream=None):
    """In-place solve of one window; tensors are float64 on the GPU.
    Returns (report bytes tensor, trace bytes tensor or None, workspace)."""
    import torch
    dev = poses.device
    workspace = _workspace(window, settings, workspace, dev)
    if report is None:
        report = torch.zeros(REPORT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    _check(lib().ba_solve(window.handle, ctypes.byref(settings.c()), _ptr(poses), _ptr(points),
                          _ptr(obs_uv), _ptr(obs_w), _ptr(workspace), workspace.numel(),
                          _ptr(report), _ptr(trace), _stream(stream)))
    return report, trace, workspace


def solve_noalloc(window: Window, settings: Settings, poses, points, obs_uv, obs_w=None,
                  report=None, trace=None, stream=None):
    """ba_solve on the library's per-device scratch (no workspace argument; the
    call allocates nothing on the device when `report` is given).  Returns
    (report bytes tensor, trace bytes tensor or None)."""
    import torch
    if report is None:
        report = torch.zeros(REPORT_DTYPE.itemsize, dtype=torch.uint8, device=poses.device)
    _check(lib().ba_solve_noalloc(window.handle, ctypes.byref(settings.c()), _ptr(poses),
                                  _ptr(points), _ptr(obs_uv), _ptr(obs_w), _ptr(report),
                                  _ptr(trace), _stream(stream)))
    return report, trace


def solve_batched(batch: Batch, settings: Settings, poses, points, obs_uv, obs_w=None,
                  workspace=None, reports=None, traces=None, stream=None):
    import torch
    dev = poses.device
    workspace = _workspace(batch, settings, workspace, dev)
    if reports is None:
        reports = torch.zeros(REPORT_DTYPE.itemsize * batch.n_windows, dtype=torch.uint8, device=dev)
    _check(lib().ba_solve_batched(batch.handle, ctypes.byref(settings.c()), _ptr(poses),
                                  _ptr(points), _ptr(obs_uv), _ptr(obs_w), _ptr(workspace),
                                  workspace.numel(), _ptr(reports), _ptr(traces), _stream(stream)))
    return reports, traces, workspace


def adjoint(plan, settings: Settings, poses, points, obs_uv, obs_w, grad_poses, grad_points,
            grad_uv, grad_w, workspace=None, reports=None, stream=None):
    import torch
    dev = poses.device
    workspace = _workspace(plan, settings, workspace, dev)
    n = plan.n_windows if isinstance(plan, Batch) else 1
    if reports is None:
        reports = torch.zeros(REPORT_DTYPE.itemsize * n, dtype=torch.uint8, device=dev)
    w = plan.handle if isinstance(plan, Window) else None
    b = plan.handle if isinstance(plan, Batch) else None
    _check(lib().ba_adjoint(w, b, ctypes.byref(settings.c()), _ptr(poses), _ptr(points),
                            _ptr(obs_uv), _ptr(obs_w), _ptr(grad_poses), _ptr(grad_points),
                            _ptr(grad_uv), _ptr(grad_w), _ptr(workspace), workspace.numel(),
                            _ptr(reports), _stream(stream)))
    return reports, workspace


def parse_reports(reports) -> np.ndarray:
    return np.frombuffer(reports.cpu().numpy().tobytes(), dtype=REPORT_DTYPE)


def parse_traces(traces, n_windows, max_iters) -> np.ndarray:
    return np.frombuffer(traces.cpu().numpy().tobytes(), dtype=TRACE_DTYPE).reshape(n_windows, max_iters)


class Rig:
    """A camera rig resident on the current device (for motion-only solves)."""

    def __init__(self, intrinsics, extrinsics=None):
        K = _host(intrinsics, np.float64).reshape(-1, 4)
        E = None if extrinsics is None else _host(extrinsics, np.float64).reshape(-1, 12)
        self.n_cams = K.shape[0]
        self._h = ctypes.c_void_p()
        _check(lib().ba_rig_create(self.n_cams, K.ctypes.data_as(ctypes.c_void_p),
                                   None if E is None else E.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.byref(self._h)))

    def set_waves_per_frame(self, waves_per_frame: int):
        """1, 2 or 4 waves share each frame; 0 chooses from the launch shape."""
        _check(lib().ba_rig_set_waves_per_frame(self._h, int(waves_per_frame)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ba_rig_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pnp_solve(rig: Rig, settings: Settings, frame_obs_begin, poses, points, obs_point, obs_uv,
              obs_cam=None, obs_w=None, frame_transform=None, reports=None, traces=None,
              stream=None):
    """In-place motion-only solve of every frame (device tensors: int32 index
    arrays, float64 values).  Returns (report bytes tensor, trace bytes or None)."""
    import torch
    n_frames = frame_obs_begin.numel() - 1
    if reports is None:
        reports = torch.zeros(REPORT_DTYPE.itemsize * max(n_frames, 1), dtype=torch.uint8,
                              device=poses.device)
    _check(lib().ba_pnp_solve(rig._h, ctypes.byref(settings.c()), n_frames, obs_point.numel(),
                              points.shape[0], _ptr(frame_obs_begin), _ptr(poses), _ptr(points),
                              _ptr(obs_point), _ptr(obs_cam), _ptr(obs_uv), _ptr(obs_w),
                              _ptr(frame_transform), _ptr(reports), _ptr(traces), _stream(stream)))
    return reports, traces


def triangulate(rig: Rig, settings: Settings, point_obs_begin, poses, obs_pose, obs_uv, points,
                obs_cam=None, obs_w=None, reports=None, traces=None, stream=None):
    """Triangulate every landmark from its observations with the poses fixed
    (device tensors: int32 index arrays, float64 values; ``points`` is written).
    Returns (report bytes tensor, trace bytes or None)."""
    import torch
    n_points = point_obs_begin.numel() - 1
    if reports is None:
        reports = torch.zeros(REPORT_DTYPE.itemsize * max(n_points, 1), dtype=torch.uint8,
                              device=points.device)
    _check(lib().ba_triangulate(rig._h, ctypes.byref(settings.c()), n_points, obs_pose.numel(),
                                poses.shape[0], _ptr(point_obs_begin), _ptr(poses), _ptr(obs_pose),
                                _ptr(obs_cam), _ptr(obs_uv), _ptr(obs_w), _ptr(points), _ptr(reports),
                                _ptr(traces), _stream(stream)))
    return reports, traces


PLAN_TABLES = ("col_of_pose", "pose_of_col", "lev_ptr", "blk_ptr", "blk_row", "upd_ptr", "upd_a",
               "upd_b", "fwd_ptr", "fwd_blk", "fwd_col", "asm_ptr", "asm_edge", "rhs_ptr", "rhs_edge")


class Graph:
    """A pose graph's structure (host arrays); planned for the current device
    unless ``host_only``."""

    def __init__(self, n_poses, edge_i, edge_j, pose_fixed=None, host_only=False):
        ei = _host(edge_i, np.int32)
        ej = _host(edge_j, np.int32)
        fx = None if pose_fixed is None else _host(pose_fixed, np.uint8)
        self.n_poses, self.n_edges = int(n_poses), int(ei.shape[0])
        self._h = ctypes.c_void_p()
        _check(lib().ba_graph_create(self.n_poses, self.n_edges, ei.ctypes.data_as(ctypes.c_void_p),
                                     ej.ctypes.data_as(ctypes.c_void_p),
                                     None if fx is None else fx.ctypes.data_as(ctypes.c_void_p),
                                     BA_CREATE_HOST_ONLY if host_only else 0, ctypes.byref(self._h)))

    def info(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ba_graph_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(n_free=a.value, n_levels=b.value, n_blocks=c.value)

    def plan(self):
        """Every plan table as a numpy array (copies)."""
        out = {}
        for k, name in enumerate(PLAN_TABLES):
            ptr = ctypes.POINTER(ctypes.c_int32)()
            n = ctypes.c_int64()
            _check(lib().ba_graph_plan_array(self._h, k, ctypes.byref(ptr), ctypes.byref(n)))
            out[name] = np.ctypeslib.as_array(ptr, shape=(n.value,)).copy() if n.value else np.zeros(0, np.int32)
        return out

    def workspace_size(self):
        n = ctypes.c_size_t()
        _check(lib().ba_graph_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ba_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pgo_solve(graph: Graph, settings: Settings, poses, deltas, workspace, edge_w=None, report=None,
              traces=None, stream=None):
    """In-place pose-graph solve (device tensors, float64; ``workspace`` a uint8
    tensor of at least ``graph.workspace_size()`` bytes).  Returns (report bytes
    tensor, trace bytes or None)."""
    import torch
    if report is None:
        report = torch.zeros(REPORT_DTYPE.itemsize, dtype=torch.uint8, device=poses.device)
    _check(lib().ba_pgo_solve(graph._h, ctypes.byref(settings.c()), _ptr(poses), _ptr(deltas), _ptr(edge_w),
                              _ptr(workspace), workspace.numel(), _ptr(report), _ptr(traces), _stream(stream)))
    return report, traces


class _BorrowedWindow(Window):
    """A plan owned by a map (not destroyed by this object)."""

    def __init__(self, handle, n_poses, n_points, n_obs):
        self._h = ctypes.c_void_p(handle)
        self.n_poses, self.n_points, self.n_obs = n_poses, n_points, n_obs

    def close(self):
        self._h = ctypes.c_void_p()


class Map:
    """Sliding-window local map (ba_map_*): host index lists, device values."""

    def __init__(self, max_keyframes, intrinsics, extrinsics=None, host_only=False):
        K = _host(intrinsics, np.float64).reshape(-1, 4)
        E = None if extrinsics is None else _host(extrinsics, np.float64).reshape(-1, 12)
        h = ctypes.c_void_p()
        _check(lib().ba_map_create(int(max_keyframes), int(K.shape[0]), K.ctypes.data_as(ctypes.c_void_p),
                                   None if E is None else E.ctypes.data_as(ctypes.c_void_p),
                                   BA_CREATE_HOST_ONLY if host_only else 0, ctypes.byref(h)))
        self._h = h
        self.host_only = bool(host_only)

    def add_keyframe(self, pose, new_ids=(), new_points=None, obs_kf=(), obs_lm=(), obs_cam=None, obs_uv=None,
                     obs_w=None, stream=None) -> int:
        P = _host(pose, np.float64).reshape(12)
        ni = _host(np.asarray(new_ids, np.int64).reshape(-1), np.int64)
        npts = _host(np.zeros((0, 3)) if new_points is None else new_points, np.float64).reshape(-1, 3)
        ok = _host(np.asarray(obs_kf, np.int32).reshape(-1), np.int32)
        ol = _host(np.asarray(obs_lm, np.int64).reshape(-1), np.int64)
        n = ok.shape[0]
        oc = None if obs_cam is None else _host(obs_cam, np.int32)
        ouv = _host(np.zeros((0, 2)) if obs_uv is None else obs_uv, np.float64).reshape(-1, 2)
        ow = None if obs_w is None else _host(obs_w, np.float64)
        vp = lambda a: None if a is None or a.size == 0 else a.ctypes.data_as(ctypes.c_void_p)
        nd = ctypes.c_int32()
        st = None if self.host_only else _stream(stream)
        _check(lib().ba_map_add_keyframe(self._h, vp(P), int(ni.shape[0]), vp(ni), vp(npts), int(n), vp(ok),
                                         vp(ol), vp(oc), vp(ouv), vp(ow), ctypes.byref(nd), st))
        return nd.value

    def info(self):
        k, p, o = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().ba_map_info(self._h, ctypes.byref(k), ctypes.byref(p), ctypes.byref(o)))
        return k.value, p.value, o.value

    def lists(self):
        k, p, o = self.info()
        op, oj, oc = (np.empty(o, np.int32) for _ in range(3))
        ids = np.empty(p, np.int64)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
        _check(lib().ba_map_lists(self._h, vp(op), vp(oj), vp(oc), vp(ids)))
        return dict(obs_pose=op, obs_point=oj, obs_cam=oc, landmark_ids=ids)

    def arrays(self):
        """Device addresses of the values: (poses, points, obs_uv, obs_w), valid
        until the next insertion."""
        ptrs = [ctypes.c_void_p() for _ in range(4)]
        _check(lib().ba_map_arrays(self._h, *[ctypes.byref(x) for x in ptrs]))
        return tuple(p.value for p in ptrs)

    def read(self):
        """Host copies of the values: poses (K, 3, 4), points (M, 3), obs_uv (n, 2), obs_w (n,)."""
        k, p, o = self.info()
        P, L, uv, w = np.empty((k, 3, 4)), np.empty((p, 3)), np.empty((o, 2)), np.empty(o)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
        _check(lib().ba_map_read(self._h, vp(P), vp(L), vp(uv), vp(w)))
        return P, L, uv, w

    def window(self) -> Window:
        h = ctypes.c_void_p()
        _check(lib().ba_map_window(self._h, ctypes.byref(h)))
        k, p, o = self.info()
        return _BorrowedWindow(h.value, k, p, o)

    def solve(self, settings: Settings, workspace=None, report=None, trace=None, stream=None):
        import torch
        w = self.window()
        dev = torch.device("cuda", torch.cuda.current_device())
        workspace = _workspace(w, settings, workspace, dev)
        if report is None:
            report = torch.zeros(REPORT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        _check(lib().ba_map_solve(self._h, ctypes.byref(settings.c()), _ptr(workspace), workspace.numel(),
                                  _ptr(report), _ptr(trace), _stream(stream)))
        return report, trace, workspace

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ba_map_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vi_preintegrate(sample_begin, gyro, accel, dt, bias_bar, noise, out=None, stream=None):
    """Preintegrated IMU factors on the GPU: sample_begin (n + 1) int32, gyro and
    accel (n_samples, 3), bias_bar (n, 6) float64 device tensors; noise: 4 floats.
    Returns the (n, VI_PREINT_DOUBLES) float64 records."""
    import torch
    n = int(sample_begin.numel()) - 1
    if out is None:
        out = torch.empty((max(n, 0), VI_PREINT_DOUBLES), dtype=torch.float64, device=gyro.device)
    nz = _host(noise, np.float64)
    _check(lib().ba_vi_preintegrate(n, _ptr(sample_begin), _ptr(gyro), _ptr(accel), float(dt), _ptr(bias_bar),
                                    nz.ctypes.data_as(ctypes.c_void_p), _ptr(out), _stream(stream)))
    return out


def vi_workspace_size(window: Window, settings: Settings) -> int:
    n = ctypes.c_size_t()
    _check(lib().ba_vi_workspace_size(window.handle, ctypes.byref(settings.c()), ctypes.byref(n)))
    return n.value


def vi_solve(window: Window, settings: Settings, preint, gravity, poses, points, states, obs_uv, obs_w=None,
             workspace=None, report=None, trace=None, stream=None):
    """Visual-inertial solve of one window in place (poses, points, states
    n_poses x 9: v, b^a, b^w).  Returns (report, trace, workspace)."""
    import torch
    dev = poses.device
    need = vi_workspace_size(window, settings)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    if report is None:
        report = torch.zeros(REPORT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    g = _host(gravity, np.float64)
    _check(lib().ba_vi_solve(window.handle, ctypes.byref(settings.c()), _ptr(preint),
                             g.ctypes.data_as(ctypes.c_void_p), _ptr(poses), _ptr(points), _ptr(states),
                             _ptr(obs_uv), _ptr(obs_w), _ptr(workspace), workspace.numel(), _ptr(report),
                             _ptr(trace), _stream(stream)))
    return report, trace, workspace
