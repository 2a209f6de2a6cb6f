"""FP64 CPU oracle for sliding-window sparse Levenberg-Marquardt bundle adjustment.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import
it; the library under ``paper_2506_04359_amd/`` never does, and the oracle imports
nothing from the library (they share no code).

What it computes (paper: Sec. 2.2, "3D module", Eq. 2 and Eq. 3):
  * per-observation reprojection residual  r = pi(T_cb_k T_bw_i p_j) - o   (Eq. 2)
  * the robust sum of squared residuals over all observations            (Eq. 3)
  * minimised by Levenberg-Marquardt; the linear system is solved "poses first,
    then points" with the Schur complement (text after Eq. 3), here as a dense
    reference (``backend='dense'``) and as the textbook block-Schur form
    (``backend='schur'``), which must agree.
  * the implicit-function adjoint of the converged solution with respect to the
    2D keypoints and the observation weights (``adjoint``);
  * visual-inertial bundle adjustment (Eq. 9): IMU preintegration, the IMU
    factor and a dense LM over poses, velocities, biases and points (``imu``).

The paper leaves the solver's details open; the readings taken here are a Huber
robust kernel on the pixel residual, Marquardt diagonal damping with x10 / /10,
the left SE(3) perturbation, strict-decrease acceptance and a fixed attempt
count.  Each function is pinned by tests against values fixed by the paper or by
the mathematics (closed forms, finite differences, library solvers, brute force).
"""
from .se3 import skew, exp_so3, left_jacobian_so3, exp_se3, retract_pose, rotation_angle
from .model import Problem, transform, residuals, jacobians, huber, cost
from .lm import LMSettings, normal_equations_dense, normal_equations_blocks, lm_solve
from .adjoint import exact_hessian_dense, adjoint_dense, chordal_loss, ambient_to_tangent
from .metrics import rms, align_scale, rotation_errors

__all__ = [
    "skew", "exp_so3", "left_jacobian_so3", "exp_se3", "retract_pose", "rotation_angle",
    "Problem", "transform", "residuals", "jacobians", "huber", "cost",
    "LMSettings", "normal_equations_dense", "normal_equations_blocks", "lm_solve",
    "exact_hessian_dense", "adjoint_dense", "chordal_loss", "ambient_to_tangent",
    "rms", "align_scale", "rotation_errors",
]
