"""torch.autograd.Function around the bundle adjuster.

forward : the LM solve (library kernels) from an initial state to x*.
backward: the implicit-function adjoint at x* (library kernels): the incoming
          cotangent of the [R | t] poses and of the points is passed as is; the
          library maps it to the left-perturbation tangent, solves with the exact
          Hessian and returns d(loss)/d(keypoints) and d(loss)/d(weights).
By the implicit-function theorem the converged state does not depend on the
initial state, so no gradient flows to it.
"""
import torch

from . import _binding as B


class BASolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, poses0, points0, obs_uv, obs_w, plan, settings):
        poses = poses0.detach().clone().contiguous()
        points = points0.detach().clone().contiguous()
        uv = obs_uv.detach().contiguous()
        w = None if obs_w is None else obs_w.detach().contiguous()
        if isinstance(plan, B.Batch):
            B.solve_batched(plan, settings, poses, points, uv, w)
        else:
            B.solve(plan, settings, poses, points, uv, w)
        ctx.plan = plan
        ctx.settings = settings
        ctx.has_w = w is not None
        ctx.save_for_backward(poses, points, uv, w if w is not None else uv.new_empty(0))
        return poses, points

    @staticmethod
    def backward(ctx, g_poses, g_points):
        poses, points, uv, w = ctx.saved_tensors
        w = w if ctx.has_w else None
        gp = torch.zeros_like(poses) if g_poses is None else g_poses.contiguous().to(torch.float64)
        gl = None if g_points is None else g_points.contiguous().to(torch.float64)
        grad_uv = torch.empty_like(uv)
        grad_w = torch.empty(uv.shape[0], dtype=torch.float64, device=uv.device)
        B.adjoint(ctx.plan, ctx.settings, poses, points, uv, w, gp, gl, grad_uv, grad_w)
        return None, None, grad_uv, (grad_w if ctx.needs_input_grad[3] else None), None, None
