"""Implicit-function adjoint of the converged solution (test infrastructure, FP64).

At a minimum x* of F(x; o, w) (Sec. 2.2, Eq. 3) the gradient vanishes, so the
solution map satisfies  H* dx* = -d(grad F)/d(o, w) d(o, w)  with H* the exact
Hessian of F in the left-perturbation chart.  For a loss L(x*) the chain rule
gives, with a = H*^-1 dL/dx:

  dL/do_o = w_o (rho' I + 2 rho'' r r^T) J_o a
  dL/dw_o = -rho' r_o^T J_o a

Exact Hessian per observation (the Gauss-Newton part plus second-order terms):
  H*_o = w [ rho' (J^T J + sum_k r_k Hess(r_k)) + 2 rho'' (J^T r)(J^T r)^T ]
  sum_k r_k Hess(r_k) = J_c^T P J_c + M(a_b)
    J_c = R_c [I, -[x_b]x, R_i]                      (3 x 9: rho, phi, point)
    P   = r_u Hess(pi_u) + r_v Hess(pi_v) in x_c:  P_XZ = -r_u fx / Z^2,
          P_YZ = -r_v fy / Z^2,  P_ZZ = 2 (r_u fx X + r_v fy Y) / Z^3
    a_b = R_c^T A^T r    (the residual-weighted projection gradient, base frame)
    M_phiphi = (x a^T + a x^T)/2 - (a.x) I,  M_phirho = -[a]x / 2,
    M_phip   = -[a]x R_i,  all other blocks 0 (x = x_b).
The second-order terms come from the second derivatives of x_b(Exp(xi) T p).
"""
import numpy as np
import scipy.linalg

from .model import huber, jacobians, projection_jacobian, residuals, skew_batch, transform


def second_order_terms(poses, points, prob):
    """sum_k r_k Hess(r_k) per observation, (n, 9, 9) in (rho, phi, point) order."""
    xb, xc = transform(poses, points, prob)
    r = residuals(poses, points, prob)
    K = prob.intrinsics[prob.obs_cam]
    A = projection_jacobian(xc, K)
    Rc = prob.extrinsics[prob.obs_cam, :, :3]
    Ri = poses[prob.obs_pose, :, :3]
    n = xb.shape[0]
    X, Y, Z = xc[:, 0], xc[:, 1], xc[:, 2]
    P = np.zeros((n, 3, 3))
    P[:, 0, 2] = P[:, 2, 0] = -r[:, 0] * K[:, 0] / Z ** 2
    P[:, 1, 2] = P[:, 2, 1] = -r[:, 1] * K[:, 1] / Z ** 2
    P[:, 2, 2] = 2.0 * (r[:, 0] * K[:, 0] * X + r[:, 1] * K[:, 1] * Y) / Z ** 3
    Jc_b = np.concatenate([np.broadcast_to(np.eye(3), (n, 3, 3)), -skew_batch(xb), Ri], axis=2)
    Jc = np.einsum("nab,nbc->nac", Rc, Jc_b)                             # (n, 3, 9)
    T = np.einsum("nai,nab,nbj->nij", Jc, P, Jc)
    a = np.einsum("nba,nb->na", Rc, np.einsum("nka,nk->na", A, r))      # R_c^T A^T r
    ax = np.sum(a * xb, axis=1)
    M = np.zeros((n, 9, 9))
    M[:, 3:6, 3:6] = 0.5 * (xb[:, :, None] * a[:, None, :] + a[:, :, None] * xb[:, None, :]) \
        - ax[:, None, None] * np.eye(3)
    Sa = skew_batch(a)
    M[:, 3:6, 0:3] = -0.5 * Sa
    M[:, 0:3, 3:6] = np.transpose(M[:, 3:6, 0:3], (0, 2, 1))
    M[:, 3:6, 6:9] = -np.einsum("nab,nbc->nac", Sa, Ri)
    M[:, 6:9, 3:6] = np.transpose(M[:, 3:6, 6:9], (0, 2, 1))
    return T + M


def _obs_columns(prob):
    """Column of each of the 9 per-observation variables in the dense system (-1: fixed)."""
    nf = prob.n_free
    fi = prob.free_index()[prob.obs_pose]
    cols = np.empty((prob.n_obs, 9), np.int64)
    for c in range(6):
        cols[:, c] = np.where(fi >= 0, 6 * fi + c, -1)
    for c in range(3):
        cols[:, 6 + c] = 6 * nf + 3 * prob.obs_point + c
    return cols


def exact_hessian_dense(poses, points, prob, delta):
    r = residuals(poses, points, prob)
    s = np.sum(r * r, axis=1)
    _, d1, d2 = huber(s, delta)
    Jp, Jl = jacobians(poses, points, prob)
    J = np.concatenate([Jp, Jl], axis=2)                                  # (n, 2, 9)
    Jr = np.einsum("nai,na->ni", J, r)
    Ho = prob.obs_w[:, None, None] * (
        d1[:, None, None] * (np.einsum("nai,naj->nij", J, J) + second_order_terms(poses, points, prob))
        + 2.0 * d2[:, None, None] * Jr[:, :, None] * Jr[:, None, :])
    nvar = 6 * prob.n_free + 3 * prob.n_points
    H = np.zeros((nvar, nvar))
    cols = _obs_columns(prob)
    for i in range(9):
        for j in range(9):
            m = (cols[:, i] >= 0) & (cols[:, j] >= 0)
            np.add.at(H, (cols[m, i], cols[m, j]), Ho[m, i, j])
    return H


def gradient_dense(poses, points, prob, delta):
    """Analytic gradient of F over the free variables (free poses, then points)."""
    r = residuals(poses, points, prob)
    s = np.sum(r * r, axis=1)
    _, d1, _ = huber(s, delta)
    Jp, Jl = jacobians(poses, points, prob)
    J = np.concatenate([Jp, Jl], axis=2)
    go = (prob.obs_w * d1)[:, None] * np.einsum("nai,na->ni", J, r)
    g = np.zeros(6 * prob.n_free + 3 * prob.n_points)
    cols = _obs_columns(prob)
    for i in range(9):
        m = cols[:, i] >= 0
        np.add.at(g, cols[m, i], go[m, i])
    return g


def adjoint_dense(poses, points, prob, delta, grad_x):
    """dL/d(obs_uv) (n, 2) and dL/d(obs_w) (n,) for the tangent cotangent grad_x."""
    H = exact_hessian_dense(poses, points, prob, delta)
    a = scipy.linalg.solve(H, grad_x, assume_a="sym")
    r = residuals(poses, points, prob)
    s = np.sum(r * r, axis=1)
    _, d1, d2 = huber(s, delta)
    Jp, Jl = jacobians(poses, points, prob)
    cols = _obs_columns(prob)
    ax = np.where(cols >= 0, a[np.maximum(cols, 0)], 0.0)                # (n, 9)
    Ja = np.einsum("nai,ni->na", Jp, ax[:, :6]) + np.einsum("nai,ni->na", Jl, ax[:, 6:])
    rJa = np.sum(r * Ja, axis=1)
    g_uv = prob.obs_w[:, None] * (d1[:, None] * Ja + 2.0 * d2[:, None] * r * rJa[:, None])
    g_w = -d1 * rJa
    return g_uv, g_w


def chordal_loss(poses, poses_ref, free_mask):
    """L = sum over free poses ||R - R_ref||_F^2 + ||t - t_ref||^2 and its ambient gradient."""
    d = (poses - poses_ref) * np.asarray(free_mask, float)[:, None, None]
    return float(np.sum(d * d)), 2.0 * d


def ambient_to_tangent(poses, G):
    """Map an ambient cotangent G (N, 3, 4) of [R | t] to the left-perturbation
    tangent cotangent (N, 6) = (dL/drho, dL/dphi):
      M = G_R R^T + G_t t^T,  dL/drho = G_t,  dL/dphi = (M32-M23, M13-M31, M21-M12)."""
    R, t = poses[:, :, :3], poses[:, :, 3]
    GR, Gt = G[:, :, :3], G[:, :, 3]
    M = np.einsum("nab,ncb->nac", GR, R) + Gt[:, :, None] * t[:, None, :]
    phi = np.stack([M[:, 2, 1] - M[:, 1, 2], M[:, 0, 2] - M[:, 2, 0], M[:, 1, 0] - M[:, 0, 1]], 1)
    return np.concatenate([Gt, phi], axis=1)


def newton_polish(poses, points, prob, delta, iters=8):
    """Unconditional Newton steps with the exact Hessian from a point near a
    minimum.  LM's cost-decrease test stops at about sqrt(machine epsilon) in the
    state; finite differences of the solution map need the stationary point to
    near machine precision, which Newton's quadratic convergence gives."""
    from .lm import apply_step
    P, L = poses.copy(), points.copy()
    for _ in range(iters):
        g = gradient_dense(P, L, prob, delta)
        H = exact_hessian_dense(P, L, prob, delta)
        step = scipy.linalg.solve(H, -g, assume_a="sym")
        P, L = apply_step(P, L, prob, step)
        if np.abs(step).max() < 1e-15 * max(1.0, np.abs(L).max()):
            break
    return P, L
