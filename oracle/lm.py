"""Levenberg-Marquardt of the oracle (test infrastructure, FP64).

Paper Sec. 2.2 (Eq. 3 and the sentence after it): the SBA objective is minimised
by solving for the poses first through the Schur complement and for the points
afterwards.  The paper gives no schedule; the oracle takes the textbook
Marquardt form (diagonal damping, x10 on rejection, /10 on acceptance) and runs
a fixed number of solve attempts.  One attempt:

  1. linearise at x (only after an accepted step or at the start):
       H = sum_o w_o rho'(s_o) J_o^T J_o,   g = sum_o w_o rho'(s_o) J_o^T r_o
     over the free variables (free poses first, 6 each, then points, 3 each);
  2. H_lam = H + lam * diag(max(H_kk, 1e-9));
  3. solve H_lam d = -g by Cholesky; a non-positive or non-finite pivot rejects
     the attempt;
  4. candidate T_i' = Exp(d_i) T_i, p_j' = p_j + d_j; a candidate with any camera
     depth Z <= min_depth is rejected;
  5. accept iff F(x') < F(x) (strict): x <- x', lam <- max(lam / 10, lam_min);
     otherwise lam <- min(10 lam, lam_max) and H, g are kept.

Per-window freeze (the paper gives no stopping rule; both tests are off at 0):
  * gradient test, before step 3: with b~ = -g_p + sum_j W_j V*_j^-1 g_l,j (the
    right-hand side of the reduced camera system, V*_j the damped landmark
    blocks) and g_l the landmark gradient, the window freezes when
    max(|b~|_inf, |g_l|_inf) <= grad_tol (not when a V*_j is not positive
    definite);
  * step test, after an accepted attempt: the window freezes when the step's
    max-norm (pose tangents and point moves) is <= step_tol.
A frozen window runs no more attempts: each remaining one is recorded with
status "frozen", not accepted, no candidate, cost and lam unchanged, and is
not counted in ``iters``.

``backend='dense'`` assembles the sparse Jacobian explicitly and forms J^T W J
(the plain definition).  ``backend='schur'`` assembles the same H in blocks
(U per pose, V per landmark, W per pose-landmark pair) and solves it by the
Schur complement on the poses followed by point back-substitution.  The two must
agree; the tests pin that.
"""
import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg
import scipy.sparse

from .model import cost, huber, jacobians, residuals, transform
from .se3 import retract_pose

DIAG_FLOOR = 1e-9


@dataclasses.dataclass
class LMSettings:
    max_iters: int = 10
    lambda_init: float = 1e-3
    lambda_up: float = 10.0
    lambda_down: float = 10.0
    lambda_min: float = 1e-10
    lambda_max: float = 1e10
    huber_delta: float = 1.0
    min_depth: float = 1e-3
    grad_tol: float = 0.0
    step_tol: float = 0.0


@dataclasses.dataclass
class LMResult:
    poses: np.ndarray
    points: np.ndarray
    initial_cost: float
    final_cost: float
    final_lambda: float
    accepted: int
    chol_failures: int
    trace: List[dict]
    iters: int = 0


def _weights(poses, points, prob, delta):
    r = residuals(poses, points, prob)
    s = np.sum(r * r, axis=1)
    _, d1, _ = huber(s, delta)
    return r, prob.obs_w * d1


# ---------------------------------------------------------------------------
# linear systems
# ---------------------------------------------------------------------------

def sparse_jacobian(poses, points, prob):
    """The full (2n x n_var) Jacobian, free poses first then points."""
    Jp, Jl = jacobians(poses, points, prob)
    n = prob.n_obs
    nf = prob.n_free
    fi = prob.free_index()[prob.obs_pose]
    rows, cols, vals = [], [], []
    obs = np.arange(n)
    for a in range(2):
        free = fi >= 0
        for c in range(6):
            rows.append(2 * obs[free] + a)
            cols.append(6 * fi[free] + c)
            vals.append(Jp[free, a, c])
        for c in range(3):
            rows.append(2 * obs + a)
            cols.append(6 * nf + 3 * prob.obs_point + c)
            vals.append(Jl[:, a, c])
    nvar = 6 * nf + 3 * prob.n_points
    return scipy.sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                           np.concatenate(cols))),
                                   shape=(2 * n, nvar)).tocsr()


def normal_equations_dense(poses, points, prob, delta):
    """Dense H = J^T W J and g = J^T W r (W = diag of w rho', per pixel row)."""
    r, wt = _weights(poses, points, prob, delta)
    J = sparse_jacobian(poses, points, prob)
    Wd = scipy.sparse.diags(np.repeat(wt, 2))
    H = (J.T @ Wd @ J).toarray()
    g = J.T @ (Wd @ r.reshape(-1))
    return H, np.asarray(g).reshape(-1)


@dataclasses.dataclass
class BlockSystem:
    U: np.ndarray          # (nf, 6, 6)
    V: np.ndarray          # (M, 3, 3)
    W: np.ndarray          # (n_pairs, 6, 3)
    gp: np.ndarray         # (nf, 6)
    gl: np.ndarray         # (M, 3)
    pair_pose: np.ndarray  # (n_pairs,) free-pose slot
    pair_point: np.ndarray  # (n_pairs,)


def normal_equations_blocks(poses, points, prob, delta):
    """The same H and g as ``normal_equations_dense``, kept in blocks."""
    r, wt = _weights(poses, points, prob, delta)
    Jp, Jl = jacobians(poses, points, prob)
    nf, M = prob.n_free, prob.n_points
    fi = prob.free_index()[prob.obs_pose]
    free = fi >= 0
    U = np.zeros((nf, 6, 6))
    gp = np.zeros((nf, 6))
    np.add.at(U, fi[free], wt[free, None, None] * np.einsum("nai,naj->nij", Jp[free], Jp[free]))
    np.add.at(gp, fi[free], wt[free, None] * np.einsum("nai,na->ni", Jp[free], r[free]))
    V = np.zeros((M, 3, 3))
    gl = np.zeros((M, 3))
    np.add.at(V, prob.obs_point, wt[:, None, None] * np.einsum("nai,naj->nij", Jl, Jl))
    np.add.at(gl, prob.obs_point, wt[:, None] * np.einsum("nai,na->ni", Jl, r))
    key = prob.obs_point[free] * max(nf, 1) + fi[free]
    ukey, inv = np.unique(key, return_inverse=True)
    W = np.zeros((ukey.size, 6, 3))
    np.add.at(W, inv, wt[free, None, None] * np.einsum("nai,naj->nij", Jp[free], Jl[free]))
    return BlockSystem(U=U, V=V, W=W, gp=gp, gl=gl, pair_pose=ukey % max(nf, 1),
                       pair_point=ukey // max(nf, 1))


def _damp(A, lam):
    """A + lam * diag(max(A_kk, 1e-9)) for a batch of square blocks or one matrix."""
    A = A.copy()
    idx = np.arange(A.shape[-1])
    d = A[..., idx, idx]
    A[..., idx, idx] = d + lam * np.maximum(d, DIAG_FLOOR)
    return A


def _chol_solve(A, b):
    """Cholesky solve; None when a pivot is non-positive or anything is non-finite."""
    if not (np.all(np.isfinite(A)) and np.all(np.isfinite(b))):
        return None
    try:
        c = scipy.linalg.cho_factor(A, lower=False, check_finite=False)
    except np.linalg.LinAlgError:
        return None
    x = scipy.linalg.cho_solve(c, b, check_finite=False)
    return x if np.all(np.isfinite(x)) else None


def solve_dense(H, g, lam):
    return _chol_solve(_damp(H, lam), -g)


def _pairs_of_pairs(sys: BlockSystem):
    """All (a, b), a <= b, of pairs that share a landmark (pairs are point-major)."""
    a_idx, b_idx = [], []
    bounds = np.flatnonzero(np.diff(sys.pair_point)) + 1
    starts = np.concatenate([[0], bounds])
    ends = np.concatenate([bounds, [sys.pair_point.size]])
    for s, e in zip(starts, ends):
        for a in range(s, e):
            for b in range(a, e):
                a_idx.append(a)
                b_idx.append(b)
    return np.asarray(a_idx, np.int64), np.asarray(b_idx, np.int64)


def solve_schur(sys: BlockSystem, lam, pp=None):
    """Reduced camera system S dp = b~ then dl_j = V*_j^-1 (-g_l - sum W^T dp)."""
    nf, M = sys.U.shape[0], sys.V.shape[0]
    Us = _damp(sys.U, lam)
    Vs = _damp(sys.V, lam)
    if not np.all(np.isfinite(Vs)):
        return None
    try:
        np.linalg.cholesky(Vs)           # every V*_j must be positive definite
    except np.linalg.LinAlgError:
        return None
    Vinv = np.linalg.inv(Vs)
    Y = np.einsum("pij,pjk->pik", sys.W, Vinv[sys.pair_point])        # W V*^-1
    if pp is None:
        pp = _pairs_of_pairs(sys)
    a, b = pp
    blocks = np.einsum("qik,qjk->qij", Y[a], sys.W[b])                # Y_a W_b^T
    S4 = np.zeros((nf, nf, 6, 6))
    np.add.at(S4, (sys.pair_pose[a], sys.pair_pose[b]), -blocks)
    off = a != b
    np.add.at(S4, (sys.pair_pose[b[off]], sys.pair_pose[a[off]]),
              -np.transpose(blocks[off], (0, 2, 1)))
    S4[np.arange(nf), np.arange(nf)] += Us
    S = S4.transpose(0, 2, 1, 3).reshape(6 * nf, 6 * nf)
    bt = -sys.gp.copy()
    np.add.at(bt, sys.pair_pose, np.einsum("pij,pj->pi", Y, sys.gl[sys.pair_point]))
    dp = _chol_solve(S, bt.reshape(-1)) if nf > 0 else np.zeros(0)
    if dp is None:
        return None
    dp = dp.reshape(nf, 6)
    rhs = -sys.gl.copy()
    np.add.at(rhs, sys.pair_point, -np.einsum("pij,pi->pj", sys.W, dp[sys.pair_pose]))
    dl = np.einsum("mij,mj->mi", Vinv, rhs)
    return np.concatenate([dp.reshape(-1), dl.reshape(-1)])


def reduced_gradient_norm(system, backend, lam, n_free):
    """max(|b~|_inf, |g_l|_inf) of the freeze test: b~ = -g_p + sum_j W_j V*_j^-1 g_l,j
    with V*_j = V_j + lam diag(max(V_j,kk, 1e-9)); NaN when a V*_j is not
    positive definite (the test then never freezes)."""
    if backend == "dense":
        H, g = system
        n = 6 * n_free
        M = (H.shape[0] - n) // 3
        gp, gl = g[:n], g[n:].reshape(M, 3)
        idx = n + 3 * np.arange(M)
        V = np.stack([H[i:i + 3, i:i + 3] for i in idx]) if M else np.zeros((0, 3, 3))
        Wt = H[:n, n:]
    else:
        gp, gl, V = system.gp.reshape(-1), system.gl, system.V
    Vs = _damp(V, lam)
    if _not_pd(Vs):
        return math.nan
    y = np.linalg.solve(Vs, gl[..., None])[..., 0] if gl.size else gl
    if backend == "dense":
        bt = -gp + Wt @ y.reshape(-1)
    else:
        bt = -system.gp.copy()
        np.add.at(bt, system.pair_pose, np.einsum("pij,pj->pi", system.W, y[system.pair_point]))
        bt = bt.reshape(-1)
    parts = [np.abs(bt).max() if bt.size else 0.0, np.abs(gl).max() if gl.size else 0.0]
    return float(max(parts))


def _not_pd(Vs):
    """True when any block of the batch is not positive definite (or not finite)."""
    if not np.all(np.isfinite(Vs)):
        return True
    try:
        np.linalg.cholesky(Vs)
    except np.linalg.LinAlgError:
        return True
    return False


# ---------------------------------------------------------------------------
# the LM loop
# ---------------------------------------------------------------------------

def apply_step(poses, points, prob, delta_x):
    nf = prob.n_free
    new_p = poses.copy()
    for i, f in enumerate(prob.free_index()):
        if f >= 0:
            new_p[i] = retract_pose(poses[i], delta_x[6 * f: 6 * f + 6])
    new_l = points + delta_x[6 * nf:].reshape(-1, 3)
    return new_p, new_l


def lm_solve(poses0, points0, prob, settings: LMSettings = None, backend: str = "dense",
             decisions: Optional[List[bool]] = None) -> LMResult:
    """Run exactly ``settings.max_iters`` LM attempts.

    ``decisions`` (optional) replays a given accept/reject sequence instead of the
    oracle's own test; a replayed acceptance of an invalid candidate raises."""
    st = settings or LMSettings()
    poses = np.array(poses0, float, copy=True)
    points = np.array(points0, float, copy=True)
    delta = st.huber_delta
    F = cost(poses, points, prob, delta)
    F0 = F
    lam = st.lambda_init
    system = None
    pp = None
    trace = []
    n_acc = n_chol = n_run = 0
    frozen = False
    for it in range(st.max_iters):
        if frozen:
            trace.append(dict(iter=it, cost=F, lam=lam, cand_cost=math.nan, status="frozen", accepted=False,
                              cost_after=F, lam_after=lam))
            continue
        if system is None:
            if backend == "dense":
                system = normal_equations_dense(poses, points, prob, delta)
            else:
                system = normal_equations_blocks(poses, points, prob, delta)
                if pp is None:
                    pp = _pairs_of_pairs(system)
        if st.grad_tol > 0:
            gn = reduced_gradient_norm(system, backend, lam, prob.n_free)
            if gn <= st.grad_tol:
                frozen = True
                trace.append(dict(iter=it, cost=F, lam=lam, cand_cost=math.nan, status="frozen", accepted=False,
                                  cost_after=F, lam_after=lam, grad_norm=gn))
                continue
        n_run += 1
        if backend == "dense":
            step = solve_dense(system[0], system[1], lam)
        else:
            step = solve_schur(system, lam, pp)
        rec = dict(iter=it, cost=F, lam=lam, cand_cost=math.nan, status="ok")
        valid = step is not None
        if not valid:
            rec["status"] = "chol_fail"
            n_chol += 1
        else:
            cp, cl = apply_step(poses, points, prob, step)
            _, xc = transform(cp, cl, prob)
            if np.any(~(xc[:, 2] > st.min_depth)):
                valid = False
                rec["status"] = "depth"
            else:
                Fc = cost(cp, cl, prob, delta)
                rec["cand_cost"] = Fc
        accept = valid and rec["cand_cost"] < F
        if decisions is not None:
            forced = bool(decisions[it])
            if forced and not valid:
                raise ValueError(f"replayed acceptance of an invalid candidate at attempt {it}")
            rec["own_decision"] = accept
            accept = forced
        if accept:
            poses, points, F = cp, cl, rec["cand_cost"]
            lam = max(lam / st.lambda_down, st.lambda_min)
            system = None
            n_acc += 1
            rec["step_norm"] = float(np.abs(step).max()) if step.size else 0.0
            if st.step_tol > 0 and rec["step_norm"] <= st.step_tol:
                frozen = True
        else:
            lam = min(lam * st.lambda_up, st.lambda_max)
        rec["accepted"] = accept
        rec["cost_after"] = F
        rec["lam_after"] = lam
        trace.append(rec)
    return LMResult(poses=poses, points=points, initial_cost=F0, final_cost=F,
                    final_lambda=lam, accepted=n_acc, chol_failures=n_chol, trace=trace, iters=n_run)
