"""Central finite differences of the converged-solution map of one window
(test infrastructure; FP64, oracle only).

The implicit-function adjoint (Sec. 2.2, Eq. 3: the gradient of the loss of
the minimiser with respect to the keypoints and weights) is checked against
the derivative it claims to be: perturb one keypoint coordinate or one weight
by +-h, solve the window again to its stationary point, and difference the
loss of the two solutions.

A re-solve starts at the unperturbed minimum x* and iterates
x <- x [+] (-H*^-1 g(x)) with H* the exact Hessian factored once at x*
(a chord iteration).  Its fixed point is where the gradient of the perturbed
cost vanishes, whatever matrix is used: the matrix only sets the rate, and
the iteration runs until the step is at rounding level (below 1e-13 of the
state's scale, or no longer shrinking tenfold), after which the caller
asserts that the gradient of the perturbed cost has vanished.  So an error in H*
would slow the re-solve, never move what is differenced.
"""
import math

import numpy as np
import scipy.linalg

import oracle
from oracle import adjoint as oadj
from oracle.lm import apply_step


def loss_of(P, w, free):
    return oracle.chordal_loss(P, w.poses_gt, free)[0]


def tight_solution(w, prob, delta=1.0, iters=50):
    """LM from the window's start, then Newton steps with the exact Hessian to
    the stationary point (rounding level)."""
    res = oracle.lm_solve(w.poses_init, w.points_init, prob,
                          oracle.LMSettings(max_iters=iters, lambda_init=1e-3, huber_delta=delta),
                          backend="schur")
    return oadj.newton_polish(res.poses, res.points, prob, delta)


def perturbed(prob, o, comp, h):
    uv, ww = prob.obs_uv.copy(), prob.obs_w.copy()
    if comp < 2:
        uv[o, comp] += h
    else:
        ww[o] += h
    return oracle.Problem(**{**prob.__dict__, "obs_uv": uv, "obs_w": ww})


class SolutionMap:
    """x*(o, w) near the stationary point (P0, L0) of prob."""

    def __init__(self, P0, L0, prob, delta=1.0):
        self.P0, self.L0, self.prob, self.delta = P0, L0, prob, delta
        H = oadj.exact_hessian_dense(P0, L0, prob, delta)
        self.cho = scipy.linalg.cho_factor(H)
        self.g0 = float(np.abs(oadj.gradient_dense(P0, L0, prob, delta)).max())

    def resolve(self, pr, max_iters=30):
        P, L = self.P0, self.L0
        scale = max(1.0, float(np.abs(L).max()))
        prev = math.inf
        for _ in range(max_iters):
            g = oadj.gradient_dense(P, L, pr, self.delta)
            step = -scipy.linalg.cho_solve(self.cho, g)
            size = float(np.abs(step).max())
            P, L = apply_step(P, L, pr, step)
            if size <= 1e-13 * scale or size > 0.1 * prev:
                break
            prev = size
        gn = float(np.abs(oadj.gradient_dense(P, L, pr, self.delta)).max())
        return P, L, gn

    def derivative(self, w, free, o, comp, h):
        """Central difference of the loss of the solution for coordinate
        (observation o, comp 0 = u, 1 = v, 2 = weight) with step h, and the
        largest gradient left at the two re-solves."""
        vals, gmax = [], 0.0
        for sgn in (1.0, -1.0):
            P, _, gn = self.resolve(perturbed(self.prob, o, comp, sgn * h))
            vals.append(loss_of(P, w, free))
            gmax = max(gmax, gn)
        return (vals[0] - vals[1]) / (2.0 * h), gmax


def pick_coordinates(prob, P, L, n_uv=80, n_w=20, seed=5, delta=1.0, kink=1e-3):
    """n_uv keypoint coordinates and n_w weights of distinct random observations,
    none within `kink` px of the Huber threshold (its second derivative jumps
    there, so a central difference across it is not the derivative)."""
    r = oracle.residuals(P, L, prob)
    norm = np.sqrt(np.sum(r * r, axis=1))
    ok = np.flatnonzero(np.abs(norm - delta) >= kink)
    rng = np.random.default_rng(seed)
    obs = rng.choice(ok, size=n_uv + n_w, replace=False)
    comps = np.concatenate([rng.integers(0, 2, size=n_uv), np.full(n_w, 2)])
    return [(int(o), int(c)) for o, c in zip(obs, comps)]


def dense_adjoint_at(w, prob, P, L, delta=1.0):
    free = ~prob.pose_fixed
    _, G = oracle.chordal_loss(P, w.poses_gt, free)
    gx = np.concatenate([oracle.ambient_to_tangent(P, G)[free].reshape(-1), np.zeros(3 * prob.n_points)])
    return oracle.adjoint_dense(P, L, prob, delta, gx)


def adjoint_value(g_uv, g_w, o, comp):
    return float(g_uv[o, comp]) if comp < 2 else float(g_w[o])


def rms_of(g_uv, g_w):
    v = np.concatenate([g_uv.reshape(-1), g_w])
    return math.sqrt(float(np.mean(v * v)))
