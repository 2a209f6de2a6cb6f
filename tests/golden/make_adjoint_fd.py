"""Write adjoint_cfg5_fd.json: central finite differences of the converged
solution map of the first window of the adjoint workload (10 keyframes, 2000
landmarks, keyframes 0 and 1 fixed, chordal pose loss), computed by the FP64
oracle alone.

    python tests/golden/make_adjoint_fd.py

100 coordinates: 80 keypoint coordinates and 20 observation weights of
distinct random observations away from the Huber kink; each differenced with
h = 1e-4 (px, or weight units) and h / 2 (a Richardson self-check).  The loss
is L = sum over free poses |R - R_gt|_F^2 + |t - t_gt|^2 (Sec. 2.2, Eq. 3:
the minimiser the adjoint differentiates).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import bagen  # noqa: E402
import oracle  # noqa: E402
import adjoint_fd as F  # noqa: E402

H = 1e-4
OUT = os.path.join(HERE, "adjoint_cfg5_fd.json")


def main():
    w = bagen.make_window(5, 0)
    prob = oracle.Problem.from_window(w)
    free = ~prob.pose_fixed
    P, L = F.tight_solution(w, prob)
    M = F.SolutionMap(P, L, prob)
    g_uv, g_w = F.dense_adjoint_at(w, prob, P, L)
    coords = F.pick_coordinates(prob, P, L)
    g_init = float(np.abs(oracle.adjoint.gradient_dense(w.poses_init, w.points_init, prob, 1.0)).max())
    rows = []
    worst_grad = 0.0
    for o, c in coords:
        d1, r1 = M.derivative(w, free, o, c, H)
        d2, r2 = M.derivative(w, free, o, c, H / 2)
        worst_grad = max(worst_grad, r1, r2)
        rows.append({"obs": o, "comp": c, "fd_h": d1, "fd_h2": d2})
    doc = {
        "window": {"config": 5, "index": 0, "n_obs": int(w.n_obs), "n_points": int(w.n_points)},
        "loss": "chordal: sum over free poses |R - R_gt|_F^2 + |t - t_gt|^2",
        "h": H, "huber_delta": 1.0,
        "comp": "0 = u, 1 = v (keypoint px), 2 = observation weight",
        "adjoint_rms": F.rms_of(g_uv, g_w),
        "loss_at_solution": F.loss_of(P, w, free),
        "max_gradient_after_resolve": worst_grad, "gradient_at_start": g_init,
        "coordinates": rows,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT, len(rows), "coordinates; largest gradient left", worst_grad)


if __name__ == "__main__":
    main()
