"""The oracle's dense implicit-function adjoint on a full window of the adjoint
workload (10 keyframes, 2000 landmarks, about 19k observations) against
central finite differences of the converged-solution map (Sec. 2.2, Eq. 3).

The 100 differences (80 keypoint coordinates, 20 weights; h = 1e-4 and h / 2)
are stored in tests/golden/adjoint_cfg5_fd.json by make_adjoint_fd.py, which
calls only the oracle; this test recomputes some of them, checks the stored
set against the dense adjoint, and checks that a planted mistake in the
oracle (the Huber second derivative dropped) is caught by them.
"""
import json
import os

import numpy as np
import pytest

import bagen
import oracle
from oracle import adjoint as oadj
import adjoint_fd as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adjoint_cfg5_fd.json")
TOL = 1e-6   # per coordinate, times the RMS of the adjoint over all coordinates


@pytest.fixture(scope="module")
def setup():
    doc = json.load(open(GOLDEN))
    w = bagen.make_window(5, 0)
    prob = oracle.Problem.from_window(w)
    P, L = F.tight_solution(w, prob)
    g_uv, g_w = F.dense_adjoint_at(w, prob, P, L)
    return doc, w, prob, P, L, g_uv, g_w


def test_stored_differences_match_dense_adjoint(setup):
    doc, w, prob, P, L, g_uv, g_w = setup
    assert doc["window"]["n_obs"] == w.n_obs
    rms = F.rms_of(g_uv, g_w)
    assert abs(rms - doc["adjoint_rms"]) <= 1e-8 * rms
    # every re-solve ended at a stationary point (gradient at rounding level)
    assert doc["max_gradient_after_resolve"] <= 1e-12 * doc["gradient_at_start"]
    rows = doc["coordinates"]
    assert len(rows) == 100 and sum(r["comp"] == 2 for r in rows) == 20
    assert len({r["obs"] for r in rows}) == 100
    r = oracle.residuals(P, L, prob)
    norm = np.sqrt(np.sum(r * r, axis=1))
    outl = 0
    for row in rows:
        o, c = row["obs"], row["comp"]
        assert abs(norm[o] - 1.0) >= 1e-3            # away from the Huber kink
        outl += norm[o] > 1.0
        a = F.adjoint_value(g_uv, g_w, o, c)
        # Richardson self-check: halving h moves the difference by rounding only
        assert abs(row["fd_h"] - row["fd_h2"]) <= 2 * TOL * rms, row
        assert abs(row["fd_h"] - a) <= TOL * rms, (row, a)
    assert outl >= 5      # some coordinates sit on the outer (linear) Huber branch


def test_differences_reproduce(setup):
    doc, w, prob, P, L, g_uv, g_w = setup
    M = F.SolutionMap(P, L, prob)
    free = ~prob.pose_fixed
    rms = doc["adjoint_rms"]
    rows = doc["coordinates"]
    for row in rows[:4] + rows[-4:]:
        d, gleft = M.derivative(w, free, row["obs"], row["comp"], doc["h"])
        assert gleft <= 1e-12 * doc["gradient_at_start"]
        assert abs(d - row["fd_h"]) <= TOL * rms, (row, d)


def test_planted_mistake_is_caught(setup, monkeypatch):
    # the adjoint with rho'' taken as zero (both in H* and in the gather) must
    # miss the differences on the outer Huber branch
    doc, w, prob, P, L, _, _ = setup
    real = oadj.huber

    def no_second_derivative(s, delta):
        rho, d1, d2 = real(s, delta)
        return rho, d1, np.zeros_like(d2)

    monkeypatch.setattr(oadj, "huber", no_second_derivative)
    g_uv, g_w = F.dense_adjoint_at(w, prob, P, L)
    rms = doc["adjoint_rms"]
    bad = sum(abs(row["fd_h"] - F.adjoint_value(g_uv, g_w, row["obs"], row["comp"])) > TOL * rms
              for row in doc["coordinates"])
    assert bad >= 5, bad
