"""The pose-graph solver's host plan (nested-dissection order, factor pattern,
level schedule, gather lists), checked on the CPU: the damped normal equations
gathered by the plan's assembly lists equal the oracle's dense matrix, a
left-looking block Cholesky that follows the plan's update lists level by level
equals numpy's Cholesky of the permuted matrix (and every nonzero of that
factor lies in the plan's pattern), and the plan's forward and back
substitution solve the system."""
import numpy as np
import pytest

import bagen
from oracle import pgo


def _plan(d):
    import paper_2506_04359_amd as ba
    g = ba.Graph(d.n_poses, d.edge_i, d.edge_j, d.pose_fixed, host_only=True)
    return g.info(), g.plan()


@pytest.mark.parametrize("laps,per_lap,seed", [(2, 30, 1), (3, 25, 2), (1, 40, 3)])
def test_plan_factorises_the_normal_equations(laps, per_lap, seed):
    d = bagen.make_pose_graph(laps=laps, per_lap=per_lap, seed=seed)
    info, P = _plan(d)
    G = pgo.PoseGraph(d.n_poses, d.edge_i, d.edge_j, d.deltas, d.edge_w, d.pose_fixed.astype(bool))
    H, g, _ = pgo.normal_equations(d.poses_init, G)
    lam = 1e-3
    nf = info["n_free"]
    assert nf == int((~G.pose_fixed).sum())
    # oracle slots are free poses in pose order
    free = np.nonzero(~G.pose_fixed)[0]
    slot = {int(p): k for k, p in enumerate(free)}
    perm = np.array([slot[int(p)] for p in P["pose_of_col"]])
    Hd = H.copy()
    idx = np.arange(H.shape[0])
    Hd[idx, idx] = H[idx, idx] + lam * np.maximum(H[idx, idx], 1e-9)
    sel = (6 * perm[:, None] + np.arange(6)[None, :]).reshape(-1)
    Hp = Hd[np.ix_(sel, sel)]
    bp = -g[sel]
    # per-edge terms and the plan's gather
    terms = []
    for e in range(G.n_edges):
        r, B = pgo.edge_jacobian(d.poses_init[d.edge_i[e]], d.poses_init[d.edge_j[e]], d.deltas[e])
        terms.append((B.T @ B, B.T @ r))
    nb = info["n_blocks"]
    blk_ptr, blk_row = P["blk_ptr"], P["blk_row"]
    col_of_blk = np.repeat(np.arange(nf), np.diff(blk_ptr))
    L = np.zeros((nb, 6, 6))
    for b in range(nb):
        v = np.zeros((6, 6))
        for q in range(P["asm_ptr"][b], P["asm_ptr"][b + 1]):
            ce = P["asm_edge"][q]
            v += -terms[ce >> 1][0] if ce & 1 else terms[ce >> 1][0]
        r, c = blk_row[b], col_of_blk[b]
        if r == c:
            v[np.arange(6), np.arange(6)] += lam * np.maximum(np.diag(v), 1e-9)
        assert np.abs(v - Hp[6 * r:6 * r + 6, 6 * c:6 * c + 6]).max() < 1e-9 * max(1.0, np.abs(Hp).max())
        L[b] = v
    y = np.zeros((nf, 6))
    for c in range(nf):
        for q in range(P["rhs_ptr"][c], P["rhs_ptr"][c + 1]):
            ce = P["rhs_edge"][q]
            y[c] += -terms[ce >> 1][1] if ce & 1 else terms[ce >> 1][1]
    assert np.abs(y.reshape(-1) - bp).max() < 1e-9 * max(1.0, np.abs(bp).max())
    # the pattern holds every nonzero of the factor
    Lref = np.linalg.cholesky(Hp)
    in_pattern = np.zeros((nf, nf), bool)
    in_pattern[blk_row, col_of_blk] = True
    for r in range(nf):
        for c in range(r + 1):
            if not in_pattern[r, c]:
                assert np.abs(Lref[6 * r:6 * r + 6, 6 * c:6 * c + 6]).max() < 1e-12
    # left-looking factorisation in the plan's level order
    lev = P["lev_ptr"]
    for l in range(len(lev) - 1):
        cols = range(lev[l], lev[l + 1])
        for c in cols:
            for b in range(blk_ptr[c], blk_ptr[c + 1]):
                for u in range(P["upd_ptr"][b], P["upd_ptr"][b + 1]):
                    L[b] -= L[P["upd_a"][u]] @ L[P["upd_b"][u]].T
            for f in range(P["fwd_ptr"][c], P["fwd_ptr"][c + 1]):
                y[c] -= L[P["fwd_blk"][f]] @ y[P["fwd_col"][f]]
        for c in cols:
            Lc = np.linalg.cholesky(L[blk_ptr[c]])
            L[blk_ptr[c]] = Lc
            y[c] = np.linalg.solve(Lc, y[c])
            for b in range(blk_ptr[c] + 1, blk_ptr[c + 1]):
                L[b] = np.linalg.solve(Lc, L[b].T).T
    for b in range(nb):
        r, c = blk_row[b], col_of_blk[b]
        assert np.abs(L[b] - Lref[6 * r:6 * r + 6, 6 * c:6 * c + 6]).max() < 1e-8 * max(1.0, np.abs(Lref).max())
    x = np.zeros((nf, 6))
    for l in range(len(lev) - 2, -1, -1):
        for c in range(lev[l], lev[l + 1]):
            v = y[c].copy()
            for b in range(blk_ptr[c] + 1, blk_ptr[c + 1]):
                v -= L[b].T @ x[blk_row[b]]
            x[c] = np.linalg.solve(L[blk_ptr[c]].T, v)
    ref = np.linalg.solve(Hp, bp)
    assert np.abs(x.reshape(-1) - ref).max() < 1e-8 * max(1.0, np.abs(ref).max())
    # every column's parent is on a later level
    level_of = np.repeat(np.arange(len(lev) - 1), np.diff(lev))
    for c in range(nf):
        rows = blk_row[blk_ptr[c] + 1:blk_ptr[c + 1]]
        if rows.size:
            assert level_of[rows.min()] > level_of[c]


def test_nested_dissection_keeps_the_tree_shallow():
    d = bagen.make_pgo_workload("pgo-helix-3x500")
    info, _ = _plan(d)
    assert info["n_free"] == 1499 and info["n_levels"] <= 64
    assert info["n_blocks"] < 10 * info["n_free"]


def test_graph_argument_errors():
    import paper_2506_04359_amd as ba
    with pytest.raises(RuntimeError, match="out of range"):
        ba.Graph(3, [0, 1], [1, 5], host_only=True)
    with pytest.raises(RuntimeError, match="itself"):
        ba.Graph(3, [0, 1], [1, 1], host_only=True)
