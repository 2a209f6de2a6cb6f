"""GPU parity of the pose-graph solver (ba_pgo_solve) against the FP64 oracle
(oracle/pgo.py), through the C ABI.

The oracle follows the GPU's accept/reject sequence (a flip must be a near-tie
in the oracle's own numbers); the cost of every attempt, the final cost and the
final poses agree to 1e-9 relative (costs with an absolute 1e-20 allowance for
graphs whose minimum is zero, poses to 1e-9 * max(1, |T|)).  The
1500-pose benchmark graph is checked the same way with the oracle's sparse
backend.
"""
import math

import numpy as np
import pytest

import bagen
from oracle import pgo
from oracle.lm import LMSettings

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
COST_ABS = 1e-20   # a tree of edges solves to a cost of pure rounding noise (about 1e-29)


def _gpu(d, s, edge_w=None, fixed=None, with_trace=True):
    import torch
    import paper_2506_04359_amd as ba
    dev = torch.device("cuda:0")
    g = ba.Graph(d.n_poses, d.edge_i, d.edge_j, d.pose_fixed if fixed is None else fixed)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    P = t(d.poses_init.reshape(-1, 12))
    ws = torch.empty(g.workspace_size() + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + g.workspace_size()]
    tr = torch.zeros(32 * max(1, s.max_iters), dtype=torch.uint8, device=dev) if with_trace else None
    rep, tr = ba.pgo_solve(g, s, P, t(d.deltas.reshape(-1, 12)), ws,
                           edge_w=None if edge_w is None else t(edge_w), traces=tr)
    torch.cuda.synchronize()
    out = dict(poses=P.cpu().numpy().reshape(-1, 3, 4), report=ba.parse_reports(rep)[0], info=g.info())
    if with_trace:
        out["trace"] = ba.parse_traces(tr, 1, max(1, s.max_iters))[0]
    return out


def _check(d, s, g, edge_w=None, backend="dense", fixed=None):
    G = pgo.PoseGraph(d.n_poses, d.edge_i, d.edge_j, d.deltas, d.edge_w if edge_w is None else edge_w,
                      (d.pose_fixed if fixed is None else fixed).astype(bool))
    tr = g["trace"]
    ref = pgo.pgo_solve(d.poses_init, G, LMSettings(max_iters=s.max_iters, lambda_init=s.lambda_init),
                        backend=backend, decisions=[bool(a) for a in tr["accepted"]])
    for t, gt in zip(ref.trace, tr):
        if t["own_decision"] != bool(gt["accepted"]):
            assert abs(t["cand_cost"] - t["cost"]) <= 1e-12 * abs(t["cost"]) + COST_ABS, (t, gt)
        assert abs(t["cost"] - gt["cost"]) <= TOL64 * abs(t["cost"]) + COST_ABS, (t, gt)
        if math.isfinite(t["cand_cost"]) and gt["status"] == 0:
            assert abs(t["cand_cost"] - gt["cand_cost"]) <= TOL64 * abs(t["cand_cost"]) + COST_ABS, (t, gt)
    r = g["report"]
    assert abs(r["final_cost"] - ref.final_cost) <= TOL64 * ref.final_cost + COST_ABS
    assert r["accepted"] == ref.accepted and r["chol_failures"] == ref.chol_failures
    assert np.abs(g["poses"] - ref.poses).max() <= TOL64 * max(1.0, np.abs(ref.poses).max())
    return ref


@pytest.mark.parametrize("laps,per_lap,seed", [(2, 30, 11), (3, 20, 12), (1, 25, 13)])
def test_graphs_match_oracle(laps, per_lap, seed):
    import paper_2506_04359_amd as ba
    d = bagen.make_pose_graph(laps=laps, per_lap=per_lap, seed=seed, sigma_rot=0.01, sigma_trans=0.05)
    s = ba.Settings(max_iters=10, precision=ba.BA_FP64)
    ref = _check(d, s, _gpu(d, s))
    assert ref.final_cost <= ref.initial_cost + COST_ABS


def test_weights_and_several_fixed_poses():
    import paper_2506_04359_amd as ba
    d = bagen.make_pose_graph(laps=2, per_lap=20, seed=14)
    w = np.random.default_rng(5).uniform(0.2, 3.0, d.n_edges)
    fixed = d.pose_fixed.copy()
    fixed[[7, 23]] = 1
    s = ba.Settings(max_iters=8, precision=ba.BA_FP64)
    _check(d, s, _gpu(d, s, edge_w=w, fixed=fixed), edge_w=w, fixed=fixed)


def test_reversed_and_repeated_edges():
    """Edges stored j -> i (with the inverse delta) and an edge given twice."""
    import paper_2506_04359_amd as ba
    d = bagen.make_pose_graph(laps=2, per_lap=20, seed=16)
    ei, ej, D = d.edge_i.copy(), d.edge_j.copy(), d.deltas.copy()
    for e in range(0, d.n_edges, 3):
        ei[e], ej[e] = d.edge_j[e], d.edge_i[e]
        D[e] = pgo.inverse(d.deltas[e])
    ei = np.concatenate([ei, ei[5:6]])
    ej = np.concatenate([ej, ej[5:6]])
    D = np.concatenate([D, D[5:6]])
    r = bagen.PoseGraphData(poses_gt=d.poses_gt, poses_init=d.poses_init, edge_i=ei, edge_j=ej, deltas=D,
                            edge_w=np.ones(ei.shape[0]), pose_fixed=d.pose_fixed, loop=np.zeros(ei.shape[0], bool))
    s = ba.Settings(max_iters=8, precision=ba.BA_FP64)
    _check(r, s, _gpu(r, s))


def test_degenerate_graphs():
    """Negative weights (every factorisation fails: poses kept), every pose
    fixed, and a graph without edges."""
    import paper_2506_04359_amd as ba
    d = bagen.make_pose_graph(laps=2, per_lap=10, seed=15)
    s = ba.Settings(max_iters=4, precision=ba.BA_FP64)
    g = _gpu(d, s, edge_w=-np.ones(d.n_edges))
    assert g["report"]["chol_failures"] == 4 and g["report"]["accepted"] == 0
    assert np.array_equal(g["poses"], d.poses_init)
    g = _gpu(d, s, fixed=np.ones(d.n_poses, np.uint8))
    assert g["info"]["n_free"] == 0 and np.array_equal(g["poses"], d.poses_init)
    e = bagen.PoseGraphData(poses_gt=d.poses_gt, poses_init=d.poses_init, edge_i=np.zeros(0, np.int32),
                            edge_j=np.zeros(0, np.int32), deltas=np.zeros((0, 3, 4)), edge_w=np.zeros(0),
                            pose_fixed=d.pose_fixed, loop=np.zeros(0, bool))
    g = _gpu(e, s)
    assert g["report"]["final_cost"] == 0.0 and np.array_equal(g["poses"], d.poses_init)


def test_benchmark_graph():
    """The 1500-pose, 2988-edge helix the benchmark times (oracle: SuperLU)."""
    import paper_2506_04359_amd as ba
    d = bagen.make_pgo_workload("pgo-helix-3x500")
    s = ba.Settings(max_iters=d.max_iters, precision=ba.BA_FP64, lambda_init=d.lambda_init)
    g = _gpu(d, s)
    assert g["info"]["n_levels"] <= 64
    ref = _check(d, s, g, backend="sparse")
    assert ref.final_cost < 0.2 * ref.initial_cost


def test_graph_replays_equal_the_eager_solve():
    """ba_pgo_solve captured in a HIP graph: every replay (with eager work and a
    synchronisation between replays) gives the eager solve's poses and report
    bit for bit."""
    import torch
    import paper_2506_04359_amd as ba
    dev = torch.device("cuda:0")
    d = bagen.make_pose_graph(laps=2, per_lap=60, seed=17)
    g = ba.Graph(d.n_poses, d.edge_i, d.edge_j, d.pose_fixed)
    s = ba.Settings(max_iters=6, precision=ba.BA_FP64)
    P0 = torch.tensor(d.poses_init.reshape(-1, 12), dtype=torch.float64, device=dev)
    P = P0.clone()
    D = torch.tensor(d.deltas.reshape(-1, 12), dtype=torch.float64, device=dev)
    raw = torch.empty(g.workspace_size() + 256, dtype=torch.uint8, device=dev)
    off = (-raw.data_ptr()) % 256
    ws = raw[off:off + g.workspace_size()]
    rep = torch.zeros(48, dtype=torch.uint8, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ba.pgo_solve(g, s, P, D, ws, report=rep)
    torch.cuda.synchronize()
    eager_P, eager_rep = P.clone(), rep.clone()
    graph = torch.cuda.CUDAGraph()
    P.copy_(P0)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=side):
        ba.pgo_solve(g, s, P, D, ws, report=rep)
    for _ in range(3):
        P.copy_(P0)
        rep.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(P, eager_P) and torch.equal(rep, eager_rep)
