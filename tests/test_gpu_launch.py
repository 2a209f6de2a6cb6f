"""Launch shapes of the batched solve (one launch per stage and size class): the shape is read
back as set, invalid shapes are refused without changing the plan, every shape
solves to the mixed-precision bar against the oracle, running the size
classes on one stream instead of as concurrent chains changes nothing (bit for
bit), and the tuner picks a valid shape that fits the workspace."""
import numpy as np
import pytest

import bagen
from helpers import gpu_solve_batched, mixed_check, settings_for

pytestmark = pytest.mark.gpu


def _windows():
    # windows of all four size classes (free poses up to 8, 16, 23, 32)
    ws = [bagen.make_window(3, i) for i in range(40)]
    nf = [int(np.sum(w.pose_fixed == 0)) for w in ws]
    picked, seen = [], set()
    for w, f in zip(ws, nf):
        c = 0 if f <= 8 else 1 if f <= 16 else 2 if f <= 23 else 3
        if c not in seen:
            seen.add(c)
            picked.append(w)
    assert len(picked) == 4
    return picked


def test_launch_config_round_trip_and_refusals():
    import paper_2506_04359_amd as ba
    ws = _windows()
    B = ba.Batch([ba.Window.from_problem(w, host_only=True) for w in ws])
    B.set_launch_config(3000, tile_pairs=64, class_chunk_mult=(1, 2, 3, 4), class_streams=0)
    want = dict(chunk_obs=3000, tile_pairs=64, class_chunk_mult=[1, 2, 3, 4], class_streams=0)
    assert B.get_launch() == want
    bad = [dict(chunk_obs=100), dict(chunk_obs=2048, tile_pairs=128), dict(chunk_obs=2048, class_chunk_mult=(0, 1, 1, 1)),
           dict(chunk_obs=2048, class_chunk_mult=(1, 1, 1, 5)), dict(chunk_obs=2048, class_streams=2)]
    for kw in bad:
        with pytest.raises(ba.BAError) as e:
            B.set_launch_config(**kw)
        assert e.value.status == ba.BA_ERR_INVALID_ARG
        assert B.get_launch() == want
    B.set_launch(4096)   # chunk_obs only; the other fields stay
    assert B.get_launch() == dict(want, chunk_obs=4096)


@pytest.mark.parametrize("launch", [
    dict(chunk_obs=2048, tile_pairs=64),
    dict(chunk_obs=1024, class_chunk_mult=(1, 1, 2, 4)),
    dict(chunk_obs=8192, class_chunk_mult=(4, 2, 1, 1), class_streams=0),
])
def test_every_shape_meets_the_bar(launch):
    ws = _windows()
    s = settings_for(ws[0], max_iters=8)
    out = gpu_solve_batched(ws, s, launch=launch)
    for w, o in zip(ws, out):
        assert o["report"]["status"] == 0
        mixed_check(w, o, align=True, s=s)


def test_one_stream_equals_class_chains():
    ws = _windows()
    s = settings_for(ws[0], max_iters=6)
    a = gpu_solve_batched(ws, s, launch=dict(chunk_obs=2048, class_streams=1))
    b = gpu_solve_batched(ws, s, launch=dict(chunk_obs=2048, class_streams=0))
    for x, y in zip(a, b):
        assert np.array_equal(x["poses"], y["poses"]) and np.array_equal(x["points"], y["points"])
        assert x["report"].tobytes() == y["report"].tobytes()


def test_autotune_picks_a_valid_shape():
    import torch
    import paper_2506_04359_amd as ba
    ws = _windows()
    dev = torch.device("cuda:0")
    B = ba.Batch([ba.Window.from_problem(w, host_only=True) for w in ws])
    s = settings_for(ws[0], max_iters=5)
    P = torch.tensor(np.concatenate([w.poses_init for w in ws]), dtype=torch.float64, device=dev)
    L = torch.tensor(np.concatenate([w.points_init for w in ws]), dtype=torch.float64, device=dev)
    uv = torch.tensor(np.concatenate([w.obs_uv for w in ws]), dtype=torch.float64, device=dev)
    B.set_launch(1024)
    ws_bytes = B.workspace_size(s) + 256
    work = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    chunk = B.autotune(s, P.clone(), L.clone(), uv, None, work)
    cfg = B.get_launch()
    assert cfg["chunk_obs"] == chunk and chunk in (1024, 2048, 4096, 8192, 16384)
    assert cfg["tile_pairs"] in (0, 64) and cfg["class_streams"] in (0, 1)
    assert all(1 <= m <= 4 for m in cfg["class_chunk_mult"])
    assert B.workspace_size(s) <= ws_bytes
