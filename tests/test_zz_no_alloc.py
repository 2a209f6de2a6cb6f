"""ba_solve_noalloc (the solve on the library's per-device scratch) against
ba_solve with a caller workspace: the same kernels on the same plan, so the
results are equal bit for bit, on two calls in a row (the second on a smaller
window, so the scratch holds the first call's contents), and a window whose
workspace exceeds the scratch is refused before any device work."""
import numpy as np
import pytest

import bagen

pytestmark = pytest.mark.gpu


def _run(w, s, noalloc):
    import torch
    import paper_2506_04359_amd as ba
    dev = torch.device("cuda:0")
    W = ba.Window.from_problem(w)
    P = torch.tensor(w.poses_init, dtype=torch.float64, device=dev)
    L = torch.tensor(w.points_init, dtype=torch.float64, device=dev)
    uv = torch.tensor(w.obs_uv, dtype=torch.float64, device=dev)
    rep = torch.zeros(48, dtype=torch.uint8, device=dev)
    tr = torch.zeros(32 * s.max_iters, dtype=torch.uint8, device=dev)
    if noalloc:
        from paper_2506_04359_amd._binding import NOALLOC_SCRATCH_BYTES
        assert W.workspace_size(s) <= NOALLOC_SCRATCH_BYTES
        ba.solve_noalloc(W, s, P, L, uv, None, report=rep, trace=tr)
    else:
        ba.solve(W, s, P, L, uv, None, report=rep, trace=tr)
    torch.cuda.synchronize()
    return P.cpu().numpy(), L.cpu().numpy(), rep.cpu().numpy(), tr.cpu().numpy()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_equals_workspace_solve(precision):
    import paper_2506_04359_amd as ba
    from paper_2506_04359_amd._binding import REPORT_DTYPE
    prec = ba.BA_MIXED if precision == "mixed" else ba.BA_FP64
    big = bagen.make_window(2)          # stereo window, about 60k observations
    small = bagen.make_window(1)        # mono window, about 800 observations
    for w in (big, small):
        s = ba.Settings(max_iters=w.max_iters, precision=prec, lambda_init=w.lambda_init,
                        huber_delta=w.huber_delta)
        ref = _run(w, s, noalloc=False)
        got = _run(w, s, noalloc=True)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        r = np.frombuffer(got[2].tobytes(), dtype=REPORT_DTYPE)[0]
        assert r["status"] == 0 and r["final_cost"] < r["initial_cost"]


def test_noalloc_refuses_a_window_beyond_the_scratch():
    import torch
    import paper_2506_04359_amd as ba
    from paper_2506_04359_amd._binding import NOALLOC_SCRATCH_BYTES
    # 1.5M landmarks seen twice each by two poses: the FP64 workspace (24 B per
    # observation of packed observations alone) exceeds 64 MiB
    n_lm = 1_500_000
    obs_pose = np.tile(np.array([0, 1], np.int32), n_lm)
    obs_point = np.repeat(np.arange(n_lm, dtype=np.int32), 2)
    W = ba.Window(2, n_lm, obs_pose, obs_point, np.array([[400.0, 400.0, 320.0, 240.0]]))
    s = ba.Settings(max_iters=1, precision=ba.BA_FP64)
    assert W.workspace_size(s) > NOALLOC_SCRATCH_BYTES
    dev = torch.device("cuda:0")
    P = torch.zeros((2, 3, 4), dtype=torch.float64, device=dev)
    L = torch.zeros((n_lm, 3), dtype=torch.float64, device=dev)
    uv = torch.zeros((2 * n_lm, 2), dtype=torch.float64, device=dev)
    with pytest.raises(ba.BAError) as e:
        ba.solve_noalloc(W, s, P, L, uv)
    assert e.value.status == ba.BA_ERR_WORKSPACE_TOO_SMALL
    assert str(NOALLOC_SCRATCH_BYTES) in str(e.value)
