#!/usr/bin/env python3
"""Benchmark of the MI355X bundle adjuster.

One step = one batched mixed-precision LM solve (15 attempts per window) of
256 independent mono windows of uneven size (5-30 keyframes, 500-8000
landmarks, tracks of 2-10 frames, about 6.2M observations), replayed from a
HIP graph that also restores the initial state (two device-to-device copies).
Inputs are resident in HBM before the timed region.

Printed as one JSON line:
  value              LM attempts per second over all windows (whole job)
  obs_jacobians_per_s  n_obs * (1 + accepted) per window, per second
  plain_fp64         the same 256 windows solved one at a time in FP64 (ba_solve),
                     sequentially on one stream: LM attempts per second and the
                     speed-up of the batched mixed solve over it
  adjoint            64 windows of 10 keyframes / 2000 landmarks, forward solve
                     then the implicit-function adjoint: observations per second
  pnp                motion-only refinement of 4096 stereo frames (300 landmarks
                     each) and of 512 frames of the 32-camera rig: frames and
                     LM attempts per second
  local_map          a 50-keyframe stereo sequence through a 20-keyframe local map:
                     per keyframe the insertion, the plan rebuild and the solve
  visual_inertial    a 10-keyframe mono window with 200 Hz IMU samples: the
                     preintegration and the visual-inertial solve beside the
                     visual-only solve of the same window, with the trajectory's
                     scale against ground truth
  triangulation      every landmark of the 256 windows re-triangulated from its
                     observations (poses at ground truth): landmarks per second
  pgo                pose-graph optimisation of a 1500-pose, 2988-edge helix
                     (odometry and loop closures): LM attempts per second
  rms_check          final RMS of sampled windows against the FP64 oracle (1e-3 px)
  roofline           the linearise + Schur kernel (pass A) against the FP32 ALU peak
                     (pnp.*.roofline, triangulation.roofline: the motion-only and
                     triangulation kernels against the FP64 peak)
  cpu_baseline       the FP64 oracle on the host cores, on a bounded sample
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LM iters/s & obs-Jacobians/s, batched+adjoint vs plain FP64, at oracle RMS"
PEAK_FP32_TFLOPS = 157.3     # MI355X published FP32 vector peak
PEAK_VALU_FP64 = 78.6        # MI355X FP64 vector peak (also the FP32 rate without packed FP32)
# motion-only pass, per observation: x_b = X p (18), x_c (18), projection and
# residual (9), s (3), w rho and the cost sum (2), the rows of A R_c (20),
# w rho' (1), the two cross products (18), w J rows (12), U (21 x 4), g (6 x 4)
PNP_FLOPS_PER_OBS_PASS = 209
# triangulation, per observation with the world-to-camera transforms of a
# workgroup's poses composed in LDS (every workgroup of the benchmark batch): a
# pass x_c (18), projection and residual (9), s (3), w rho and the sum (2), the
# rows of A R_cw, the Jacobian (20), w rho' (1), w J (6), V (6 x 4), g (3 x 4);
# the ray start once: normalised pixel (4), ray direction and centre (33),
# normalisation (9), d.c (5), M and b (30)
TRI_FLOPS_PER_OBS_PASS = 95
TRI_FLOPS_PER_OBS_START = 81
# pose-graph edge: D^-1 T_i^-1 T_j (120), Log (60), J^-1 (60), the series of Q
# (about 8 terms of 3 3x3 products, 1300), M, N (240), B^T B (21 x 12), B^T r
# (72), |r|^2 (12)
PGO_FLOPS_PER_EDGE = 2100
N_WINDOWS = 256
ITERS = 15

# algorithmic flops of pass A, counted from the kernel source per unit of work:
#   per observation: transform (double) + projection + Huber + 2x6 / 2x3 Jacobians
#                    + the U, W, V, gradient block products          350
#   per free pair  : Z = W L^-T |D|^-1/2 (6 rows) + reduced rhs        90
#   per landmark   : sum of the pair blocks, damping, 3x3 L D L^T      60
#   per Schur block: off-diagonal 6x6 (36 x 3 FMA + scaling)          234
#                    diagonal (21 entries)                            144
FLOP_OBS, FLOP_FREE_PAIR, FLOP_LM, FLOP_BLK_OFF, FLOP_BLK_DIAG = 350, 90, 60, 234, 144


def pass_a_flops(infos):
    f = 0
    for i in infos:
        off = i["schur_blocks"] - i["n_free_pairs"]
        f += (FLOP_OBS * i["n_obs"] + FLOP_FREE_PAIR * i["n_free_pairs"] + FLOP_LM * i["n_points"]
              + FLOP_BLK_OFF * off + FLOP_BLK_DIAG * i["n_free_pairs"])
    return f


def _cpu_worker(job):
    """Oracle solve of one window (spawned process; no torch, one BLAS thread).
    job = (config, index): the window's generator and its index in the config."""
    import bagen
    import oracle
    cfg, index = job
    w = bagen.make_window(cfg, index)
    prob = oracle.Problem.from_window(w)
    st = oracle.LMSettings(max_iters=w.max_iters, lambda_init=w.lambda_init, huber_delta=w.huber_delta)
    t = time.perf_counter()
    res = oracle.lm_solve(w.poses_init, w.points_init, prob, st, backend="schur")
    dt = time.perf_counter() - t
    return cfg, index, dt, oracle.rms(res.poses, res.points, prob), res.poses, res.points


def cpu_pool(jobs):
    """Run the oracle jobs over the host cores: one process per window, one
    BLAS thread each; returns the results, the wall time and the process count."""
    import multiprocessing as mp
    procs = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    t = time.perf_counter()
    with ctx.Pool(procs) as pool:
        out = pool.map(_cpu_worker, jobs, chunksize=1)
    wall = time.perf_counter() - t
    return out, wall, procs


def host_description():
    """CPU model and the BLAS numpy links (for the CPU baseline)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = "unknown"
    try:
        import numpy as np
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        blas = f"{b.get('name', '?')} {b.get('version', '')}".strip()
    except Exception:
        pass
    return model, blas


def state_errors(P, L, prob, ref_poses, ref_rms, mono):
    """|dRMS| (px), largest rotation angle (rad) and largest relative translation
    error of one GPU result against the oracle's (after scale alignment about
    the first camera for mono windows)."""
    import numpy as np
    import oracle
    d_rms = abs(oracle.rms(P, L, prob) - ref_rms)
    if mono:
        P, L, _ = oracle.align_scale(P, L, ref_poses)
    ang, dt = oracle.rotation_errors(P, ref_poses)
    tn = np.maximum(np.linalg.norm(ref_poses[:, :, 3], axis=1), 1.0)
    return d_rms, float(ang.max()), float((dt / tn).max())


def kernels_sha():
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.hpp", "geometry.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2506_04359_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(per_launch_flops_units):
    """HBM bytes of one pass-A launch from the committed rocprofv3 counter
    summary, when it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pass_a_batch256_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernels_sha") != kernels_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 baseline")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-pnp", action="store_true", help="skip the motion-only frames")
    ap.add_argument("--no-tri", action="store_true", help="skip the triangulation leg")
    ap.add_argument("--no-pgo", action="store_true", help="skip the pose-graph leg")
    ap.add_argument("--chunk-obs", type=int, default=None,
                    help="fixed observations per work item instead of the autotuned value")
    ap.add_argument("--no-map", action="store_true", help="skip the sliding-window local map leg")
    ap.add_argument("--no-vi", action="store_true", help="skip the visual-inertial window leg")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-window legs (mono, stereo and rig windows)")
    ap.add_argument("--cpu-sample", type=int, default=N_WINDOWS,
                    help="windows of the batch solved by the oracle (all by default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import bagen
    import paper_2506_04359_amd as ba

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    ws = [bagen.make_window(3, i) for i in range(N_WINDOWS)]
    log(f"generated {N_WINDOWS} windows in {time.time() - t0:.1f}s, "
        f"{sum(w.n_obs for w in ws)} observations")
    wins = [ba.Window.from_problem(w, host_only=True) for w in ws]
    batch = ba.Batch(wins)
    infos = [batch.info(k) for k in range(N_WINDOWS)]
    n_obs = np.array([w.n_obs for w in ws])
    s_mixed = ba.Settings(max_iters=ITERS, precision=ba.BA_MIXED, lambda_init=1e-3, huber_delta=1.0)

    P0 = torch.tensor(np.concatenate([w.poses_init for w in ws]), dtype=torch.float64, device=dev)
    L0 = torch.tensor(np.concatenate([w.points_init for w in ws]), dtype=torch.float64, device=dev)
    uv = torch.tensor(np.concatenate([w.obs_uv for w in ws]), dtype=torch.float64, device=dev)
    P = P0.clone()
    L = L0.clone()
    reports = torch.zeros(48 * N_WINDOWS, dtype=torch.uint8, device=dev)

    chunk = None
    if args.chunk_obs is not None:
        batch.set_launch(args.chunk_obs)
        chunk = args.chunk_obs
        log(f"chunk_obs = {chunk} (fixed)")
    elif not args.no_tune:
        big = torch.empty(max(batch.workspace_size(s_mixed), 1), dtype=torch.uint8, device=dev)
        # room for the finest candidate shape
        batch.set_launch(1024)
        big = torch.empty(batch.workspace_size(s_mixed) + 256, dtype=torch.uint8, device=dev)
        chunk = batch.autotune(s_mixed, P, L, uv, None, big)
        del big
        log(f"autotuned launch shape: {batch.get_launch()}")
    ws_bytes = batch.workspace_size(s_mixed)
    work = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())

    def step():
        P.copy_(P0)
        L.copy_(L0)
        ba.solve_batched(batch, s_mixed, P, L, uv, None, work, reports)

    with torch.cuda.stream(side):
        step()                        # eager run before capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        step()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    for k in range(args.steps):
        graph.replay()
        log(f"step {k + 1}/{args.steps} enqueued")
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    rep = ba.parse_reports(reports)
    assert np.all(rep["iters"] == ITERS), rep["iters"]
    lm_iters_per_s = N_WINDOWS * ITERS / (ms_per_step / 1e3)
    obs_jac = float(np.sum(n_obs * (1 + rep["accepted"]))) / (ms_per_step / 1e3)
    log(f"batched mixed: {ms_per_step:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}), "
        f"{lm_iters_per_s:.4g} LM iters/s")
    P_final = P.cpu().numpy()
    L_final = L.cpu().numpy()

    # per-stage device times (HIP events on the launch stream), same solve
    P.copy_(P0)
    L.copy_(L0)
    stages = batch.profile_stages(s_mixed, P, L, uv, None, work, reports)
    pass_a_ms = stages["pass_a"] / ITERS
    flops = pass_a_flops(infos)
    achieved = flops / (pass_a_ms / 1e3) / 1e12
    log(f"stages (ms over {ITERS} attempts): {stages}")

    out = {
        "metric": METRIC, "value": lm_iters_per_s, "unit": "LM iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": bagen.WORKLOAD_NAMES[3], "windows": N_WINDOWS,
                   "observations": int(n_obs.sum()), "landmarks": int(sum(w.n_points for w in ws)),
                   "lm_attempts_per_window": ITERS, "precision": "mixed (FP32 bulk, FP64 Cholesky)",
                   "graph_captured": True, "chunk_obs": chunk, "launch": batch.get_launch()},
        "obs_jacobians_per_s": obs_jac,
        "stage_ms_per_attempt": {k: v / ITERS for k, v in stages.items()},
    }
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                       "traffic": traffic_from_profile(flops), "kernel": "k_pass_a<float,256>",
                       "flops_per_launch": flops, "avg_launch_ms": pass_a_ms}

    # plain FP64: one window at a time on one stream
    if not args.no_fp64:
        s64 = ba.Settings(max_iters=ITERS, precision=ba.BA_FP64, lambda_init=1e-3, huber_delta=1.0)
        singles = [ba.Window.from_problem(w) for w in ws]
        po = np.cumsum([0] + [w.n_poses for w in ws])
        lo = np.cumsum([0] + [w.n_points for w in ws])
        oo = np.cumsum([0] + [w.n_obs for w in ws])
        need = max(sw.workspace_size(s64) for sw in singles)
        w64 = torch.empty(need, dtype=torch.uint8, device=dev)
        rep64 = torch.zeros(48 * N_WINDOWS, dtype=torch.uint8, device=dev)
        Pw, Lw = P0.clone(), L0.clone()
        views = [(Pw[po[k]:po[k + 1]], Lw[lo[k]:lo[k + 1]], uv[oo[k]:oo[k + 1]], rep64[48 * k:48 * (k + 1)])
                 for k in range(N_WINDOWS)]
        for k in range(2):   # warm-up
            ba.solve(singles[k], s64, views[k][0], views[k][1], views[k][2], None, w64, views[k][3])
        Pw.copy_(P0)
        Lw.copy_(L0)
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record()
        for k in range(N_WINDOWS):
            ba.solve(singles[k], s64, views[k][0], views[k][1], views[k][2], None, w64, views[k][3])
        f1.record()
        torch.cuda.synchronize()
        ms64 = f0.elapsed_time(f1)
        r64 = ba.parse_reports(rep64)
        it64 = N_WINDOWS * ITERS / (ms64 / 1e3)
        out["plain_fp64"] = {"value": it64, "unit": "LM iters/s", "ms_total": ms64,
                             "obs_jacobians_per_s": float(np.sum(n_obs * (1 + r64["accepted"]))) / (ms64 / 1e3),
                             "speedup_batched_mixed": lm_iters_per_s / it64}
        log(f"plain FP64 sequential: {ms64:.1f} ms, {it64:.4g} LM iters/s")
        P64, L64 = Pw.cpu().numpy(), Lw.cpu().numpy()
        del singles

    # single windows: the mono window (5 keyframes), the stereo window (20
    # keyframes, 2 cameras) and the 32-camera rig, each solved alone in mixed
    # and in FP64 precision, replayed from a HIP graph
    singles_out = {}
    if not args.no_single:
        for cfg in (1, 2, 4):
            w = bagen.make_window(cfg)
            name = bagen.WORKLOAD_NAMES[cfg]
            win = ba.Window.from_problem(w)
            one = ba.Batch([ba.Window.from_problem(w, host_only=True)])
            Ps0 = torch.tensor(w.poses_init, dtype=torch.float64, device=dev)
            Ls0 = torch.tensor(w.points_init, dtype=torch.float64, device=dev)
            uvs = torch.tensor(w.obs_uv, dtype=torch.float64, device=dev)
            leg = {"observations": int(w.n_obs), "landmarks": int(w.n_points), "poses": int(w.n_poses),
                   "cameras": int(w.n_cams), "free_poses": int(np.sum(w.pose_fixed == 0)),
                   "lm_attempts": int(w.max_iters),
                   "precision_of_config": "mixed" if w.mixed else "fp64"}
            for pname, prec in (("mixed", ba.BA_MIXED), ("fp64", ba.BA_FP64)):
                ss = ba.Settings(max_iters=w.max_iters, precision=prec, lambda_init=w.lambda_init,
                                 huber_delta=w.huber_delta)
                Ps, Ls = Ps0.clone(), Ls0.clone()
                wk = torch.empty(max(win.workspace_size(ss), 256), dtype=torch.uint8, device=dev)
                rp = torch.zeros(48, dtype=torch.uint8, device=dev)

                def sstep():
                    Ps.copy_(Ps0)
                    Ls.copy_(Ls0)
                    ba.solve(win, ss, Ps, Ls, uvs, None, wk, rp)

                with torch.cuda.stream(side):
                    sstep()
                torch.cuda.synchronize()
                sg = torch.cuda.CUDAGraph()
                with torch.cuda.graph(sg, stream=side):
                    sstep()
                torch.cuda.synchronize()
                for _ in range(args.warmup):
                    sg.replay()
                torch.cuda.synchronize()
                c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                c0.record()
                for _ in range(args.steps):
                    sg.replay()
                c1.record()
                torch.cuda.synchronize()
                ms_s = c0.elapsed_time(c1) / args.steps
                rr = ba.parse_reports(rp)[0]
                d = {"ms_per_solve": ms_s, "lm_iters_per_s": w.max_iters / (ms_s / 1e3),
                     "obs_jacobians_per_s": w.n_obs * (1 + int(rr["accepted"])) / (ms_s / 1e3),
                     "accepted": int(rr["accepted"]), "final_cost": float(rr["final_cost"]),
                     "poses": Ps.cpu().numpy(), "points": Ls.cpu().numpy()}
                # pass A of this window alone, its device time per attempt
                Ps.copy_(Ps0)
                Ls.copy_(Ls0)
                wk1 = torch.empty(max(one.workspace_size(ss), 256), dtype=torch.uint8, device=dev)
                st1 = one.profile_stages(ss, Ps, Ls, uvs, None, wk1, rp)
                pa_ms = st1["pass_a"] / w.max_iters
                fl = pass_a_flops([one.info(0)])
                peak = PEAK_FP32_TFLOPS if prec == ba.BA_MIXED else PEAK_VALU_FP64
                d["stage_ms_per_attempt"] = {k: v / w.max_iters for k, v in st1.items()}
                d["roofline"] = {"bound": "alu", "achieved": fl / (pa_ms / 1e3) / 1e12, "peak": peak,
                                 "unit": "TFLOP/s", "frac": fl / (pa_ms / 1e3) / 1e12 / peak,
                                 "traffic": None,
                                 "kernel": "k_pass_a<float>" if prec == ba.BA_MIXED else "k_pass_a<double>",
                                 "flops_per_launch": fl, "avg_launch_ms": pa_ms}
                leg[pname] = d
                del sg
            leg["speedup_mixed_over_fp64"] = leg["fp64"]["ms_per_solve"] / leg["mixed"]["ms_per_solve"]
            singles_out[cfg] = (name, w, leg)
            log(f"{name}: mixed {leg['mixed']['ms_per_solve']:.3f} ms, fp64 {leg['fp64']['ms_per_solve']:.3f} ms "
                f"per {w.max_iters}-attempt solve")
            del win, one

    # the sliding-window local map: a stereo keyframe sequence through a
    # 20-keyframe window, each keyframe inserted (slide, new landmarks and
    # observations, device gather), the window's plan rebuilt on the host and
    # the window solved (mixed, 10 attempts)
    if not args.no_map:
        seq = bagen.make_stereo_sequence(n_keyframes=50, births=250, seed=11100)
        NW = 20
        mp = ba.Map(NW, seq.intrinsics, seq.extrinsics.reshape(-1, 12))
        sm = ba.Settings(max_iters=10, precision=ba.BA_MIXED, lambda_init=1e-3, huber_delta=1.0)
        wsm = torch.empty(256, dtype=torch.uint8, device=dev)
        rows = []
        for i, kf in enumerate(seq.keyframes):
            kfi = np.full(kf.obs_lm.shape[0], min(i + 1, NW) - 1, np.int32)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mp.add_keyframe(kf.pose_init, kf.new_ids, kf.new_points, kfi, kf.obs_lm, kf.obs_cam, kf.obs_uv)
            t1 = time.perf_counter()
            if i == 0:
                continue
            Wm = mp.window()
            t2 = time.perf_counter()
            need = Wm.workspace_size(sm)
            if wsm.numel() < need:
                wsm = torch.empty(2 * need, dtype=torch.uint8, device=dev)
            torch.cuda.synchronize()
            m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t3 = time.perf_counter()
            m0.record()
            mp.solve(sm, workspace=wsm)
            m1.record()
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            K_, M_, n_ = mp.info()
            rows.append((t1 - t0, t2 - t1, m0.elapsed_time(m1) / 1e3, t4 - t3, K_, M_, n_))
        steady = [r for r in rows if r[4] == NW]
        A = np.array([r[:4] for r in steady])
        per_kf = float(A[:, 0].mean() + A[:, 1].mean() + A[:, 3].mean())
        out["local_map"] = {
            "workload": "stereo-sequence-50kf-window20", "keyframes": len(seq.keyframes), "window": NW,
            "steady_keyframes": len(steady), "mean_points": float(np.mean([r[5] for r in steady])),
            "mean_observations": float(np.mean([r[6] for r in steady])),
            "insert_ms": 1e3 * float(A[:, 0].mean()), "plan_ms": 1e3 * float(A[:, 1].mean()),
            "solve_ms": 1e3 * float(A[:, 2].mean()), "solve_wall_ms": 1e3 * float(A[:, 3].mean()),
            "keyframes_per_s": 1.0 / per_kf, "lm_attempts_per_window": 10, "precision": "mixed"}
        log(f"local map: insert {out['local_map']['insert_ms']:.2f} ms, plan {out['local_map']['plan_ms']:.2f} ms, "
            f"solve {out['local_map']['solve_ms']:.2f} ms per keyframe ({out['local_map']['mean_observations']:.0f} obs)")
        del mp

    # visual-inertial window (Eq. 9): 10 keyframes 0.25 s apart, 400 landmarks,
    # 200 Hz IMU samples; the preintegration of its 9 factors, the VI solve and
    # the visual-only solve of the same window (10 attempts each), replayed
    # from HIP graphs that restore the initial state
    if not args.no_vi:
        vw = bagen.make_vi_window(seed=9300, n_kf=10, n_lm=400)
        wv = vw.window
        winv = ba.Window.from_problem(wv)
        nkf = wv.n_poses
        tv = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        sbv = tv(np.concatenate([[0], np.cumsum([g.shape[0] for g in vw.gyro])]), torch.int32)
        gyv, acv = tv(np.concatenate(vw.gyro)), tv(np.concatenate(vw.accel))
        bbv = tv(np.tile(np.concatenate([vw.ba_init[0], vw.bg_init[0]]), (nkf - 1, 1)))
        pre = torch.empty((nkf - 1, ba.VI_PREINT_DOUBLES), dtype=torch.float64, device=dev)
        Pv0, Lv0, uvv = tv(wv.poses_init), tv(wv.points_init), tv(wv.obs_uv)
        Xv0 = tv(np.concatenate([vw.vel_init, vw.ba_init, vw.bg_init], axis=1))
        Pv, Lv, Xv = Pv0.clone(), Lv0.clone(), Xv0.clone()
        vi_out = {"workload": f"vi-mono-{nkf}kf-{wv.n_points}lm-200hz", "observations": int(wv.n_obs),
                  "landmarks": int(wv.n_points), "keyframes": nkf, "imu_samples": int(gyv.shape[0]),
                  "lm_attempts": 10}

        def graph_ms(fn):
            with torch.cuda.stream(side):
                fn()
            torch.cuda.synchronize()
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr, stream=side):
                fn()
            torch.cuda.synchronize()
            for _ in range(args.warmup):
                gr.replay()
            torch.cuda.synchronize()
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record()
            for _ in range(args.steps):
                gr.replay()
            c1.record()
            torch.cuda.synchronize()
            return c0.elapsed_time(c1) / args.steps

        def centres(Pn):
            return -np.einsum("kji,kj->ki", Pn[:, :, :3], Pn[:, :, 3])

        cg = centres(wv.poses_gt)
        vi_out["preintegrate_ms"] = graph_ms(lambda: ba.vi_preintegrate(sbv, gyv, acv, vw.dt, bbv, vw.noise, out=pre))
        for pname, prec in (("mixed", ba.BA_MIXED), ("fp64", ba.BA_FP64)):
            sv = ba.Settings(max_iters=10, precision=prec, lambda_init=1e-3, huber_delta=1.0)
            wkv = torch.empty(ba.vi_workspace_size(winv, sv), dtype=torch.uint8, device=dev)
            wko = torch.empty(max(winv.workspace_size(sv), 256), dtype=torch.uint8, device=dev)
            rpv = torch.zeros(48, dtype=torch.uint8, device=dev)
            rpo = torch.zeros(48, dtype=torch.uint8, device=dev)

            def vstep():
                Pv.copy_(Pv0)
                Lv.copy_(Lv0)
                Xv.copy_(Xv0)
                ba.vi_solve(winv, sv, pre, vw.gravity, Pv, Lv, Xv, uvv, None, wkv, rpv)

            def ostep():
                Pv.copy_(Pv0)
                Lv.copy_(Lv0)
                ba.solve(winv, sv, Pv, Lv, uvv, None, wko, rpo)

            d = {"vi_ms_per_solve": graph_ms(vstep)}
            Pn = Pv.cpu().numpy()
            rr = ba.parse_reports(rpv)[0]
            c = centres(Pn)
            d["vi_accepted"] = int(rr["accepted"])
            d["vi_scale"] = float(np.linalg.norm(c[-1] - c[0]) / np.linalg.norm(cg[-1] - cg[0]))
            d["vi_centre_rms_m"] = float(np.sqrt(np.mean(np.sum((c - cg) ** 2, axis=1))))
            d["vi_velocity_rms"] = float(np.sqrt(np.mean((Xv[:, :3].cpu().numpy() - vw.vel_gt) ** 2)))
            d["visual_ms_per_solve"] = graph_ms(ostep)
            c = centres(Pv.cpu().numpy())
            d["visual_scale"] = float(np.linalg.norm(c[-1] - c[0]) / np.linalg.norm(cg[-1] - cg[0]))
            d["visual_centre_rms_m"] = float(np.sqrt(np.mean(np.sum((c - cg) ** 2, axis=1))))
            vi_out[pname] = d
        out["visual_inertial"] = vi_out
        log(f"visual-inertial: preintegration {vi_out['preintegrate_ms']:.3f} ms; mixed VI "
            f"{vi_out['mixed']['vi_ms_per_solve']:.3f} ms vs visual {vi_out['mixed']['visual_ms_per_solve']:.3f} ms "
            f"per 10-attempt solve; scale {vi_out['mixed']['vi_scale']:.4f} (VI) vs "
            f"{vi_out['mixed']['visual_scale']:.4f} (visual)")
        del winv

    # adjoint on 64 windows of 10 keyframes / 2000 landmarks
    if not args.no_adjoint:
        wa = [bagen.make_window(5, i) for i in range(64)]
        ba_wins = [ba.Window.from_problem(w, host_only=True) for w in wa]
        badj = ba.Batch(ba_wins)
        sa = ba.Settings(max_iters=50, precision=ba.BA_MIXED, lambda_init=1e-3, huber_delta=1.0)
        Pa = torch.tensor(np.concatenate([w.poses_init for w in wa]), dtype=torch.float64, device=dev)
        La = torch.tensor(np.concatenate([w.points_init for w in wa]), dtype=torch.float64, device=dev)
        uva = torch.tensor(np.concatenate([w.obs_uv for w in wa]), dtype=torch.float64, device=dev)
        Pgt = torch.tensor(np.concatenate([w.poses_gt for w in wa]), dtype=torch.float64, device=dev)
        free = torch.tensor(np.concatenate([1 - w.pose_fixed for w in wa]), dtype=torch.float64, device=dev)
        wsa = torch.empty(badj.workspace_size(sa), dtype=torch.uint8, device=dev)
        ba.solve_batched(badj, sa, Pa, La, uva, None, wsa)
        gP = (2.0 * (Pa - Pgt) * free[:, None, None]).contiguous()     # chordal loss gradient
        guv = torch.empty_like(uva)
        gw = torch.empty(uva.shape[0], dtype=torch.float64, device=dev)
        ba.adjoint(badj, sa, Pa, La, uva, None, gP, None, guv, gw, wsa)
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(args.steps):
            ba.adjoint(badj, sa, Pa, La, uva, None, gP, None, guv, gw, wsa)
        a1.record()
        torch.cuda.synchronize()
        ms_adj = a0.elapsed_time(a1) / args.steps
        nobs_a = sum(w.n_obs for w in wa)
        out["adjoint"] = {"workload": bagen.WORKLOAD_NAMES[5], "windows": 64, "observations": nobs_a,
                          "ms_per_call": ms_adj, "obs_per_s": nobs_a / (ms_adj / 1e3),
                          "windows_per_s": 64 / (ms_adj / 1e3),
                          "finite": bool(torch.isfinite(guv).all().item())}
        log(f"adjoint: {ms_adj:.3f} ms for {nobs_a} observations")

    # motion-only frames (stereo PnP refinement and the 32-camera rig)
    if not args.no_pnp:
        out["pnp"] = {}
        for name in ("pnp-4096x-stereo-300lm", "pnp-512x-rig32-400lm"):
            pb = bagen.make_pnp_workload(name)
            rig = ba.Rig(pb.intrinsics, pb.extrinsics.reshape(-1, 12))
            sp = ba.Settings(max_iters=pb.max_iters, precision=ba.BA_MIXED, lambda_init=pb.lambda_init,
                             huber_delta=pb.huber_delta)
            tt = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
            PP0 = tt(pb.poses_init, torch.float64)
            PP = PP0.clone()
            fb, pts = tt(pb.frame_obs_begin, torch.int32), tt(pb.points, torch.float64)
            op, oc, ouv = tt(pb.obs_point, torch.int32), tt(pb.obs_cam, torch.int32), tt(pb.obs_uv, torch.float64)
            prep = torch.zeros(48 * pb.n_frames, dtype=torch.uint8, device=dev)
            for _ in range(2):
                PP.copy_(PP0)
                ba.pnp_solve(rig, sp, fb, PP, pts, op, ouv, obs_cam=oc, reports=prep)
            torch.cuda.synchronize()
            # one event pair per call on the launch stream; the pose restore
            # between calls is outside the timed spans
            evs = []
            for _ in range(args.steps):
                PP.copy_(PP0)
                b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                b0.record()
                ba.pnp_solve(rig, sp, fb, PP, pts, op, ouv, obs_cam=oc, reports=prep)
                b1.record()
                evs.append((b0, b1))
            torch.cuda.synchronize()
            ms_p = sum(a.elapsed_time(b) for a, b in evs) / args.steps
            pr = ba.parse_reports(prep)[: pb.n_frames]
            n_f = np.diff(pb.frame_obs_begin).astype(np.float64)
            # every pass linearises: the first, then one per attempt whose
            # Cholesky succeeded
            passes = 1 + pr["iters"].astype(np.float64) - pr["chol_failures"]
            flops = float(np.sum(n_f * passes)) * PNP_FLOPS_PER_OBS_PASS
            out["pnp"][name] = {"frames": pb.n_frames, "observations": pb.n_obs,
                                "lm_attempts_per_frame": pb.max_iters, "ms_per_call": ms_p,
                                "frames_per_s": pb.n_frames / (ms_p / 1e3),
                                "lm_iters_per_s": pb.n_frames * pb.max_iters / (ms_p / 1e3),
                                "obs_jacobians_per_s": float(np.sum(n_f * (1 + pr["accepted"]))) / (ms_p / 1e3),
                                "all_reduced": bool(np.all(pr["final_cost"] < pr["initial_cost"])),
                                "roofline": {"bound": "alu", "achieved": flops / (ms_p * 1e-3) / 1e12,
                                             "peak": PEAK_VALU_FP64, "unit": "TFLOP/s",
                                             "frac": flops / (ms_p * 1e-3) / 1e12 / PEAK_VALU_FP64,
                                             "traffic": None, "kernel": "k_pnp",
                                             "flops_per_launch": flops, "avg_launch_ms": ms_p}}
            log(f"{name}: {ms_p:.3f} ms for {pb.n_frames} frames ({pb.n_obs} observations)")
            del rig

    # triangulation of every landmark of the 256 windows from its observations,
    # poses at ground truth
    if not args.no_tri:
        tb = bagen.make_tri_batch(ws, max_iters=10)
        rig = ba.Rig(tb.intrinsics, tb.extrinsics.reshape(-1, 12))
        st = ba.Settings(max_iters=tb.max_iters, precision=ba.BA_MIXED, lambda_init=tb.lambda_init,
                         huber_delta=tb.huber_delta)
        tt = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        targs = (tt(tb.point_obs_begin, torch.int32), tt(tb.poses.reshape(-1, 12), torch.float64),
                 tt(tb.obs_pose, torch.int32), tt(tb.obs_uv, torch.float64))
        tpts = torch.empty((tb.n_points, 3), dtype=torch.float64, device=dev)
        toc = tt(tb.obs_cam, torch.int32)
        trep = torch.zeros(48 * tb.n_points, dtype=torch.uint8, device=dev)
        for _ in range(2):
            ba.triangulate(rig, st, *targs, tpts, obs_cam=toc, reports=trep)
        torch.cuda.synchronize()
        b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b0.record()
        for _ in range(args.steps):
            ba.triangulate(rig, st, *targs, tpts, obs_cam=toc, reports=trep)
        b1.record()
        torch.cuda.synchronize()
        ms_t = b0.elapsed_time(b1) / args.steps
        tr_ = ba.parse_reports(trep)[: tb.n_points]
        n_l = np.diff(tb.point_obs_begin).astype(np.float64)
        ok = tr_["status"] == 0
        passes = np.where(ok, 1 + tr_["iters"].astype(np.float64) - tr_["chol_failures"], 0.0)
        flops = float(np.sum(n_l * (passes * TRI_FLOPS_PER_OBS_PASS + TRI_FLOPS_PER_OBS_START)))
        out["triangulation"] = {
            "workload": "tri-256x-mono-uneven", "landmarks": tb.n_points, "observations": tb.n_obs,
            "lm_attempts_per_landmark": tb.max_iters, "ms_per_call": ms_t,
            "landmarks_per_s": tb.n_points / (ms_t / 1e3), "obs_per_s": tb.n_obs / (ms_t / 1e3),
            "refined_fraction": float(ok.mean()),
            "roofline": {"bound": "alu", "achieved": flops / (ms_t * 1e-3) / 1e12, "peak": PEAK_VALU_FP64,
                         "unit": "TFLOP/s", "frac": flops / (ms_t * 1e-3) / 1e12 / PEAK_VALU_FP64,
                         "traffic": None, "kernel": "k_tri", "flops_per_launch": flops,
                         "avg_launch_ms": ms_t}}
        log(f"triangulation: {ms_t:.3f} ms for {tb.n_points} landmarks ({tb.n_obs} observations)")
        del rig

    # pose-graph optimisation of the 1500-pose helix
    if not args.no_pgo:
        pg = bagen.make_pgo_workload("pgo-helix-3x500")
        graph = ba.Graph(pg.n_poses, pg.edge_i, pg.edge_j, pg.pose_fixed)
        sg = ba.Settings(max_iters=pg.max_iters, precision=ba.BA_FP64, lambda_init=pg.lambda_init)
        P0g = torch.tensor(pg.poses_init.reshape(-1, 12), dtype=torch.float64, device=dev)
        Pg = P0g.clone()
        Dg = torch.tensor(pg.deltas.reshape(-1, 12), dtype=torch.float64, device=dev)
        wsz = graph.workspace_size()
        wsg_raw = torch.empty(wsz + 256, dtype=torch.uint8, device=dev)
        o = (-wsg_raw.data_ptr()) % 256
        wsg = wsg_raw[o:o + wsz]
        rg = torch.zeros(48, dtype=torch.uint8, device=dev)

        def pgo_step():
            Pg.copy_(P0g)
            ba.pgo_solve(graph, sg, Pg, Dg, wsg, report=rg)

        # one solve is about 700 small launches: replay it from a HIP graph
        # (restore of the poses included), as the window step is
        with torch.cuda.stream(side):
            pgo_step()
        torch.cuda.synchronize()
        ggraph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(ggraph, stream=side):
            pgo_step()
        torch.cuda.synchronize()
        for _ in range(2):
            ggraph.replay()
        torch.cuda.synchronize()
        b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b0.record()
        for _ in range(args.steps):
            ggraph.replay()
        b1.record()
        torch.cuda.synchronize()
        ms_g = b0.elapsed_time(b1) / args.steps
        rep_g = ba.parse_reports(rg)[0]
        info = graph.info()
        plan = ba.Graph(pg.n_poses, pg.edge_i, pg.edge_j, pg.pose_fixed, host_only=True).plan()
        n_upd = int(plan["upd_ptr"][-1])
        n_offd = info["n_blocks"] - info["n_free"]
        # per attempt: the edges at the candidate, the factorisation (updates
        # 432, diagonal blocks 182, panel rows 6 x 36), forward and back
        # substitution (72 per block each)
        flops_att = (pg.n_edges * PGO_FLOPS_PER_EDGE + n_upd * 432 + info["n_free"] * 182
                     + n_offd * 6 * 36 + info["n_blocks"] * 144)
        flops_g = flops_att * pg.max_iters
        out["pgo"] = {"workload": "pgo-helix-3x500", "poses": pg.n_poses, "edges": pg.n_edges,
                      "free_poses": info["n_free"], "factor_blocks": info["n_blocks"],
                      "tree_levels": info["n_levels"], "lm_attempts": pg.max_iters, "ms_per_solve": ms_g,
                      "graph_captured": True,
                      "lm_iters_per_s": pg.max_iters / (ms_g / 1e3),
                      "edges_per_s": pg.n_edges * (1 + pg.max_iters) / (ms_g / 1e3),
                      "initial_cost": float(rep_g["initial_cost"]), "final_cost": float(rep_g["final_cost"]),
                      "roofline": {"bound": "alu", "achieved": flops_g / (ms_g * 1e-3) / 1e12,
                                   "peak": PEAK_VALU_FP64, "unit": "TFLOP/s",
                                   "frac": flops_g / (ms_g * 1e-3) / 1e12 / PEAK_VALU_FP64, "traffic": None,
                                   "kernel": "k_pgo_* (one solve)", "flops_per_launch": flops_g,
                                   "avg_launch_ms": ms_g}}
        log(f"pgo: {ms_g:.3f} ms per solve ({pg.n_poses} poses, {pg.n_edges} edges, "
            f"{info['n_levels']} levels)")
        del ggraph, graph

    # the oracle on the host: every window of the batch (and the single
    # windows), one process per window; the RMS check of every result
    sample = list(range(min(args.cpu_sample, N_WINDOWS)))
    if not args.no_cpu:
        import oracle
        jobs = [(3, k) for k in sample]
        res, wall_cpu, procs = cpu_pool(jobs)
        iters_cpu = len(sample) * ITERS / wall_cpu
        po = np.cumsum([0] + [w.n_poses for w in ws])
        lo = np.cumsum([0] + [w.n_points for w in ws])
        tol = {"drms_px": 1e-3, "rot_rad": 1e-4, "trans_rel": 1e-4}
        worst = {"mixed": [0.0, 0.0, 0.0], "plain_fp64": [0.0, 0.0, 0.0]}
        drms_mixed_fp64 = 0.0
        for cfg, idx, dt, rms_o, Po, Lo in res:
            w = ws[idx]
            prob = oracle.Problem.from_window(w)
            sl_p, sl_l = slice(po[idx], po[idx + 1]), slice(lo[idx], lo[idx + 1])
            results = {"mixed": (P_final[sl_p], L_final[sl_l])}
            if not args.no_fp64:
                results["plain_fp64"] = (P64[sl_p], L64[sl_l])
                drms_mixed_fp64 = max(drms_mixed_fp64, abs(oracle.rms(*results["mixed"], prob)
                                                           - oracle.rms(*results["plain_fp64"], prob)))
            for key, (Pg, Lg) in results.items():
                e = state_errors(Pg, Lg, prob, Po, rms_o, mono=True)
                worst[key] = [max(a, b) for a, b in zip(worst[key], e)]
        chk = {"windows": len(sample), "tol": tol}
        ok = True
        for key, (a, b, c) in worst.items():
            if key == "plain_fp64" and args.no_fp64:
                continue
            passed = a <= tol["drms_px"] and b <= tol["rot_rad"] and c <= tol["trans_rel"]
            ok = ok and passed
            chk[key] = {"max_abs_drms_px": a, "max_rot_err_rad": b, "max_trans_err_rel": c, "pass": passed}
        chk["pass"] = ok
        out["rms_check"] = chk
        if "plain_fp64" in out:
            out["plain_fp64"]["max_abs_drms_vs_mixed_px"] = drms_mixed_fp64
        model, blas = host_description()
        out["cpu_baseline"] = {"value": iters_cpu, "unit": "LM iters/s", "cores": procs,
                               "kind": "oracle",
                               "sample": f"windows 0-{len(sample) - 1} of the 256, {ITERS} LM attempts each, "
                                         f"block-Schur FP64 oracle, one process per window, one BLAS thread",
                               "cpu_model": model, "blas": blas, "wall_s": wall_cpu}
        log(f"cpu oracle: {wall_cpu:.1f}s for {len(sample)} windows on {procs} processes; check {chk}")
        # the single windows against their own oracle solves
        if singles_out:
            sres, swall, _ = cpu_pool([(cfg, 0) for cfg in singles_out])
            for cfg, _, dt, rms_o, Po, Lo in sres:
                name, w, leg = singles_out[cfg]
                prob = oracle.Problem.from_window(w)
                for pname in ("mixed", "fp64"):
                    d = leg[pname]
                    a, b, c = state_errors(d["poses"], d["points"], prob, Po, rms_o, mono=(w.n_cams == 1))
                    d["vs_oracle"] = {"abs_drms_px": a, "rot_err_rad": b, "trans_err_rel": c,
                                      "pass": bool(a <= 1e-3 and b <= 1e-4 and c <= 1e-4)}
                leg["oracle_s"] = dt
                leg["oracle_rms_px"] = rms_o
    for cfg, (name, w, leg) in singles_out.items():
        for pname in ("mixed", "fp64"):
            leg[pname].pop("poses", None)
            leg[pname].pop("points", None)
        out.setdefault("single_windows", {})[name] = leg
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
