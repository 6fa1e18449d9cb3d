#!/usr/bin/env python3
"""Throughput of the VOLDOR window solver on one MI355X.

Default workload (the headline): a batch of 32 windows of uneven shape and T
(320x240, 640x480 and 1242x375, T from 4 to 8, 4 EM iterations, 1024 / 2048 /
4096 P3P groups per frame by shape), solved by voldor_window_batch over
concurrent streams in one HIP graph per step, flows resident in device memory.
One step = the whole batch: for every window the bootstrap, then every EM
iteration (pose of each frame, the directional depth/rigidness sweeps, the
unsmoothed rigidness and the gauge), finally the log-likelihood.

Metric: pixel-frame EM updates/s = sum over windows of T*H*W*n_iters per
second.  Windows/s is reported beside it, and the indoor (T=6, 640x480) and
driving (T=8, 1242x375) single windows as sub-objects.  --workload indoor,
driving, small time one window shape alone; learned, vo and resfit the
extensions.

Roofline: the dominant kernel, the fused directional sweep, against HBM:
algorithmic bytes per launch = the flow stack read once (8 B per pixel-frame)
plus the depth read and written (8 B per pixel), divided by the mean launch
duration from device timestamps written on the stream each launch runs on (a
one-thread kernel reading the real-time counter at each phase boundary; unlike
HIP events it also runs inside the captured graph).  Its ALU view
beside it counts 3 candidate-frame evaluations x (8 transcendental + 50 FP32)
operations per pixel-frame and sweep against the FP32 peak.  The cpu_baseline
object times the FP64 CPU oracle on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of one sweep launch on the indoor workload, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) scaled by what the same
# counters read for a plain 256 MiB copy (x2.000 and x1.000); valid only while
# the sweep kernel's sources hash to SWEEP_SOURCES_SHA (profile:
# profiles/k_sweep_hbm_traffic.md)
SWEEP_TRAFFIC_INDOOR = {"fetch_bytes": 44.90e6, "write_bytes": 1.23e6}
SWEEP_SOURCES_SHA = "cae795f93c1e31cf"
SWEEP_SOURCES = ("vo_sweep.hip", "vo_device.hpp")   # the sweep's device code
# Issue peak of non-packed FP32 VALU lane-instructions: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz = 39.3 T/s; the all-pixel candidate scoring (--pose-start
# allpixel) is bound by it and reported against it.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def _sweep_traffic(workload):
    """Measured HBM bytes per sweep launch, or None if not measured for this
    workload or if the kernel changed since the counters were taken."""
    if workload != "indoor" or _sweep_sources_sha() != SWEEP_SOURCES_SHA:
        return None
    return SWEEP_TRAFFIC_INDOOR["fetch_bytes"] + SWEEP_TRAFFIC_INDOOR["write_bytes"]


def _sweep_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_06789_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# HBM traffic of one residual-binning pass (k_resid_bins + k_resid_reduce) on the
# indoor window flows, 40 bins: FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
# scaled by the copy calibration above; valid while vo_resfit.hip hashes to
# RESFIT_SOURCE_SHA (profile: profiles/k_resid_bins_indoor_hbm_traffic.md)
RESFIT_TRAFFIC = ((14454.046875 + 1140.5) * 1.99980 + 1125.0 + 1.25) * 1024
RESFIT_SOURCE_SHA = "40f42a8ae96ba6f1"


def _resfit_traffic():
    import hashlib
    with open(os.path.join(ROOT, "paper_2104_06789_amd", "csrc", "vo_resfit.hip"), "rb") as fh:
        ok = hashlib.sha256(fh.read()).hexdigest()[:16] == RESFIT_SOURCE_SHA
    return RESFIT_TRAFFIC if ok else None


CAND_EVAL_VALU_OPS = 46    # one (candidate, pixel) evaluation of k_cand_score: 1484 of the 1676 VALU
                           # instructions of its 32-evaluation candidate loop are not transcendental


def _cumulative(rel):
    import numpy as np
    M = [np.concatenate([np.eye(3).ravel(), np.zeros(3)])]
    for r in np.asarray(rel, dtype=np.float64).reshape(-1, 12):
        R, t = r[:9].reshape(3, 3), r[9:]
        Rm, tm = M[-1][:9].reshape(3, 3), M[-1][9:]
        M.append(np.concatenate([(R @ Rm).ravel(), R @ tm + t]))
    return np.array(M)


def _allpixel_roofline(vo, torch, solver, w, spec, p_ap, out, reps=3):
    """Live figure of the all-pixel candidate scoring (k_cand_score): every
    frame's pose step at the window's final state, through the step entry point
    on the current stream, timed with HIP events once with the all-pixel start
    and once with the KDE start; the difference is the scoring's time, and the
    candidates x pixels it scored come from the step's own score list."""
    import numpy as np
    T, H, W = spec.T, spec.H, spec.W
    poses = out[0].cpu().numpy()
    M = _cumulative(poses)
    p_kde = vo.default_params(n_iters=spec.n_iters, n_pose_groups=spec.n_groups, seed=p_ap.seed,
                              criterion=p_ap.criterion, pose_start=0, residual_model=p_ap.residual_model)
    flows = torch.from_numpy(w["flows"]).cuda()
    ms = {0: 0.0, 1: 0.0}
    evals = 0
    for rep in range(reps + 1):
        for t in range(1, T + 1):
            for key, pp in ((1, p_ap), (0, p_kde)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                solver.pose_step(out[1], out[2], flows, w["K"], pp, M, t, spec.n_iters - 1, prevT=poses[t - 1])
                e1.record()
                torch.cuda.synchronize()
                if rep > 0:   # the first pass warms up
                    ms[key] += e0.elapsed_time(e1)
                    if key == 1:
                        evals += len(solver.pose_scores()) * H * W
    launches = reps * T
    launch_ms = (ms[1] - ms[0]) / launches
    ops = evals / launches * CAND_EVAL_VALU_OPS
    achieved = ops / (launch_ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": "k_cand_score", "achieved": achieved, "peak": VALU_PEAK_TOPS,
            "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
            "alg_ops_per_launch": ops, "evals_per_launch": evals / launches, "launch_ms": launch_ms,
            "note": "k_cand_score time = pose step with the all-pixel start minus the same step with the "
                    "KDE start, HIP events on the stream; ops = candidates x pixels x 46 non-transcendental VALU instructions"}


def _pose_error(poses, gt):
    import numpy as np
    rot, tdir = [], []
    for k, (R, t) in enumerate(gt):
        Re = poses[k, :9].reshape(3, 3)
        te = poses[k, 9:]
        c = (np.trace(Re @ R.T) - 1) / 2
        rot.append(math.acos(max(-1.0, min(1.0, c))))
        ct = te @ t / (np.linalg.norm(te) * np.linalg.norm(t))
        tdir.append(math.acos(max(-1.0, min(1.0, ct))))
    return float(np.mean(rot)), float(np.mean(tdir))


BATCH_ITERS = 4
# lanes of the batch workload per mode.  A replayed graph runs the work of at
# most four lanes at once here (device timestamps: lanes 4-7 of eight start as
# lanes 0-3 end, also with eight hardware queues), so more lanes only split the
# batch into rounds, each with its own bootstrap and first pose steps; measured
# on one box, lockstep: 2 lanes 30.3 ms per step, 3 lanes 28.7, 4 lanes 27.6,
# 5 lanes 32.4, 6 lanes 30.2, 8 lanes 28.5; stream-order lanes 34.7 ms at 4
BATCH_LOCKSTEP_LANES = 4
BATCH_STREAM_LANES = 4
# algorithmic FP32 work of one pixel-frame in one sweep: three candidate-frame
# evaluations (previous depth, random sample, propagated neighbour), each about
# 8 transcendental and 50 other FP32 operations
ALG_OPS_PER_PF_SWEEP = 3 * (8 + 50)
FP32_PEAK_TFLOPS = 157.3


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_job(job):
    """One whole window by the FP64 oracle in this process: (status, seconds)."""
    import oracle
    flows, K, kw = job
    t0 = time.perf_counter()
    st, *_ = oracle.window(flows, K, oracle.params(**kw))
    return st, time.perf_counter() - t0


def _cpu_baseline_batch(wins, seed, iters):
    """The oracle on a bounded sample of the batch, run before the GPU is
    touched: the batch's 320x240 windows, first one alone on one core, then one
    window per process on up to 16 cores at once (the oracle is serial C;
    windows are independent, so this is how the oracle uses a multi-core host)."""
    import multiprocessing as mp

    import synthflow
    small = [w for w in wins if (w["spec"].W, w["spec"].H) == (320, 240)]
    if not small:
        return None
    cores = max(1, min(16, os.cpu_count() or 1))
    jobs = []
    for k in range(cores):
        w = small[k % len(small)]
        kw = dict(n_iters=iters, n_pose_groups=synthflow.BATCH_GROUPS[(320, 240)], seed=seed)
        jobs.append((w["flows"], w["K"], kw))
    pf = [j[0].shape[0] * j[0].shape[1] * j[0].shape[2] * iters for j in jobs]
    st1, s1 = _oracle_job(jobs[0])
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_job, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    ok = st1 == 0 and all(r[0] == 0 for r in res)
    return {"value": sum(pf) / wall, "unit": "pixel-frame updates/s", "cores": cores, "kind": "oracle",
            "single_core_value": pf[0] / s1,
            "sample": f"{cores} windows of the batch's 320x240 shape (its {len(small)} such windows, repeated), "
                      f"{iters} EM iterations, FP64 oracle, one window per process on {cores} processes at once: "
                      f"{wall:.1f} s wall; one window alone on one core: {s1:.1f} s; status {'ok' if ok else 'FAILED'}",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


def _single_window_figures(vo, torch, name, seed, steps):
    """One window shape solved sequentially (the per-window latency view)."""
    import synthflow
    w = synthflow.make_window(name, seed)
    spec = w["spec"]
    T, H, W = spec.T, spec.H, spec.W
    flows = torch.from_numpy(w["flows"]).to("cuda:0")
    p = vo.default_params(n_iters=spec.n_iters, n_pose_groups=spec.n_groups, seed=seed)
    solver = vo.Solver(T, H, W, spec.n_groups)
    solver.autotune(flows, w["K"], p)
    solver.set_timing(True)
    dev = flows.device
    out = (torch.empty((T, 12), dtype=torch.float64, device=dev), torch.empty((H, W), dtype=torch.float32, device=dev),
           torch.empty((T, H, W), dtype=torch.float32, device=dev), torch.empty(2, dtype=torch.float64, device=dev))
    status = torch.full((steps + 2,), -1, dtype=torch.int32, device=dev)
    for i in range(2):
        solver.window_async(flows, w["K"], p, out, status[i])
    torch.cuda.synchronize()
    solver.timing_summary()
    t0 = time.perf_counter()
    for i in range(steps):
        solver.window_async(flows, w["K"], p, out, status[2 + i])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ph, n = solver.timing_summary()
    if any(int(x) != 0 for x in status.cpu().tolist()):
        print(f"{name}: a window reported a nonzero status", file=sys.stderr)
        sys.exit(1)
    sweep_us = ph["sweeps"] / max(ph["sweep_launches"], 1.0) * 1e3
    alg_bytes = 8.0 * T * H * W + 8.0 * H * W
    gbs = alg_bytes / (sweep_us * 1e-6) / 1e9
    rot, tdir = _pose_error(out[0].cpu().numpy(), w["poses"])
    tuning = solver.sweep_tuning()
    solver.close()
    return {"workload": f"{name}: T={T}, {W}x{H}, {spec.n_iters} EM iterations, {spec.n_groups} P3P groups/frame",
            "ms_per_window": ms, "windows_per_s": 1e3 / ms,
            "pixel_frame_updates_per_s": T * H * W * spec.n_iters / (ms * 1e-3),
            "phase_ms": {k: float(ph[k]) for k in ["bootstrap", "pose", "sweeps", "rigidness", "loglik", "window"]},
            "sweep_launch_us": sweep_us, "sweep_hbm_GBs": gbs, "sweep_hbm_frac": gbs / HBM_PEAK_GBS,
            "sweep_tuning": [list(t) for t in tuning],
            "pose_error_vs_gt": {"rot_rad": rot, "tdir_rad": tdir}}


def run_batch(args):
    """One step = one batch of windows of uneven shape and T solved by
    voldor_window_batch over concurrent streams (one HIP graph per step)."""
    import synthflow
    # generated in forked workers, and the CPU baseline run, before anything
    # touches the GPU
    wins = synthflow.make_batch(args.batch, args.seed, workers=min(16, os.cpu_count() or 1))
    cpu = None if args.no_cpu_baseline else _cpu_baseline_batch(wins, args.seed, BATCH_ITERS)
    import numpy as np
    import torch

    import paper_2104_06789_amd as vo

    dev = torch.device("cuda:0")
    p = vo.default_params(n_iters=BATCH_ITERS, n_pose_groups=2048, seed=args.seed)
    flows = [torch.from_numpy(w["flows"]).to(dev) for w in wins]
    shapes = [tuple(f.shape[:3]) for f in flows]
    groups = [synthflow.BATCH_GROUPS[(W, H)] for T, H, W in shapes]
    outs = [vo.Batch.outputs(T, H, W) for T, H, W in shapes]
    items = [(f, w["K"], o, None, g) for f, w, o, g in zip(flows, wins, outs, groups)]
    Tm, Hm, Wm = (max(x[k] for x in shapes) for k in range(3))
    status = torch.full((len(wins),), -1, dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()
    lockstep = args.batch_mode == "lockstep"
    lanes = args.lanes or (BATCH_LOCKSTEP_LANES if lockstep else BATCH_STREAM_LANES)
    solver = vo.Batch(lanes, Tm, Hm, Wm, max(groups), graph=not args.no_graph, lockstep=lockstep)
    with torch.cuda.stream(stream):
        solver.autotune(items, p, stream=stream)
    solver.set_timing(True)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            solver.solve(items, p, status, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            solver.solve(items, p, status, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bad = [int(x) for x in status.cpu().tolist() if x != 0]
    if bad:
        print(f"window status {vo.status_str(bad[0])} in {len(bad)} of {len(wins)} windows", file=sys.stderr)
        sys.exit(1)
    # phase sums over the windows of the last timed step (the graph replays the
    # event records of every captured window)
    ph, n_timed = solver.timing_summary()
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)
    pf_win = [T * H * W for T, H, W in shapes]
    pf = sum(pf_win) * BATCH_ITERS
    value = pf / (ms * 1e-3)
    n_sweeps = BATCH_ITERS * p.sweeps_per_iter
    alg_bytes = sum(n_sweeps * (8.0 * T * H * W + 8.0 * H * W) for T, H, W in shapes)
    alg_ops = sum(n_sweeps * ALG_OPS_PER_PF_SWEEP * T * H * W for T, H, W in shapes)
    # the sweep kernels' device time: the union of every window's sweep
    # intervals over the lanes (the chip ran at least one sweep), which a
    # kernel trace's per-dispatch durations add up to when sweeps do not
    # overlap; the lanes' own interval sums count overlapping time once per lane
    sweep_s = ph["sweeps_busy"] * 1e-3
    launches = ph["sweep_launches"]
    achieved_gbs = alg_bytes / sweep_s / 1e9 if sweep_s > 0 else None
    errs = [_pose_error(o[0].cpu().numpy(), w["poses"]) for o, w in zip(outs, wins)]
    mix = {}
    for T, H, W in shapes:
        mix[f"{W}x{H}"] = mix.get(f"{W}x{H}", 0) + 1
    tuning = []
    line = {
        "metric": "pixel-frame EM updates/s",
        "value": value,
        "unit": "pixel-frame updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch: {len(wins)} windows, shapes drawn from 320x240 (CPU-sized generator, "
                               f"intrinsics x2), 640x480 (indoor) and 1242x375 (driving), T from 4..8, "
                               f"{BATCH_ITERS} EM iterations, P3P groups per frame 1024 / 2048 / 4096 by shape, "
                               f"seed {args.seed}",
                   "windows": len(wins), "shapes": mix, "frames": sum(x[0] for x in shapes),
                   "lanes": lanes, "graph": not args.no_graph,
                   "mode": ("lockstep: the windows of a lane advance together, one launch per kernel over "
                            "their (window, frame) and (window, chain) items") if lockstep
                   else "windows in stream order per lane",
                   "parallelism": "single GPU, one batch per step over concurrent streams"},
        "windows_per_s": len(wins) * 1e3 / ms,
        "pose_error_vs_gt": {"rot_rad": float(np.mean([e[0] for e in errs])),
                             "tdir_rad": float(np.mean([e[1] for e in errs]))},
        ("phase_ms_summed_over_lanes" if lockstep else "phase_ms_summed_over_windows"):
            {k: float(ph[k]) for k in ["bootstrap", "pose", "sweeps", "rigidness", "loglik", "window"]},
        ("timed_lanes" if lockstep else "timed_windows"): n_timed,
        "roofline": {"bound": "hbm", "kernel": "k_sweep_multi" if lockstep else "k_sweep",
                     "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS if achieved_gbs else None,
                     "traffic": BATCH_SWEEP_TRAFFIC_PER_LAUNCH if _batch_sweep_counters_valid(lockstep) else None,
                     "fetch_bytes_per_launch": (BATCH_SWEEP_FETCH_PER_LAUNCH
                                                if _batch_sweep_counters_valid(lockstep) else None),
                     "alg_bytes_per_launch": alg_bytes / max(launches, 1.0),
                     "launch_ms": ph["sweeps_busy"] / max(launches, 1.0), "launches": launches,
                     "launch_ms_concurrent": ph["sweeps"] / max(launches, 1.0),
                     "step_aggregate_GBs": alg_bytes / (ms * 1e-3) / 1e9,
                     "note": "a launch here is one window's sweep of one direction (in lockstep mode one kernel "
                             "launch serves those of several windows); algorithmic bytes of a sweep: the flow stack "
                             "read once (8 B per pixel-frame) and the depth read and written (8 B per pixel); "
                             "launch_ms = the time during which the chip ran sweeps in the last timed step (union of "
                             "the lanes' sweep intervals between device timestamps on the lane streams) per launch; "
                             "launch_ms_concurrent = the lanes' sweep intervals summed, per launch, stretched where "
                             "lanes overlap"},
        "alu_view": {"achieved_TFLOPs": alg_ops / sweep_s / 1e12 if sweep_s > 0 else None,
                     "peak_TFLOPs": FP32_PEAK_TFLOPS,
                     "frac": alg_ops / sweep_s / 1e12 / FP32_PEAK_TFLOPS if sweep_s > 0 else None,
                     "ops_per_pixel_frame_sweep": ALG_OPS_PER_PF_SWEEP,
                     "note": "3 candidate-frame evaluations x (8 transcendental + 50 FP32) operations per "
                             "pixel-frame and sweep, over the same launch time"},
        "cpu_baseline": cpu,
    }
    solver.close()
    if not args.no_single:
        line["single_window"] = {name: _single_window_figures(vo, torch, name, args.seed, 10)
                                 for name in ("indoor", "driving")}
    print(json.dumps(line))


# HBM bytes of the sweeps of one batch step (rocprofv3 FETCH_SIZE and
# WRITE_SIZE of k_sweep_multi, summed over the step's launches, per window-sweep,
# scaled by the copy calibration); valid while the sweep's sources hash to
# BATCH_SWEEP_SOURCES_SHA (profiles/k_sweep_hbm_traffic.md).  On these sources
# only the FETCH_SIZE pass was taken, so the traffic (read + write) is None and
# the read bytes are reported on their own.
BATCH_SWEEP_FETCH_PER_LAUNCH = 32.83e6   # at 4 lockstep lanes
BATCH_SWEEP_TRAFFIC_PER_LAUNCH = None
BATCH_SWEEP_SOURCES_SHA = "cae795f93c1e31cf"
BATCH_SWEEP_TRAFFIC_LOCKSTEP = True    # the batch mode the counters were taken in


def _batch_sweep_counters_valid(lockstep):
    if BATCH_SWEEP_SOURCES_SHA is None or lockstep != BATCH_SWEEP_TRAFFIC_LOCKSTEP:
        return False
    return _sweep_sources_sha() == BATCH_SWEEP_SOURCES_SHA


LEARN_T, LEARN_H, LEARN_W = 6, 480, 640
LEARN_PLAIN_ITERS, LEARN_ITERS, LEARN_GROUPS = 4, 2, 2048


def _he_params(T, seed):
    """He-normal weights in the proposal's packed layout (zero padded channels)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for k in range(6):
        ci, co = 32, (16 if k == 5 else 32)
        ci_real = 2 * T if k == 0 else ci
        co_real = 1 + T if k == 5 else co
        w = np.zeros((3, 3, ci, co), np.float32)
        w[:, :, :ci_real, :co_real] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci_real)), (3, 3, ci_real, co_real))
        out.append(w.ravel())
        out.append(np.zeros(co, np.float32))
    return np.concatenate(out)


def _vo_starts(N, T, stride):
    s, out = 0, [0]
    while s + T < N:
        s = min(s + stride, N - T)
        out.append(s)
    return out


def _vo_chain(wposes, starts, N):
    """Trajectory from per-window relative poses, each window in its own gauge:
    window i's scale relative to window i - 1 is the length, in window i - 1's
    units, of the frame pair window i starts with."""
    import numpy as np
    scale = [1.0]
    for i in range(1, len(starts)):
        scale.append(scale[-1] * np.linalg.norm(wposes[i - 1][starts[i] - starts[i - 1]][9:]))
    M = [np.concatenate([np.eye(3).ravel(), np.zeros(3)])]
    for k in range(N):
        i = max(j for j, st in enumerate(starts) if st <= k)
        r = wposes[i][k - starts[i]]
        R, t = r[:9].reshape(3, 3), r[9:] * scale[i]
        Rm, tm = M[-1][:9].reshape(3, 3), M[-1][9:]
        M.append(np.concatenate([(R @ Rm).ravel(), R @ tm + t]))
    return np.array(M)


def _trajectory_error(M, gt_rel):
    """Mean rotation error (rad) of the camera poses, and the RMS camera-centre
    error after the least-squares scale, relative to the mean distance travelled."""
    import numpy as np
    G = [np.eye(4)]
    for R, t in gt_rel:
        A = np.eye(4)
        A[:3, :3], A[:3, 3] = R, t
        G.append(A @ G[-1])
    rot, ce, cg = [], [], []
    for k in range(1, len(M)):
        Re, te = M[k][:9].reshape(3, 3), M[k][9:]
        Rg, tg = G[k][:3, :3], G[k][:3, 3]
        D = Re @ Rg.T
        rot.append(float(np.arccos(np.clip((np.trace(D) - 1) / 2, -1, 1))))
        ce.append(-Re.T @ te)
        cg.append(-Rg.T @ tg)
    ce, cg = np.array(ce), np.array(cg)
    s = float((ce * cg).sum() / (ce * ce).sum())
    ate = float(np.sqrt(((s * ce - cg) ** 2).sum(axis=1).mean()) / np.linalg.norm(cg, axis=1).mean())
    return float(np.mean(rot)), ate


def run_vo(args):
    """Sliding-window VO over an indoor-shaped sequence (640x480, windows of T=6,
    per-frame speed varying in [0.6, 1.4] x 5 cm): windows seeded from the
    previous window's estimate on the device (voldor_vo_sequence), against the
    same windows each bootstrapped on its own and chained the same way."""
    import numpy as np
    import torch

    import paper_2104_06789_amd as vo
    import synthflow

    N, T, stride = args.vo_flows, 6, args.vo_stride
    w = synthflow.make_window("indoor", args.seed, T=N, speed_range=(0.6, 1.4))
    spec = w["spec"]
    H, W = spec.H, spec.W
    flows = torch.from_numpy(w["flows"]).to("cuda:0")
    p = vo.default_params(n_iters=spec.n_iters, n_pose_groups=spec.n_groups, seed=args.seed)
    solver = vo.Solver(T, H, W, spec.n_groups)
    solver.set_timing(True)
    for _ in range(max(args.warmup, 1)):
        traj, wposes, wst, depth, rig = solver.vo_sequence(flows, w["K"], p, T, stride)
    torch.cuda.synchronize()
    solver.timing_summary()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        traj, wposes, wst, depth, rig = solver.vo_sequence(flows, w["K"], p, T, stride)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    if not (wst.cpu().numpy() == 0).all():
        print(f"vo: window statuses {wst.cpu().tolist()}", file=sys.stderr)
        sys.exit(1)
    phases, n_timed = solver.timing_summary()
    starts = _vo_starts(N, T, stride)
    rot_s, ate_s = _trajectory_error(traj.cpu().numpy(), w["poses"])
    # the same windows, each bootstrapped from its own first flow
    outs = []
    status = torch.full((len(starts),), -1, dtype=torch.int32, device=flows.device)
    for i, s0 in enumerate(starts):
        o = (torch.empty((T, 12), dtype=torch.float64, device=flows.device),
             torch.empty((H, W), dtype=torch.float32, device=flows.device),
             torch.empty((T, H, W), dtype=torch.float32, device=flows.device), None)
        solver.window_async(flows[s0:s0 + T], w["K"], p, o, status[i], want_loglik=False)
        outs.append(o)
    torch.cuda.synchronize()
    plain = _vo_chain([o[0].cpu().numpy() for o in outs], starts, N)
    rot_p, ate_p = _trajectory_error(plain, w["poses"])
    launches = float(phases["sweep_launches"])
    sweep_ms = float(phases["sweeps"]) / max(launches, 1.0)
    alg_bytes = 8.0 * T * H * W + 8.0 * H * W
    achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9
    line = {
        "metric": "frames/s of sliding-window VO",
        "value": N / (ms * 1e-3),
        "unit": "frames/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"vo: indoor-shaped sequence of {N} flows ({W}x{H}), windows of T={T} every "
                               f"{stride} frame(s), {spec.n_iters} EM iterations, {spec.n_groups} P3P groups/frame, "
                               f"per-frame speed x[0.6, 1.4], seed {args.seed}",
                   "windows": len(starts), "parallelism": "single GPU, windows seeded in sequence on one stream"},
        "seeded": {"rot_err_rad": rot_s, "ate_rel": ate_s},
        "bootstrapped_each": {"rot_err_rad": rot_p, "ate_rel": ate_p},
        "phase_ms": {k: float(phases[k]) for k in ["bootstrap", "pose", "sweeps", "rigidness", "window"]},
        "roofline": {"bound": "hbm", "kernel": "k_sweep", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg_bytes, "launch_ms": sweep_ms},
    }
    print(json.dumps(line))


def run_resfit(args):
    """Regression of the Fisk laws on residuals (Fig. 4b procedure): the noisy
    flows of an indoor window (T=6, 640x480, no moving objects) against the same
    scene's exact flows, 40 bins of |v|.  The binning pass streams both flow
    fields once (16 bytes per item): HBM-bound."""
    import numpy as np
    import torch

    import paper_2104_06789_amd as vo
    import synthflow

    w = synthflow.make_window("indoor", args.seed, outliers=False)
    g = synthflow.make_window("indoor", args.seed, noise=False, outliers=False)
    X = torch.from_numpy(w["flows"]).cuda()
    G = torch.from_numpy(g["flows"]).cuda()
    n = X.numel() // 2
    nb = 40
    v_max = float(np.ceil(np.nanpercentile(np.linalg.norm(w["flows"].reshape(-1, 2), axis=1), 99.5)))
    work = torch.empty(int(vo.lib().voldor_residual_workspace(n, nb)), dtype=torch.float64, device="cuda")
    out = torch.empty((nb, 4), dtype=torch.float64, device="cuda")
    for _ in range(max(args.warmup, 1)):
        vo.residual_bins(X, G, nb, v_max, work=work, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        vo.residual_bins(X, G, nb, v_max, work=work, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    launch_ms = e0.elapsed_time(e1) / max(args.steps, 1)
    laws, bins = vo.residual_fit(X, G, nb, v_max)
    spec = w["spec"]
    alg_bytes = 16.0 * n
    gbs = alg_bytes / (launch_ms * 1e-3) / 1e9
    line = {
        "metric": "residual items/s binned for the Fisk-law regression",
        "value": n / (ms * 1e-3), "unit": "items/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64 sums of f32 flows",
        "data": "synthetic",
        "config": {"workload": f"resfit: indoor window T=6 640x480 noisy vs exact flows, {nb} bins over |v| < {v_max}, "
                               f"seed {args.seed}", "items": n},
        "laws": {"a1": laws[0], "a2": laws[1], "b1": laws[2], "b2": laws[3]},
        # the generator draws the end-point error from Fisk(c1 |v| + c0, beta), so
        # its square follows Fisk((c1 |v| + c0)^2, beta / 2)
        "generator_law_of_squared_epe": {"A": f"({spec.noise_c1} |v| + {spec.noise_c0})^2",
                                         "B": spec.noise_beta / 2},
        "roofline": {"bound": "hbm", "kernel": "k_resid_bins + k_resid_reduce", "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": _resfit_traffic(),
                     "alg_bytes_per_launch": alg_bytes, "launch_ms": launch_ms},
    }
    if not args.no_cpu_baseline:
        from oracle import resfit as oracle_resfit
        c0 = time.perf_counter()
        ref = oracle_resfit.bin_stats(w["flows"].reshape(-1, 2), g["flows"].reshape(-1, 2), nb, v_max)
        oracle_resfit.fit(ref, min_count=64)
        c1 = time.perf_counter()
        line["cpu_baseline"] = {"value": n / (c1 - c0), "unit": "items/s", "cores": 1, "kind": "oracle",
                                "sample": f"the whole workload ({n} items): FP64 binning and fit with numpy, "
                                          f"{c1 - c0:.2f} s"}
    print(json.dumps(line))


def run_learned(args):
    """The learned proposal: train it on windows labelled by the plain EM, then
    compare EM at LEARN_ITERS iterations from the proposal (falling back to the
    bootstrap's state where that explains the window better) against the plain
    EM at LEARN_PLAIN_ITERS iterations on held-out windows.

    --gen cpu: every window generated on the host before the GPU is touched,
    labelled once, trained over for --epochs.  --gen gpu: windows generated on
    the device (synthflow.torchgen, the same scene and noise laws) in chunks of
    --chunk, each chunk labelled, trained over once per epoch and dropped, so
    that training sets far larger than device memory stream through."""
    import synthflow
    n_train, n_eval = args.train_windows, args.eval_windows
    gen_gpu = args.gen == "gpu"
    shapes = (("small", LEARN_W, LEARN_H),)
    train_seeds = [((args.seed + 1) << 16) + i for i in range(n_train)]
    held_seeds = [((args.seed + 2) << 16) + i for i in range(n_eval)]
    train = held = None
    if not gen_gpu:
        # the CPU-sized generator at 640x480 with its intrinsics scaled x4, in
        # forked workers before anything touches the GPU
        workers = min(16, os.cpu_count() or 1)
        train = synthflow.make_batch(n_train, args.seed + 1, shapes=shapes, T_range=(LEARN_T, LEARN_T),
                                     workers=workers)
        held = synthflow.make_batch(n_eval, args.seed + 2, shapes=shapes, T_range=(LEARN_T, LEARN_T),
                                    workers=workers)
    import numpy as np
    import torch

    import paper_2104_06789_amd as vo

    dev = torch.device("cuda:0")
    T, H, W = LEARN_T, LEARN_H, LEARN_W
    stream = torch.cuda.Stream()
    gen_ms = [0.0]

    def generate(seeds):
        from synthflow.torchgen import make_window_torch
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        out = []
        for sd in seeds:
            w = make_window_torch("small", sd, dev, T=T, H=H, W=W)
            out.append({"flows": w["flows"], "K": w["K"], "poses": w["poses"]})
        torch.cuda.synchronize()
        gen_ms[0] += (time.perf_counter() - g0) * 1e3
        return out

    def dev_flows(w):
        f = w["flows"]
        return f if isinstance(f, torch.Tensor) else torch.from_numpy(f).to(dev)

    def solve(wins, iters, props=None):
        p = vo.default_params(n_iters=iters, n_pose_groups=LEARN_GROUPS, seed=args.seed)
        flows = [dev_flows(w) for w in wins]
        outs = [vo.Batch.outputs(T, H, W) for _ in wins]
        st = torch.full((len(wins),), -1, dtype=torch.int32, device=dev)
        ch = torch.full((len(wins),), -1, dtype=torch.int32, device=dev)
        items = []
        for k, (f, w, o) in enumerate(zip(flows, wins, outs)):
            items.append((f, w["K"], o) if props is None else (f, w["K"], o, (props[0][k], props[1][k], ch[k:k + 1])))
        b = vo.Batch(4, T, H, W, LEARN_GROUPS, graph=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            b.solve(items, p, st, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        b.close()
        if any(int(x) != 0 for x in st.cpu().tolist()):
            print("a window reported a nonzero status", file=sys.stderr)
            sys.exit(1)
        return outs, ms, ch

    net = vo.Net(T, args.learn_batch, H, W)
    net.set_params(_he_params(T, args.seed))
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    nb = args.learn_batch
    losses = []
    steps = 0
    train_s = 0.0
    label_ms = 0.0
    rng = np.random.default_rng(args.seed)

    def train_over(tflows, tdepth, trig):
        # one pass over the given windows in a random order, nb per Adam step
        nonlocal steps, train_s
        ep_loss = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        order = rng.permutation(tflows.shape[0])
        for i in range(0, tflows.shape[0] - nb + 1, nb):
            idx = torch.from_numpy(order[i:i + nb]).to(dev)
            net.train_step(tflows[idx].contiguous(), tdepth[idx].contiguous(), trig[idx].contiguous(), args.lr,
                           loss=loss)
            ep_loss.append(loss.clone())
            steps += 1
        torch.cuda.synchronize()
        train_s += time.perf_counter() - t0
        return ep_loss

    if not gen_gpu:
        # labels: the plain EM's depth and final rigidness
        labels, label_ms, _ = solve(train, LEARN_PLAIN_ITERS)
        tflows = torch.stack([torch.from_numpy(w["flows"]) for w in train]).to(dev)
        tdepth = torch.stack([o[1] for o in labels])
        trig = torch.stack([o[2] for o in labels])
        for ep in range(args.epochs):
            losses.append(float(torch.stack(train_over(tflows, tdepth, trig)).mean()))
    else:
        for ep in range(args.epochs):
            ep_loss = []
            for c0 in range(0, n_train, args.chunk):
                wins = generate(train_seeds[c0:c0 + args.chunk])
                labels, ms, _ = solve(wins, LEARN_PLAIN_ITERS)
                if ep == 0:
                    label_ms += ms
                tflows = torch.stack([w["flows"] for w in wins])
                tdepth = torch.stack([o[1] for o in labels])
                trig = torch.stack([o[2] for o in labels])
                ep_loss += train_over(tflows, tdepth, trig)
                del wins, labels, tflows, tdepth, trig
                print(f"epoch {ep} windows {min(c0 + args.chunk, n_train)}/{n_train} "
                      f"loss {float(torch.stack(ep_loss[-16:]).mean()):.4f}", file=sys.stderr, flush=True)
            losses.append(float(torch.stack(ep_loss).mean()))
        held = generate(held_seeds)

    # matrix-core rate of the forward pass on one training batch, HIP events on its stream
    fb = torch.stack([dev_flows(w) for w in held[:nb]]).contiguous()
    with torch.cuda.stream(stream):
        net.forward(fb, stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reps = 10
        for _ in range(reps):
            net.forward(fb, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    conv_flops = 2.0 * nb * H * W * 9 * 32 * (5 * 32 + 16)   # six layers, padded widths
    achieved = conv_flops / (fwd_ms * 1e-3) / 1e12

    # held-out windows: plain EM vs proposal + shorter EM
    plain, plain_ms, _ = solve(held, LEARN_PLAIN_ITERS)
    hflows = torch.stack([dev_flows(w) for w in held])
    pdepth = torch.empty((n_eval, H, W), device=dev)
    prig = torch.empty((n_eval, T, H, W), device=dev)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for i in range(0, n_eval, nb):
        j = min(n_eval, i + nb)
        net.forward(hflows[i:j].contiguous(), depth=pdepth[i:j], rig=prig[i:j])
    torch.cuda.synchronize()
    prop_ms = (time.perf_counter() - p0) * 1e3
    learned, learned_ms, choice = solve(held, LEARN_ITERS, props=(pdepth, prig))
    shorter, shorter_ms, _ = solve(held, LEARN_ITERS)

    def errs(outs):
        e = [_pose_error(o[0].cpu().numpy(), w["poses"]) for o, w in zip(outs, held)]
        return {"rot_rad": float(np.mean([x[0] for x in e])), "tdir_rad": float(np.mean([x[1] for x in e]))}

    ds = [float(np.median(np.abs(np.log(pdepth[k].cpu().numpy()) - np.log(plain[k][1].cpu().numpy()))))
          for k in range(n_eval)]
    learned_total = learned_ms + prop_ms
    line = {
        "metric": "windows/s at equal pose error, learned vs plain EM",
        "value": n_eval * 1e3 / learned_total,
        "unit": "windows/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": learned_total,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 network, f32 sweeps",
        "data": "synthetic",
        "config": {"workload": f"learned proposal: {n_train} training and {n_eval} held-out windows, T={T}, "
                               f"{W}x{H}, CPU-sized scene generator with intrinsics x4; plain EM "
                               f"{LEARN_PLAIN_ITERS} iterations vs proposal + EM {LEARN_ITERS} iterations, "
                               f"{LEARN_GROUPS} P3P groups/frame, seed {args.seed}",
                   "epochs": args.epochs, "batch": nb, "lr": args.lr,
                   "parallelism": "single GPU, four stream lanes"},
        "plain": {"windows_per_s": n_eval * 1e3 / plain_ms, "pose_error_vs_gt": errs(plain)},
        "learned": {"windows_per_s": n_eval * 1e3 / learned_total, "pose_error_vs_gt": errs(learned),
                    "proposal_used": float(np.mean(choice.cpu().numpy() == 1)),
                    "proposal_ms": prop_ms, "em_ms": learned_ms,
                    "median_abs_log_depth_vs_plain": float(np.mean(ds))},
        "bootstrap_em_short": {"windows_per_s": n_eval * 1e3 / shorter_ms, "pose_error_vs_gt": errs(shorter)},
        "training": {"loss_per_epoch": losses, "steps": steps, "seconds": train_s, "label_ms": label_ms,
                     "generator": ("device (synthflow.torchgen), chunks of %d windows" % args.chunk) if gen_gpu
                     else "host (synthflow.make_batch)", "generate_ms": gen_ms[0]},
        "roofline": {"bound": "mfma", "kernel": "k_net_input + k_net_fused (six layers, forward)", "achieved": achieved,
                     "peak": 2500.0, "unit": "TFLOP/s", "frac": achieved / 2500.0, "traffic": None,
                     "flops_per_pass": conv_flops, "pass_ms": fwd_ms},
    }
    print(json.dumps(line))


def _concurrent(vo, torch, T, H, W, spec, flows, w, p, out, dev, args, pf, lanes=4, per_batch=8, widths=(0, 0)):
    """The same windows solved `lanes` at a time (voldor_window_batch): independent
    windows overlap one window's latency-bound pose chain with the others' sweeps."""
    conc = vo.Batch(lanes, T, H, W, spec.n_groups, graph=True)
    conc.set_sweep_threads(*widths)
    couts = [vo.Batch.outputs(T, H, W) for _ in range(per_batch)]
    citems = [(flows, w["K"], o) for o in couts]
    cstat = torch.full((per_batch,), -1, dtype=torch.int32, device=dev)
    cstream = torch.cuda.Stream()
    with torch.cuda.stream(cstream):
        conc.solve(citems, p, cstat, stream=cstream)
    torch.cuda.synchronize()
    reps = max(1, args.steps // per_batch)
    c0 = time.perf_counter()
    with torch.cuda.stream(cstream):
        for _ in range(reps):
            conc.solve(citems, p, cstat, stream=cstream)
    torch.cuda.synchronize()
    cms = (time.perf_counter() - c0) * 1e3 / (reps * per_batch)
    if any(int(x) != 0 for x in cstat.cpu().tolist()):
        print("a concurrent window reported a nonzero status", file=sys.stderr)
        sys.exit(1)
    for o in couts:
        if not all(torch.equal(a, b) for a, b in zip(o, out)):
            print("a concurrent window differs from the sequential one", file=sys.stderr)
            sys.exit(1)
    return {"lanes": lanes, "windows_per_call": per_batch, "calls": reps, "value": pf / (cms * 1e-3),
            "unit": "pixel-frame updates/s", "windows_per_s": 1e3 / cms, "ms_per_window": cms,
            "note": "same workload, windows solved four at a time by voldor_window_batch "
                    "(HIP graph); results equal the sequential windows bit for bit"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch", choices=["indoor", "driving", "small", "batch", "learned", "vo", "resfit"])
    ap.add_argument("--vo-flows", type=int, default=18, help="flows of the sequence (--workload vo)")
    ap.add_argument("--vo-stride", type=int, default=1, help="frames between window starts (--workload vo)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--criterion", default="mie", choices=["mie", "mle"],
                    help="depth M-step: maximum inlier (Eq. 10) or maximum likelihood (Eq. 9)")
    ap.add_argument("--residual-model", default="fisk", choices=["fisk", "gauss"],
                    help="density of rho and mu: Fisk (Eq. 5) or the Gaussian flow error of the ablations")
    ap.add_argument("--pose-start", default="kde", choices=["kde", "allpixel"],
                    help="mean-shift start: densest of 64 seeds, or every candidate scored over all pixels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=32, help="windows per step (--workload batch)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="concurrent streams of --workload batch (default: 4 in either mode)")
    ap.add_argument("--batch-mode", choices=["lockstep", "lanes"], default="lockstep",
                    help="lockstep: the windows of each lane advance together, one launch per kernel over all "
                         "of them; lanes: each lane solves its windows one after another")
    ap.add_argument("--no-graph", action="store_true", help="enqueue launches instead of a HIP graph")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-window indoor and driving figures of the batch workload")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the four-lane figure (profiles of the sequential windows alone)")
    ap.add_argument("--train-windows", type=int, default=20000, help="(--workload learned)")
    ap.add_argument("--eval-windows", type=int, default=512, help="(--workload learned)")
    ap.add_argument("--epochs", type=int, default=1, help="(--workload learned)")
    ap.add_argument("--learn-batch", type=int, default=4, help="(--workload learned)")
    ap.add_argument("--lr", type=float, default=1e-3, help="(--workload learned)")
    ap.add_argument("--gen", default="gpu", choices=["cpu", "gpu"],
                    help="(--workload learned) where the windows are generated; gpu streams the training set "
                         "in chunks")
    ap.add_argument("--chunk", type=int, default=500, help="(--workload learned --gen gpu) windows per chunk")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: windows are independent, so more GPUs would "
              "each solve their own share; runs with --gpus > 1 are not supported.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "learned":
        run_learned(args)
        return
    if args.workload == "vo":
        run_vo(args)
        return
    if args.workload == "resfit":
        run_resfit(args)
        return

    import numpy as np
    import torch

    import paper_2104_06789_amd as vo
    import synthflow

    w = synthflow.make_window(args.workload, args.seed)
    spec = w["spec"]
    T, H, W = spec.T, spec.H, spec.W
    flows = torch.from_numpy(w["flows"]).to("cuda:0")
    crit = 1 if args.criterion == "mle" else 0
    pstart = 1 if args.pose_start == "allpixel" else 0
    rmodel = 1 if args.residual_model == "gauss" else 0
    p = vo.default_params(n_iters=spec.n_iters, n_pose_groups=spec.n_groups, seed=args.seed, criterion=crit,
                          pose_start=pstart, residual_model=rmodel)
    solver = vo.Solver(T, H, W, spec.n_groups)
    # sweep widths for this shape (every width gives the same result)
    widths = solver.autotune(flows, w["K"], p)
    solver.set_timing(True)
    dev = flows.device
    out = (torch.empty((T, 12), dtype=torch.float64, device=dev),
           torch.empty((H, W), dtype=torch.float32, device=dev),
           torch.empty((T, H, W), dtype=torch.float32, device=dev),
           torch.empty(2, dtype=torch.float64, device=dev))
    # windows are enqueued back to back on the stream, each reporting its device
    # status into its own element; the host waits once, after the last one
    status = torch.full((max(args.steps, args.warmup, 1),), -1, dtype=torch.int32, device=dev)
    for i in range(args.warmup):
        solver.window_async(flows, w["K"], p, out, status[i])
    torch.cuda.synchronize()
    solver.timing_summary()   # start the phase count at the timed windows
    t0 = time.perf_counter()
    for i in range(args.steps):
        solver.window_async(flows, w["K"], p, out, status[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)
    pf = T * H * W * spec.n_iters
    value = pf / (ms * 1e-3)
    bad = [int(x) for x in status[:args.steps].cpu().tolist() if x != 0]
    if bad:
        print(f"window status {vo.status_str(bad[0])} in {len(bad)} of {args.steps} timed windows",
              file=sys.stderr)
        sys.exit(1)

    phases, n_timed = solver.timing_summary()   # mean over the timed windows (last 32 at most)
    keys = ["bootstrap", "pose", "sweeps", "rigidness", "loglik", "window"]
    ph = {k: float(phases[k]) for k in keys}
    launches = float(phases["sweep_launches"])
    sweep_ms = ph["sweeps"] / max(launches, 1.0)
    alg_bytes = 8.0 * T * H * W + 8.0 * H * W
    achieved_gbs = alg_bytes / (sweep_ms * 1e-3) / 1e9
    alg_ops = float(ALG_OPS_PER_PF_SWEEP) * T * H * W
    achieved = alg_ops / (sweep_ms * 1e-3) / 1e12

    rot_err, tdir_err = _pose_error(out[0].cpu().numpy(), w["poses"])

    # the same windows solved LANES at a time (voldor_window_batch): independent
    # windows overlap one window's latency-bound pose chain with the others' sweeps
    conc_line = None if args.no_concurrent else _concurrent(vo, torch, T, H, W, spec, flows, w, p, out, dev,
                                                             args, pf, widths=widths)

    line = {
        "metric": "pixel-frame EM updates/s",
        "value": value,
        "unit": "pixel-frame updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: T={T}, {W}x{H}, {spec.n_iters} EM iterations, "
                               f"{spec.n_groups} P3P groups/frame, seed {args.seed}"
                               + (", depth criterion MLE (Eq. 9)" if crit else "")
                               + (", all-pixel mean-shift start" if pstart else "")
                               + (", Gaussian residual model" if rmodel else ""),
                   "criterion": args.criterion, "pose_start": args.pose_start,
                   "residual_model": args.residual_model,
                   "sweep_threads": {"rows": widths[0], "cols": widths[1]},
                   "T": T, "H": H, "W": W, "n_iters": spec.n_iters, "n_pose_groups": spec.n_groups,
                   "parallelism": "single GPU, one window per step, enqueued back to back on one stream"},
        "windows_per_s": 1e3 / ms,
        "phase_ms": ph,
        "phase_windows": n_timed,
        "concurrent": conc_line,
        "pose_error_vs_gt": {"rot_rad": rot_err, "tdir_rad": tdir_err},
        "roofline": {"bound": "hbm", "kernel": "k_sweep", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
                     "traffic": _sweep_traffic(args.workload) if not (crit or rmodel) else None,
                     "alg_bytes_per_launch": alg_bytes, "launch_ms": sweep_ms},
        "alu_view": {"achieved_TFLOPs": achieved, "peak_TFLOPs": FP32_PEAK_TFLOPS,
                     "frac": achieved / FP32_PEAK_TFLOPS, "ops_per_pixel_frame_sweep": ALG_OPS_PER_PF_SWEEP},
    }

    if pstart:
        # the dominant kernel of this variant is the candidate scoring
        line["roofline_sweep"] = line["roofline"]
        line["roofline"] = _allpixel_roofline(vo, torch, solver, w, spec, p, out)

    if pstart and not args.no_cpu_baseline:
        # the FP64 oracle scores ~10^9 candidate-pixel pairs per pose step here:
        # hours per window, far beyond a bounded sample of the same workload
        line["cpu_baseline"] = None
        line["cpu_baseline_note"] = "not run for the all-pixel start (hours of FP64 work per window)"
    elif not args.no_cpu_baseline:
        import oracle
        kw = dict(n_iters=spec.n_iters, n_pose_groups=spec.n_groups, seed=args.seed, criterion=crit,
                  pose_start=pstart, residual_model=rmodel)
        c0 = time.perf_counter()
        st, *_ = oracle.window(w["flows"], w["K"], oracle.params(**kw))
        c1 = time.perf_counter()
        line["cpu_baseline"] = {"value": pf / (c1 - c0), "unit": "pixel-frame updates/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"one whole {args.workload} window (T={T}, {W}x{H}, "
                                          f"{spec.n_iters} iterations), FP64 oracle, single thread, "
                                          f"{c1 - c0:.1f} s, status {st}"}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
