#!/usr/bin/env python3
"""Throughput of the VOLDOR window solver on one MI355X.

One step = one whole window solved by the HIP library (bootstrap, then every
EM iteration: pose of each frame, the directional depth/rigidness sweeps, the
unsmoothed rigidness and the gauge; finally the log-likelihood), on a seeded
synthetic window whose flows are already resident in device memory.

Metric: pixel-frame EM updates/s = T*H*W*n_iters / (seconds per window).
Default workload: the indoor shape (T=6, 640x480, 4 iterations, 2048 P3P
groups per frame); --workload driving runs T=8, 1242x375.

The roofline object reports the dominant GPU kernel, the fused directional
sweep, against the VALU issue rate it is bound by.  Algorithmic work per
launch = 3 emission evaluations per pixel-frame (previous depth, random sample,
propagated neighbour: what the serial walk needs) x EMISSION_VALU_OPS FP32
VALU lane-instructions each, divided by the mean sweep duration measured with
HIP events on the solver's stream; the peak is 256 CUs x 64 lanes x 2.4 GHz.
The HBM view of the same launch (flow stack read + depth read/write) is kept
alongside for reference.  The cpu_baseline object times the FP64 CPU oracle on
one window of the same workload.
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
# profiles/k_sweep_indoor_hbm_traffic.md)
SWEEP_TRAFFIC_INDOOR = {"fetch_bytes": 25142.82421875 * 1024 * 1.99983,
                        "write_bytes": 1266.16796875 * 1024 * 1.0}
SWEEP_SOURCES_SHA = "6734fc834195be18"
SWEEP_SOURCES = ("vo_sweep.hip", "vo_device.hpp", "vo_internal.hpp")
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12     # FP32 lane-instructions/s (non-packed), 39.3 T
EMISSION_VALU_OPS = 160                      # VALU instructions of one emission evaluation (gfx950 ISA),
                                             # 12 of them transcendental


def _sweep_traffic(workload):
    """Measured HBM bytes per sweep launch, or None if not measured for this
    workload or if the kernel changed since the counters were taken."""
    import hashlib
    if workload != "indoor":
        return None
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_06789_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != SWEEP_SOURCES_SHA:
        return None
    return SWEEP_TRAFFIC_INDOOR["fetch_bytes"] + SWEEP_TRAFFIC_INDOOR["write_bytes"]


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


BATCH_ITERS, BATCH_GROUPS = 4, 2048


def run_batch(args):
    """One step = one batch of windows of uneven shape and T solved by
    voldor_window_batch over concurrent streams (one HIP graph per step)."""
    import synthflow
    # generated in forked workers before anything touches the GPU
    wins = synthflow.make_batch(args.batch, args.seed, workers=min(16, os.cpu_count() or 1))
    import numpy as np
    import torch

    import paper_2104_06789_amd as vo

    dev = torch.device("cuda:0")
    p = vo.default_params(n_iters=BATCH_ITERS, n_pose_groups=BATCH_GROUPS, seed=args.seed)
    flows = [torch.from_numpy(w["flows"]).to(dev) for w in wins]
    shapes = [tuple(f.shape[:3]) for f in flows]
    outs = [vo.Batch.outputs(T, H, W) for T, H, W in shapes]
    items = [(f, w["K"], o) for f, w, o in zip(flows, wins, outs)]
    Tm, Hm, Wm = (max(x[k] for x in shapes) for k in range(3))
    status = torch.full((len(wins),), -1, dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()
    solver = vo.Batch(args.lanes, Tm, Hm, Wm, BATCH_GROUPS, graph=not args.no_graph)
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
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)
    pf_win = [T * H * W for T, H, W in shapes]
    pf = sum(pf_win) * BATCH_ITERS
    value = pf / (ms * 1e-3)
    # every sweep of the batch: 3 emission evaluations per pixel-frame
    alg_ops = 3.0 * sum(pf_win) * EMISSION_VALU_OPS * BATCH_ITERS * p.sweeps_per_iter
    achieved = alg_ops / (ms * 1e-3) / 1e12
    errs = [_pose_error(o[0].cpu().numpy(), w["poses"]) for o, w in zip(outs, wins)]
    mix = {}
    for T, H, W in shapes:
        mix[f"{W}x{H}"] = mix.get(f"{W}x{H}", 0) + 1
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
        "config": {"workload": f"batch: {len(wins)} windows of shapes drawn from 320x240, 640x480, "
                               f"1242x375 and T from 4..8, {BATCH_ITERS} EM iterations, {BATCH_GROUPS} P3P "
                               f"groups/frame, seed {args.seed}",
                   "windows": len(wins), "shapes": mix, "frames": sum(x[0] for x in shapes),
                   "lanes": args.lanes, "graph": not args.no_graph,
                   "parallelism": "single GPU, one batch per step over concurrent streams"},
        "windows_per_s": len(wins) * 1e3 / ms,
        "pose_error_vs_gt": {"rot_rad": float(np.mean([e[0] for e in errs])),
                             "tdir_rad": float(np.mean([e[1] for e in errs]))},
        "roofline": {"bound": "alu", "kernel": "k_sweep (all sweeps of the batch over the whole step)",
                     "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TFLOP/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "alg_ops_per_step": alg_ops},
    }
    if not args.no_cpu_baseline:
        import oracle
        k = int(np.argmin(pf_win))   # the smallest window of the batch
        c0 = time.perf_counter()
        st, *_ = oracle.window(wins[k]["flows"], wins[k]["K"],
                               oracle.params(n_iters=BATCH_ITERS, n_pose_groups=BATCH_GROUPS, seed=args.seed))
        c1 = time.perf_counter()
        T, H, W = shapes[k]
        line["cpu_baseline"] = {"value": pf_win[k] * BATCH_ITERS / (c1 - c0), "unit": "pixel-frame updates/s",
                                "cores": 1, "kind": "oracle",
                                "sample": f"window {k} of the batch (T={T}, {W}x{H}, {BATCH_ITERS} iterations), "
                                          f"FP64 oracle, single thread, {c1 - c0:.1f} s, status {st}"}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="indoor", choices=["indoor", "driving", "small", "batch"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=32, help="windows per step (--workload batch)")
    ap.add_argument("--lanes", type=int, default=4, help="concurrent streams (--workload batch)")
    ap.add_argument("--no-graph", action="store_true", help="enqueue launches instead of a HIP graph")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: windows are independent, so more GPUs would "
              "each solve their own share; runs with --gpus > 1 are not supported.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args)
        return

    import numpy as np
    import torch

    import paper_2104_06789_amd as vo
    import synthflow

    w = synthflow.make_window(args.workload, args.seed)
    spec = w["spec"]
    T, H, W = spec.T, spec.H, spec.W
    flows = torch.from_numpy(w["flows"]).to("cuda:0")
    p = vo.default_params(n_iters=spec.n_iters, n_pose_groups=spec.n_groups, seed=args.seed)
    solver = vo.Solver(T, H, W, spec.n_groups)
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
    alg_ops = 3.0 * T * H * W * EMISSION_VALU_OPS
    achieved = alg_ops / (sweep_ms * 1e-3) / 1e12

    rot_err, tdir_err = _pose_error(out[0].cpu().numpy(), w["poses"])

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
                               f"{spec.n_groups} P3P groups/frame, seed {args.seed}",
                   "T": T, "H": H, "W": W, "n_iters": spec.n_iters, "n_pose_groups": spec.n_groups,
                   "parallelism": "single GPU, one window per step, enqueued back to back on one stream"},
        "windows_per_s": 1e3 / ms,
        "phase_ms": ph,
        "phase_windows": n_timed,
        "pose_error_vs_gt": {"rot_rad": rot_err, "tdir_rad": tdir_err},
        "roofline": {"bound": "alu", "kernel": "k_sweep", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": _sweep_traffic(args.workload),
                     "alg_ops_per_launch": alg_ops, "launch_ms": sweep_ms,
                     "hbm_view": {"alg_bytes_per_launch": alg_bytes, "achieved_GBs": achieved_gbs,
                                  "frac_of_8TBs": achieved_gbs / HBM_PEAK_GBS}},
    }

    if not args.no_cpu_baseline:
        import oracle
        kw = dict(n_iters=spec.n_iters, n_pose_groups=spec.n_groups, seed=args.seed)
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
