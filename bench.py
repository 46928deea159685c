#!/usr/bin/env python3
"""Benchmark of the relocalization hot path on one MI355X.

Metric: hypothesis x orientation evaluations per second, SMAD + TAM
(SMAD evals = N_p x circular shifts, 1 shift when the FoV covers >= 90 % of
the turn; TAM evals = hypotheses evaluated by TAM x N_theta), plus p50/p99
latency of one relocalization.

One step = one relocalization of the plain-large workload (2000 x 2000
warehouse at 0.05 m, 20 000 hypotheses, 270 deg / 720-beam scan with
clutter, 0.5 deg TAM orientations, 64 hypotheses per stage, tau = 0.95):
ray cast + SMAD for every hypothesis, SMAD order, TAM stages with early
termination, ranking. Map, hypotheses and the scan's tables are resident in
HBM before timing starts (reloc_prepare); each step is one reloc_run.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9      # int32 lane-ops/s: CUs x SIMDs x lanes x clock
DDA_OPS_PER_STEP = 10                      # compare, 2 selects, D update, 2 bounds, 3 address, 1 bit test


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(w, hyp, n_theta, batch_k, stages_gpu, budget_s):
    """The oracle as it stands, on a bounded sample of the same workload:
    ray cast + SMAD for a hypothesis subsample and TAM for the first stages."""
    import numpy as np
    import oracle
    pr = oracle.prep(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                     range_min=w.range_min, range_max=w.range_max, n_theta=n_theta)
    k = oracle.edt(w.occ)
    threads = oracle.num_threads()
    # size the sample from a short probe so the whole leg stays near budget_s
    probe = hyp[:200]
    t = time.perf_counter()
    _, z = oracle.raycast(w.occ, probe, pr["Ns"], pr["Ng"], w.resolution, w.range_max)
    oracle.smad(z, pr)
    per_hyp = (time.perf_counter() - t) / len(probe)
    q = np.repeat(hyp[:2], n_theta, axis=0)
    kk = np.tile(np.arange(n_theta), 2)
    t = time.perf_counter()
    oracle.tam(k, w.resolution, pr, q, kk)
    per_tam_hyp = (time.perf_counter() - t) / 2
    n_sm = int(min(len(hyp), max(200, 0.6 * budget_s / per_hyp)))
    n_st = int(min(stages_gpu, max(1, 0.4 * budget_s / (per_tam_hyp * batch_k))))
    t0 = time.perf_counter()
    _, z = oracle.raycast(w.occ, hyp[:n_sm], pr["Ns"], pr["Ng"], w.resolution, w.range_max)
    sm, _ = oracle.smad(z, pr)
    n_tam = min(len(sm), n_st * batch_k)
    q = np.repeat(hyp[:n_tam], n_theta, axis=0)
    kk = np.tile(np.arange(n_theta), n_tam)
    oracle.tam(k, w.resolution, pr, q, kk)
    dt = time.perf_counter() - t0
    evals = n_sm * pr["n_shifts"] + n_tam * n_theta
    return {"value": evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": "ray cast + direct-sum SMAD of %d of %d hypotheses, TAM of %d "
                      "hypotheses x %d orientations (%d stages); %.1f s"
                      % (n_sm, len(hyp), n_tam, n_theta, n_st, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tau", default="0.95")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--variant", type=int, default=0,
                    help="ray-cast kernel: 0 tuned default, 1 bit tiles, 2 distance skipping")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB (counter scale)")
    ap.add_argument("--traffic", default=None,
                    help="JSON file with measured HBM bytes per launch of the ray-cast kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2511_01219_amd as reloc
    from synth import make_config

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.calibrate_copy)
        del src, dst
    tau = None if args.tau.lower() in ("none", "nan") else float(args.tau)
    n_theta, batch_k = 720, 64
    log("generating the plain-large workload")
    w = make_config(2)
    ctx = reloc.Context(0)
    m = ctx.load_map(w.occ, w.resolution, w.origin)
    s = w.sample
    sid, n_hyp = ctx.sample_hypotheses(m, s["n_target"], s["min_spacing"], s["robot_radius"],
                                       seed=s["seed"])
    hyp = ctx.read_hypotheses(sid)
    rid = ctx.prepare(m, sid, w.ranges, w.angle_min, w.angle_increment, w.range_min,
                      w.range_max, n_theta=n_theta, batch_k=batch_k, tau=tau, k_out=10,
                      variant=args.variant)
    log("map %dx%d, %d hypotheses, warmup %d" % (w.occ.shape[1], w.occ.shape[0], n_hyp,
                                               args.warmup))
    for _ in range(args.warmup):
        ctx.run(rid)
    torch.cuda.synchronize()
    lat, evals, ray_ms, tam_ms, tot_ms = [], 0, [], [], []
    last = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        poses, st = ctx.run(rid)
        lat.append(time.perf_counter() - ts)
        evals += st["smad_evals"] + st["tam_evals"]
        ray_ms.append(st["ms_raycast"])
        tam_ms.append(st["ms_tam"])
        tot_ms.append(st["ms_total"])
        last = (poses, st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    poses, st = last
    log("timed %d steps in %.3f s; stages %d, early stop %d" % (args.steps, elapsed,
                                                              st["stages"], st["early_stopped"]))

    # roofline of the dominant kernel (fused ray cast + SMAD): algorithmic
    # integer ops = DDA iterations x ops per iteration, counted once outside
    # the timed region with the same kernel's step output
    _, _, steps = ctx.debug_raycast(rid, n_hyp, reloc.scan_info(
        w.ranges, w.angle_min, w.angle_increment, w.resolution, w.range_min, w.range_max,
        n_theta=n_theta)["Ns"], steps=True)
    dda_steps = int(steps.astype(np.int64).sum())
    t_ray = float(np.mean(ray_ms)) * 1e-3
    achieved = dda_steps * DDA_OPS_PER_STEP / t_ray
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        traffic = json.load(open(args.traffic)).get("bytes_per_launch")
    roofline = {"kernel": "raycast_smad_kernel", "bound": "alu",
                "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s (int32 lane-ops)", "frac": achieved / VALU_PEAK_OPS,
                "traffic": traffic, "dda_steps": dda_steps,
                "avg_ms": t_ray * 1e3}
    out = {
        "metric": "hypothesis x orientation evals/s (SMAD+TAM)",
        "value": evals / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f32+f64",
        "data": "synthetic",
        "config": {"workload": "plain-large: warehouse 2000x2000 @0.05 m, 20000 hypotheses, "
                               "270 deg 720 beams, 0.5 deg TAM, top-64 per stage",
                   "tau": tau, "n_hyp": n_hyp, "n_theta": n_theta, "batch_k": batch_k},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3)},
        "per_step": {"smad_evals": st["smad_evals"], "tam_evals": st["tam_evals"],
                     "stages": st["stages"], "early_stopped": st["early_stopped"],
                     "device_ms": float(np.mean(tot_ms)), "raycast_ms": float(np.mean(ray_ms)),
                     "tam_ms": float(np.mean(tam_ms)), "rays": st["rays"],
                     "rays_per_s": st["rays"] / t_ray, "tam_lookups": st["tam_lookups"]},
        "best_pose": {k: poses[0][k] for k in ("x", "y", "theta", "tam", "hyp", "k")},
        "true_pose": list(w.pose),
        "roofline": roofline,
    }
    ctx.release(rid)
    if not args.no_cpu:
        log("cpu baseline (oracle) ~%.0f s" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(w, hyp, n_theta, batch_k, st["stages"],
                                           args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
