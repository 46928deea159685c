#!/usr/bin/env python3
"""Benchmark of the relocalization hot path on one MI355X.

Metric: hypothesis x orientation evaluations per second, SMAD + TAM
(SMAD evals = N_p x circular shifts, 1 shift when the FoV covers >= 90 % of
the turn; TAM evals = hypotheses evaluated by TAM x N_theta), plus p50/p99
latency of one relocalization.

Default workload (stress): 8000 x 8000 mixed warehouse and rooms map at
0.05 m, 200 000 hypotheses, panoramic 1440-beam scan taken in a perturbed
copy of the map with 15 % short-return clutter, 1440 TAM orientations
(0.25 deg), 256 hypotheses per stage, tau = 0.95. Each timed step is one
whole relocalization through reloc_relocalize, from the host scan to the
host poses: scan preprocessing and table upload, fused ray cast + SMAD of
every hypothesis, SMAD order, TAM stages with early termination, ranking,
release. Map and hypothesis set are resident before timing starts; the
ray-cast launch shape is tuned once for the map, outside the timed region.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload ...]
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

FP64_ADD_PEAK = 256 * 4 * 16 * 2.4e9       # FP64 adds/s (lane-ops; FP64 runs at the FP32 rate)
# Algorithmic work of one iteration of the jump traversal (one free-space
# jump test, one exact crossing, one walk-word test): int32 VALU operations
# of that path in the compiled loop of the fused kernel.
OPS_PER_ITER = 50
COARSE = {"smad": 0, "smad-direct": 1, "caer": 2, "none": 3}
FINE = {"tam": 0, "tam-mean": 1, "baseline": 2, "lf": 3}
RAYCAST_SOURCES = ("paper_2511_01219_amd/csrc/k_raycast.hip",
                   "paper_2511_01219_amd/csrc/raycast.h")
# counter summaries of the dominant kernel on the default workload
TRAFFIC_FILE = "profiles/raycast_smad_kernel_stress_traffic.txt"
COUNTERS_FILE = "profiles/raycast_smad_kernel_stress_counters.txt"
WORKLOADS = {   # config number, TAM orientations, hypotheses per stage
    "plain-small": (1, 360, 10),
    "plain-large": (2, 720, 64),
    "stress": (5, 1440, 256),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def exact_crossings(hit, hyp, Ns, W, H, rcells, chunk=4096):
    """Cell crossings of the plain step-by-step traversal of every ray: for a
    hit |dx| + |dy| to the hit cell; for a miss the crossings done when the
    ray first passes the map edge or the cut-off (continuous geometry).
    Hypotheses are taken chunk by chunk to bound host memory."""
    import numpy as np
    n = len(hyp)
    hit = hit.reshape(n, Ns)
    ang = 2.0 * np.pi * np.arange(Ns) / Ns
    ux, uy = np.cos(ang)[None, :], np.sin(ang)[None, :]
    ux = np.where(np.abs(ux) < 1e-12, 0.0, ux)
    uy = np.where(np.abs(uy) < 1e-12, 0.0, uy)
    ax, ay = np.abs(ux), np.abs(uy)
    total = 0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        ix0 = hyp[a:b, 0:1].astype(np.int64)
        iy0 = hyp[a:b, 1:2].astype(np.int64)
        h = hit[a:b].astype(np.int64)
        hx, hy = h % W, h // W
        steps = np.where(h >= 0, np.abs(hx - ix0) + np.abs(hy - iy0), 0)
        lx = np.minimum(rcells, np.where(ux > 0, W - 1 - ix0, np.where(ux < 0, ix0, rcells)))
        ly = np.minimum(rcells, np.where(uy > 0, H - 1 - iy0, np.where(uy < 0, iy0, rcells)))
        with np.errstate(divide="ignore", invalid="ignore"):
            tx = np.where(ax > 0, (0.5 + lx) / ax, np.inf)
            ty = np.where(ay > 0, (0.5 + ly) / ay, np.inf)
            te = np.minimum(tx, ty)
            cx = np.where(ax > 0, np.floor(te * ax - 0.5) + 1, 0)
            cy = np.where(ay > 0, np.floor(te * ay - 0.5) + 1, 0)
        total += int(np.where(h >= 0, steps, cx + cy).sum())
    return total


def _summary(path):
    """key: value lines of a committed counter summary, or None when the file
    is missing or the ray-cast sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    hs = hashlib.sha256()
    for f in RAYCAST_SOURCES:
        hs.update(open(os.path.join(ROOT, f), "rb").read())
    if kv.get("source_sha256") != hs.hexdigest():
        return None
    return kv


def measured_traffic():
    """HBM bytes per launch of the fused ray-cast kernel on the default
    workload from the committed FETCH_SIZE / WRITE_SIZE summary, or None when
    the kernel sources changed since it was taken."""
    kv = _summary(TRAFFIC_FILE)
    try:
        return float(kv["bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def measured_counters():
    """Executed VALU wave-instructions and L2 read requests per launch of the
    fused ray-cast kernel on the default workload (committed counter summary,
    same pass as its duration), or None when stale."""
    kv = _summary(COUNTERS_FILE)
    try:
        return {k: float(kv[k]) for k in ("valu_insts_per_launch", "tcp_tcc_read_req_per_launch",
                                          "duration_ns")} if kv else None
    except (KeyError, ValueError):
        return None


def _oracle_steps(w, hyp, pr, k, n_tam, n_theta, budget_s, threads):
    """Whole oracle steps (ray cast and direct-sum SMAD of every hypothesis in
    hyp, TAM of the first n_tam in SMAD order) until budget_s has passed."""
    import numpy as np
    import oracle
    steps, evals = 0, 0
    t0 = time.perf_counter()
    while True:
        _, z = oracle.raycast(w.occ, hyp, pr["Ns"], pr["Ng"], w.resolution, w.range_max,
                              threads=threads)
        sm, _ = oracle.smad(z, pr, threads=threads)
        order = np.lexsort((np.arange(len(sm)), sm))[:n_tam]
        q = np.repeat(hyp[order], n_theta, axis=0)
        kk = np.tile(np.arange(n_theta), n_tam)
        oracle.tam(k, w.resolution, pr, q, kk, threads=threads)
        steps += 1
        evals += len(hyp) * pr["n_shifts"] + n_tam * n_theta
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            return steps, evals, dt


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, hyp, n_theta, batch_k, stages_gpu, budget_s):
    """The oracle as it stands on the host cores: whole steps of the same
    workload (ray cast and direct-sum SMAD of every hypothesis, TAM of the
    stages the GPU ran), repeated until about budget_s has passed; then the
    same steps on one thread over the first 1/16 of the hypotheses (at
    least 64), TAM of the same share of the evaluated ones, for about
    budget_s / 3."""
    import oracle
    pr = oracle.prep(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                     range_min=w.range_min, range_max=w.range_max, n_theta=n_theta)
    k = oracle.edt(w.occ)
    threads = oracle.num_threads()
    n_tam = min(len(hyp), stages_gpu * batch_k)
    steps, evals, dt = _oracle_steps(w, hyp, pr, k, n_tam, n_theta, budget_s, 0)
    sub = hyp[:max(64, len(hyp) // 16)]
    n_sub = max(1, min(len(sub), round(n_tam * len(sub) / len(hyp))))
    s1, e1, d1 = _oracle_steps(w, sub, pr, k, n_sub, n_theta, budget_s / 3, 1)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": "%d whole steps: ray cast + direct-sum SMAD of all %d hypotheses, "
                      "TAM of the first %d in SMAD order x %d orientations; %.1f s"
                      % (steps, len(hyp), n_tam, n_theta, dt),
            "single_thread": {"value": e1 / d1, "unit": "evals/s", "cores": 1,
                              "sample": "%d steps over the first %d hypotheses, TAM of %d "
                                        "x %d orientations; %.1f s"
                                        % (s1, len(sub), n_sub, n_theta, d1)},
            "host": {"cpu_model": _cpu_model(), "cpu_count": os.cpu_count(),
                     "affinity": affinity}}


def accuracy(pose, truth, st):
    """Error of the best pose against the true pose, with the success
    criterion of Sec. IV-C (position error below 0.5 m and heading error
    below 30 deg), and the run's ambiguity statistics (Remark 1)."""
    d = math.hypot(pose["x"] - truth[0], pose["y"] - truth[1])
    phi = abs((pose["theta"] - truth[2] + math.pi) % (2 * math.pi) - math.pi)
    deg = math.degrees(phi)
    return {"d_err_m": d, "phi_err_deg": deg, "success": bool(d < 0.5 and deg < 30.0),
            "best_margin": st["best_margin"], "ambiguous": st["ambiguous"]}


def _load_multi(ctx, w):
    mids, sids = [], []
    for m, occ in enumerate(w.maps):
        mid = ctx.load_map(occ, w.resolution)
        sid, _ = ctx.sample_hypotheses(mid, w.sample["n_target"][m], w.sample["min_spacing"],
                                       w.sample["robot_radius"], seed=w.sample["seeds"][m])
        mids.append(mid)
        sids.append(sid)
    return mids, sids


def _scan_args(q):
    return (q.ranges, q.angle_min, q.angle_increment, q.range_min, q.range_max)


def bench_batched(args):
    """64 queries over 8 resident maps: the batched form (one reloc_run_batch)
    against the plain path (reloc_run of one request after another)."""
    import numpy as np
    import torch
    import paper_2511_01219_amd as reloc
    from synth import make_batched
    log("generating the batched workload")
    w = make_batched(64)
    ctx = reloc.Context(0)
    mids, sids = _load_multi(ctx, w)
    rids = [ctx.prepare(mids[q.map_index], sids[q.map_index], *_scan_args(q), n_hyp=q.n_hyp,
                        k_out=10, **q.search) for q in w.queries]
    log("%d requests prepared, %d hypotheses" % (len(rids), sum(q.n_hyp for q in w.queries)))
    for _ in range(args.warmup):
        ref = ctx.run_batch(rids)
        plain = [ctx.run(r) for r in rids]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain = [ctx.run(r) for r in rids]
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.run_batch(rids)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    same = all(a[0][0]["hyp"] == b[0][0]["hyp"] and a[0][0]["k"] == b[0][0]["k"] and
               a[0][0]["tam"] == b[0][0]["tam"] and a[1]["n_eval"] == b[1]["n_eval"]
               for a, b in zip(plain, res))
    evals = sum(st["smad_evals"] + st["tam_evals"] for _, st in res)
    st0 = res[0][1]
    out = {
        "metric": "hypothesis x orientation evals/s (SMAD+TAM)",
        "value": evals / t_batch, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32+f32+f64", "data": "synthetic",
        "config": {"workload": "batched: 64 queries over 8 maps (rooms and warehouse at "
                               "500^2, 1000^2, 2000^2, 4000^2), 1k-50k hypotheses, FoV "
                               "180-360 deg, 360-1080 beams, N_theta 360, top-64, tau 0.95",
                   "n_queries": len(rids), "n_hyp_total": int(sum(st["n_hyp"] for _, st in res))},
        "plain": {"value": evals / t_plain, "ms_per_step": t_plain * 1e3},
        "speedup_vs_plain": t_plain / t_batch,
        "identical_to_plain": bool(same),
        "phases_ms": {k: st0[k] for k in ("ms_raycast", "ms_smad", "ms_sort", "ms_tam",
                                          "ms_rank")},
        "stages": {"max": int(max(st["stages"] for _, st in res)),
                   "total": int(sum(st["stages"] for _, st in res))},
    }
    for r in rids:
        ctx.release(r)
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_sweep(args):
    """Dense sweeps on the plain-small map (Sec. IV Case 1 analogues): the
    SMAD map over every feasible cell (Fig. 7) and TAM and baseline over a
    0.1 m x 10 deg lattice of 15 x 36 poses around the true pose (Fig. 8);
    one step = both sweeps."""
    import numpy as np
    import torch
    import paper_2511_01219_amd as reloc
    from synth import make_config
    w = make_config(1)
    ctx = reloc.Context(0)
    m = ctx.load_map(w.occ, w.resolution, w.origin)
    k = ctx.read_edt(m)
    F = (w.occ >= 0) & (w.occ < 65) & (k >= 18)
    ys, xs = np.nonzero(F)
    cells = np.stack([xs, ys], 1).astype(np.int32)
    n = len(cells)
    sid = ctx.set_hypotheses(m, cells)
    scan = (w.ranges, w.angle_min, w.angle_increment, w.range_min, w.range_max)
    rid = ctx.prepare(m, sid, *scan, n_theta=360, batch_k=10)
    rid_b = ctx.prepare(m, sid, *scan, n_theta=360, batch_k=10, fine_metric=2)
    Ng = 1440
    c0 = np.floor((np.asarray(w.pose[:2]) - np.asarray(w.origin)) / w.resolution).astype(int)
    g0 = int(round(w.pose[2] * Ng / (2 * math.pi))) % Ng
    lx = np.array([(c0[0] + 2 * t, c0[1]) for t in range(-7, 8) for _ in range(36)], np.int32)
    lg = np.array([(g0 + 40 * j) % Ng for _ in range(-7, 8) for j in range(36)], np.int32)
    log("sweep: %d feasible cells, %d lattice poses" % (n, len(lg)))
    for _ in range(args.warmup):
        ctx.coarse_scores(rid, n)
        ctx.score_poses(rid, lx, lg)
        ctx.score_poses(rid_b, lx, lg)
    torch.cuda.synchronize()
    dev_c, dev_t, dev_b = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, _, st = ctx.coarse_scores(rid, n)
        dev_c.append(st["ms_total"])
        _, ms = ctx.score_poses(rid, lx, lg)
        dev_t.append(ms)
        _, ms = ctx.score_poses(rid_b, lx, lg)
        dev_b.append(ms)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    evals = args.steps * (st["smad_evals"] + 2 * len(lg))
    out = {
        "metric": "hypothesis x orientation evals/s (SMAD+TAM)",
        "value": evals / elapsed, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32+f32+f64", "data": "synthetic",
        "config": {"workload": "sweep: plain-small map, SMAD over all %d feasible cells "
                               "(480 shifts), TAM and baseline at 15 x 36 lattice poses" % n},
        "heatmap": {"cells": n, "device_ms": float(np.mean(dev_c)),
                    "rays_per_s": st["rays"] / (float(np.mean(dev_c)) * 1e-3),
                    "smad_evals": st["smad_evals"]},
        "lattice": {"poses": len(lg), "tam_ms": float(np.mean(dev_t)),
                    "baseline_ms": float(np.mean(dev_b))},
        "cpu_baseline": None,
    }
    ctx.release(rid)
    ctx.release(rid_b)
    ctx.free_hypotheses(sid)
    ctx.close()
    print(json.dumps(out), flush=True)


def cpu_baseline_sampled(w, hyp, n_theta, n_eval, budget_s):
    """The oracle on seeded 1 % subsamples of the workload (ray cast and
    direct-sum SMAD of 1 % of the hypotheses, TAM of 1 % of the evaluated
    ones over every orientation), one subsample after another until about
    budget_s has passed; the x100 extrapolation of one subsample's time is
    reported as such."""
    import numpy as np
    import oracle
    pr = oracle.prep(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                     range_min=w.range_min, range_max=w.range_max, n_theta=n_theta)
    k = oracle.edt(w.occ)
    n = len(hyp)
    n_sub = max(1, n // 100)
    n_tam = max(1, n_eval // 100)
    t0 = time.perf_counter()
    samples, evals = 0, 0
    while True:
        sub = np.sort(np.random.default_rng([5, 6, samples]).choice(n, n_sub, replace=False))
        _, z = oracle.raycast(w.occ, hyp[sub], pr["Ns"], pr["Ng"], w.resolution, w.range_max)
        oracle.smad(z, pr)
        q = np.repeat(hyp[sub[:n_tam]], n_theta, axis=0)
        oracle.tam(k, w.resolution, pr, q, np.tile(np.arange(n_theta), n_tam))
        samples += 1
        evals += n_sub * pr["n_shifts"] + n_tam * n_theta
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": evals / dt, "unit": "evals/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d seeded 1 %% subsamples, each: ray cast + direct-sum SMAD of %d "
                      "hypotheses, TAM of %d x %d orientations; %.1f s in all; x100 "
                      "extrapolation of one relocalization: %.1f s"
                      % (samples, n_sub, n_tam, n_theta, dt, 100 * dt / samples),
            "extrapolated_step_s": 100 * dt / samples,
            "host": {"cpu_model": _cpu_model(), "cpu_count": os.cpu_count(),
                     "affinity": affinity}}


def bench_single(args):
    """One relocalization per step on a single map: plain-small, plain-large
    or stress (the default)."""
    import numpy as np
    import torch
    import paper_2511_01219_amd as reloc
    from synth import make_config

    cid, n_theta, batch_k = WORKLOADS[args.workload]
    tau = None if args.tau.lower() in ("none", "nan") else float(args.tau)
    log("measuring device peaks")
    peaks = reloc.measure_peaks(0)
    log("peaks: int32 VALU %.1f T lane-ops/s, L2 gathers %.0f G/s, HBM read %.2f TB/s"
        % (peaks["valu_i32_ops"] / 1e12, peaks["l2_gathers"] / 1e9, peaks["hbm_read"] / 1e12))
    if args.calibrate_copy:
        # one device-to-device copy (a plain copy kernel): reads and writes
        # exactly this many bytes, the scale of the HBM byte counters
        nbytes = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(nbytes, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.calibrate_copy)
        del src, dst
    log("generating the %s workload" % args.workload)
    w = make_config(cid)
    ctx = reloc.Context(0)
    m = ctx.load_map(w.occ, w.resolution, w.origin)
    s = w.sample
    sid, n_hyp = ctx.sample_hypotheses(m, s["n_target"], s["min_spacing"], s["robot_radius"],
                                       seed=s["seed"])
    hyp = ctx.read_hypotheses(sid)
    rrt = None
    if args.sampler == "rrt":
        # Algorithm 1 from the first cell of the deterministic set as the
        # tree root, spacing rho of the workload; the set replaces the grid one
        p0 = ((hyp[0, 0] + 0.5) * w.resolution + w.origin[0],
              (hyp[0, 1] + 0.5) * w.resolution + w.origin[1])
        ctx.free_hypotheses(sid)
        t0 = time.perf_counter()
        sid, n_hyp, info = ctx.sample_rrt(m, p0, rho=s["min_spacing"],
                                          robot_radius=s["robot_radius"], seed=s["seed"])
        rrt = dict(info, seconds=time.perf_counter() - t0, n_hyp=n_hyp)
        log("RRT: %d hypotheses from %d nodes in %d rounds, %.2f s" % (
            n_hyp, info["nodes"], info["rounds"], rrt["seconds"]))
        hyp = ctx.read_hypotheses(sid)
    scan = (w.ranges, w.angle_min, w.angle_increment, w.range_min, w.range_max)
    search = dict(n_theta=n_theta, batch_k=batch_k, tau=tau, k_out=10, variant=args.variant,
                  refine_k=args.refine_k, refine_cells=args.refine_cells,
                  coarse_metric=COARSE[args.coarse], fine_metric=FINE[args.fine])
    tuned = None
    if args.variant == 0 and args.tune:
        # the ray-cast launch shape is picked once for the map (every shape
        # gives bit-identical results), outside the timed region; later
        # requests of the map with the same beam grid start from it
        rid = ctx.prepare(m, sid, *scan, **search)
        tv, tc, tms = ctx.autotune(rid, reps=2)
        ctx.release(rid)
        tuned = {"variant": tv, "shape": tc, "ms": tms}
        log("ray-cast shape tuned for the map: variant %d, shape %d, %.3f ms" % (tv, tc, tms))
    log("map %dx%d, %d hypotheses, warmup %d" % (w.occ.shape[1], w.occ.shape[0], n_hyp,
                                               args.warmup))
    for _ in range(args.warmup):
        ctx.relocalize(m, sid, *scan, **search)
    torch.cuda.synchronize()
    lat, evals, ray_ms, smad_ms, tam_ms, tot_ms = [], 0, [], [], [], []
    last = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        poses, st = ctx.relocalize(m, sid, *scan, **search)
        lat.append(time.perf_counter() - ts)
        evals += st["smad_evals"] + st["tam_evals"]
        ray_ms.append(st["ms_raycast"])
        smad_ms.append(st["ms_smad"])
        tam_ms.append(st["ms_tam"])
        tot_ms.append(st["ms_total"])
        last = (poses, st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    poses, st = last
    log("timed %d steps in %.3f s; stages %d, early stop %d" % (args.steps, elapsed,
                                                              st["stages"], st["early_stopped"]))

    # roofline of the dominant kernel, the fused ray cast + SMAD (its mean
    # launch time from the hipEvents the library records around it on its
    # own stream in every timed step)
    info = reloc.scan_info(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                           w.range_min, w.range_max, n_theta=n_theta)
    Ns, pano = info["Ns"], info["n_shifts"] == 1
    iterations = crossings = 0
    if not args.no_roofline:
        rid = ctx.prepare(m, sid, *scan, **search)
        hit, _, iters = ctx.debug_raycast(rid, n_hyp, Ns, steps=True)
        ctx.release(rid)
        rcells = int(math.ceil(w.range_max / w.resolution)) + 2
        crossings = exact_crossings(hit, hyp[:n_hyp], Ns, w.occ.shape[1], w.occ.shape[0],
                                    rcells)
        del hit
        iterations = int(iters.astype(np.int64).sum())
        del iters
    t_ray = float(np.mean(ray_ms)) * 1e-3
    shape = tuned["shape"] if tuned else None
    refill = {3: 8, 4: 16, 5: 32}.get(tuned["variant"]) if tuned else None
    kname = ("raycast_smad_kernel<%s,%s,%s>" % (shape or "default", refill or 16,
                                                "pano" if pano else "shifts")
             if args.variant == 0 and COARSE[args.coarse] == 0 else "split ray cast")
    alg_ops = iterations * OPS_PER_ITER / t_ray
    cnt = measured_counters() if args.workload == "stress" else None
    traffic = measured_traffic() if args.workload == "stress" else None
    roofline = {"kernel": kname, "bound": "alu", "unit": "TOP/s (int32 lane-ops)",
                "peak": peaks["valu_i32_ops"] / 1e12, "traffic": traffic,
                "avg_ms": t_ray * 1e3}
    if cnt:
        # executed VALU lane-ops per launch (counters of the same kernel,
        # workload and sources) over this run's mean launch time
        ex = cnt["valu_insts_per_launch"] * 64.0
        roofline.update(achieved=ex / t_ray / 1e12, frac=ex / t_ray / peaks["valu_i32_ops"],
                        basis="executed VALU lane-ops (committed counters) / live launch time")
        roofline["gather"] = {
            "l2_requests_per_s": cnt["tcp_tcc_read_req_per_launch"] / t_ray,
            "peak_l2_random_gathers_per_s": peaks["l2_gathers"],
            "frac": cnt["tcp_tcc_read_req_per_launch"] / t_ray / peaks["l2_gathers"]}
    else:
        roofline.update(achieved=alg_ops / 1e12, frac=alg_ops / peaks["valu_i32_ops"],
                        basis="algorithmic: traversal iterations x %d ops / live launch time"
                              % OPS_PER_ITER)
    roofline["algorithmic"] = {"unit": "traversal iteration (jump test + crossing)",
                               "iterations_per_launch": iterations,
                               "ops_per_iteration": OPS_PER_ITER,
                               "achieved": alg_ops / 1e12,
                               "frac": alg_ops / peaks["valu_i32_ops"]}
    roofline["dda_crossing_rate"] = {
        "note": "cells a step-by-step traversal visits; the jump traversal skips most of them",
        "crossings_per_launch": crossings, "crossings_per_s": crossings / t_ray}
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
        "config": {"workload": {
            "plain-small": "plain-small: rooms 200x200 @0.05 m, 300 hypotheses, 270 deg 360 "
                           "beams, 1 deg TAM, top-10 per stage",
            "plain-large": "plain-large: warehouse 2000x2000 @0.05 m, 20000 hypotheses, 270 deg "
                           "720 beams, 0.5 deg TAM, top-64 per stage",
            "stress": "stress: mixed 8000x8000 @0.05 m, 200000 hypotheses, 360 deg 1440 beams "
                      "(perturbed map, 15 % clutter), 0.25 deg TAM, top-256 per stage"}[
                          args.workload],
                   "tau": tau, "n_hyp": n_hyp, "n_theta": n_theta, "batch_k": batch_k,
                   "refine_k": args.refine_k,
                   "refine_cells": args.refine_cells if args.refine_k else None,
                   "coarse": args.coarse, "fine": args.fine, "sampler": args.sampler,
                   "timed_step": "reloc_relocalize: prepare + run + release"},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "what": "submit to poses on the host, whole relocalization"},
        "value_by_kind": {"smad_evals_per_s": args.steps * st["smad_evals"] / elapsed,
                          "tam_evals_per_s": args.steps * st["tam_evals"] / elapsed},
        "per_step": {"smad_evals": st["smad_evals"], "tam_evals": st["tam_evals"],
                     "stages": st["stages"], "early_stopped": st["early_stopped"],
                     "device_ms": float(np.mean(tot_ms)), "raycast_ms": float(np.mean(ray_ms)),
                     "smad_ms": float(np.mean(smad_ms)),
                     "tam_ms": float(np.mean(tam_ms)), "rays": st["rays"],
                     "rays_per_s": st["rays"] / t_ray, "tam_lookups": st["tam_lookups"],
                     "tam_lookups_per_s": st["tam_lookups"] / max(1e-9, float(np.mean(tam_ms))
                                                                  * 1e-3),
                     "refined": st["refined"], "refine_points": st["refine_points"]},
        "best_pose": {k: poses[0][k] for k in ("x", "y", "theta", "tam", "hyp", "k", "g",
                                               "refined")},
        "true_pose": list(w.pose),
        "accuracy": accuracy(poses[0], w.pose, st),
        "peaks": peaks,
        "roofline": roofline,
        "autotune": tuned,
        "rrt": rrt,
    }
    if COARSE[args.coarse] in (1, 2):
        # the direct coarse kernel: one FP64 subtract and one FP64 add (of an
        # absolute value) per (hypothesis, shift, FoV beam) term for CAER, one
        # add for direct-sum SMAD; FP64 add peak = 256 CUs x 64 lanes x 2.4 GHz
        caer = COARSE[args.coarse] == 2
        nsh = info["Ns"] if caer else info["n_shifts"]
        terms = n_hyp * nsh * info["n_fov"]
        t_c = float(np.mean(smad_ms)) * 1e-3
        ops = terms * (2 if caer else 1)
        out["coarse_roofline"] = {"kernel": "coarse_direct_kernel", "bound": "alu",
                                  "achieved": ops / t_c / 1e12, "peak": FP64_ADD_PEAK / 1e12,
                                  "unit": "TOP/s (fp64 lane-ops)",
                                  "frac": ops / t_c / FP64_ADD_PEAK, "terms": terms,
                                  "avg_ms": t_c * 1e3}
    if tau is not None and not args.no_full_search and args.workload != "stress":
        # untimed: the same search without early termination, so the line
        # shows what the stop test at tau gave up (Sec. IV-C criterion)
        pf, sf = ctx.relocalize(m, sid, *scan, **dict(search, tau=None))
        out["accuracy"]["full_search"] = dict(accuracy(pf[0], w.pose, sf), tam=pf[0]["tam"],
                                              rank=pf[0]["rank"], ms=sf["ms_total"])
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)
    ctx.close()
    if args.no_cpu:
        out["cpu_baseline"] = None
    elif args.workload == "stress":
        log("cpu baseline (oracle, 1 %% subsamples) ~%.0f s" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline_sampled(w, hyp[:n_hyp], n_theta, st["n_eval"],
                                                   args.cpu_seconds)
    else:
        log("cpu baseline (oracle) ~%.0f s" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(w, hyp, n_theta, batch_k, st["stages"],
                                           args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """Open-loop Poisson replay over 16 resident maps: served (reloc_submit /
    reloc_poll, continuous batching) against plain FIFO (reloc_relocalize of
    one request after another in arrival order) on the same trace."""
    import threading
    import numpy as np
    import torch
    import paper_2511_01219_amd as reloc
    from synth import make_serving
    log("generating the serving workload")
    w = make_serving(1.0, args.requests)        # arrivals at rate 1, rescaled per rate
    ctx = reloc.Context(0)
    mids, sids = _load_multi(ctx, w)
    qs = w.queries
    base = np.array([q.arrival for q in qs])

    def call_args(q):
        return (mids[q.map_index], sids[q.map_index]) + _scan_args(q)

    for q in qs[:8]:                            # warm-up
        ctx.relocalize(*call_args(q), n_hyp=q.n_hyp, **q.search)
    torch.cuda.synchronize()
    rows = []
    for rate in [float(x) for x in args.rates.split(",")]:
        arr = base / rate
        # served
        ctx.serve_configure(max_inflight=args.max_inflight, max_admit=args.max_admit)
        sub = []
        start = time.perf_counter()

        def submitter():
            for i, q in enumerate(qs):
                d = start + arr[i] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tc = time.perf_counter()
                sub.append((i, ctx.submit(*call_args(q), n_hyp=q.n_hyp, **q.search), tc))

        th = threading.Thread(target=submitter)
        th.start()
        lat_s, fin_s, served = [], [], {}
        idx = 0
        while idx < len(qs):
            while idx >= len(sub):
                time.sleep(0.0002)
            i, t, tc = sub[idx]
            idx += 1
            poses, st = ctx.poll(t, wait_ms=-1)
            done = tc + st["ms_total"] * 1e-3
            lat_s.append(done - (start + arr[i]))
            fin_s.append(done)
            served[i] = (poses[0]["hyp"], poses[0]["k"], poses[0]["tam"],
                         st["smad_evals"] + st["tam_evals"])
        th.join()
        span_s = max(fin_s) - start
        sstats = ctx.serve_stats()
        # plain FIFO
        lat_f, same = [], True
        start = time.perf_counter()
        for i, q in enumerate(qs):
            d = start + arr[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            poses, st = ctx.relocalize(*call_args(q), n_hyp=q.n_hyp, **q.search)
            lat_f.append(time.perf_counter() - (start + arr[i]))
            same &= served[i][:3] == (poses[0]["hyp"], poses[0]["k"], poses[0]["tam"])
        span_f = time.perf_counter() - start
        evals = sum(v[3] for v in served.values())
        rows.append({
            "rate_per_s": rate, "requests": len(qs),
            "served": {"p50_ms": float(np.percentile(lat_s, 50) * 1e3),
                       "p99_ms": float(np.percentile(lat_s, 99) * 1e3),
                       "evals_per_s": evals / span_s, "req_per_s": len(qs) / span_s,
                       "rounds": int(sstats["ticks"])},
            "fifo": {"p50_ms": float(np.percentile(lat_f, 50) * 1e3),
                     "p99_ms": float(np.percentile(lat_f, 99) * 1e3),
                     "evals_per_s": evals / span_f, "req_per_s": len(qs) / span_f},
            "identical_best_pose": bool(same)})
        log("rate %.0f/s: served p50 %.1f ms p99 %.1f ms, fifo p50 %.1f ms p99 %.1f ms"
            % (rate, rows[-1]["served"]["p50_ms"], rows[-1]["served"]["p99_ms"],
               rows[-1]["fifo"]["p50_ms"], rows[-1]["fifo"]["p99_ms"]))
    out = {"metric": "p50/p99 relocalization latency and evals/s under Poisson load",
           "unit": "ms", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "config": {"workload": "serving: 16 maps (4 each of 1000^2, 2000^2, 3000^2, "
                                  "4000^2), 2k-40k hypotheses, FoV 270/360 deg, 540-1440 "
                                  "beams, N_theta 360, top-64, tau 0.95",
                      "requests_per_rate": len(qs), "max_inflight": args.max_inflight,
                      "max_admit": args.max_admit},
           "serving": rows}
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_peaks(args):
    """The device's measured peaks alone (reloc_measure_peaks)."""
    import paper_2511_01219_amd as reloc
    p = reloc.measure_peaks(0)
    print(json.dumps({"metric": "measured peaks", "peaks": p, "n_gpus": 1}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tau", default="0.95")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-full-search", action="store_true",
                    help="skip the untimed search without early termination that the "
                         "accuracy report of a tau run adds (profiler runs that count "
                         "the timed launches only)")
    ap.add_argument("--no-roofline", action="store_true",
                    help="skip the untimed debug ray cast behind the roofline fields "
                         "(profiler runs that count the timed launches only)")
    ap.add_argument("--tune", action="store_true",
                    help="tune the ray-cast launch shape once for the map (untimed) instead "
                         "of the default shape")
    ap.add_argument("--variant", type=int, default=0,
                    help="ray-cast kernel: 0 fused default, 1 bit tiles, 2-5 split skipping")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="stress",
                    choices=("stress", "plain-large", "plain-small", "batched", "serving",
                             "sweep", "peaks"))
    ap.add_argument("--rates", default="50,100,200,500", help="serving: arrivals per second")
    ap.add_argument("--requests", type=int, default=400, help="serving: requests per rate")
    ap.add_argument("--max-inflight", type=int, default=64)
    ap.add_argument("--max-admit", type=int, default=16)
    ap.add_argument("--refine-k", type=int, default=0,
                    help="plain workloads: poses refined per stage (local TAM lattice search)")
    ap.add_argument("--refine-cells", type=int, default=3,
                    help="refinement lattice half-width in cells")
    ap.add_argument("--sampler", default="grid", choices=("grid", "rrt"),
                    help="plain workloads: hypothesis sampler (grid: fixed count; rrt: Alg. 1)")
    ap.add_argument("--coarse", default="smad", choices=tuple(COARSE),
                    help="plain workloads: coarse metric (ablation)")
    ap.add_argument("--fine", default="tam", choices=tuple(FINE),
                    help="plain workloads: fine metric (ablation)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "peaks":
        return bench_peaks(args)
    return bench_single(args)


if __name__ == "__main__":
    main()
