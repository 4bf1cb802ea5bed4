"""Benchmark of the MI scan-alignment hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload all|uneven|c2f|batched|serving|accuracy|surface]
                    [--calibrate-copy]

Default (--workload all) prints one JSON line whose headline is the uneven
batch: 64 surface-sampled scan pairs, points log-uniform in 10k-300k, voxels
0.25 / 0.5 / 1 m (grids up to 640 x 640 x 40), count + z-variance features at
32 bins, 4096 candidate 6-DOF poses per pair (262,144 MI evaluations), all in
one batch per step.  A step is one execution of that batch; K steps are timed
after W warm-up steps, inputs resident in HBM.  The same line carries, under
"workloads", the other configured workloads, each with its own throughput,
roofline and CPU-oracle baseline:

  c2f      a realistic pair: two 64-ring spinning-scanner scans (~115k points
           each) of a 160 x 160 m urban scene, 0.5 m voxels over 320 x 320 x 20,
           both features at 32 bins; 3 coarse-to-fine levels of 5^6 poses, and
           a finer search (7,7,5,5,5,9 nodes, 6 levels, shrink 2) for accuracy;
  batched  the tiny pair (~20k / ~14k points, 1 m voxels, 64 x 64 x 10, count at
           32 bins) with 8^6 = 262,144 poses in one batch, replayed as one
           captured HIP graph;
  serving  alignment requests (surface-sampled pairs, 20k-250k points, 0.5 or
           1 m voxels, 3 levels x 4^6 poses) arriving as Poisson processes at
           50, 200 and 800 req/s, 2,000 requests per rate, served by the
           continuous-batching loop: throughput and p50/p99 latency against one
           request at a time.

Each workload alone: --workload NAME (its own line).  accuracy and surface
run the paper's accuracy protocol and cost surfaces on synthetic stand-ins.
--calibrate-copy runs a plain 1 GiB device copy, the reference kernel that
scales the HBM byte counters of a profile.  --calibrate KIND|all runs the
roofline microbenchmarks (LDS atomics and compare-and-swap, HBM stream read,
FP64 issue); their committed results (profiles/roofline_calibration.md) give
each roofline a measured peak beside the published one.

Rooflines: the evaluator is bound by FP64/integer ALU work (no dense
contraction, so no MFMA); achieved = 27 algorithmic FP64 operations per
(point, pose) x the point-poses of a launch / the launch's mean duration
(HIP events on the launch stream during the timed region), against
256 CU x 4 SIMD x 16 lanes x 2.4 GHz.  traffic is the launch's HBM bytes from
the committed counter profile of that workload, while the kernel source is
unchanged since it was taken.  cpu_baseline is the FP64 CPU oracle timed on
a bounded sample of the same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz = 3.93e13 FP64 lane-ops/s
# (78.6 TFLOP/s counts a fused multiply-add as two; the voxel arithmetic has none).
PEAK_FP64_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic FP64 operations per (point, pose): 9 mul + 9 add for R p + t,
# 3 sub + 3 mul + 3 floor for the voxel coordinate and index.
OPS_PER_POINT_POSE = 27

EVAL_SOURCE = os.path.join(ROOT, "paper_1709_06948_amd", "csrc", "k_eval.hip")
TRAFFIC_FILES = {
    "uneven": os.path.join(ROOT, "profiles", "k_eval_uneven_64pairs_traffic.md"),
    "c2f": os.path.join(ROOT, "profiles", "k_eval_urban_c2f_traffic.md"),
}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=96)
    ap.add_argument("--cpu-per-pair", type=int, default=16,
                    help="uneven batch: poses of each pair the CPU oracle times")
    ap.add_argument("--workload", choices=("all", "uneven", "c2f", "batched", "serving",
                                           "accuracy", "surface"), default="all")
    ap.add_argument("--seeds", type=int, default=3)
    ap.add_argument("--features", choices=("count+zvar", "joint", "weighted"), default="count+zvar",
                    help="c2f workload: the features and objective (default: both features, "
                         "search on MI-VARZ)")
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--rates", default="50,200,800")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=24)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--serial", action="store_true",
                    help="generate the synthetic pairs in this process (no worker pool), as "
                         "under a profiler")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--calibrate", choices=("lds_u32", "lds_u64", "lds_cas", "hbm_read", "fp64",
                                            "all"),
                    help="roofline microbenchmarks: measured peaks of the units the evaluator uses")
    return ap.parse_args()


def _cores() -> int:
    return len(os.sched_getaffinity(0))


def _measured_traffic(workload):
    """HBM bytes per evaluator launch from the committed counter profile of the
    workload, or None when there is none or the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = TRAFFIC_FILES.get(workload)
    if not path:
        return None
    try:
        text = open(path).read()
        src = hashlib.sha256(open(EVAL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("k_eval.hip sha256") != src:
        return None
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def _roofline(prof, workload, **extra):
    """ALU roofline of the evaluator from the library's stage timings (HIP
    events recorded on the launch stream around every evaluator launch)."""
    launches = max(prof["eval_launches"], 1)
    ms = prof["eval_ms"] / launches
    pp = prof["point_poses"] / launches
    achieved = OPS_PER_POINT_POSE * pp / (ms * 1e-3) if ms > 0 else 0.0
    out = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
           "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_OPS,
           "traffic": _measured_traffic(workload), "kernel": "k_eval", "avg_launch_ms": ms,
           "point_poses_per_launch": pp, "eval_launches": prof["eval_launches"]}
    peaks = _measured_peaks()
    if peaks.get("fp64_lane_ops_per_s"):
        # the same work against the FP64 issue rate measured on this GPU
        out["measured_peak"] = peaks["fp64_lane_ops_per_s"] / 1e12
        out["frac_of_measured_peak"] = achieved / peaks["fp64_lane_ops_per_s"]
    out.update(extra)
    return out


SERIAL = False


def _parallel(fn, args):
    """fn over args in forked worker processes (before any GPU work), in order;
    in this process, printing progress, with --serial."""
    import multiprocessing as mp
    n = max(1, min(16, _cores(), len(args)))
    if n == 1 or SERIAL:
        out = []
        for i, x in enumerate(args):
            out.append(fn(x))
            if SERIAL and (i + 1) % 8 == 0:
                print(json.dumps({"generated": i + 1, "of": len(args)}), file=sys.stderr,
                      flush=True)
        return out
    with mp.get_context("fork").Pool(n) as pool:
        return pool.map(fn, args, chunksize=1)


def _line(metric, value, unit, steps, warmup, ms_per_step, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": config}
    out.update(extra)
    return out


CALIB_KINDS = {"lds_u32": (0, 2000, "LDS 32-bit atomic add lane-ops/s"),
               "lds_u64": (1, 2000, "LDS 64-bit atomic add lane-ops/s"),
               "lds_cas": (2, 2000, "LDS compare-and-swap lane-ops/s"),
               "hbm_read": (3, 1, "HBM stream read bytes/s"),
               "fp64": (4, 20000, "FP64 VALU mul/add lane-ops/s (no contraction)")}
CALIB_FILE = os.path.join(ROOT, "profiles", "roofline_calibration.md")


def _calibrate(a):
    """Each microbenchmark launched 5 times after a warm-up, timed with HIP
    events on the launch stream; the best rate is reported."""
    import torch

    from paper_1709_06948_amd import mi

    torch.cuda.set_device(0)
    kinds = list(CALIB_KINDS) if a.calibrate == "all" else [a.calibrate]
    out = {}
    for name in kinds:
        kind, size, what = CALIB_KINDS[name]
        nbytes = (4 << 30) if name == "hbm_read" else (1 << 20)
        scratch = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        s = torch.cuda.current_stream()
        mi.calibrate_launch(kind, size, scratch, stream=s)
        best = 0.0
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            ops = mi.calibrate_launch(kind, size, scratch, stream=s)
            e1.record(s)
            e1.synchronize()
            best = max(best, ops / (e0.elapsed_time(e1) * 1e-3))
        out[name] = {"rate": best, "unit": what}
        del scratch
    print(json.dumps({"calibration": out}), flush=True)


def _measured_peaks():
    """Peaks measured by --calibrate all (the committed profile), or {}."""
    vals = {}
    try:
        text = open(CALIB_FILE).read()
    except OSError:
        return vals
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            try:
                vals[k.strip()] = float(v.strip().strip("`"))
            except ValueError:
                pass
    return vals


def _calibrate_copy():
    import torch
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "dispatches": 3}),
          flush=True)


# --------------------------------------------------------------- uneven batch

UNEVEN_DESC = ("uneven batch: {n} surface-sampled scan pairs, points log-uniform in 10k-300k, "
               "voxels 0.25/0.5/1 m (grids up to 640x640x40), count + z-variance 32 bins, 4096 "
               "random 6-DOF poses per pair, all in one batch per step")


def _uneven_pair(j):
    from paper_1709_06948_amd import synth
    return synth.uneven_pair(j)


def _run_uneven(a, work):
    import torch

    from paper_1709_06948_amd import mi

    items = []
    for pair, poses in work:
        grid = mi.Grid(pair.origin, pair.dims, pair.voxel,
                       features=mi.FEAT_COUNT | mi.FEAT_ZVAR, nb_count=32, nb_zvar=32)
        items.append(mi.WorkItem(mi.Ref(grid, pair.A), pair.B, poses))
    torch.cuda.synchronize()
    batch = mi.Batch(items)
    K = sum(it.K for it in items)
    point_poses = sum(it.K * it.xyz_b.shape[1] for it in items)
    for _ in range(a.warmup):
        batch.execute()
    torch.cuda.synchronize()
    mi.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        batch.execute()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = mi.profile_read()
    mi.profile_enable(False)
    value = K * a.steps / dt
    res = {"value": value, "ms_per_step": dt * 1e3 / a.steps, "steps": a.steps,
           "warmup": a.warmup,
           "config": {"workload": UNEVEN_DESC.format(n=len(items)), "evals_per_step": K,
                      "pairs": len(items), "point_poses_per_step": point_poses},
           "gpoint_transforms_per_s": point_poses * a.steps / dt / 1e9,
           "roofline": _roofline(prof, "uneven",
                                 frames_ms_per_step=prof["frames_ms"] / a.steps)}
    del batch
    res["cpu_baseline"] = None
    if not a.no_cpu_baseline and a.cpu_per_pair > 0:
        import oracle as O
        cores = _cores()
        n_eval, tc = 0, 0.0
        for j, (pair, poses) in enumerate(work):
            og = O.Grid(pair.origin, pair.dims, pair.voxel, features=3, nb_count=32, nb_zvar=32)
            rng = np.random.default_rng(1000 + j)
            sel = np.sort(rng.choice(len(poses), min(a.cpu_per_pair, len(poses)), replace=False))
            t0 = time.perf_counter()
            O.eval_poses(og, pair.A, pair.B, poses[sel], nthreads=cores)
            tc += time.perf_counter() - t0
            n_eval += len(sel)
        res["cpu_baseline"] = {
            "value": n_eval / tc, "unit": "MI pose evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{a.cpu_per_pair} seeded random poses of each of the {len(work)} pairs "
                      f"({n_eval} evaluations) of the same batch, FP64 dense oracle, {tc:.1f} s"}
    return res


# ------------------------------------------------------------- coarse-to-fine

# A finer search than the configured one (nodes per axis, levels, shrink), with
# the same level-0 half-ranges: it recovers the urban pair's true pose.
FINE_SAMPLES = (7, 7, 5, 5, 5, 9)
FINE_LEVELS, FINE_SHRINK = 6, 2.0


def _run_c2f(a, pair):
    import torch

    from paper_1709_06948_amd import mi, synth

    c2f = synth.urban_c2f_params()
    fkw = dict(features=mi.FEAT_COUNT | mi.FEAT_ZVAR, nb_count=32, nb_zvar=32)
    slot, weights, fdesc = 1, None, "count + z-variance 32 bins, search on MI-VARZ"
    if a.features == "joint":
        fkw = dict(features=mi.FEAT_JOINT, nb_count=8, nb_zvar=8)
        slot, fdesc = 0, "joint count x z-variance feature (8 x 8 part bins, 50 values)"
    elif a.features == "weighted":
        weights, fdesc = (0.5, 0.5), "count + z-variance 32 bins, search on 0.5 MI-N + 0.5 MI-VARZ"
    grid = mi.Grid(pair.origin, pair.dims, pair.voxel, **fkw)
    A = torch.from_numpy(pair.A).cuda()
    B = torch.from_numpy(pair.B).cuda()
    n_b = B.shape[1]
    init = np.zeros(6)
    levels = int(c2f["levels"])
    K_level = int(np.prod(c2f["samples"]))
    evals_per_step = levels * K_level

    def step():
        ref = mi.Ref(grid, A)
        return mi.align_coarse_to_fine(ref, B, init, c2f["half"], c2f["samples"], levels,
                                       c2f["shrink"], feature_slot=slot, weights=weights)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    mi.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        pose, best = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = mi.profile_read()
    mi.profile_enable(False)
    value = evals_per_step * a.steps / dt
    ref = mi.Ref(grid, A)
    fine_pose, _ = mi.align_coarse_to_fine(ref, B, init, c2f["half"], FINE_SAMPLES, FINE_LEVELS,
                                           FINE_SHRINK, feature_slot=slot, weights=weights)
    res = {"value": value, "unit": "evals/s", "ms_per_step": dt * 1e3 / a.steps,
           "steps": a.steps, "warmup": a.warmup,
           "config": {"workload": "urban scan pair, 6-DOF coarse-to-fine: 2 x ~115k-point 64-ring "
                                  f"scans, 0.5 m voxels 320x320x20, {fdesc}, 3 levels x 5^6 poses",
                      "evals_per_step": evals_per_step, "n_b": int(n_b), "n_a": int(A.shape[1])},
           "gpoint_transforms_per_s": evals_per_step * n_b * a.steps / dt / 1e9,
           "roofline": _roofline(prof, "c2f" if a.features == "count+zvar" else "",
                                 frames_ms_per_step=prof["frames_ms"] / a.steps,
                                 eval_ms_per_step=prof["eval_ms"] / a.steps),
           "result": {"pose": [float(v) for v in pose], "mi": best,
                      "abs_err_vs_truth": [float(v) for v in np.abs(pose - pair.eta_gt)]},
           "fine_search": {"samples": list(FINE_SAMPLES), "levels": FINE_LEVELS,
                           "shrink": FINE_SHRINK, "pose": [float(v) for v in fine_pose],
                           "abs_err_vs_truth": [float(v) for v in np.abs(fine_pose - pair.eta_gt)]}}
    if a.plain_sample > 0:
        P0 = synth.level_poses(init, c2f["half"], c2f["samples"])
        rng = np.random.default_rng(1)
        Ps = P0[np.sort(rng.choice(len(P0), a.plain_sample, replace=False))]
        mi.eval_poses_plain(ref, B, Ps[:4])
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        mi.eval_poses_plain(ref, B, Ps)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        res["plain_path"] = {"evals_per_s": len(Ps) / tp, "sample": f"{len(Ps)} level-0 poses",
                             "batched_speedup": value / (len(Ps) / tp)}
    res["cpu_baseline"] = None
    if not a.no_cpu_baseline:
        import oracle as O
        og = O.Grid(pair.origin, pair.dims, pair.voxel, **fkw)
        Ps = synth.level_poses(init, c2f["half"], c2f["samples"])
        cores = _cores()
        O.eval_poses(og, pair.A, pair.B, Ps[:cores], nthreads=cores)
        tc0 = time.perf_counter()
        O.eval_poses(og, pair.A, pair.B, Ps, nthreads=cores)
        tc = time.perf_counter() - tc0
        res["cpu_baseline"] = {
            "value": len(Ps) / tc, "unit": "MI pose evals/s", "cores": cores, "kind": "oracle",
            "sample": f"all {len(Ps)} poses of level 0 of the same workload, FP64 dense oracle, "
                      f"{tc:.1f} s"}
    return res


# -------------------------------------------------------------------- batched

def _run_batched(a, pair):
    import torch

    from paper_1709_06948_amd import mi, synth

    grid = mi.Grid(pair.origin, pair.dims, pair.voxel, features=mi.FEAT_COUNT, nb_count=32)
    poses = synth.grid8_poses(8)
    items = [mi.WorkItem(mi.Ref(grid, pair.A), pair.B, poses)]
    torch.cuda.synchronize()
    batch = mi.Batch(items)
    K = len(poses)
    point_poses = K * pair.B.shape[1]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.execute(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.execute()
    for _ in range(a.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        graph.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # stage events cannot sit inside a graph: the evaluator's duration comes from
    # eager executions of the same batch right after the timed replays
    mi.profile_enable(True)
    for _ in range(2):
        batch.execute()
    torch.cuda.synchronize()
    prof = mi.profile_read()
    mi.profile_enable(False)
    value = K * a.steps / dt
    res = {"value": value, "unit": "evals/s", "ms_per_step": dt * 1e3 / a.steps,
           "steps": a.steps, "warmup": a.warmup,
           "config": {"workload": "tiny scan pair, 8^6 = 262,144 6-DOF poses in one batch (one "
                                  "captured HIP graph per step): ~20k / ~14k surface points, 1 m "
                                  "voxels 64x64x10, count 32 bins", "evals_per_step": K},
           "gpoint_transforms_per_s": point_poses * a.steps / dt / 1e9,
           "roofline": _roofline(prof, "batched", timed_on="2 eager executions after the replays")}
    res["cpu_baseline"] = None
    if not a.no_cpu_baseline:
        import oracle as O
        og = O.Grid(pair.origin, pair.dims, pair.voxel, features=1, nb_count=32)
        Ps = poses[::128]
        cores = _cores()
        tc0 = time.perf_counter()
        O.eval_poses(og, pair.A, pair.B, Ps, nthreads=cores)
        tc = time.perf_counter() - tc0
        res["cpu_baseline"] = {
            "value": len(Ps) / tc, "unit": "MI pose evals/s", "cores": cores, "kind": "oracle",
            "sample": f"every 128th of the 262,144 poses ({len(Ps)}), FP64 dense oracle, {tc:.1f} s"}
        # the tiny plain search (11 x 11 x 11 x, y, yaw poses, count in 16 bins) in full,
        # on one thread: the oracle's single-core rate on the smallest workload
        og1 = O.Grid(pair.origin, pair.dims, pair.voxel, features=1, nb_count=16)
        P1 = synth.tiny_search_poses()
        t10 = time.perf_counter()
        O.eval_poses(og1, pair.A, pair.B, P1, nthreads=1)
        t1 = time.perf_counter() - t10
        res["cpu_baseline"]["tiny_search_one_thread"] = {
            "value": len(P1) / t1, "unit": "MI pose evals/s", "cores": 1, "poses": len(P1),
            "seconds": t1}
    return res


# ------------------------------------------------- accuracy and cost surfaces

NM_STEP = [8.0, 8.0, 1.0, 0.1, 0.1, 0.8]
# Success: final error under one voxel (1 m) in translation and 2 deg in rotation.
SUCCESS_M, SUCCESS_DEG = 1.0, 2.0


def _bench_accuracy(a):
    """Accuracy protocol of Sec. IV (Figs. 4, 5) on synthetic displaced scans:
    every query aligned from the identity by mi_align_nelder_mead (one start,
    the paper's simplex), and again with four starts advancing together."""
    import math

    import torch

    from paper_1709_06948_amd import mi, synth

    torch.cuda.set_device(0)
    d2r = math.pi / 180.0
    starts4 = np.array([[0, 0, 0, 0, 0, 0], [4, 4, 0, 0, 0, 0.3], [-4, 4, 0, 0, 0, -0.3],
                        [0, -5, 0, 0, 0, 0]], np.float64)
    methods = [("nm", np.zeros((1, 6))), ("nm_4starts", starts4)]
    res = {}
    n_align, t_align, iters = 0, 0.0, []
    for study, cfg in (("translation", 6), ("rotation", 7)):
        for sd in range(a.seeds):
            D = synth.displaced_scans(seed=synth.seed_for(cfg, sd), study=study)
            grid = mi.Grid(D.origin, D.dims, D.voxel, features=mi.FEAT_COUNT | mi.FEAT_ZVAR,
                           nb_count=32, nb_zvar=32)
            ref = mi.Ref(grid, D.A)
            for i, (B, g) in enumerate(zip(D.B, D.eta_gt)):
                Bd = torch.from_numpy(B).cuda()
                for mname, starts in methods:
                    for slot, fname in ((0, "mi_n"), (1, "mi_varz")):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        pose, _, it = mi.align_nelder_mead(ref, Bd, starts, NM_STEP, 400, 1e-7,
                                                           1e-3, feature_slot=slot)
                        torch.cuda.synchronize()
                        t_align += time.perf_counter() - t0
                        n_align += 1
                        iters += [int(x) for x in it]
                        et = float(np.linalg.norm(pose[:3] - g[:3]))
                        er = float(np.linalg.norm(pose[3:] - g[3:]) / d2r)
                        key = (study, mname, fname, float(D.levels[i]))
                        res.setdefault(key, []).append((et, er))
    summary = {}
    for (study, mname, fname, lv), v in sorted(res.items()):
        e = np.array(v)
        ok = (e[:, 0] < SUCCESS_M) & (e[:, 1] < SUCCESS_DEG)
        summary.setdefault(study, {}).setdefault(mname, {}).setdefault(fname, {})[f"{lv:g}"] = {
            "median_t_err_m": round(float(np.median(e[:, 0])), 3),
            "median_r_err_deg": round(float(np.median(e[:, 1])), 3),
            "success": round(float(ok.mean()), 3)}
    overall = {}
    for (study, mname, fname, lv), v in res.items():
        e = np.array(v)
        ok = (e[:, 0] < SUCCESS_M) & (e[:, 1] < SUCCESS_DEG)
        overall.setdefault(f"{study}/{mname}/{fname}", []).extend(ok.tolist())
    out = {
        "metric": "NM alignments/s", "value": n_align / t_align, "unit": "alignments/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": t_align * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"accuracy protocol: {a.seeds} seeded urban scenes per study, "
                                "reference scan at the origin, 10 query scans each at 1-10 m "
                                "(translation study) or 2-20 deg heading (rotation study), 64-ring "
                                "scans at 0.4 deg azimuth (~57k points), 1 m voxels 160x160x10, "
                                "count + z-variance 32 bins, simplex search from the identity "
                                f"with initial simplex {NM_STEP}, max 400 iterations"),
                   "alignments": n_align},
        "mean_nm_iterations": float(np.mean(iters)),
        "success_rule": f"translation error < {SUCCESS_M} m and rotation error < {SUCCESS_DEG} deg",
        "success_rate": {k: round(float(np.mean(v)), 3) for k, v in sorted(overall.items())},
        "accuracy": summary,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def _local_maxima_2d(S):
    """Interior nodes strictly above all 8 neighbours."""
    c = S[1:-1, 1:-1]
    m = np.ones_like(c, dtype=bool)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            if dx or dy:
                m &= c > S[1 + dx:S.shape[0] - 1 + dx, 1 + dy:S.shape[1] - 1 + dy]
    return int(m.sum())


def _bench_surface(a):
    """Cost surfaces of Fig. 6 around the true pose of a displaced query scan
    (6 m away): MI over a +-10 m (tx, ty) grid at 0.25 m and over +-30 deg of
    heading at 0.25 deg, every other parameter at the truth, both features."""
    import math

    import torch

    from paper_1709_06948_amd import mi, synth

    torch.cuda.set_device(0)
    d2r = math.pi / 180.0
    D = synth.displaced_scans(seed=synth.seed_for(8), study="translation", levels=[6.0])
    g = D.eta_gt[0]
    grid = mi.Grid(D.origin, D.dims, D.voxel, features=mi.FEAT_COUNT | mi.FEAT_ZVAR,
                   nb_count=32, nb_zvar=32)
    ref = mi.Ref(grid, D.A)
    B = torch.from_numpy(D.B[0]).cuda()
    P, xs, ys, Y, yaws = synth.surface_poses(g)
    Pall = np.concatenate([P, Y])
    plan = mi.Plan(ref, B.shape[1], Pall)
    o = torch.empty((2, len(Pall)), dtype=torch.float64, device="cuda")
    for _ in range(max(a.warmup, 1)):
        plan.execute(B, o)
    torch.cuda.synchronize()
    mi.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        plan.execute(B, o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = mi.profile_read()
    mi.profile_enable(False)
    M = o.cpu().numpy()
    n = len(xs)
    feats = {}
    for f, fname in ((0, "mi_n"), (1, "mi_varz")):
        S = M[f, :n * n].reshape(n, n)
        h = M[f, n * n:]
        i, j = np.unravel_index(int(np.argmax(S)), S.shape)
        feats[fname] = {
            "xy_argmax_err_m": round(float(math.hypot(xs[i] - g[0], ys[j] - g[1])), 3),
            "xy_local_maxima": _local_maxima_2d(S),
            "heading_argmax_err_deg": round(float(abs(yaws[int(np.argmax(h))] - g[5]) / d2r), 3),
            "heading_local_maxima": int(((h[1:-1] > h[:-2]) & (h[1:-1] > h[2:])).sum()),
            "mi_max": float(S.max())}
    K = len(Pall)
    eval_ms_avg = prof["eval_ms"] / max(prof["eval_launches"], 1)
    pp_per_launch = prof["point_poses"] / max(prof["eval_launches"], 1)
    achieved = OPS_PER_POINT_POSE * pp_per_launch / (eval_ms_avg * 1e-3)
    out = {
        "metric": "MI pose evals/s", "value": K * a.steps / dt, "unit": "evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt * 1e3 / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("cost surfaces: query scan 6 m from the reference (~57k points "
                                "each), 1 m voxels 160x160x10, count + z-variance 32 bins; "
                                f"{n}x{n} (tx, ty) nodes over +-10 m and {len(yaws)} headings over "
                                "+-30 deg around the true pose, one batch per step"),
                   "evals_per_step": K},
        "gpoint_transforms_per_s": K * B.shape[1] * a.steps / dt / 1e9,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_OPS, "traffic": None,
                     "kernel": "k_eval", "avg_launch_ms": eval_ms_avg},
        "surfaces": feats,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


# -------------------------------------------------------------------- serving

def _serving_request(spec):
    """One request of the serving pool: a surface-sampled pair as the serving
    workload specifies (points log-uniform in [20k, 250k], voxel 0.5 or 1 m,
    160 x 160 x 10 m scenes) with a seeded prior near its true pose."""
    import math

    from paper_1709_06948_amd import synth
    d2r = math.pi / 180.0
    pair = synth.make_request(spec)
    rng = np.random.default_rng(spec["seed"] + 1)
    init = pair.eta_gt + np.array([rng.normal(0, 0.5), rng.normal(0, 0.5), 0.0, 0.0, 0.0,
                                   rng.normal(0, 2 * d2r)])
    return dict(origin=pair.origin, dims=pair.dims, voxel=pair.voxel, A=pair.A, B=pair.B,
                init=init, eta_gt=pair.eta_gt)


def _serving_specs(n_pool):
    from paper_1709_06948_amd import synth
    _, specs = synth.serving_requests(1.0, n_pool)
    return specs


SERVE_HALF = (3.0, 3.0, 0.2, 2.0 * np.pi / 180, 2.0 * np.pi / 180, 10.0 * np.pi / 180)
SERVE_SAMPLES = (4, 4, 4, 4, 4, 4)
SERVE_LEVELS, SERVE_SHRINK = 3, 4.0


def _fifo_latency(arrivals, service):
    """One request at a time, in arrival order: completion - arrival."""
    t_free, lat = 0.0, []
    for a, s in zip(arrivals, service):
        start = max(a, t_free)
        t_free = start + s
        lat.append(t_free - a)
    return np.array(lat)


def _run_serving(a, pool):
    import threading

    import torch

    from paper_1709_06948_amd import mi, synth

    K_req = SERVE_LEVELS * int(np.prod(SERVE_SAMPLES))

    def submit(srv, q):
        return srv.submit(q["origin"], q["dims"], q["voxel"], q["A"], q["B"], q["init"], SERVE_HALF,
                          SERVE_SAMPLES, SERVE_LEVELS, SERVE_SHRINK, features=3, nb_count=32,
                          nb_zvar=32, feature_slot=0)

    # one request at a time: batched per request (every pool pair), and the plain
    # per-pose path on a sample of one level
    service = []
    for q in pool:
        g = mi.Grid(q["origin"], q["dims"], q["voxel"], features=3, nb_count=32, nb_zvar=32)
        A = torch.from_numpy(q["A"]).cuda()
        B = torch.from_numpy(q["B"]).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref = mi.Ref(g, A)
        mi.align_coarse_to_fine(ref, B, q["init"], SERVE_HALF, SERVE_SAMPLES, SERVE_LEVELS,
                                SERVE_SHRINK, feature_slot=0)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
    service[0] = service[1] if len(service) > 1 else service[0]   # the first call warms up
    q = pool[0]
    g = mi.Grid(q["origin"], q["dims"], q["voxel"], features=3, nb_count=32, nb_zvar=32)
    ref = mi.Ref(g, q["A"])
    P = synth.level_poses(q["init"], SERVE_HALF, SERVE_SAMPLES)[::64]
    mi.eval_poses_plain(ref, q["B"], P[:2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mi.eval_poses_plain(ref, q["B"], P)
    torch.cuda.synchronize()
    plain_rate = len(P) / (time.perf_counter() - t0)
    mean_pts = float(np.mean([p["B"].shape[1] for p in pool]))
    plain_service = K_req / plain_rate * mean_pts / q["B"].shape[1]

    per_rate = []
    prof_all = {"eval_ms": 0.0, "eval_launches": 0, "point_poses": 0, "frames_ms": 0.0}
    for rate in [float(r) for r in a.rates.split(",")]:
        rng = np.random.default_rng(int(rate))
        gaps = rng.exponential(1.0 / rate, a.requests)
        arrivals = np.cumsum(gaps) - gaps[0]
        order = rng.integers(0, len(pool), a.requests)
        srv = mi.Server(arena_bytes=48 << 30, step_bytes=16 << 30, max_active=a.slots)
        ids = [None] * a.requests
        late = []
        t_start = time.perf_counter()

        def producer():
            for j in range(a.requests):
                dt = arrivals[j] - (time.perf_counter() - t_start)
                if dt > 0:
                    time.sleep(dt)
                late.append(time.perf_counter() - t_start - arrivals[j])
                ids[j] = submit(srv, pool[order[j]])

        th = threading.Thread(target=producer)
        mi.profile_enable(True)
        th.start()
        done, steps, lat, t_step = set(), 0, {}, 0.0
        pending = list(range(a.requests))
        while len(done) < a.requests:
            ts = time.perf_counter()
            na, nq = srv.step()
            t_step += time.perf_counter() - ts
            steps += 1
            now = time.perf_counter() - t_start
            still = []
            for j in pending:
                if ids[j] is None:
                    still.append(j)
                    continue
                st = srv.poll(ids[j])
                if st["state"] in (mi.REQ_DONE, mi.REQ_FAILED):
                    if st["state"] != mi.REQ_DONE:
                        raise RuntimeError(f"request {j} failed: status {st['status']}")
                    done.add(j)
                    lat[j] = now - arrivals[j]
                    srv.release(ids[j])
                else:
                    still.append(j)
            pending = still
            if na == 0 and nq == 0 and len(done) < a.requests:
                time.sleep(0.0005)
        th.join()
        elapsed = time.perf_counter() - t_start
        prof = mi.profile_read()
        mi.profile_enable(False)
        for k in prof_all:
            prof_all[k] += prof[k]
        srv.close()
        L = np.array([lat[j] for j in range(a.requests)])
        svc = np.array([service[o] for o in order])
        one = _fifo_latency(arrivals, svc)
        plain_one = _fifo_latency(arrivals, np.full(a.requests, plain_service))
        # the second half of the requests: the latency a request meets once the queue has
        # reached the state this rate drives it to
        half = slice(a.requests // 2, a.requests)
        per_rate.append({
            "rate_req_s": rate, "requests": a.requests, "steps": steps,
            "throughput_req_s": a.requests / elapsed,
            "evals_per_s": a.requests * K_req / elapsed,
            "p50_s": float(np.percentile(L, 50)), "p99_s": float(np.percentile(L, 99)),
            "p50_s_second_half": float(np.percentile(L[half], 50)),
            "p99_s_second_half": float(np.percentile(L[half], 99)),
            "offered_req_s": float(a.requests / max(arrivals[-1], 1e-9)),
            "max_submit_late_s": float(max(late)),
            "time_in_steps_s": t_step, "elapsed_s": elapsed,
            "gpu_frames_ms": prof["frames_ms"], "gpu_eval_ms": prof["eval_ms"],
            "eval_launches": prof["eval_launches"], "point_poses": prof["point_poses"],
            "one_at_a_time_batched": {"p50_s": float(np.percentile(one, 50)),
                                      "p99_s": float(np.percentile(one, 99)),
                                      "capacity_req_s": 1.0 / float(np.mean(svc))},
            "one_at_a_time_plain": {"p50_s": float(np.percentile(plain_one, 50)),
                                    "p99_s": float(np.percentile(plain_one, 99)),
                                    "capacity_req_s": 1.0 / plain_service},
        })
        print(json.dumps({"serving_rate": per_rate[-1]}), file=sys.stderr, flush=True)
    best = max(per_rate, key=lambda r: r["evals_per_s"])
    res = {"value": best["evals_per_s"], "unit": "evals/s", "steps": a.requests, "warmup": 0,
           "ms_per_step": 1e3 / best["throughput_req_s"],
           "config": {"workload": "serving: Poisson arrivals of alignment requests (surface-sampled "
                                  "pairs, 20k-250k points, 0.5/1 m voxels, count + z-variance 32 "
                                  "bins, 3 levels x 4^6 poses), continuous batching, "
                                  f"{a.slots} slots", "pool": len(pool), "rates": a.rates,
                      "requests_per_rate": a.requests},
           "serving": per_rate,
           "one_request_service_s": {"batched_mean": float(np.mean(service)),
                                     "plain_estimate": plain_service,
                                     "plain_evals_per_s": plain_rate},
           "roofline": _roofline(prof_all, "serving", over="every evaluator launch of all rates")}
    res["cpu_baseline"] = None
    if not a.no_cpu_baseline:
        import oracle as O
        cores = _cores()
        q = pool[0]
        og = O.Grid(q["origin"], q["dims"], q["voxel"], features=3, nb_count=32, nb_zvar=32)
        P = synth.level_poses(q["init"], SERVE_HALF, SERVE_SAMPLES)[::8]
        tc0 = time.perf_counter()
        O.eval_poses(og, q["A"], q["B"], P, nthreads=cores)
        tc = time.perf_counter() - tc0
        per_eval = tc / len(P) * mean_pts / q["B"].shape[1]
        res["cpu_baseline"] = {
            "value": len(P) / tc, "unit": "MI pose evals/s", "cores": cores, "kind": "oracle",
            "request_latency_s_estimate": per_eval * K_req,
            "capacity_req_s_estimate": 1.0 / (per_eval * K_req),
            "sample": f"every 8th pose of level 0 of pool request 0 ({len(P)} evaluations, "
                      f"{q['B'].shape[1]} points), FP64 dense oracle, {tc:.1f} s; one request "
                      "at a time scaled to the pool's mean point count"}
    return res



# ------------------------------------------------------------------------ main

def _sub(res, metric="MI pose evals/s"):
    """A workload's result as a nested record of the benchmark line."""
    out = {"metric": metric}
    out.update(res)
    return out


def _bench_all(a):
    """Every configured workload; the uneven batch is the headline."""
    from paper_1709_06948_amd import synth

    t_gen = time.perf_counter()
    # generation runs in forked workers before this process touches the GPU
    work = _parallel(_uneven_pair, list(range(a.pairs)))
    pool = _parallel(_serving_request, _serving_specs(a.pool))
    urban = synth.urban_pair()
    tiny = synth.tiny_pair()
    t_gen = time.perf_counter() - t_gen
    import torch
    torch.cuda.set_device(0)

    def done(name, res):
        print(json.dumps({"workload_done": name, "value": res["value"],
                          "frac": (res.get("roofline") or {}).get("frac")}), file=sys.stderr,
              flush=True)
        return res

    print(json.dumps({"generated_s": round(t_gen, 1)}), file=sys.stderr, flush=True)
    head = done("uneven", _run_uneven(a, work))
    del work
    sub = {"c2f": _sub(done("c2f", _run_c2f(a, urban))),
           "batched": _sub(done("batched", _run_batched(a, tiny)))}
    sub["serving"] = _sub(done("serving", _run_serving(a, pool)))
    out = _line("MI pose evals/s", head["value"], "evals/s", head["steps"], head["warmup"],
                head["ms_per_step"], head["config"],
                gpoint_transforms_per_s=head["gpoint_transforms_per_s"],
                roofline=head["roofline"], cpu_baseline=head["cpu_baseline"],
                workloads=sub, generation_s=t_gen)
    print(json.dumps(out), flush=True)


def _bench_one(a):
    """One workload alone, on its own line."""
    from paper_1709_06948_amd import synth
    if a.workload == "uneven":
        work = _parallel(_uneven_pair, list(range(a.pairs)))
    elif a.workload == "serving":
        pool = _parallel(_serving_request, _serving_specs(a.pool))
    import torch
    torch.cuda.set_device(0)
    if a.workload == "uneven":
        res = _run_uneven(a, work)
    elif a.workload == "c2f":
        res = _run_c2f(a, synth.urban_pair())
    elif a.workload == "batched":
        res = _run_batched(a, synth.tiny_pair())
    else:
        res = _run_serving(a, pool)
    extra = {k: v for k, v in res.items()
             if k not in ("value", "unit", "steps", "warmup", "ms_per_step", "config")}
    print(json.dumps(_line("MI pose evals/s", res["value"], "evals/s", res["steps"],
                           res["warmup"], res["ms_per_step"], res["config"], **extra)), flush=True)


def main():
    global SERIAL
    a = _args()
    SERIAL = a.serial
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; pose sets are not "
                                   "sharded over several GPUs",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    if a.calibrate_copy:
        _calibrate_copy()
        return
    if a.calibrate:
        return _calibrate(a)
    if a.workload == "all":
        return _bench_all(a)
    if a.workload == "accuracy":
        return _bench_accuracy(a)
    if a.workload == "surface":
        return _bench_surface(a)
    return _bench_one(a)


if __name__ == "__main__":
    main()
