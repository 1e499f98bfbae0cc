"""Benchmark of the elevation-map fusion hot path on one MI355X.

Headline workload: one robot.
  * A 400x400 map at 0.04 m (16 x 16 m).
  * 300k-point frames: a 64-beam dome LiDAR plus four depth frustums.
  * The frames follow a seeded smooth trajectory over a synthetic terrain.
One step is one frame through the whole per-frame path, the ABI calls in
order: move_fuse_points (the robot-centric move inside the fusion),
clear_visibility, normals_traversability (the normals and the traversability
filter in one pass).  Every frame is generated on the device before timing
starts.
  * value: the timed frames submitted back to back (inputs resident in HBM),
    points per second of wall time between two device synchronisations.
  * latency_ms: the same frames with the host waiting for each one
    (submission to completion).
  * roofline: the dominant kernel of the plain path, its per-launch duration
    taken with events on its stream around each launch.

Also reported, each with its plain per-frame comparison:
  * batched: 16 maps of uneven sizes, one frame each, in one batched launch
    (emx_pipeline_batch) against 16 per-frame plain pipelines;
  * server: 64 robots sending frames by Poisson arrival at 20 Hz each into the
    continuous-batching server, against the per-frame plain loop on the same
    arrival trace; and both with every frame queued at once (saturated).
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points fused/sec and p99 update latency: batched server vs per-frame plain"
HBM_PEAK_GBS = 8000.0
STAGES = ("move_fuse_points", "clear_visibility", "normals_traversability")
TUNING_FILE = os.path.join(ROOT, "paper_2204_12876_amd", "tuning_mi355x.json")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_400x400_300k.txt")


def say(*a):
    print("#", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--points", type=int, default=300000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=50)
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-features", action="store_true")
    ap.add_argument("--skip-server", action="store_true")
    ap.add_argument("--batched-reps", type=int, default=20)
    ap.add_argument("--server-seconds", type=float, default=1.0)
    ap.add_argument("--server-robots", type=int, default=64)
    ap.add_argument("--server-lanes", type=int, default=2)
    ap.add_argument("--tuning", default=None, help="batch tuning JSON (default: the tuned file)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 256 MiB device to device once (a known-size kernel that "
                         "calibrates hardware byte counters)")
    ap.add_argument("--autotune", default=None, metavar="OUT",
                    help="tune the batched executor on the 16-map workload, write OUT, exit")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def frame_stats(cell: np.ndarray, acc: np.ndarray) -> dict:
    return dict(touched=np.unique(cell[cell >= 0]).size,
                updated=np.unique(cell[acc.astype(bool)]).size)


def kernel_alg_bytes(name: str, n: int, C: int, touched: float, updated: float,
                     moved: float = 0.0) -> float:
    """Bytes each kernel must move at the least, per launch.
      fusion pass 1: the points (12 B) and the prior h, v of each distinct
        in-map cell they hit (8 B);
      fusion pass 2: prior h, v read and h, v, t_upd, valid written for each
        updated cell (8 + 13 B); with the move folded in (a frame whose centre
        cell changes), also every layer read and written once (2 x 29 B);
      clearing: setup reads the points and h, t_upd, valid per cell for the
        block maxima (9 B); the march reads each cell's h, v, t_upd, valid and
        normal once (25 B) and resets the removed cells in place;
      normals: h, valid in (5 B), three components out (12 B);
      traversability: h, valid in, one float out (9 B);
      normals and traversability in one pass: h, valid in, four floats out
        (21 B);
      move: every layer read and written once (2 x 29 B)."""
    return {
        "k_fuse_chunk": 12 * n + 8 * touched,
        "k_fuse_tile": 21 * updated + 58 * C * moved,
        "k_clear_setup": 12 * n + 9 * C,
        "k_clear_march": 25 * C,
        "k_normals": 17 * C,
        "k_trav": 9 * C,
        "k_normals_trav": 21 * C,
        "k_move": 58 * C,
    }.get(name, 0.0)


KERNEL_SOURCE = {"k_fuse_chunk": "emx_fuse.hip", "k_fuse_tile": "emx_fuse.hip",
                 "k_clear_setup": "emx_clear.hip", "k_clear_march": "emx_clear.hip",
                 "k_move": "emx_cells.hip",
                 "k_normals": "emx_cells.hip", "k_trav": "emx_cells.hip",
                 "k_normals_trav": "emx_cells.hip",
                 "k_fill_prior": "emx_cells.hip"}


def kernel_source_hash(kernel: str) -> str:
    """Hash of the source file holding ``kernel`` and the headers it includes."""
    d = os.path.join(ROOT, "paper_2204_12876_amd", "csrc")
    h = hashlib.sha256()
    for f in (KERNEL_SOURCE[kernel], "emx_device.h", "emx_kernels.h"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of ``kernel`` from the committed counter summary,
    or None if it is absent or was taken from different kernel sources."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get(f"{kernel}.source_sha256_16") != kernel_source_hash(kernel):
            return None
        f = float(kv[f"{kernel}.fetch_kib"]) * float(kv["fetch_factor"])
        w = float(kv[f"{kernel}.write_kib"]) * float(kv["write_factor"])
        return 1024.0 * (f + w)
    except (OSError, KeyError, ValueError):
        return None


def load_tuning(args):
    if args.tuning:
        return args.tuning
    if os.path.exists(TUNING_FILE):
        with open(TUNING_FILE) as fh:
            return json.dumps(json.load(fh)["tuning"])
    return None


# ------------------------------------------------------------- plain, one robot
def plain_single_robot(args, dev):
    import torch

    import synth
    from paper_2204_12876_amd import ElevationMap, _emx

    K, W = args.steps, args.warmup
    t_gen = time.perf_counter()
    d = synth.cfg1(n_frames=W + K, device=dev, n_points=args.points)
    torch.cuda.synchronize()
    say(f"generated {W + K} frames of {args.points} points in {time.perf_counter() - t_gen:.1f} s")
    frames = [(f.x.contiguous(), f.y.contiguous(), f.z.contiguous(), f.pose, f.t_ms)
              for f in d["frames"]]
    centers = d["centers"]
    params = d["params"]
    C = params["nx"] * params["ny"]
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    stream = torch.cuda.current_stream(dev)
    probe = ElevationMap(params, device=dev)
    scratch = probe.scratch(args.points)
    probe.close()

    def run(m, k, ev=None, cell=None, acc=None):
        x, y, z, pose, t = frames[k]
        if ev is not None:
            ev[0].record(stream)
        m.move_fuse_points(*centers[k], x, y, z, pose, t, scratch=scratch, out_cell=cell,
                           out_accept=acc)
        if ev is not None:
            ev[1].record(stream)
        m.clear_visibility(x, y, z, pose, t, scratch=scratch)
        if ev is not None:
            ev[2].record(stream)
        m.normals_traversability(w)
        if ev is not None:
            ev[3].record(stream)

    def fresh():
        m = ElevationMap(params, centers[0][0], centers[0][1], 0, device=dev)
        for k in range(W):
            run(m, k)
        torch.cuda.synchronize()
        return m

    # ---- timed: frames back to back, inputs resident; wall clock between syncs
    m = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(K):
        run(m, W + j)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m.close()
    n_pts = sum(frames[W + j][0].numel() for j in range(K))
    say(f"plain back to back: {wall / K * 1e3:.3f} ms/frame")

    # ---- latency: the host waits for every frame; events per stage
    m = fresh()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(STAGES) + 1)]
           for _ in range(K)]
    lat = np.zeros(K)
    for j in range(K):
        s = time.perf_counter()
        run(m, W + j, evs[j])
        stream.synchronize()
        lat[j] = time.perf_counter() - s
    stage_ms = {name: float(np.mean([evs[j][i].elapsed_time(evs[j][i + 1]) for j in range(K)]))
                for i, name in enumerate(STAGES)}
    m.close()

    # ---- per-kernel durations: the frames back to back again, each kernel
    # bracketed by events on its stream
    m = fresh()
    _emx.timing_begin()
    for j in range(K):
        run(m, W + j)
    kt = _emx.timing_end()
    m.close()

    # ---- frame statistics for the algorithmic bytes (untimed)
    m = fresh()
    cell = torch.empty(args.points, dtype=torch.int32, device=dev)
    acc = torch.empty(args.points, dtype=torch.uint8, device=dev)
    stats = []
    for j in range(K):
        run(m, W + j, cell=cell, acc=acc)
        n = frames[W + j][0].numel()
        stats.append(frame_stats(cell[:n].cpu().numpy(), acc[:n].cpu().numpy()))
    m.close()
    touched = float(np.mean([s["touched"] for s in stats]))
    updated = float(np.mean([s["updated"] for s in stats]))
    n_mean = n_pts / K
    # the share of timed frames whose centre cell changes (the move is folded
    # into fusion pass 2 for those)
    r = params["resolution"]
    cell_of = [(math.floor(cx / r), math.floor(cy / r)) for cx, cy in centers]
    moved = float(np.mean([cell_of[W + j] != cell_of[W + j - 1] for j in range(K)]))
    kernels = {}
    for name, (cnt, tot_ms) in kt.items():
        avg_us = tot_ms / cnt * 1e3
        ab = kernel_alg_bytes(name, n_mean, C, touched, updated, moved)
        kernels[name] = {"launches": cnt, "avg_us": avg_us, "alg_bytes": ab,
                         "alg_GBps": ab / (avg_us * 1e-6) / 1e9 if avg_us > 0 else None}
    dom = max((k for k in kernels if k != "k_fill_prior"),
              key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    dk = kernels[dom]
    traffic = measured_traffic(dom)

    out = {
        "value": n_pts / wall,
        "ms_per_step": wall / K * 1e3,
        "config": {"workload": "plain single robot: 400x400 map at 0.04 m, 300k-point frames "
                               "(dome LiDAR + 4 depth frustums), full pipeline per frame",
                   "map_cells": C, "points_per_frame": args.points, "frames": K,
                   "mode": "per-frame plain calls (move_fuse_points, clear_visibility, "
                           "normals_traversability), frames submitted back to back"},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "max": float(lat.max() * 1e3),
                       "note": "host waits for each frame before the next"},
        "maps_per_s": K / wall,
        "stage_ms": stage_ms,
        "kernels": kernels,
        "cells_touched": touched, "cells_updated": updated, "frames_moved": moved,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dk["alg_GBps"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dk["alg_GBps"] / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "alg_bytes_per_launch": dk["alg_bytes"], "avg_launch_us": dk["avg_us"]},
    }
    return out, dict(frames=frames, centers=centers, params=params)


# --------------------------------------------------- optional per-map features
def features(args, dev, ctx):
    """The features beyond the base path, on the same workload and frames: a
    map with time variance, the wall/edge rule and the upper bound layer on,
    run through the extended per-frame sequence (move, drift compensation,
    fusion, clearing with the bound, normals, traversability, overlap
    clearance, inpainting).  Each feature is then timed per kernel over the
    frames; algorithmic bytes per call are stated in ``FEATURE_BYTES``."""
    import torch

    import synth
    from paper_2204_12876_amd import ElevationMap, _emx, smooth

    frames, centers, params = ctx["frames"], ctx["centers"], ctx["params"]
    W = min(args.warmup, len(frames) // 2)
    K = min(args.steps, len(frames) - W, 20)
    C = params["nx"] * params["ny"]
    pe = dict(params, time_variance=1e-4, wall_min_count=8, upper_bound=1)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    m = ElevationMap(pe, centers[0][0], centers[0][1], 0, device=dev)
    scratch = m.scratch(max(f[0].numel() for f in frames))
    trav_min = 0.0

    def frame(k):
        x, y, z, pose, t = frames[k]
        m.move_map(*centers[k])
        m.compensate_drift(x, y, z, pose, t, trav_min, scratch=scratch)
        m.fuse_points(x, y, z, pose, t, scratch=scratch)
        m.clear_visibility(x, y, z, pose, t, scratch=scratch)
        m.normals_traversability(w)
        m.overlap_clear(pose[:, 3], 1.0, 1.5)
        return m.inpaint_min()

    for k in range(W):
        frame(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(K):
        frame(W + j)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    say(f"extended sequence: {wall / K * 1e3:.3f} ms/frame")

    g = m.state_numpy()
    valid = float((g["valid"] != 0).sum())
    n_mean = float(np.mean([frames[W + j][0].numel() for j in range(K)]))
    cell = torch.empty(int(n_mean) + 1024, dtype=torch.int32, device=dev)
    m2 = ElevationMap(params, centers[W][0], centers[W][1], 0, device=dev)
    x, y, z, pose, t = frames[W]
    m2.fuse_points(x, y, z, pose, t, out_cell=cell[:x.numel()])
    c = cell[:x.numel()].cpu().numpy()
    touched = float(np.unique(c[c >= 0]).size)
    m2.close()
    filled = m.inpaint_min()

    def timed(fn, reps=K):
        _emx.timing_begin()
        for j in range(reps):
            fn(j)
        kt = _emx.timing_end()
        return {k: v for k, v in kt.items()}

    x0 = frames[W]
    ops = {
        "drift_compensation": (
            lambda j: m.compensate_drift(*frames[W + j][:5], trav_min, scratch=scratch),
            12 * n_mean + 9 * touched + C + 8 * valid),
        "wall_rule_and_time_variance_fusion": (
            lambda j: m.fuse_points(*frames[W + j][:5], scratch=scratch), None),
        "upper_bound_clearing": (
            lambda j: m.clear_visibility(*frames[W + j][:5], scratch=scratch), None),
        "overlap_clearance": (lambda j: m.overlap_clear(x0[3][:, 3], 1.0, 1.5), 5 * C),
        "inpaint_min": (lambda j: m.inpaint_min(), 9 * C),
        "smooth_box_5": (lambda j: smooth(filled, "box", 5), 8 * C),
        "smooth_gaussian_5": (lambda j: smooth(filled, "gaussian", 5, 1.0), 8 * C),
        "smooth_median_5": (lambda j: smooth(filled, "median", 5), 8 * C),
    }
    out = {"workload": "the plain workload's map and frames with time_variance, "
                       "wall_min_count=8 and upper_bound on",
           "extended_ms_per_frame": wall / K * 1e3, "frames": K}
    for name, (fn, ab) in ops.items():
        kt = timed(fn)
        per_call_us = sum(tot for _, tot in kt.values()) / K * 1e3
        ent = {"kernels": {k: {"launches": cnt, "avg_us": tot / cnt * 1e3}
                           for k, (cnt, tot) in kt.items()},
               "us_per_call": per_call_us}
        if ab is not None and per_call_us > 0:
            gbps = ab / (per_call_us * 1e-6) / 1e9
            ent.update(alg_bytes=ab, alg_GBps=gbps, frac_hbm=gbps / HBM_PEAK_GBS)
        out[name] = ent
    # the feature kernels inside the extended fusion: counts and time variance
    fk = out["wall_rule_and_time_variance_fusion"]["kernels"]
    extra = {k: fk[k] for k in ("k_zero_u32", "k_fuse_count", "k_time_variance") if k in fk}
    ab = {"k_zero_u32": 4 * C, "k_fuse_count": 12 * n_mean + 8 * touched,
          "k_time_variance": 2 * C + 8 * valid}
    for k, e in extra.items():
        e["alg_bytes"] = ab[k]
        e["alg_GBps"] = ab[k] / (e["avg_us"] * 1e-6) / 1e9
    m.close()
    return out


# ------------------------------------------------------------ batched, 16 maps
def batched_maps(args, dev, tuning):
    import torch

    import synth
    from paper_2204_12876_amd import BatchEntry, ElevationMap, PipelineBatch

    t_gen = time.perf_counter()
    d = synth.cfg2(device=dev)
    torch.cuda.synchronize()
    items = d["items"]
    pts = sum(it["frames"][0].n for it in items)
    say(f"generated 16 maps / {pts} points in {time.perf_counter() - t_gen:.1f} s")
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    fr = [(it["frames"][0].x.contiguous(), it["frames"][0].y.contiguous(),
           it["frames"][0].z.contiguous(), it["frames"][0].pose) for it in items]
    R = args.batched_reps
    stream = torch.cuda.current_stream(dev)

    def maps():
        return [ElevationMap(it["params"], 0.0, 0.0, 0, device=dev) for it in items]

    # batched
    mb = maps()
    pb = PipelineBatch(tuning, device=dev)

    def batch(rep):
        pb.run([BatchEntry(m, x, y, z, pose, 100 * rep, center=(0.0, 0.0), weights=w)
                for m, (x, y, z, pose) in zip(mb, fr)])

    for rep in range(3):
        batch(rep)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for rep in range(3, 3 + R):
        batch(rep)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / R
    lat_b = []
    for rep in range(3 + R, 3 + 2 * R):
        s = time.perf_counter()
        batch(rep)
        stream.synchronize()
        lat_b.append(time.perf_counter() - s)

    # 16 per-frame plain pipelines
    mp = maps()
    scratch = max((m.scratch(f[0].numel()) for m, f in zip(mp, fr)), key=lambda t: t.numel())

    def plain(rep):
        for m, (x, y, z, pose) in zip(mp, fr):
            m.move_fuse_points(0.0, 0.0, x, y, z, pose, 100 * rep, scratch=scratch)
            m.clear_visibility(x, y, z, pose, 100 * rep, scratch=scratch)
            m.normals_traversability(w)

    for rep in range(3):
        plain(rep)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for rep in range(3, 3 + R):
        plain(rep)
    torch.cuda.synchronize()
    t_p = (time.perf_counter() - t0) / R
    lat_p = []
    for rep in range(3 + R, 3 + 2 * R):
        s = time.perf_counter()
        plain(rep)
        stream.synchronize()
        lat_p.append(time.perf_counter() - s)
    # identical results, as the batched path promises
    same = all(torch.equal(a.export_state(), b.export_state()) for a, b in zip(mb, mp))
    for m in mb + mp:
        m.close()
    pb.close()
    say(f"batched {t_b * 1e3:.3f} ms vs plain {t_p * 1e3:.3f} ms per 16 maps")
    return {
        "workload": "16 maps, sides U{200..1000} at 0.02-0.1 m, one frame each of "
                    "logU[20k, 1M] points, full pipeline",
        "points_per_batch": int(pts),
        "batched": {"ms": t_b * 1e3, "points_per_s": pts / t_b, "maps_per_s": 16 / t_b,
                    "p50_ms": float(np.percentile(lat_b, 50) * 1e3),
                    "p99_ms": float(np.percentile(lat_b, 99) * 1e3)},
        "plain": {"ms": t_p * 1e3, "points_per_s": pts / t_p, "maps_per_s": 16 / t_p,
                  "p50_ms": float(np.percentile(lat_p, 50) * 1e3),
                  "p99_ms": float(np.percentile(lat_p, 99) * 1e3)},
        "speedup": t_p / t_b,
        "results_identical": bool(same),
        "tuning": pb_tuning_text(tuning),
    }


def pb_tuning_text(tuning):
    return json.loads(tuning) if tuning else "library defaults"


# -------------------------------------------------------------- server, 64 robots
def serving(args, dev, tuning):
    import torch

    import synth
    from paper_2204_12876_amd import ElevationMap
    from paper_2204_12876_amd.server import (GpuExecutor, Request, Server, latency_summary,
                                             run_plain_trace, run_trace)

    t_gen = time.perf_counter()
    d = synth.cfg3(device=dev, n_robots=args.server_robots, n_frames=1)
    torch.cuda.synchronize()
    items = d["items"]
    say(f"generated {len(items)} robot frames in {time.perf_counter() - t_gen:.1f} s")
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    host = []
    for it in items:
        f = it["frames"][0]
        xyz = torch.empty((3, f.n), dtype=torch.float32, pin_memory=True)
        xyz[0].copy_(f.x)
        xyz[1].copy_(f.y)
        xyz[2].copy_(f.z)
        host.append((xyz, f.pose, it["centers"][0]))
    largest = max((it["params"] for it in items), key=lambda p: p["nx"] * p["ny"])
    rng = np.random.default_rng(12876 + 3)

    def trace(seconds, saturated_frames=0):
        reqs, seq = [], 0
        for k, it in enumerate(items):
            xyz, pose, c = host[k]
            if saturated_frames:
                times = np.zeros(saturated_frames)
            else:
                gaps = rng.exponential(1.0 / it["rate_hz"], int(seconds * it["rate_hz"] * 3) + 8)
                times = np.cumsum(gaps)
                times = times[times < seconds]
            for j, t in enumerate(times):
                # the robot re-observes from its pose; the centre alternates by one cell
                cx = c[0] + (it["params"]["resolution"] if j % 2 else 0.0)
                reqs.append(Request(robot=k, xyz=xyz, pose=pose, t_ms=100 * (j + 1),
                                    center=(cx, c[1]), arrival=float(t), seq=seq))
                seq += 1
        return reqs

    budget = 32 << 30

    def run_server(reqs, warm):
        ex = GpuExecutor(largest, lanes=args.server_lanes, max_items=64,
                         max_batch_points=8_000_000, pool_points=24_000_000, weights=w,
                         device=dev)
        srv = Server(ex, budget)
        for k, it in enumerate(items):
            srv.add_map(k, it["params"], *host[k][2])
        run_trace(srv, warm)  # a short trace of the same kind: graph captures, clocks
        srv.completed.clear()
        srv.batch_sizes.clear()
        b0, c0 = ex.graph_stats()
        run_trace(srv, reqs, timeout_s=120)
        b1, c1 = ex.graph_stats()
        s = latency_summary(reqs)
        s["mean_batch_items"] = float(np.mean(srv.batch_sizes))
        s["batches"] = len(srv.batch_sizes)
        s["batched_calls"] = b1 - b0
        s["graph_captures_in_trace"] = c1 - c0
        s["hbm_budget_bytes"] = budget
        s["hbm_reserved_bytes"] = srv.budget.used
        return s

    def run_plain(reqs):
        maps = {k: ElevationMap(it["params"], *host[k][2], 0, device=dev)
                for k, it in enumerate(items)}
        mx = max(h[0].shape[1] for h in host)
        run_plain_trace(maps, trace(0, saturated_frames=1), w, device=dev, max_points=mx)
        run_plain_trace(maps, reqs, w, device=dev, max_points=mx)
        for m in maps.values():
            m.close()
        return latency_summary(reqs)

    poisson = trace(args.server_seconds)
    offered = sum(r.n for r in poisson) / args.server_seconds
    say(f"server trace: {len(poisson)} frames, offered {offered / 1e6:.0f} M points/s")
    srv_p = run_server(poisson, trace(0.3))
    say(f"server p50 {srv_p['p50_ms']:.3f} p99 {srv_p['p99_ms']:.3f} ms")
    pln_p = run_plain(_fresh(poisson))
    say(f"plain  p50 {pln_p['p50_ms']:.3f} p99 {pln_p['p99_ms']:.3f} ms")
    sat = trace(0, saturated_frames=6)
    srv_s = run_server(sat, trace(0, saturated_frames=2))
    pln_s = run_plain(_fresh(sat))
    say(f"saturated: server {srv_s['points_per_s'] / 1e9:.2f} vs plain "
        f"{pln_s['points_per_s'] / 1e9:.2f} G points/s")
    return {
        "workload": f"{len(items)} robots, maps U{{256..800}}^2 at 0.04 m, frames "
                    "logU[50k, 500k] points, Poisson arrivals at 20 Hz each, full pipeline, "
                    "frames copied from pinned host memory, 32 GiB device budget",
        "offered_points_per_s": offered,
        "poisson": {"server": srv_p, "plain": pln_p},
        "saturated": {"frames_per_robot": 6, "server": srv_s, "plain": pln_s},
    }


def autotune_batched(dev, out_path):
    """Tune the batched executor on the 16-map workload; write the result."""
    import torch

    import synth
    from paper_2204_12876_amd import BatchEntry, ElevationMap
    from paper_2204_12876_amd.autotune import autotune, default_tuning, time_tuning
    d = synth.cfg2(device=dev)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    maps, frames = [], []
    for it in d["items"]:
        f = it["frames"][0]
        maps.append(ElevationMap(it["params"], 0.0, 0.0, 0, device=dev))
        frames.append((f.x.contiguous(), f.y.contiguous(), f.z.contiguous(), f.pose))

    def run_batch(pb, rep):
        pb.run([BatchEntry(m, x, y, z, pose, 100 * rep, center=(0.0, 0.0), weights=w)
                for m, (x, y, z, pose) in zip(maps, frames)])

    start = default_tuning()
    best, _, hist = autotune(run_batch, start, device=dev, log=say)
    t_def = time_tuning(run_batch, start, device=dev)
    t_best = time_tuning(run_batch, best, device=dev)
    out = {"tuning": best,
           "workload": "16 maps, sides U{200..1000} at 0.02-0.1 m, one frame each of "
                       "logU[20k, 1M] points, full pipeline",
           "points_per_batch": int(sum(f[0].numel() for f in frames)),
           "ms_best": t_best * 1e3, "ms_default": t_def * 1e3,
           "device": torch.cuda.get_device_name(dev), "candidates_timed": len(hist)}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def _fresh(reqs):
    """Copies of requests with their timing fields reset."""
    from paper_2204_12876_amd.server import Request
    return [Request(robot=r.robot, xyz=r.xyz, pose=r.pose, t_ms=r.t_ms, center=r.center,
                    arrival=r.arrival, seq=r.seq) for r in reqs]


# ------------------------------------------------------------------- CPU oracle
def cpu_baseline(args, ctx):
    import oracle as O
    import synth
    params, frames, centers = ctx["params"], ctx["frames"], ctx["centers"]
    p = O.Params.from_dict(params)
    nfr = max(1, args.cpu_frames)
    st = O.init_map(p, centers[0][0], centers[0][1], 0)
    wts = synth.trav_weights()
    t_cpu, pts = 0.0, 0
    host = [(frames[k][0].cpu().numpy(), frames[k][1].cpu().numpy(),
             frames[k][2].cpu().numpy()) for k in range(nfr)]
    for k in range(nfr):
        xs, ys, zs = host[k]
        pose, t = frames[k][3], frames[k][4]
        s = time.perf_counter()
        st = O.move_map(p, st, *centers[k])
        r = O.fuse(p, st, xs, ys, zs, pose, t)
        st = r.state
        mk = O.clear_visibility(p, st, xs, ys, zs, pose, t)
        st = O.apply_clear(p, st, mk)
        st.nrm[:] = O.compute_normals(p, st.h, st.valid).astype(np.float32)
        T, _ = O.traversability(st.h, st.valid, wts)
        st.trav[:] = T.astype(np.float32)
        t_cpu += time.perf_counter() - s
        pts += xs.size
    return {"value": pts / t_cpu, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"first {nfr} frames of the same workload, full pipeline, "
                      f"{t_cpu:.1f} s on one thread; {cpu_model()}, "
                      f"{os.cpu_count()} host threads visible"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every map and frame "
              "of this workload fits one MI355X.", file=sys.stderr)
        sys.exit(2)
    import torch
    dev = torch.device("cuda:0")
    if args.autotune:
        autotune_batched(dev, args.autotune)
        return
    tuning = load_tuning(args)
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        say("calibration copy: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    plain, ctx = plain_single_robot(args, dev)
    out = {
        "metric": METRIC,
        "value": plain.pop("value"),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": plain.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
    }
    out.update(plain)
    if not args.skip_features:
        out["features"] = features(args, dev, ctx)
    if not args.skip_batched:
        out["batched"] = batched_maps(args, dev, tuning)
    if not args.skip_server:
        out["server"] = serving(args, dev, tuning)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
