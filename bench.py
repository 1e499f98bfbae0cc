"""Benchmark of the elevation-map fusion hot path on one MI355X.

Workload: one robot.
  * A 400x400 map at 0.04 m (16 x 16 m).
  * 300k-point frames: a 64-beam dome LiDAR plus four depth frustums.
  * The frames follow a seeded smooth trajectory over a synthetic terrain.
One step is one frame through the whole per-frame path, the ABI calls in
order: move_map, fuse_points, clear_visibility, compute_normals,
traversability.
Every frame is generated on the device before timing starts.  The plain loop
waits for each frame before submitting the next, so the recorded per-frame
latency is submission to completion.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points fused/sec and p99 update latency: batched server vs per-frame plain"
HBM_PEAK_GBS = 8000.0
STAGES = ("move_map", "fuse_points", "clear_visibility", "compute_normals", "traversability")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--points", type=int, default=300000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=12)
    return ap.parse_args()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def algorithmic_bytes(cell: np.ndarray, acc: np.ndarray, n: int, C: int) -> dict:
    """Bytes the method must move per call, by stage.
    fuse: points (12 B) + prior h, v of each distinct in-map cell hit (8 B) +
    h, v, t_upd, valid written for each updated cell (13 B)."""
    touched = np.unique(cell[cell >= 0]).size
    updated = np.unique(cell[acc.astype(bool)]).size
    return dict(
        fuse_points=12 * n + 8 * touched + 13 * updated,
        clear_visibility=12 * n + 25 * C + 1 * C,
        compute_normals=5 * C + 12 * C,
        traversability=5 * C + 4 * C,
        move_map=2 * 29 * C,
        touched=touched, updated=updated)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every map and frame "
              "of this workload fits one MI355X.", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_2204_12876_amd import ElevationMap, aligned_empty

    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    t_gen = time.perf_counter()
    d = synth.cfg1(n_frames=W + K, device=dev, n_points=args.points)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    print(f"# generated {W + K} frames of {args.points} points in {t_gen:.1f} s", file=sys.stderr,
          flush=True)
    frames = [(f.x.contiguous(), f.y.contiguous(), f.z.contiguous(), f.pose, f.t_ms)
              for f in d["frames"]]
    centers = d["centers"]
    params = d["params"]
    C = params["nx"] * params["ny"]
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    m = ElevationMap(params, centers[0][0], centers[0][1], 0, device=dev)
    scratch = m.scratch(args.points)
    stream = torch.cuda.current_stream(dev)

    def step(k, ev=None):
        x, y, z, pose, t = frames[k]
        cx, cy = centers[k]
        if ev is not None:
            ev[0].record(stream)
        m.move_map(cx, cy)
        if ev is not None:
            ev[1].record(stream)
        m.fuse_points(x, y, z, pose, t, scratch=scratch)
        if ev is not None:
            ev[2].record(stream)
        m.clear_visibility(x, y, z, pose, t)
        if ev is not None:
            ev[3].record(stream)
        m.compute_normals()
        if ev is not None:
            ev[4].record(stream)
        m.traversability(w)
        if ev is not None:
            ev[5].record(stream)

    for k in range(W):
        step(k)
    torch.cuda.synchronize()

    # ---- timed: plain per-frame loop, host waits for every frame
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(K)]
    lat = np.zeros(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(K):
        s = time.perf_counter()
        step(W + j, evs[j])
        stream.synchronize()
        lat[j] = time.perf_counter() - s
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = {name: float(np.mean([evs[j][i].elapsed_time(evs[j][i + 1]) for j in range(K)]))
                for i, name in enumerate(STAGES)}
    step_ms = float(np.mean([evs[j][0].elapsed_time(evs[j][5]) for j in range(K)]))
    n_pts = sum(frames[W + j][0].numel() for j in range(K))

    # ---- the same frames submitted back to back (no host wait): device rate
    m2 = ElevationMap(params, centers[0][0], centers[0][1], 0, device=dev)
    for k in range(W):
        x, y, z, pose, t = frames[k]
        m2.move_map(*centers[k])
        m2.fuse_points(x, y, z, pose, t, scratch=scratch)
        m2.clear_visibility(x, y, z, pose, t)
        m2.compute_normals()
        m2.traversability(w)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for j in range(K):
        x, y, z, pose, t = frames[W + j]
        m2.move_map(*centers[W + j])
        m2.fuse_points(x, y, z, pose, t, scratch=scratch)
        m2.clear_visibility(x, y, z, pose, t)
        m2.compute_normals()
        m2.traversability(w)
    e1.record(stream)
    torch.cuda.synchronize()
    async_ms = e0.elapsed_time(e1) / K
    m2.close()

    # ---- algorithmic bytes: replay the run untimed with per-point outputs
    m3 = ElevationMap(params, centers[0][0], centers[0][1], 0, device=dev)
    cell = torch.empty(args.points, dtype=torch.int32, device=dev)
    acc = torch.empty(args.points, dtype=torch.uint8, device=dev)
    ab = {s: [] for s in STAGES}
    ab["touched"], ab["updated"] = [], []
    for k in range(W + K):
        x, y, z, pose, t = frames[k]
        m3.move_map(*centers[k])
        m3.fuse_points(x, y, z, pose, t, out_cell=cell, out_accept=acc, scratch=scratch)
        m3.clear_visibility(x, y, z, pose, t)
        m3.compute_normals()
        m3.traversability(w)
        if k >= W:
            n = x.numel()
            b = algorithmic_bytes(cell[:n].cpu().numpy(), acc[:n].cpu().numpy(), n, C)
            for s in b:
                ab[s].append(b[s])
    m3.close()
    alg = {s: float(np.mean(ab[s])) for s in ab}
    dominant = max(STAGES, key=lambda s: stage_ms[s])
    dom_gbs = alg[dominant] / (stage_ms[dominant] * 1e-3) / 1e9

    value = n_pts / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain single robot: 400x400 map at 0.04 m, 300k-point frames "
                               "(dome LiDAR + 4 depth frustums), full pipeline per frame",
                   "map_cells": C, "points_per_frame": args.points, "frames": K,
                   "mode": "per-frame plain (host waits each frame)"},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "max": float(lat.max() * 1e3)},
        "device_ms_per_step": step_ms,
        "async_ms_per_step": async_ms,
        "async_points_per_s": args.points / (async_ms * 1e-3),
        "maps_per_s": 1e3 / (wall / K * 1e3),
        "stage_ms": stage_ms,
        "stage_alg_bytes": {s: alg[s] for s in STAGES},
        "stage_alg_GBps": {s: alg[s] / (stage_ms[s] * 1e-3) / 1e9 for s in STAGES},
        "cells_touched": alg["touched"], "cells_updated": alg["updated"],
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": dom_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS,
                     "traffic": None},
    }

    # ---- CPU oracle on a bounded sample of the same workload
    if not args.no_cpu_baseline:
        import oracle as O
        p = O.Params.from_dict(params)
        nfr = max(1, args.cpu_frames)
        st = O.init_map(p, centers[0][0], centers[0][1], 0)
        wts = synth.trav_weights()
        t_cpu = 0.0
        pts = 0
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
            nrm = O.compute_normals(p, st.h, st.valid)
            st.nrm[:] = nrm.astype(np.float32)
            T, _ = O.traversability(st.h, st.valid, wts)
            st.trav[:] = T.astype(np.float32)
            t_cpu += time.perf_counter() - s
            pts += xs.size
        out["cpu_baseline"] = {"value": pts / t_cpu, "unit": "points/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {nfr} frames of the same workload, full "
                                         f"pipeline, {t_cpu:.1f} s; {cpu_model()}, "
                                         f"{os.cpu_count()} host threads visible"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
