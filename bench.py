"""Benchmark of the elevation-map fusion hot path on one MI355X.

Headline: the serving workload, continuous batching against per-frame plain
launches (points fused per second and p99 update latency).
  * 64 simulated robots; maps U{256..800}^2 at 0.04 m; frames of logU[50k, 500k]
    points (a dome LiDAR plus four depth frustums) already in device memory
    when the timed region starts; the full per-frame path (move, fusion,
    visibility clearing, normals, traversability); every map resident in
    device memory under a 32 GiB budget.
  * One step serves one frame of every robot.  Robots are closed-loop
    clients: each submits its next frame as soon as the previous one has
    completed, so the server always holds every robot's next frame.  W steps
    warm up, then K steps are timed between two device synchronisations.
  * value: points per second through the server over the K steps.
    latency_ms: per-frame update latency (submission to completion).
    plain: the same K steps through the per-frame plain calls on one stream.
  * sweep: the seeded Poisson arrival trace (20 Hz per robot; a warm-up
    second and a measured window) replayed at x1, x2, x4, ... time
    compression through both, until each stops keeping up.
  * roofline: the dominant kernel of the headline's server run, from a second
    pass of the K steps with every kernel bracketed by events on its stream.
  * pcie_inclusive: the same closed loop with every frame copied from pinned
    host memory inside the timed region (server and plain).

Sub-records, each with its plain comparison where one exists:
  * single_robot: the 400x400 map with 300k-point frames through the plain
    calls (per-kernel timings);
  * features: the further per-map steps on the same map and frames;
  * batched: 16 maps of uneven sizes, one frame each, in one batched launch
    against 16 plain pipelines; warm, and cold with a rotation over copies
    larger than the 256 MB last-level cache;
  * stress: the 2000x2000 map with 4M-point LiDAR frames, plain, and batched
    together with 8 400x400 maps;
  * cpu_baseline: the oracle on a bounded sample of the headline workload, on
    the host cores, one map per process; the 16-map batch and the stress mix,
    one map per process (clearing on sampled rays, scaled); and on the 128x128
    fusion case.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
BUDGET_BYTES = 32 << 30
SLO_S = 0.05          # one frame period at 20 Hz: a later update lags the robot by a frame
# host copies of the batched and stress workloads' maps and frames, for the
# oracle baseline: (params, centre, x, y, z, pose) per map
HOST_SPECS = {}


def say(*a):
    print("#", *a, file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed steps of the headline (one frame of every robot per step)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--robots", type=int, default=64)
    ap.add_argument("--lanes", type=int, default=2)
    ap.add_argument("--sweep-warm", type=float, default=1.0)
    ap.add_argument("--sweep-window", type=float, default=10.0)
    ap.add_argument("--sweep-max", type=int, default=64, help="largest time compression")
    ap.add_argument("--single-frames", type=int, default=30)
    ap.add_argument("--points", type=int, default=300000)
    ap.add_argument("--batched-reps", type=int, default=20)
    ap.add_argument("--stress-frames", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle seconds per process in the CPU baseline")
    ap.add_argument("--cpu-procs", type=int, default=0, help="0: min(16, host cores)")
    for leg in ("pcie", "sweep", "single", "features", "batched", "stress"):
        ap.add_argument(f"--skip-{leg}", action="store_true")
    ap.add_argument("--skip-stress-batch", action="store_true",
                    help="time the 2000x2000 map's plain calls only")
    ap.add_argument("--skip-serving", action="store_true",
                    help="profiling runs of one leg: no headline (value is null), no CPU "
                         "baseline, no PCIe or sweep legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default=None, help="batch tuning JSON (default: the tuned file)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 256 MiB device to device once (a known-size kernel that "
                         "calibrates hardware byte counters)")
    ap.add_argument("--autotune", default=None, metavar="OUT",
                    help="tune the batched executor on the 16-map workload, write OUT, exit")
    return ap.parse_args(argv)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else math.nan


# ------------------------------------------------------------ algorithmic bytes
def frame_bytes(n: float, C: float, touched: float, updated: float, entering: float) -> dict:
    """Bytes each stage of one frame must move at the least, by kernel role.
      fuse_chunk: the points (12 B) and the prior h, v of each distinct in-map
        cell they hit (8 B);
      fuse_tile: prior h, v read and h, v, t_upd, valid written for each
        updated cell (8 + 13 B);
      clear_setup: the points, and h, t_upd, valid per cell for the block
        maxima (9 B); clear_march: each cell's h, v, t_upd, valid and normal
        read once (25 B);
      cells: normals and traversability from h, valid (5 B in, 16 B out);
      move (a frame whose centre cell changes): the ring turns and the cells
      entering the map are written once (29 B each)."""
    return {"fuse_chunk": 12 * n + 8 * touched, "fuse_tile": 21 * updated,
            "clear_setup": 12 * n + 9 * C, "clear_march": 25 * C, "cells": 21 * C,
            "move": 29 * entering}


def ray_samples(x, y, z, pose, min_range: float, ray_step: float) -> int:
    """Samples of one frame's clearing rays, S = sum of K - 1 over the valid
    points, with K = ceil(max(|dx|, |dy|) / ray_step) for the ray d from the
    sensor to the point (Sec. II-E): the march's unit of work, whether a
    sample lies in the map or not.  Counted in float64 from the rotated point
    (the ray does not depend on the translation), so a ray at a rounding
    boundary may count one sample more or less than the kernels' float32
    evaluation: a throughput unit, not a parity check."""
    p = np.stack([np.asarray(v, np.float64) for v in (x, y, z)])
    d2 = (p * p).sum(axis=0)
    ok = np.isfinite(d2) & (d2 >= float(min_range) ** 2)
    r = np.asarray(pose, np.float64)[:3, :3] @ p[:, ok]
    m = np.maximum(np.abs(r[0]), np.abs(r[1])) * (1.0 / float(ray_step))
    k = np.ceil(m[m < 2.0 ** 24])
    return int(np.maximum(k - 1.0, 0.0).sum())


def add_sample_rate(kernels: dict, samples: dict) -> None:
    """Ray samples per launch and per second of each clearing march in
    ``kernels``, from the total samples of its timed launches."""
    for name, tot in samples.items():
        e = kernels.get(name)
        if e and e["launches"] > 0 and e["total_ms"] > 0:
            e["samples_per_launch"] = tot / e["launches"]
            e["G_samples_per_s"] = tot / (e["total_ms"] * 1e-3) / 1e9


PLAIN_KERNEL = {"fuse_chunk": "k_fuse_chunk", "fuse_tile": "k_fuse_tile",
                "clear_setup": "k_clear_setup", "clear_march": "k_clear_march",
                "cells": "k_normals_trav", "move": "k_move"}
BATCH_KERNEL = {"fuse_chunk": "k_fuse_chunk_b", "fuse_tile": "k_fuse_tile_b",
                "clear_setup": "k_clear_setup_b", "clear_march": "k_clear_march_b",
                "cells": "k_cells_b", "move": "k_move_b"}
KERNEL_SOURCE = {"fuse": "emx_fuse.hip", "clear": "emx_clear.hip", "cells": "emx_cells.hip",
                 "move": "emx_cells.hip"}


def code_only(text: str) -> str:
    """C/C++ source without its comments, trailing blanks and empty lines:
    what the compiler sees, so that a comment edit keeps a kernel's hash."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).split("\n"))
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash(kernel: str) -> str:
    """Hash of the code (comments left out) of the source file holding
    ``kernel`` and the headers it includes."""
    role = kernel[2:].split("_")[0]
    src = KERNEL_SOURCE.get(role, "emx_cells.hip")
    d = os.path.join(ROOT, "paper_2204_12876_amd", "csrc")
    h = hashlib.sha256()
    for f in (src, "emx_device.h", "emx_kernels.h"):
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            h.update(f.encode() + code_only(fh.read()).encode())
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


def kernel_table(kt: dict, alg: dict) -> dict:
    """Per kernel: launches, average duration, and with ``alg`` (total
    algorithmic bytes over the same launches) bytes per launch and GB/s."""
    out = {}
    for name, (cnt, tot_ms) in kt.items():
        e = {"launches": cnt, "avg_us": tot_ms / cnt * 1e3, "total_ms": tot_ms}
        if name in alg and tot_ms > 0:
            e["alg_bytes_per_launch"] = alg[name] / cnt
            e["alg_GBps"] = alg[name] / (tot_ms * 1e-3) / 1e9
        out[name] = e
    return out


def roofline(kernels: dict) -> dict:
    """The roofline object of the kernel with the largest total time among
    those with algorithmic bytes."""
    cand = [k for k in kernels if "alg_GBps" in kernels[k]]
    dom = max(cand, key=lambda k: kernels[k]["total_ms"])
    d = kernels[dom]
    traffic = measured_traffic(dom)
    return {"bound": "hbm", "kernel": dom, "achieved": d["alg_GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": d["alg_GBps"] / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": d["alg_bytes_per_launch"], "avg_launch_us": d["avg_us"]}


def load_tuning(args):
    if args.tuning:
        return args.tuning
    if os.path.exists(TUNING_FILE):
        with open(TUNING_FILE) as fh:
            return json.dumps(json.load(fh)["tuning"])
    return None


# ---------------------------------------------------------------- serving
def serving_context(args, dev):
    """The robots' frames (one per robot, re-sent from its pose; the map centre
    alternates by one cell so that every frame also moves the map), pinned on
    the host and resident on the device, and per-robot frame statistics for
    the algorithmic bytes."""
    import torch

    import synth
    from paper_2204_12876_amd import ElevationMap

    t_gen = time.perf_counter()
    d = synth.cfg3(device=dev, n_robots=args.robots, n_frames=1)
    torch.cuda.synchronize()
    items = d["items"]
    say(f"generated {len(items)} robot frames in {time.perf_counter() - t_gen:.1f} s")
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    host, device, stats = [], [], []
    for it in items:
        f = it["frames"][0]
        xyz = torch.empty((3, f.n), dtype=torch.float32, pin_memory=True)
        xyz[0].copy_(f.x)
        xyz[1].copy_(f.y)
        xyz[2].copy_(f.z)
        host.append((xyz, f.pose, it["centers"][0]))
        device.append(xyz.to(dev))
        m = ElevationMap(it["params"], *it["centers"][0], 0, device=dev)
        cell = torch.empty(f.n, dtype=torch.int32, device=dev)
        acc = torch.empty(f.n, dtype=torch.uint8, device=dev)
        m.fuse_points(f.x.contiguous(), f.y.contiguous(), f.z.contiguous(), f.pose, 100,
                      out_cell=cell, out_accept=acc)
        c = cell.cpu().numpy()
        a = acc.cpu().numpy().astype(bool)
        m.close()
        C = it["params"]["nx"] * it["params"]["ny"]
        pr = it["params"]
        S = ray_samples(xyz[0].numpy(), xyz[1].numpy(), xyz[2].numpy(), f.pose,
                        pr.get("min_range", 0.05), pr.get("ray_step", pr["resolution"]))
        stats.append(dict(n=f.n, C=C, ny=it["params"]["ny"], touched=np.unique(c[c >= 0]).size,
                          updated=np.unique(c[a]).size, samples=S))
    largest = max((it["params"] for it in items), key=lambda p: p["nx"] * p["ny"])
    return dict(items=items, host=host, device=device, stats=stats, weights=w,
                largest=largest, data=d)


def _make_request(ctx, k, j, arrival=0.0, t_off=0, resident=True):
    """Robot k's j-th frame: its one ray-cast frame re-sent from the same pose,
    with the map centre alternating by one cell; frame times increase with j
    (and with ``t_off`` between replays on the same maps).  ``resident``: the
    points are already in device memory, else they come from pinned host
    memory and each run copies them to the device."""
    from paper_2204_12876_amd.server import Request
    xyz, pose, c = ctx["host"][k]
    if resident:
        xyz = ctx["device"][k]
    r = ctx["items"][k]["params"]["resolution"]
    cx = c[0] + (r if j % 2 else 0.0)
    return Request(robot=k, xyz=xyz, pose=pose, t_ms=t_off + 100 * (j + 1), center=(cx, c[1]),
                   arrival=float(arrival))


def _executor(args, ctx, dev, tuning=None):
    from paper_2204_12876_amd.server import GpuExecutor, Server
    ex = GpuExecutor(ctx["largest"], lanes=args.lanes, max_items=64,
                     max_batch_points=8_000_000, pool_points=24_000_000,
                     weights=ctx["weights"], tuning=tuning, device=dev)
    srv = Server(ex, BUDGET_BYTES)
    for k, it in enumerate(ctx["items"]):
        srv.add_map(k, it["params"], *ctx["host"][k][2])
    return ex, srv


def _plain_maps(ctx, dev):
    from paper_2204_12876_amd import ElevationMap
    return {k: ElevationMap(it["params"], *ctx["host"][k][2], 0, device=dev)
            for k, it in enumerate(ctx["items"])}


def serving_headline(args, dev, ctx, resident=True, kernel_timing=True):
    """Closed-loop saturation: K steps (one frame of every robot per step)
    through the server, then through the per-frame plain calls.  With
    ``resident`` the frames are in device memory when the timed region
    starts; without, every frame is copied from pinned host memory inside it."""
    import torch

    from paper_2204_12876_amd import _emx
    from paper_2204_12876_amd.server import run_closed_loop, run_plain_closed_loop

    K, W = args.steps, args.warmup
    robots = list(range(len(ctx["items"])))
    mk = lambda k, j: _make_request(ctx, k, j, resident=resident)        # noqa: E731
    mx = max(h[0].shape[1] for h in ctx["host"])

    # ---- server: W warm-up steps, then K timed steps between synchronisations
    ex, srv = _executor(args, ctx, dev)
    run_closed_loop(srv, mk, robots, max(W, 1))
    srv.completed.clear()
    srv.batch_sizes.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reqs = run_closed_loop(srv, lambda k, j: mk(k, W + j), robots, K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pts = sum(r.n for r in reqs)
    lat = np.array([r.latency for r in reqs])
    batches = list(srv.batch_sizes)
    where = "resident" if resident else "from host"
    say(f"server closed loop ({where}): {pts / wall / 1e9:.2f} G points/s, p99 "
        f"{pct(lat, 99) * 1e3:.2f} ms, mean batch {np.mean(batches):.1f}")

    # ---- per-kernel timing: the same K steps again, every kernel bracketed by
    # events on its stream; algorithmic bytes summed over the frames each
    # launch served
    kernels = roof = None
    if kernel_timing:
        kernels, roof = _serving_kernels(ctx, srv, mk, robots, K, W)
    b_stats = ex.graph_stats()
    for m in list(ex.maps):
        ex.drop_map(m)

    # ---- plain: the same steps through the per-frame calls on one stream
    maps = _plain_maps(ctx, dev)
    run_plain_closed_loop(maps, mk, robots, max(W, 1), ctx["weights"], device=dev, max_points=mx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    preqs = run_plain_closed_loop(maps, lambda k, j: mk(k, W + j), robots, K, ctx["weights"],
                                  device=dev, max_points=mx)
    torch.cuda.synchronize()
    pwall = time.perf_counter() - t0
    plat = np.array([r.latency for r in preqs])
    for m in maps.values():
        m.close()
    say(f"plain closed loop ({where}): {pts / pwall / 1e9:.2f} G points/s, p99 "
        f"{pct(plat, 99) * 1e3:.2f} ms")
    out = {
        "value": pts / wall,
        "ms_per_step": wall / K * 1e3,
        "maps_per_s": len(reqs) / wall,
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                       "max": float(lat.max() * 1e3),
                       "note": "submission to completion; closed-loop clients"},
        "server": {"mean_batch_items": float(np.mean(batches)), "batches": len(batches),
                   "lanes": args.lanes, "batched_calls_and_graph_captures": list(b_stats),
                   "hbm_budget_bytes": BUDGET_BYTES, "hbm_reserved_bytes": srv.budget.used},
        "plain": {"points_per_s": pts / pwall, "ms_per_step": pwall / K * 1e3,
                  "p50_ms": pct(plat, 50) * 1e3, "p99_ms": pct(plat, 99) * 1e3,
                  "mode": "per-frame plain calls (move_fuse_points, clear_visibility, "
                          "normals_traversability) on one stream, frames in turn"},
        "speedup_vs_plain": pwall / wall,
        "points_per_step": pts / K,
        "frames": "resident in device memory before the timed region" if resident else
                  "copied from pinned host memory inside the timed region",
    }
    if kernel_timing:
        out["kernels"] = kernels
        out["roofline"] = roof
    return out


def _serving_kernels(ctx, srv, mk, robots, K, W):
    """Per-kernel table and roofline of K more closed-loop steps."""
    from paper_2204_12876_amd import _emx
    from paper_2204_12876_amd.server import run_closed_loop
    _emx.timing_begin()
    treqs = run_closed_loop(srv, lambda k, j: mk(k, W + K + j), robots, K)
    kt = _emx.timing_end()
    alg, samples = {}, {}
    for r in treqs:
        s = ctx["stats"][r.robot]
        names = BATCH_KERNEL if r.batch_items > 1 else PLAIN_KERNEL
        # the centre alternates by one cell in x: one column enters
        for role, b in frame_bytes(s["n"], s["C"], s["touched"], s["updated"], s["ny"]).items():
            alg[names[role]] = alg.get(names[role], 0.0) + b
        march = names["clear_march"]
        samples[march] = samples.get(march, 0) + s["samples"]
    kernels = kernel_table(kt, alg)
    add_sample_rate(kernels, samples)
    return kernels, roofline(kernels)


def poisson_trace(ctx, seconds: float, seed: int = 12876 + 3):
    """Seeded Poisson arrivals (each robot at its rate) over ``seconds``:
    (robot, frame index, arrival time) sorted by time."""
    rng = np.random.default_rng(seed)
    out = []
    for k, it in enumerate(ctx["items"]):
        gaps = rng.exponential(1.0 / it["rate_hz"], int(seconds * it["rate_hz"] * 3) + 8)
        times = np.cumsum(gaps)
        for j, t in enumerate(times[times < seconds]):
            out.append((k, j, float(t)))
    out.sort(key=lambda e: e[2])
    return out


def window_summary(reqs, t_from: float, t_to: float) -> dict:
    """Requests arriving in [t_from, t_to) (compressed time): latency
    percentiles, and delivered points/s = their points over the time from
    t_from until the last of them completed."""
    sel = [r for r in reqs if t_from <= r.arrival < t_to]
    lat = np.array([r.latency for r in sel])
    pts = sum(r.n for r in sel)
    end = max(r.done for r in sel)
    return dict(frames=len(sel), points=int(pts), offered_points_per_s=pts / (t_to - t_from),
                points_per_s=pts / (end - t_from), p50_ms=pct(lat, 50) * 1e3,
                p99_ms=pct(lat, 99) * 1e3, max_ms=float(lat.max() * 1e3))


def serving_sweep(args, dev, ctx):
    """The Poisson trace replayed at x1, x2, x4, ... through the server and the
    plain loop.  A system stops at the first level where it no longer keeps
    up: delivered points/s under 95% of offered, or p99 above one frame period
    (50 ms)."""
    from paper_2204_12876_amd.server import run_plain_trace, run_trace

    warm, win = args.sweep_warm, args.sweep_window
    base = poisson_trace(ctx, warm + win)
    offered = sum(ctx["stats"][k]["n"] for k, _, t in base if t >= warm) / win
    mx = max(h[0].shape[1] for h in ctx["host"])
    levels = []
    c = 1
    while c <= args.sweep_max:
        levels.append(c)
        c *= 2
    ex, srv = _executor(args, ctx, dev)
    maps = _plain_maps(ctx, dev)
    out = {"trace": f"Poisson, 20 Hz per robot, {warm:g} s warm-up + {win:g} s window at x1; "
                    f"{len(base)} frames; offered {offered / 1e6:.0f} M points/s at x1",
           "slo_ms": SLO_S * 1e3, "levels": []}
    alive = {"server": True, "plain": True}
    for li, c in enumerate(levels):
        ent = {"compression": c}
        for name in ("server", "plain"):
            if not alive[name]:
                continue
            # frame times keep increasing from one replay to the next on the same maps
            t_off = (li + 1) * 10_000_000
            reqs = [_make_request(ctx, k, j, t / c, t_off) for k, j, t in base]
            for i, r in enumerate(reqs):
                r.seq = i
            if name == "server":
                srv.completed.clear()
                srv.batch_sizes.clear()
                run_trace(srv, reqs, timeout_s=300)
            else:
                run_plain_trace(maps, reqs, ctx["weights"], device=dev, max_points=mx)
            s = window_summary(reqs, warm / c, (warm + win) / c)
            if name == "server":
                s["mean_batch_items"] = float(np.mean([r.batch_items for r in reqs
                                                       if r.arrival >= warm / c]))
            keeps_up = s["points_per_s"] >= 0.95 * s["offered_points_per_s"] and \
                s["p99_ms"] <= SLO_S * 1e3
            s["keeps_up"] = bool(keeps_up)
            ent[name] = s
            alive[name] = keeps_up
            say(f"sweep x{c} {name}: {s['points_per_s'] / 1e9:.2f} G points/s of "
                f"{s['offered_points_per_s'] / 1e9:.2f}, p50 {s['p50_ms']:.2f} "
                f"p99 {s['p99_ms']:.2f} ms" + (f", batch {s['mean_batch_items']:.1f}"
                                              if name == "server" else ""))
        out["levels"].append(ent)
        if not alive["server"] and not alive["plain"]:
            break
    for m in list(ex.maps):
        ex.drop_map(m)
    for m in maps.values():
        m.close()
    for name in ("server", "plain"):
        ok = [e[name] for e in out["levels"] if name in e and e[name]["keeps_up"]]
        out[f"{name}_sustained_points_per_s"] = max((s["points_per_s"] for s in ok), default=0.0)
    return out


# ------------------------------------------------------------- plain, one robot
def single_robot(args, dev):
    """The 400x400 map with 300k-point frames along a trajectory, through the
    plain calls: frames back to back, then with the host waiting, then with
    every kernel timed by events."""
    import torch

    import synth
    from paper_2204_12876_amd import ElevationMap, _emx

    K = args.single_frames
    W = 5
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

    m = fresh()
    t0 = time.perf_counter()
    for j in range(K):
        run(m, W + j)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m.close()
    n_pts = sum(frames[W + j][0].numel() for j in range(K))
    say(f"single robot back to back: {wall / K * 1e3:.3f} ms/frame")

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

    # frame statistics for the algorithmic bytes (untimed), then the kernels
    m = fresh()
    cell = torch.empty(args.points, dtype=torch.int32, device=dev)
    acc = torch.empty(args.points, dtype=torch.uint8, device=dev)
    r = params["resolution"]
    cell_of = [(math.floor(cx / r), math.floor(cy / r)) for cx, cy in centers]
    alg, samples = {}, 0
    for j in range(K):
        run(m, W + j, cell=cell, acc=acc)
        n = frames[W + j][0].numel()
        fx, fy, fz, fpose = frames[W + j][:4]
        samples += ray_samples(fx.cpu().numpy(), fy.cpu().numpy(), fz.cpu().numpy(), fpose,
                               params.get("min_range", 0.05),
                               params.get("ray_step", params["resolution"]))
        c = cell[:n].cpu().numpy()
        a = acc[:n].cpu().numpy().astype(bool)
        sx = min(abs(cell_of[W + j][0] - cell_of[W + j - 1][0]), params["nx"])
        sy = min(abs(cell_of[W + j][1] - cell_of[W + j - 1][1]), params["ny"])
        entering = sx * params["ny"] + sy * params["nx"] - sx * sy
        for role, b in frame_bytes(n, C, np.unique(c[c >= 0]).size, np.unique(c[a]).size,
                                   entering).items():
            if b > 0:
                alg[PLAIN_KERNEL[role]] = alg.get(PLAIN_KERNEL[role], 0.0) + b
    m.close()
    m = fresh()
    _emx.timing_begin()
    for j in range(K):
        run(m, W + j)
    kt = _emx.timing_end()
    m.close()
    kernels = kernel_table(kt, alg)
    add_sample_rate(kernels, {PLAIN_KERNEL["clear_march"]: samples})
    return {
        "workload": "one robot: 400x400 map at 0.04 m, 300k-point frames (dome LiDAR + 4 depth "
                    "frustums) along a trajectory, full path per frame through the plain calls",
        "frames": K, "points_per_s": n_pts / wall, "ms_per_frame": wall / K * 1e3,
        "maps_per_s": K / wall,
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                       "note": "host waits for each frame"},
        "stage_ms": stage_ms, "kernels": kernels, "roofline": roofline(kernels),
    }, dict(frames=frames, centers=centers, params=params)


# --------------------------------------------------- optional per-map features
def features(args, dev, ctx):
    """The features beyond the base path on the single-robot map and frames:
    time variance, the wall/edge rule and the upper bound layer on, through the
    extended per-frame sequence (move, drift compensation, fusion, clearing
    with the bound, normals, traversability, overlap clearance, inpainting).
    Each feature is then timed per kernel over the frames."""
    import torch

    import synth
    from paper_2204_12876_amd import ElevationMap, _emx, smooth

    frames, centers, params = ctx["frames"], ctx["centers"], ctx["params"]
    W = min(5, len(frames) // 2)
    K = min(20, len(frames) - W)
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
        return _emx.timing_end()

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
    out = {"workload": "the single-robot map and frames with time_variance, "
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
    fk = out["wall_rule_and_time_variance_fusion"]["kernels"]
    ab = {"k_zero_u32": 4 * C, "k_fuse_count": 12 * n_mean + 8 * touched,
          "k_time_variance": 2 * C + 8 * valid}
    for k in ("k_zero_u32", "k_fuse_count", "k_time_variance"):
        if k in fk:
            fk[k]["alg_bytes"] = ab[k]
            fk[k]["alg_GBps"] = ab[k] / (fk[k]["avg_us"] * 1e-6) / 1e9
    m.close()
    return out


# ------------------------------------------------------------ batched, many maps
def _frame_stats(dev, params, centre, frame):
    """Points, cells, touched and updated cells of one frame fused into a
    fresh map at ``centre`` (for the algorithmic bytes; untimed)."""
    import torch

    from paper_2204_12876_amd import ElevationMap
    x, y, z, pose = frame[:4]
    m = ElevationMap(params, centre[0], centre[1], 0, device=dev)
    cell = torch.empty(x.numel(), dtype=torch.int32, device=dev)
    acc = torch.empty(x.numel(), dtype=torch.uint8, device=dev)
    m.fuse_points(x, y, z, pose, 100, out_cell=cell, out_accept=acc)
    c = cell.cpu().numpy()
    a = acc.cpu().numpy().astype(bool)
    m.close()
    return dict(n=x.numel(), C=params["nx"] * params["ny"], touched=np.unique(c[c >= 0]).size,
                updated=np.unique(c[a]).size)


def batch_vs_plain(args, dev, tuning, specs, label: str, reps: int, cold_copies: int = 0):
    """Maps of ``specs`` (params, centre, frame) through one emx_pipeline_batch
    per step against their plain per-frame pipelines; warm (the same maps and
    frames every step) and, with ``cold_copies``, rotating over that many copies
    of every map and frame."""
    import torch

    from paper_2204_12876_amd import BatchEntry, ElevationMap, PipelineBatch, _emx

    w = torch.from_numpy(__import__("synth").trav_weights()).to(dev)
    stream = torch.cuda.current_stream(dev)
    pts = sum(f[0].numel() for _, _, f in specs)
    C = sum(p["nx"] * p["ny"] for p, _, _ in specs)

    def maps():
        return [ElevationMap(p, c[0], c[1], 0, device=dev) for p, c, _ in specs]

    def frames_copy():
        return [(f[0].clone(), f[1].clone(), f[2].clone(), f[3]) for _, _, f in specs]

    def centre(c, rep, p):       # the centre alternates by one cell: every step moves
        return (c[0] + (p["resolution"] if rep % 2 else 0.0), c[1])

    pb = PipelineBatch(tuning, device=dev)
    copies = [(maps(), frames_copy()) for _ in range(max(1, cold_copies))]

    def batch(rep, copy=0):
        mb, fr = copies[copy]
        pb.run([BatchEntry(m, x, y, z, pose, 100 * (rep + 1), center=centre(c, rep, p), weights=w)
                for m, (x, y, z, pose), (p, c, _) in zip(mb, fr, specs)])

    def timed(fn, r):
        for rep in range(3):
            fn(rep)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for rep in range(3, 3 + r):
            fn(rep)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / r

    t_b = timed(batch, reps)
    lat_b = []
    for rep in range(3 + reps, 3 + 2 * reps):
        s = time.perf_counter()
        batch(rep)
        stream.synchronize()
        lat_b.append(time.perf_counter() - s)
    t_cold = None
    if cold_copies > 1:
        t_cold = timed(lambda rep: batch(rep, rep % cold_copies), reps)
    # per-kernel timing of the batched launches (direct, every kernel bracketed)
    pbd = PipelineBatch(json.dumps(dict(json.loads(tuning) if tuning else {}, graph=0)),
                        device=dev)
    mb, fr = copies[0]
    _emx.timing_begin()
    for rep in range(reps):
        pbd.run([BatchEntry(m, x, y, z, pose, 100 * (rep + 1), center=centre(c, rep, p),
                            weights=w) for m, (x, y, z, pose), (p, c, _) in zip(mb, fr, specs)])
    kt = _emx.timing_end()
    pbd.close()

    mp = maps()
    fr0 = copies[0][1]
    scratch = max((m.scratch(f[0].numel()) for m, f in zip(mp, fr0)), key=lambda t: t.numel())

    def plain(rep):
        for m, (x, y, z, pose), (p, c, _) in zip(mp, fr0, specs):
            m.move_fuse_points(*centre(c, rep, p), x, y, z, pose, 100 * (rep + 1),
                               scratch=scratch)
            m.clear_visibility(x, y, z, pose, 100 * (rep + 1), scratch=scratch)
            m.normals_traversability(w)

    t_p = timed(plain, reps)
    lat_p = []
    for rep in range(3 + reps, 3 + 2 * reps):
        s = time.perf_counter()
        plain(rep)
        stream.synchronize()
        lat_p.append(time.perf_counter() - s)
    # the batch promises the plain calls' bits: fresh maps through three steps
    # each way
    ma, mb2 = maps(), maps()
    for rep in range(3):
        pb.run([BatchEntry(m, x, y, z, pose, 100 * (rep + 1), center=centre(c, rep, p),
                           weights=w) for m, (x, y, z, pose), (p, c, _) in zip(ma, fr0, specs)])
        for m, (x, y, z, pose), (p, c, _) in zip(mb2, fr0, specs):
            m.move_fuse_points(*centre(c, rep, p), x, y, z, pose, 100 * (rep + 1),
                               scratch=scratch)
            m.clear_visibility(x, y, z, pose, 100 * (rep + 1), scratch=scratch)
            m.normals_traversability(w)
    same = all(torch.equal(a.export_state(), b.export_state()) for a, b in zip(ma, mb2))
    for m in ma + mb2:
        m.close()
    for mb_, _ in copies:
        for m in mb_:
            m.close()
    for m in mp:
        m.close()
    pb.close()
    say(f"{label}: batched {t_b * 1e3:.3f} ms vs plain {t_p * 1e3:.3f} ms per step")
    n = len(specs)
    out = {
        "points_per_step": int(pts), "cells": int(C), "maps": n,
        "batched": {"ms": t_b * 1e3, "points_per_s": pts / t_b, "maps_per_s": n / t_b,
                    "p50_ms": pct(lat_b, 50) * 1e3, "p99_ms": pct(lat_b, 99) * 1e3},
        "plain": {"ms": t_p * 1e3, "points_per_s": pts / t_p, "maps_per_s": n / t_p,
                  "p50_ms": pct(lat_p, 50) * 1e3, "p99_ms": pct(lat_p, 99) * 1e3},
        "speedup": t_p / t_b,
        "batched_kernels": {k: {"launches": c_, "avg_us": tot / c_ * 1e3}
                            for k, (c_, tot) in kt.items()},
        "tuning": json.loads(tuning) if tuning else "library defaults",
    }
    out["results_identical"] = bool(same)
    # fusion (both passes) against the HBM roofline: the algorithmic bytes of
    # every map's frame over the two batched fusion kernels' average times
    fb = 0.0
    for p_, c_, f_ in specs:
        st_ = _frame_stats(dev, p_, c_, f_)
        b_ = frame_bytes(st_["n"], st_["C"], st_["touched"], st_["updated"], 0.0)
        fb += b_["fuse_chunk"] + b_["fuse_tile"]
    t_f = sum(tot / c_ for k, (c_, tot) in kt.items() if k in ("k_fuse_chunk_b", "k_fuse_tile_b"))
    if t_f > 0:
        out["fusion_roofline"] = {
            "bound": "hbm", "kernels": ["k_fuse_chunk_b", "k_fuse_tile_b"],
            "alg_bytes_per_launch": fb, "us_per_launch": t_f * 1e3,
            "achieved": fb / (t_f * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": fb / (t_f * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "note": "12 B per point, 8 B per touched cell, 21 B per updated cell; both passes"}
    if t_cold is not None:
        out["batched_cold"] = {"ms": t_cold * 1e3, "points_per_s": pts / t_cold,
                               "copies": cold_copies,
                               "note": "each step takes the next copy of every map and frame; "
                                       "the copies together exceed the 256 MB last-level cache"}
    return out


def _host_specs(specs):
    """(params, centre, x, y, z, pose) with the points copied to host numpy."""
    return [(p, c, f[0].cpu().numpy(), f[1].cpu().numpy(), f[2].cpu().numpy(),
             np.asarray(f[3])) for p, c, f in specs]


def batched_maps(args, dev, tuning):
    import torch

    import synth
    t_gen = time.perf_counter()
    d = synth.cfg2(device=dev)
    torch.cuda.synchronize()
    specs = []
    for it in d["items"]:
        f = it["frames"][0]
        specs.append((it["params"], (0.0, 0.0), (f.x.contiguous(), f.y.contiguous(),
                                                 f.z.contiguous(), f.pose)))
    say(f"generated 16 maps / {sum(f[0].numel() for _, _, f in specs)} points in "
        f"{time.perf_counter() - t_gen:.1f} s")
    HOST_SPECS["batched"] = _host_specs(specs)
    # every copy holds the maps' state (about 30 B per cell) and the frames;
    # four copies pass 256 MB several times over
    out = batch_vs_plain(args, dev, tuning, specs, "16 maps", args.batched_reps, cold_copies=4)
    out["workload"] = ("16 maps, sides U{200..1000} at 0.02-0.1 m, one frame each of "
                       "logU[20k, 1M] points, full path")
    return out


def stress(args, dev, tuning, single_ctx):
    """The 2000x2000 map with 4M-point LiDAR frames: plain per frame along its
    trajectory, and batched together with 8 400x400 maps (300k-point frames of
    the single-robot workload)."""
    import torch

    import synth
    from paper_2204_12876_amd import ElevationMap, _emx

    S = max(2, args.stress_frames)
    t_gen = time.perf_counter()
    d = synth.cfg4(n_frames=S, device=dev)
    torch.cuda.synchronize()
    say(f"generated {S} stress frames in {time.perf_counter() - t_gen:.1f} s")
    frames = [(f.x.contiguous(), f.y.contiguous(), f.z.contiguous(), f.pose, f.t_ms)
              for f in d["frames"]]
    centers = d["centers"]
    params = d["params"]
    C = params["nx"] * params["ny"]
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    m = ElevationMap(params, *centers[0], 0, device=dev)
    scratch = m.scratch(max(f[0].numel() for f in frames))
    n_steps = 2 * S

    def run(k, t):
        x, y, z, pose, _ = frames[k % S]
        m.move_fuse_points(*centers[k % S], x, y, z, pose, t, scratch=scratch)
        m.clear_visibility(x, y, z, pose, t, scratch=scratch)
        m.normals_traversability(w)

    run(0, 100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, n_steps + 1):
        run(k, 100 * (k + 1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pts = sum(frames[k % S][0].numel() for k in range(1, n_steps + 1))
    _emx.timing_begin()
    for k in range(n_steps + 1, 2 * n_steps + 1):
        run(k, 100 * (k + 1))
    kt = _emx.timing_end()
    m.close()
    say(f"stress plain: {wall / n_steps * 1e3:.2f} ms/frame")
    out = {"workload": "2000x2000 map at 0.02 m, 4M-point frames from a 128-beam LiDAR "
                       "(30 m, 10% outliers, 500 boxes), full path per frame",
           "plain": {"frames": n_steps, "distinct_frames": S, "ms_per_frame": wall / n_steps * 1e3,
                     "points_per_s": pts / wall,
                     "kernels": {k: {"launches": c, "avg_us": tot / c * 1e3}
                                 for k, (c, tot) in kt.items()}}}
    if args.skip_stress_batch:
        return out
    # batched with 8 smaller maps
    specs = [(params, centers[0], frames[0][:4])]
    sf, sc, sp = single_ctx["frames"], single_ctx["centers"], single_ctx["params"]
    for k in range(8):
        specs.append((sp, sc[k], sf[k][:4]))
    HOST_SPECS["stress_mix"] = _host_specs(specs)
    b = batch_vs_plain(args, dev, tuning, specs, "stress batch", max(3, args.batched_reps // 4))
    b["workload"] = ("the 2000x2000 map with one 4M-point frame and 8 400x400 maps with one "
                     "300k-point frame each, one batched launch per step")
    out["batched"] = b
    return out


# ------------------------------------------------------------------- CPU oracle
def _oracle_worker(job):
    """One process: the oracle's full per-frame path on its maps' frames,
    frame after frame in turn, until ``seconds`` of oracle time have passed."""
    import oracle as O
    frames, weights, seconds = job
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    t_cpu, pts, nfr = 0.0, 0, 0
    states = {}
    while t_cpu < seconds:
        for (key, params, centre, xs, ys, zs, pose) in frames:
            p = O.Params.from_dict(params)
            st = states.get(key)
            if st is None:
                st = O.init_map(p, centre[0], centre[1], 0)
            t = 100 * (nfr + 1)
            s = time.perf_counter()
            st = O.move_map(p, st, centre[0] + (p.resolution if nfr % 2 else 0.0), centre[1])
            r = O.fuse(p, st, xs, ys, zs, pose, t)
            st = r.state
            mk = O.clear_visibility(p, st, xs, ys, zs, pose, t)
            st = O.apply_clear(p, st, mk)
            st.nrm[:] = O.compute_normals(p, st.h, st.valid).astype(np.float32)
            T, _ = O.traversability(st.h, st.valid, weights)
            st.trav[:] = T.astype(np.float32)
            t_cpu += time.perf_counter() - s
            states[key] = st
            pts += xs.size
            nfr += 1
            if t_cpu >= seconds:
                break
    return pts, t_cpu, nfr


def _oracle_map_job(job):
    """One map's frame through the oracle's full path in one process: fusion
    of every point, clearing of a seeded sample of the rays (its time scaled
    to all of them), normals and traversability of every cell.  Returns
    (points, seconds, sampled rays)."""
    import oracle as O
    params, centre, xs, ys, zs, pose, weights, ray_sample = job
    p = O.Params.from_dict(params)
    st = O.init_map(p, centre[0], centre[1], 0)
    n = xs.size
    s = time.perf_counter()
    st = O.fuse(p, st, xs, ys, zs, pose, 100).state
    t_fuse = time.perf_counter() - s
    k = min(n, ray_sample)
    idx = np.sort(np.random.default_rng(12876).choice(n, size=k, replace=False))
    s = time.perf_counter()
    mk = O.clear_visibility(p, st, xs[idx], ys[idx], zs[idx], pose, 100)
    t_clear = (time.perf_counter() - s) * (n / max(k, 1))
    st = O.apply_clear(p, st, mk)
    s = time.perf_counter()
    st.nrm[:] = O.compute_normals(p, st.h, st.valid).astype(np.float32)
    T, _ = O.traversability(st.h, st.valid, weights)
    t_cells = time.perf_counter() - s
    return n, t_fuse + t_clear + t_cells, k


def _cfg0_worker(job):
    """The oracle's fusion on the 128x128 case, 20 repetitions."""
    import oracle as O
    import synth
    reps = job
    d = synth.cfg0()
    p = O.Params.from_dict(d["params"])
    f = d["frames"][0]
    xs, ys, zs = f.numpy()
    ts = []
    for _ in range(reps):
        st = O.init_map(p, 0.0, 0.0, 0)
        s = time.perf_counter()
        O.fuse(p, st, xs, ys, zs, f.pose, f.t_ms)
        ts.append(time.perf_counter() - s)
    return xs.size, ts


def cpu_pool(args):
    """Worker processes for the oracle baseline, started before the GPU is
    touched (each is a fresh interpreter)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    procs = args.cpu_procs or min(16, os.cpu_count() or 1)
    # one thread per worker: the variables are read when each interpreter starts
    keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                           "MKL_NUM_THREADS")}
    for k in keep:
        os.environ[k] = "1"
    pool = ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn"))
    # a worker starts per task submitted while none is idle: start them all now
    list(pool.map(time.sleep, [0.5] * procs))
    for k, v in keep.items():
        if v is None:
            os.environ.pop(k)
        else:
            os.environ[k] = v
    return pool, procs


def cpu_baseline(args, ctx, pool, procs):
    """The oracle (float64 NumPy, one thread per process) on the headline
    workload: the robots' frames spread over ``procs`` processes, one map per
    process at a time, each running for about ``cpu_seconds``; then one
    process alone.  Also the 128x128 fusion case, 20 repetitions."""
    import synth
    jobs = [[] for _ in range(procs)]
    for k, it in enumerate(ctx["items"]):
        xyz, pose, c = ctx["host"][k]
        a = xyz.numpy()
        jobs[k % procs].append((k, it["params"], c, a[0].copy(), a[1].copy(), a[2].copy(),
                                np.asarray(pose)))
    wts = synth.trav_weights()
    t0 = time.perf_counter()
    res = list(pool.map(_oracle_worker, [(j, wts, args.cpu_seconds) for j in jobs if j]))
    wall = time.perf_counter() - t0
    pts = sum(r[0] for r in res)
    nfr = sum(r[2] for r in res)
    one = pool.submit(_oracle_worker, (jobs[0], wts, args.cpu_seconds)).result()
    cfg0 = pool.submit(_cfg0_worker, 20).result()
    n0, ts0 = cfg0
    used = len([j for j in jobs if j])
    # the batched and stress workloads: one map per process
    multi = {}
    for key, specs in HOST_SPECS.items():
        sample = 20000 if key == "batched" else 5000
        res_m = list(pool.map(_oracle_map_job, [(pr, c_, x_, y_, z_, po_, wts, sample)
                                                for pr, c_, x_, y_, z_, po_ in specs]))
        # maps dealt to the processes in turn; the slowest process sets the wall
        load = [0.0] * procs
        for i, (_, secs, _) in enumerate(res_m):
            load[i % procs] += secs
        n_all = sum(r[0] for r in res_m)
        multi[key] = {"points_per_s": n_all / max(load), "maps": len(res_m),
                      "cores": min(procs, len(res_m)), "points": int(n_all),
                      "seconds_slowest_process": max(load),
                      "sample": f"fusion of every point, normals and traversability of every "
                                f"cell; clearing timed on {sample} seeded rays per map and "
                                f"scaled to all of them"}
        say(f"oracle on {key}: {n_all / max(load) / 1e6:.2f} M points/s over "
            f"{min(procs, len(res_m))} processes")
    return {"value": pts / wall, "unit": "points/s", "cores": used, "kind": "oracle",
            "sample": f"the serving workload's robot frames (full path: move, fusion, clearing, "
                      f"normals, traversability), {used} processes of one thread each, each "
                      f"on its robots' maps in turn for about {args.cpu_seconds:g} s: {nfr} "
                      f"frames, {pts / 1e6:.1f} M points in {wall:.1f} s wall; {cpu_model()}, "
                      f"{os.cpu_count()} host threads visible",
            "single_core": {"value": one[0] / one[1], "frames": one[2],
                            "seconds": one[1], "cores": 1},
            "fusion_128x128_20k": {"points_per_s": n0 / float(np.median(ts0)),
                                   "median_ms": float(np.median(ts0) * 1e3), "reps": len(ts0),
                                   "cores": 1},
            "per_workload": multi}


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


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every map and frame "
              "of this workload fits one MI355X.", file=sys.stderr)
        sys.exit(2)
    pool = procs = None
    if args.skip_serving:
        args.no_cpu_baseline = args.skip_pcie = args.skip_sweep = True
    if not args.no_cpu_baseline and not args.autotune:
        pool, procs = cpu_pool(args)        # the workers start before the GPU is touched
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
    if args.skip_serving:
        ctx, head = None, {"value": None, "ms_per_step": None}
    else:
        ctx = serving_context(args, dev)
        head = serving_headline(args, dev, ctx)
    out = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving: {args.robots} robots, maps U{{256..800}}^2 at "
                               "0.04 m, frames logU[50k, 500k] points (dome LiDAR + 4 depth "
                               "frustums) resident in device memory, full path per frame, "
                               "continuous-batching server under a 32 GiB device budget",
                   "robots": args.robots, "frames_per_step": args.robots,
                   "lanes": args.lanes,
                   "mode": "closed-loop clients: each robot submits its next frame when the "
                           "previous one completes"},
    }
    out.update(head)
    if not args.skip_pcie:
        out["pcie_inclusive"] = serving_headline(args, dev, ctx, resident=False,
                                                 kernel_timing=False)
    if not args.skip_sweep:
        out["sweep"] = serving_sweep(args, dev, ctx)
    single_ctx = None
    if not args.skip_single or not args.skip_features or \
            not (args.skip_stress or args.skip_stress_batch):
        single, single_ctx = single_robot(args, dev)
        if not args.skip_single:
            out["single_robot"] = single
    if not args.skip_features:
        out["features"] = features(args, dev, single_ctx)
    if not args.skip_batched:
        out["batched"] = batched_maps(args, dev, tuning)
    if not args.skip_stress:
        out["stress"] = stress(args, dev, tuning, single_ctx)
    if pool is not None:
        out["cpu_baseline"] = cpu_baseline(args, ctx, pool, procs)
        pool.shutdown()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
