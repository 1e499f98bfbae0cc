"""Autotuner of the batched executor's launch geometry.

The batched kernels are persistent: each stage runs a fixed number of
workgroups that walk the batch's work units.  The tuning picks those counts
per stage and the clearing segment length (ray samples per queued entry).  It
never changes results: every candidate yields the same bits.

Search: coordinate descent from the library defaults.  Each knob in turn is
set to each of its candidate values with the others held, the fastest is
kept, and the sweep repeats until a round changes nothing.  A candidate is
timed as the wall time of back-to-back batches between two device
synchronisations, the median of several repeats, so host-side batch
preparation counts as it does in use.

The caller supplies the workload as a function that runs one batch; bench.py
--autotune tunes on the 16-map batched workload and writes the result that
the benchmark then loads (tuning_mi355x.json next to this file).
"""
from __future__ import annotations

import json
import time

# 65536 means one workgroup per work unit for every batch of this size class.
SPACE = {
    "grid_chunk": [256, 512, 1024, 2048, 4096, 65536],
    "grid_tile": [256, 512, 1024, 2048, 4096, 65536],
    "grid_setup": [512, 1024, 2048, 4096, 8192, 65536],
    "grid_march": [1024, 2048, 4096, 8192, 16384],
    "grid_move": [256, 512, 1024, 2048, 8192, 65536],
    "grid_cells": [256, 512, 1024, 2048, 8192, 65536],
    "seg": [16, 32, 64, 128],
}


def time_tuning(run_batch, tuning: dict, reps: int = 8, repeats: int = 3, device=None) -> float:
    """Median seconds per batch of ``run_batch(pb, rep)`` under ``tuning``."""
    import torch

    from . import PipelineBatch
    pb = PipelineBatch(json.dumps(tuning), device=device)
    rep = 0
    for _ in range(3):                       # capture the graphs of both host tables
        run_batch(pb, rep)
        rep += 1
    torch.cuda.synchronize(device)
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        for _ in range(reps):
            run_batch(pb, rep)
            rep += 1
        torch.cuda.synchronize(device)
        times.append((time.perf_counter() - t0) / reps)
    pb.close()
    times.sort()
    return times[len(times) // 2]


def autotune(run_batch, start: dict, space: dict = SPACE, reps: int = 8, max_rounds: int = 3,
             device=None, log=None):
    """Coordinate descent over ``space`` from ``start``; returns (best, seconds, history)."""
    best = dict(start)
    best_t = time_tuning(run_batch, best, reps, device=device)
    history = [(dict(best), best_t)]
    if log:
        log(f"start {best} {best_t * 1e3:.3f} ms")
    for rnd in range(max_rounds):
        changed = False
        for knob, values in space.items():
            for v in values:
                if v == best[knob]:
                    continue
                cand = dict(best)
                cand[knob] = v
                t = time_tuning(run_batch, cand, reps, device=device)
                history.append((cand, t))
                if t < best_t * 0.98:            # a clear win, not noise
                    best, best_t, changed = cand, t, True
                    if log:
                        log(f"round {rnd} {knob}={v}: {t * 1e3:.3f} ms (best)")
        if not changed:
            break
    return best, best_t, history


def default_tuning() -> dict:
    from . import PipelineBatch
    pb = PipelineBatch()
    t = json.loads(pb.tuning)
    pb.close()
    return t
