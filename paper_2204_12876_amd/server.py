"""Continuous-batching server for many robots' elevation maps on one GPU.

Robots submit frames (host point clouds with pose, time and map centre) as they
arrive.  The server
  * keeps every admitted map's state resident in device memory;
  * admits maps against a fixed device-memory budget, which also covers a pool
    for staging frames on the device and each lane's batch scratch;
  * keeps per-map FIFO order with at most one frame of a map in flight, since
    each frame updates its map's state;
  * whenever a lane is free, forms a batch from the oldest waiting frames of
    maps not in flight (up to the item limit and the staging room) and
    launches it at once.  It does not wait for a batch to fill: frames that
    arrive while other batches run join the next one (continuous batching).
  * runs lanes on separate streams, so one batch's host-to-device copies and
    kernels overlap another's.

Each batch runs the whole per-frame path (move, fusion, clearing, normals,
traversability) through emx_pipeline_batch.  That call gives every map the
same bits it would get from the plain per-frame calls, so a frame's result does
not depend on the batch it rode in.

The device side sits behind a small executor interface (GpuExecutor here), so
scheduling and admission can also run against a simulated executor.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _emx

__all__ = ["AdmissionError", "HbmBudget", "Request", "Server", "GpuExecutor", "FramePool",
           "run_trace", "run_closed_loop", "run_plain_trace", "run_plain_closed_loop",
           "latency_summary"]


class AdmissionError(RuntimeError):
    """A map or frame does not fit the device-memory budget or the limits."""


class HbmBudget:
    """Byte accounting of device memory against a fixed budget."""

    def __init__(self, total: int):
        self.total = int(total)
        self.parts: Dict[object, int] = {}

    @property
    def used(self) -> int:
        return sum(self.parts.values())

    @property
    def free(self) -> int:
        return self.total - self.used

    def reserve(self, key, nbytes: int):
        if key in self.parts:
            raise KeyError(f"{key!r} already reserved")
        if nbytes > self.free:
            raise AdmissionError(f"{key!r} needs {nbytes} bytes; {self.free} of {self.total} free")
        self.parts[key] = int(nbytes)

    def release(self, key):
        self.parts.pop(key)


class FramePool:
    """First-fit allocator over one device region that stages frames.

    Offsets and sizes are in float32 elements.  Free blocks are kept sorted
    and merged with their neighbours on release."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free_blocks = [(0, self.capacity)] if capacity > 0 else []

    def alloc(self, size: int) -> Optional[int]:
        size = max(int(size), 1)
        size = (size + 63) & ~63            # 256-byte granules
        for k, (off, sz) in enumerate(self.free_blocks):
            if sz >= size:
                if sz == size:
                    self.free_blocks.pop(k)
                else:
                    self.free_blocks[k] = (off + size, sz - size)
                return off
        return None

    def release(self, off: int, size: int):
        size = (max(int(size), 1) + 63) & ~63
        fb = self.free_blocks
        lo, hi = 0, len(fb)
        while lo < hi:
            mid = (lo + hi) // 2
            if fb[mid][0] < off:
                lo = mid + 1
            else:
                hi = mid
        fb.insert(lo, (off, size))
        # merge with the right, then the left neighbour
        if lo + 1 < len(fb) and fb[lo][0] + fb[lo][1] == fb[lo + 1][0]:
            fb[lo] = (fb[lo][0], fb[lo][1] + fb[lo + 1][1])
            fb.pop(lo + 1)
        if lo > 0 and fb[lo - 1][0] + fb[lo - 1][1] == fb[lo][0]:
            fb[lo - 1] = (fb[lo - 1][0], fb[lo - 1][1] + fb[lo][1])
            fb.pop(lo)

    @property
    def largest_free(self) -> int:
        return max((s for _, s in self.free_blocks), default=0)

    @property
    def free_total(self) -> int:
        return sum(s for _, s in self.free_blocks)


@dataclasses.dataclass
class Request:
    """One frame of one robot.  xyz: float32 [3, n], either in host memory
    (pinned for overlap; the server stages it on the device) or already in
    device memory (used in place; it must stay unchanged until the frame
    completes)."""
    robot: object
    xyz: torch.Tensor
    pose: np.ndarray
    t_ms: int
    center: tuple
    arrival: float                  # seconds on the server clock
    seq: int = 0
    launch: float = math.nan        # when its batch was enqueued
    done: float = math.nan          # when its batch finished on the device
    batch: int = -1
    lane: int = -1
    batch_items: int = 0

    @property
    def n(self) -> int:
        return int(self.xyz.shape[1])

    @property
    def resident(self) -> bool:
        """True if the points are already in device memory."""
        return bool(self.xyz.is_cuda)

    def pose12(self):
        """The pose as 12 Python floats (row-major 3x4), computed once."""
        p = self.__dict__.get("_pose12")
        if p is None:
            p = [float(v) for v in np.asarray(self.pose, dtype=np.float64).reshape(12)]
            self.__dict__["_pose12"] = p
        return p

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Lane:
    def __init__(self, k: int):
        self.k = k
        self.requests: List[Request] = []
        self.regions: List[tuple] = []
        self.busy = False


class Server:
    """Scheduler and admission over an executor (GpuExecutor or a simulation).

    The executor provides: map_bytes(params), create_map(robot, params, cx, cy,
    t0), drop_map(robot), lanes, pool_floats, lane_bytes, max_items,
    max_batch_points, now(), launch(lane, requests, regions, batch_id),
    done(lane), finish_time(lane)."""

    def __init__(self, executor, budget_bytes: int):
        self.ex = executor
        self.budget = HbmBudget(budget_bytes)
        self.budget.reserve("frame pool", 4 * executor.pool_floats)
        for k in range(executor.lanes):
            self.budget.reserve(("lane", k), executor.lane_bytes)
        self.pool = FramePool(executor.pool_floats)
        self.lanes = [_Lane(k) for k in range(executor.lanes)]
        self.maps: Dict[object, int] = {}
        self.waiting: Dict[object, collections.deque] = {}
        self.ready: set = set()          # robots with a waiting frame
        self.inflight: set = set()
        self.completed: List[Request] = []
        self.batches = 0
        self.batch_sizes: List[int] = []

    # ------------------------------------------------------------ admission
    def add_map(self, robot, params: dict, cx: float = 0.0, cy: float = 0.0, t0_ms: int = 0):
        """Admit a robot's map if its state fits the budget; else AdmissionError."""
        if robot in self.maps:
            raise KeyError(f"robot {robot!r} already has a map")
        nbytes = int(self.ex.map_bytes(params))
        self.budget.reserve(("map", robot), nbytes)
        try:
            self.ex.create_map(robot, params, cx, cy, t0_ms)
        except Exception:
            self.budget.release(("map", robot))
            raise
        self.maps[robot] = nbytes
        self.waiting[robot] = collections.deque()

    def remove_map(self, robot):
        if robot in self.inflight or self.waiting.get(robot):
            raise RuntimeError(f"robot {robot!r} still has frames queued or in flight")
        self.ex.drop_map(robot)
        self.budget.release(("map", robot))
        del self.maps[robot]
        del self.waiting[robot]

    def submit(self, req: Request):
        if req.robot not in self.maps:
            raise AdmissionError(f"robot {req.robot!r} has no admitted map")
        if req.resident and (req.xyz.dtype != torch.float32 or not req.xyz.is_contiguous()):
            raise AdmissionError("a resident frame must be a contiguous float32 [3, n] tensor")
        if req.n > self.ex.max_batch_points or (not req.resident
                                                and 3 * req.n > self.pool.capacity):
            raise AdmissionError(f"frame of {req.n} points exceeds the staging limits")
        self.waiting[req.robot].append(req)
        self.ready.add(req.robot)

    # ----------------------------------------------------------- scheduling
    def pending(self) -> int:
        return sum(len(self.waiting[r]) for r in self.ready)

    def idle(self) -> bool:
        return not self.inflight and self.pending() == 0

    def _retire(self):
        for ln in self.lanes:
            if ln.busy and self.ex.done(ln.k):
                t = self.ex.finish_time(ln.k)
                for r in ln.requests:
                    r.done = t
                    self.inflight.discard(r.robot)
                    self.completed.append(r)
                for off, size in ln.regions:
                    if off >= 0:
                        self.pool.release(off, size)
                ln.requests, ln.regions, ln.busy = [], [], False

    def _form(self) -> List[Request]:
        heads = sorted((self.waiting[robot][0].arrival, self.waiting[robot][0].seq, robot)
                       for robot in self.ready if robot not in self.inflight)
        picked, points = [], 0
        for _, _, robot in heads:
            r = self.waiting[robot][0]
            if len(picked) == self.ex.max_items:
                break
            if points + r.n > self.ex.max_batch_points:
                continue
            picked.append(r)
            points += r.n
        return picked

    def poll(self) -> int:
        """Retire finished batches, then fill every free lane.  Returns the
        number of batches launched."""
        self._retire()
        launched = 0
        for ln in self.lanes:
            if ln.busy:
                continue
            reqs = self._form()
            if not reqs:
                break
            regions, taken = [], []
            for r in reqs:
                if r.resident:                    # no staging: used in place
                    regions.append((-1, 0))
                    taken.append(r)
                    continue
                off = self.pool.alloc(3 * r.n)
                if off is None:
                    continue                      # waits for staging room
                regions.append((off, 3 * r.n))
                taken.append(r)
            if not taken:
                break
            now = self.ex.now()
            for r in taken:
                q = self.waiting[r.robot]
                q.popleft()
                if not q:
                    self.ready.discard(r.robot)
                self.inflight.add(r.robot)
                r.launch = now
                r.batch = self.batches
                r.lane = ln.k
                r.batch_items = len(taken)
            self.ex.launch(ln.k, taken, [o for o, _ in regions], self.batches)
            ln.requests, ln.regions, ln.busy = taken, regions, True
            self.batches += 1
            self.batch_sizes.append(len(taken))
            launched += 1
        return launched


# ---------------------------------------------------------------- GPU side
class GpuExecutor:
    """Device side of the server: resident maps, a staging pool, and one
    stream, batch executor and scratch buffer per lane."""

    # Batches here are mostly small and of ever-changing composition:
    #   - every stage but the march gets one workgroup per work unit, so a
    #     small batch is not folded into rounds;
    #   - launches are direct, not through captured graphs: a capture stalls
    #     the host for milliseconds, and varying batch shapes would keep
    #     capturing new graphs while frames wait.
    DEFAULT_TUNING = {"grid_move": 65536, "grid_chunk": 65536, "grid_tile": 65536,
                      "grid_setup": 65536, "grid_cells": 65536,
                      "graph": 0}

    def __init__(self, largest_params: dict, lanes: int = 2, max_items: int = 64,
                 max_batch_points: int = 4_000_000, pool_points: int = 16_000_000,
                 weights: torch.Tensor = None, tuning: str = None, single_plain: bool = True,
                 wall_rule: bool = False, device=None):
        """single_plain: run a batch of one frame through the plain calls, which
        give the same bits with less launch overhead.  wall_rule: size each
        lane's scratch for maps with the wall/edge rule (per-cell counts of
        every item); without it such maps are not admitted."""
        import json
        from . import PipelineBatch, aligned_empty
        self.device = torch.device(device if device is not None else "cuda")
        self.lanes = int(lanes)
        self.max_items = int(max_items)
        self.max_batch_points = int(max_batch_points)
        self.pool_floats = 3 * int(pool_points)
        self.weights = weights
        self.single_plain = bool(single_plain)
        tune = dict(self.DEFAULT_TUNING)
        if tuning:
            tune.update(json.loads(tuning))
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.lanes)]
        self.execs = [PipelineBatch(json.dumps(tune), device=self.device)
                      for _ in range(self.lanes)]
        self.wall_rule = bool(wall_rule)
        sized = dict(largest_params, wall_min_count=1 if self.wall_rule else 0)
        bound = _emx.batch_scratch_bound(self.execs[0].handle, _emx.make_params(sized),
                                         self.max_items, self.max_batch_points)
        if bound == 0:
            raise AdmissionError(_emx.last_error())
        self.lane_bytes = int(bound)
        for ex in self.execs:
            ex.reserve(bound)
        self.pool = aligned_empty(4 * self.pool_floats, self.device).view(torch.float32)
        self.ends = [torch.cuda.Event(enable_timing=True) for _ in range(self.lanes)]
        self.maps = {}
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_host = None
        self.start_clock()

    def start_clock(self):
        torch.cuda.synchronize(self.device)
        self.t0_event.record(torch.cuda.current_stream(self.device))
        self.t0_event.synchronize()
        self.t0_host = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0_host

    def map_bytes(self, params: dict) -> int:
        return _emx.state_bytes(_emx.make_params(params))

    def create_map(self, robot, params, cx, cy, t0):
        from . import ElevationMap
        if params.get("wall_min_count", 0) and not self.wall_rule:
            raise AdmissionError("maps with the wall/edge rule need an executor built with "
                                 "wall_rule=True (its scratch holds their counts)")
        self.maps[robot] = ElevationMap(params, cx, cy, t0, device=self.device)

    def drop_map(self, robot):
        self.maps.pop(robot).close()

    def launch(self, lane: int, requests, offsets, batch_id):
        if self.single_plain and len(requests) == 1:
            self._launch_plain(lane, requests[0], offsets[0])
            return
        st = self.streams[lane]
        base = self.pool.data_ptr()
        items = (_emx.BatchItem * len(requests))()
        wptr = self.weights.data_ptr() if self.weights is not None else None
        stages = _emx.STAGE_ALL if self.weights is not None else _emx.STAGE_ALL & ~_emx.STAGE_TRAV
        with torch.cuda.stream(st):
            for k, (r, off) in enumerate(zip(requests, offsets)):
                n = r.n
                it = items[k]
                it.map = self.maps[r.robot].handle
                f = it.frame
                if off < 0:                           # resident [3, n] rows
                    b = r.xyz.data_ptr()
                    f.x, f.y, f.z = b, b + 4 * n, b + 8 * n
                else:
                    if n:
                        self.pool[off:off + 3 * n].view(3, n).copy_(r.xyz, non_blocking=True)
                    f.x, f.y, f.z = base + 4 * off, base + 4 * (off + n), base + 4 * (off + 2 * n)
                f.n = n
                f.pose[:] = r.pose12()
                f.t_ms = r.t_ms
                it.cx, it.cy = r.center
                it.d_weights = wptr
                it.stages = stages
            self.execs[lane].run_items(items, len(requests), st.cuda_stream)
            self.ends[lane].record(st)

    def _launch_plain(self, lane: int, r, off: int):
        """One frame through the plain calls on the lane's stream; the lane's
        batch scratch (sized for a whole batch) serves as their scratch."""
        st = self.streams[lane]
        n = r.n
        m = self.maps[r.robot]
        scratch = self.execs[lane].scratch_buffer()
        with torch.cuda.stream(st):
            if off < 0:
                x, y, z = r.xyz[0], r.xyz[1], r.xyz[2]
            else:
                if n:
                    self.pool[off:off + 3 * n].view(3, n).copy_(r.xyz, non_blocking=True)
                x = self.pool[off:off + n]
                y = self.pool[off + n:off + 2 * n]
                z = self.pool[off + 2 * n:off + 3 * n]
            m.move_fuse_points(*r.center, x, y, z, r.pose, r.t_ms, scratch=scratch)
            m.clear_visibility(x, y, z, r.pose, r.t_ms, scratch=scratch)
            if self.weights is not None:
                m.normals_traversability(self.weights)
            else:
                m.compute_normals()
            self.ends[lane].record(st)

    def done(self, lane: int) -> bool:
        return self.ends[lane].query()

    def graph_stats(self):
        """(batches run through the batched call, graphs captured), all lanes."""
        st = [ex.stats() for ex in self.execs]
        return sum(a for a, _ in st), sum(b for _, b in st)

    def finish_time(self, lane: int) -> float:
        return self.t0_event.elapsed_time(self.ends[lane]) / 1e3


def run_trace(server: Server, requests: List[Request], timeout_s: float = 120.0):
    """Feed requests at their arrival times (server clock) until all finish."""
    reqs = sorted(requests, key=lambda r: (r.arrival, r.seq))
    if hasattr(server.ex, "start_clock"):
        server.ex.start_clock()
    i = 0
    t_end = server.ex.now() + timeout_s
    while i < len(reqs) or not server.idle():
        now = server.ex.now()
        while i < len(reqs) and reqs[i].arrival <= now:
            server.submit(reqs[i])
            i += 1
        server.poll()
        if now > t_end:
            raise TimeoutError("trace did not finish")
    return reqs


def run_closed_loop(server: Server, make_request, robots, frames_per_robot: int,
                    timeout_s: float = 120.0) -> List[Request]:
    """Closed-loop clients: every robot submits its first frame at once and
    each later frame as soon as its previous one has completed, so the server
    always has every robot's next frame in hand.  ``make_request(robot, j)``
    returns the robot's j-th frame; its arrival is set to the submission time.
    Returns the requests in submission order."""
    if hasattr(server.ex, "start_clock"):
        server.ex.start_clock()
    nxt = {k: 0 for k in robots}
    out: List[Request] = []

    def submit(k):
        r = make_request(k, nxt[k])
        r.arrival = server.ex.now()
        r.seq = len(out)
        nxt[k] += 1
        server.submit(r)
        out.append(r)

    for k in robots:
        submit(k)
    seen = len(server.completed)
    t_end = server.ex.now() + timeout_s
    while len(out) < frames_per_robot * len(nxt) or not server.idle():
        server.poll()
        while seen < len(server.completed):
            r = server.completed[seen]
            seen += 1
            if nxt[r.robot] < frames_per_robot:
                submit(r.robot)
        if server.ex.now() > t_end:
            raise TimeoutError("closed loop did not finish")
    return out


def _plain_points(r: Request, stage: torch.Tensor):
    """The frame's x, y, z rows on the device: in place if resident, else
    copied into the staging buffer on the current stream."""
    if r.resident:
        return r.xyz[0], r.xyz[1], r.xyz[2]
    n = r.n
    stage[:3 * n].view(3, n).copy_(r.xyz, non_blocking=True)
    return stage[:n], stage[n:2 * n], stage[2 * n:3 * n]


def run_plain_trace(maps: dict, requests: List[Request], weights: torch.Tensor, device=None,
                    max_points: int = 1_000_000):
    """The per-frame baseline: each frame, at its arrival, is copied to the
    device (unless already resident) and run through the plain calls on one
    stream (no batching)."""
    from . import aligned_empty
    device = torch.device(device if device is not None else "cuda")
    reqs = sorted(requests, key=lambda r: (r.arrival, r.seq))
    st = torch.cuda.current_stream(device)
    stage = aligned_empty(12 * max_points, device).view(torch.float32)
    # one scratch buffer serves every map: the calls run in order on one stream
    need = max(_emx.scratch_bytes(m.p, max_points) for m in maps.values())
    scratch = aligned_empty(need, device)
    ends = []
    torch.cuda.synchronize(device)
    t0e = torch.cuda.Event(enable_timing=True)
    t0e.record(st)
    t0e.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            pass
        m = maps[r.robot]
        x, y, z = _plain_points(r, stage)
        r.launch = time.perf_counter() - t0
        m.move_fuse_points(*r.center, x, y, z, r.pose, r.t_ms, scratch=scratch)
        m.clear_visibility(x, y, z, r.pose, r.t_ms, scratch=scratch)
        if weights is not None:
            m.normals_traversability(weights)
        else:
            m.compute_normals()
        e = torch.cuda.Event(enable_timing=True)
        e.record(st)
        ends.append((r, e))
    torch.cuda.synchronize(device)
    for r, e in ends:
        r.done = t0e.elapsed_time(e) / 1e3
    return reqs


def run_plain_closed_loop(maps: dict, make_request, robots, frames_per_robot: int,
                          weights: torch.Tensor, device=None,
                          max_points: int = 1_000_000) -> List[Request]:
    """The per-frame baseline under closed-loop clients: the robots' frames in
    turn, first frames first, each copied to the device and run through the
    plain calls on one stream.  A robot's next frame arrives when its previous
    one completes; on one stream in this order that is always before its turn,
    so the host never waits.  Arrival and completion times are read from
    events recorded on the stream."""
    from . import aligned_empty
    device = torch.device(device if device is not None else "cuda")
    st = torch.cuda.current_stream(device)
    stage = aligned_empty(12 * max_points, device).view(torch.float32)
    need = max(_emx.scratch_bytes(m.p, max_points) for m in maps.values())
    scratch = aligned_empty(need, device)
    torch.cuda.synchronize(device)
    t0e = torch.cuda.Event(enable_timing=True)
    t0e.record(st)
    reqs, ends = [], []
    for j in range(frames_per_robot):
        for k in robots:
            r = make_request(k, j)
            r.seq = len(reqs)
            m = maps[k]
            x, y, z = _plain_points(r, stage)
            m.move_fuse_points(*r.center, x, y, z, r.pose, r.t_ms, scratch=scratch)
            m.clear_visibility(x, y, z, r.pose, r.t_ms, scratch=scratch)
            if weights is not None:
                m.normals_traversability(weights)
            else:
                m.compute_normals()
            e = torch.cuda.Event(enable_timing=True)
            e.record(st)
            reqs.append(r)
            ends.append(e)
    torch.cuda.synchronize(device)
    last = {}
    for r, e in zip(reqs, ends):
        r.done = t0e.elapsed_time(e) / 1e3
        r.arrival = last.get(r.robot, 0.0)
        r.launch = r.arrival
        last[r.robot] = r.done
    return reqs


def latency_summary(reqs: List[Request]) -> dict:
    """Latency (completion - arrival) percentiles and throughput; the wait
    (launch - arrival) and device (completion - launch) parts as means."""
    lat = np.array([r.latency for r in reqs]) * 1e3
    wait = np.array([r.launch - r.arrival for r in reqs]) * 1e3
    pts = sum(r.n for r in reqs)
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return dict(frames=len(reqs), points=int(pts), span_s=float(span),
                points_per_s=float(pts / span) if span > 0 else math.nan,
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                max_ms=float(lat.max()), mean_ms=float(lat.mean()),
                mean_wait_ms=float(wait.mean()), mean_run_ms=float((lat - wait).mean()))
