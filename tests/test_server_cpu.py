"""Server scheduling and admission on the CPU, with a simulated executor and a
virtual clock (no GPU): budget admission, the staging pool, per-map FIFO with
one frame in flight, batch limits, and continuous batching under load."""
import numpy as np
import pytest
import torch

from paper_2204_12876_amd.server import AdmissionError, FramePool, HbmBudget, Request, Server


class SimExecutor:
    """Device stand-in: a batch takes a + b * points seconds on its lane."""

    def __init__(self, lanes=2, max_items=8, max_batch_points=100_000, pool_points=150_000,
                 a=2e-4, b=1e-9):
        self.lanes = lanes
        self.max_items = max_items
        self.max_batch_points = max_batch_points
        self.pool_floats = 3 * pool_points
        self.lane_bytes = 1 << 20
        self.a, self.b = a, b
        self.t = 0.0
        self.finish = [None] * lanes
        self.maps = {}
        self.inflight = {}             # robot -> lane
        self.regions = {}              # lane -> [(off, size)]
        self.last_seq = {}
        self.log = []

    def map_bytes(self, params):
        return params["nx"] * params["ny"] * 64

    def create_map(self, robot, params, cx, cy, t0):
        self.maps[robot] = params

    def drop_map(self, robot):
        del self.maps[robot]

    def now(self):
        return self.t

    def launch(self, lane, reqs, offsets, batch_id):
        assert self.finish[lane] is None, "lane launched while busy"
        assert 1 <= len(reqs) <= self.max_items
        assert sum(r.n for r in reqs) <= self.max_batch_points
        regs = [(o, 3 * r.n) for o, r in zip(offsets, reqs)]
        live = [g for gs in self.regions.values() for g in gs] + regs
        live.sort()
        for (o1, s1), (o2, _) in zip(live, live[1:]):
            assert o1 + s1 <= o2, "staging regions overlap"
        assert all(o + s <= self.pool_floats for o, s in live)
        for r in reqs:
            assert r.robot not in self.inflight, "a map has two frames in flight"
            assert r.seq > self.last_seq.get(r.robot, -1), "per-map order broken"
            assert r.arrival <= self.t
            self.inflight[r.robot] = lane
            self.last_seq[r.robot] = r.seq
        self.regions[lane] = regs
        self.finish[lane] = self.t + self.a + self.b * sum(r.n for r in reqs)
        self.log.append((batch_id, lane, len(reqs)))

    def done(self, lane):
        return self.finish[lane] is not None and self.finish[lane] <= self.t

    def finish_time(self, lane):
        f = self.finish[lane]
        self.finish[lane] = None
        for r, ln in list(self.inflight.items()):
            if ln == lane:
                del self.inflight[r]
        self.regions.pop(lane, None)
        return f


def _req(robot, seq, n, arrival):
    return Request(robot=robot, xyz=torch.zeros(3, n), pose=np.eye(3, 4), t_ms=seq,
                   center=(0.0, 0.0), arrival=arrival, seq=seq)


def _simulate(server, ex, reqs, horizon=100.0):
    """Event-driven driver: jump the clock to the next arrival or finish."""
    reqs = sorted(reqs, key=lambda r: (r.arrival, r.seq))
    i = 0
    while i < len(reqs) or not server.idle():
        while i < len(reqs) and reqs[i].arrival <= ex.t:
            server.submit(reqs[i])
            i += 1
        server.poll()
        nxt = [f for f in ex.finish if f is not None]
        if i < len(reqs):
            nxt.append(reqs[i].arrival)
        if not nxt:
            assert server.idle()
            break
        ex.t = max(ex.t, min(nxt))
        assert ex.t < horizon
    return reqs


def _poisson(rng, robots, rate_hz, seconds, sizes):
    out = []
    for k in robots:
        t, s = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t > seconds:
                break
            out.append(_req(k, s, int(sizes[k]), t))
            s += 1
    return out


def test_frame_pool_against_occupancy_map():
    rng = np.random.default_rng(0)
    cap = 64 * 500
    pool = FramePool(cap)
    used = np.zeros(cap, bool)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off, size = live.pop(int(rng.integers(len(live))))
            pool.release(off, size)
            g = (size + 63) & ~63
            assert used[off:off + g].all()
            used[off:off + g] = False
        else:
            size = int(rng.integers(1, 3000))
            off = pool.alloc(size)
            g = (size + 63) & ~63
            if off is None:
                # first fit fails only if no free block can hold g floats
                assert pool.largest_free < g
                continue
            assert off % 64 == 0 and not used[off:off + g].any()
            used[off:off + g] = True
            live.append((off, size))
        assert pool.free_total == cap - used.sum()
    for off, size in live:
        pool.release(off, size)
    assert pool.free_blocks == [(0, cap)]


def test_budget_admits_maps_until_full_and_after_removal():
    ex = SimExecutor()
    budget = 4 * ex.pool_floats + 2 * ex.lane_bytes + 3 * 100 * 100 * 64
    srv = Server(ex, budget)
    for k in range(3):
        srv.add_map(k, dict(nx=100, ny=100))
    with pytest.raises(AdmissionError):
        srv.add_map(3, dict(nx=100, ny=100))
    assert 3 not in ex.maps
    srv.remove_map(0)
    srv.add_map(3, dict(nx=100, ny=100))
    assert sorted(srv.maps) == [1, 2, 3]
    with pytest.raises(AdmissionError):
        srv.submit(_req(0, 0, 10, 0.0))            # robot 0 was removed
    with pytest.raises(AdmissionError):
        srv.submit(_req(1, 0, 200_000, 0.0))       # larger than a batch may hold
    assert HbmBudget(10).free == 10


def test_poisson_trace_invariants_and_continuous_batching():
    rng = np.random.default_rng(1)
    ex = SimExecutor(lanes=2, max_items=8, max_batch_points=100_000, pool_points=150_000,
                     a=3e-4, b=4e-9)
    srv = Server(ex, 1 << 40)
    robots = list(range(24))
    sizes = rng.integers(2_000, 30_000, len(robots))
    for k in robots:
        srv.add_map(k, dict(nx=64, ny=64))
    reqs = _simulate(srv, ex, _poisson(rng, robots, 40.0, 2.0, sizes))
    assert len(srv.completed) == len(reqs) > 1000
    assert all(r.done >= r.launch >= r.arrival for r in reqs)
    # per-map completion in submission order
    for k in robots:
        mine = [r for r in srv.completed if r.robot == k]
        assert [r.seq for r in mine] == sorted(r.seq for r in mine)
        assert all(a.done <= b.launch for a, b in zip(mine, mine[1:]))
    # batches formed under load, both lanes used, the limits respected
    assert max(srv.batch_sizes) > 1 and max(srv.batch_sizes) <= ex.max_items
    assert {lane for _, lane, _ in ex.log} == {0, 1}
    assert srv.pool.free_blocks == [(0, srv.pool.capacity)]


def test_staging_pressure_delays_but_never_drops():
    rng = np.random.default_rng(2)
    ex = SimExecutor(lanes=3, max_items=4, max_batch_points=60_000, pool_points=40_000)
    srv = Server(ex, 1 << 40)
    for k in range(10):
        srv.add_map(k, dict(nx=32, ny=32))
    reqs = [_req(k % 10, k // 10, int(rng.integers(5_000, 39_000)), 0.001 * (k // 10))
            for k in range(200)]
    _simulate(srv, ex, reqs)
    assert len(srv.completed) == 200
    assert srv.pool.free_blocks == [(0, srv.pool.capacity)]


def test_oldest_frames_go_first():
    ex = SimExecutor(lanes=1, max_items=2, max_batch_points=10_000, a=1.0, b=0.0)
    srv = Server(ex, 1 << 40)
    for k in range(4):
        srv.add_map(k, dict(nx=8, ny=8))
    # robot 3's frame is the oldest; robot 0 submits two frames
    reqs = [_req(3, 0, 100, 0.0), _req(0, 0, 100, 0.1), _req(0, 1, 100, 0.2),
            _req(1, 0, 100, 0.3), _req(2, 0, 100, 0.4)]
    ex.t = 0.5
    for r in reqs:
        srv.submit(r)
    srv.poll()
    first = sorted(r.robot for r in srv.lanes[0].requests)
    assert first == [0, 3]
    ex.t = 1.5
    srv.poll()
    second = sorted(r.robot for r in srv.lanes[0].requests)
    assert second == [0, 1]           # robot 0's second frame, then the next oldest


class _AutoClock(SimExecutor):
    """The simulated clock jumps to the next batch end whenever it is read."""

    def now(self):
        nxt = [f for f in self.finish if f is not None]
        if nxt:
            self.t = max(self.t, min(nxt))
        return self.t


def test_closed_loop_clients_resubmit_on_completion():
    from paper_2204_12876_amd.server import run_closed_loop
    ex = _AutoClock(lanes=2, max_items=8, max_batch_points=100_000, pool_points=150_000,
                    a=3e-4, b=4e-9)
    srv = Server(ex, 1 << 40)
    robots = list(range(12))
    for k in robots:
        srv.add_map(k, dict(nx=32, ny=32))
    reqs = run_closed_loop(srv, lambda k, j: _req(k, j, 1000 + 100 * k, 0.0), robots, 5)
    assert len(reqs) == len(srv.completed) == 60
    for k in robots:
        mine = [r for r in reqs if r.robot == k]
        assert [r.t_ms for r in mine] == list(range(5))
        # each later frame is submitted only once the previous one has completed
        assert all(b.arrival >= a.done for a, b in zip(mine, mine[1:]))
    assert all(r.done >= r.launch >= r.arrival for r in reqs)
    assert max(srv.batch_sizes) > 1
