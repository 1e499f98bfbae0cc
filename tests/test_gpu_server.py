"""The continuous-batching server on the GPU: every robot's map after a mixed,
overlapping trace equals, bit for bit, the map that the same frames give when
run alone through the plain per-frame calls.  The per-frame baseline loop is
checked the same way."""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

F32 = np.float32

SHAPES = [(64, 48, 0.05), (130, 97, 0.04), (200, 180, 0.03), (33, 200, 0.1), (96, 96, 0.02),
          (150, 150, 0.05)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_12876_amd import _emx
    _emx.lib()
    return torch.device("cuda:0")


def _params(nx, ny, r):
    return dict(nx=nx, ny=ny, resolution=r, noise_alpha=1e-3, gate_k=3.0, min_range=0.01,
                ray_step=r, clear_min_age_ms=100, clear_normal_alpha=0.2)


def _trace(seed, frames_per_robot=4, span_s=0.02):
    from paper_2204_12876_amd.server import Request
    rng = np.random.default_rng(seed)
    reqs, seq = [], 0
    for k, (nx, ny, r) in enumerate(SHAPES):
        cx = cy = 0.0
        for f in range(frames_per_robot):
            n = int(rng.integers(3000, 60000))
            ex, ey = 0.6 * nx * r, 0.6 * ny * r
            xs = rng.uniform(-ex, ex, n)
            ys = rng.uniform(-ey, ey, n)
            zs = 0.1 * np.sin(3 * xs) - 0.8 + 0.01 * rng.normal(size=n)
            zs[::13] += 0.4
            xyz = torch.from_numpy(np.stack([xs, ys, zs]).astype(F32)).pin_memory()
            cx += float(rng.integers(-4, 5)) * r
            cy += float(rng.integers(-4, 5)) * r
            yaw = float(rng.uniform(0, 2 * math.pi))
            P = np.zeros((3, 4))
            P[:, :3] = [[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0],
                        [0, 0, 1]]
            P[:, 3] = (cx, cy, 0.3)
            reqs.append(Request(robot=k, xyz=xyz, pose=P, t_ms=200 * (f + 1), center=(cx, cy),
                                arrival=float(rng.uniform(0, span_s)), seq=seq))
            seq += 1
    # per robot, frames arrive in order; every robot's first frame at time 0,
    # so that the first batches hold several frames whatever the device speed
    for k in range(len(SHAPES)):
        mine = sorted((r for r in reqs if r.robot == k), key=lambda r: r.t_ms)
        times = sorted(r.arrival for r in mine)
        times[0] = 0.0
        for r, t in zip(mine, times):
            r.arrival = t
    return reqs


def _alone(reqs, robot, w, dev):
    from paper_2204_12876_amd import ElevationMap
    m = ElevationMap(_params(*SHAPES[robot]), device=dev)
    for r in sorted((r for r in reqs if r.robot == robot), key=lambda r: r.t_ms):
        x, y, z = (r.xyz[i].to(dev) for i in range(3))
        m.move_map(*r.center)
        m.fuse_points(x, y, z, r.pose, r.t_ms)
        m.clear_visibility(x, y, z, r.pose, r.t_ms)
        m.compute_normals()
        m.traversability(w)
    torch.cuda.synchronize()
    return m


def _same_map(a, b, tag):
    assert a.info() == b.info(), tag
    sa, sb = a.export_state().cpu().numpy(), b.export_state().cpu().numpy()
    assert np.array_equal(sa, sb), f"{tag}: {(sa != sb).sum()} bytes differ"


def test_server_results_equal_alone_results(dev):
    from paper_2204_12876_amd.server import GpuExecutor, Server, latency_summary, run_trace
    print("[case] server mix vs alone", flush=True)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    reqs = _trace(5)
    largest = _params(200, 200, 0.03)
    ex = GpuExecutor(largest, lanes=2, max_items=3, max_batch_points=150_000,
                     pool_points=300_000, weights=w, device=dev)
    srv = Server(ex, budget_bytes=4 << 30)
    for k, s in enumerate(SHAPES):
        srv.add_map(k, _params(*s))
    run_trace(srv, reqs, timeout_s=60)
    torch.cuda.synchronize()
    assert len(srv.completed) == len(reqs)
    print("batches", srv.batches, "sizes", srv.batch_sizes, latency_summary(reqs), flush=True)
    assert max(srv.batch_sizes) > 1
    for k in range(len(SHAPES)):
        _same_map(ex.maps[k], _alone(reqs, k, w, dev), f"robot {k}")


def test_plain_trace_results_equal_alone_results(dev):
    from paper_2204_12876_amd import ElevationMap
    from paper_2204_12876_amd.server import run_plain_trace
    print("[case] plain trace vs alone", flush=True)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    reqs = _trace(6, frames_per_robot=3)
    maps = {k: ElevationMap(_params(*s), device=dev) for k, s in enumerate(SHAPES)}
    run_plain_trace(maps, reqs, w, device=dev, max_points=60000)
    for k in range(len(SHAPES)):
        _same_map(maps[k], _alone(reqs, k, w, dev), f"robot {k}")


def test_server_admission_budget(dev):
    from paper_2204_12876_amd.server import AdmissionError, GpuExecutor, Server
    print("[case] server admission", flush=True)
    largest = _params(200, 200, 0.03)
    ex = GpuExecutor(largest, lanes=2, max_items=4, max_batch_points=100_000,
                     pool_points=100_000, device=dev)
    fixed = 12 * 100_000 + 2 * ex.lane_bytes
    one = ex.map_bytes(largest)
    srv = Server(ex, budget_bytes=fixed + 2 * one + one // 2)
    srv.add_map(0, largest)
    srv.add_map(1, largest)
    with pytest.raises(AdmissionError):
        srv.add_map(2, largest)
    srv.remove_map(0)
    srv.add_map(2, largest)
    assert srv.budget.used <= srv.budget.total
