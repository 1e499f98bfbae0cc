"""Batched executor (emx_pipeline_batch) on the GPU.

Every map of a batch must end bit for bit where the plain calls (checked
against the oracle in test_gpu_parity) take it, whatever the batch holds, the
launch geometry, or whether a captured graph or direct launches run it.
Graphs are replayed over several frames, with the plain calls and host
synchronisation between replays, and every replay is checked.
"""
import json
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from parity_util import assert_fuse_parity, assert_normals_parity, load_state, random_state

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_12876_amd import _emx
    _emx.lib()
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def _pose(t, yaw=0.0):
    P = np.zeros((3, 4))
    c, s = math.cos(yaw), math.sin(yaw)
    P[:, :3] = [[c, -s, 0], [s, c, 0], [0, 0, 1]]
    P[:, 3] = t
    return P


# maps of uneven shape and resolution; (nx, ny, r, points per frame)
SHAPES = [(64, 48, 0.05, 30000), (130, 97, 0.04, 2049), (33, 200, 0.1, 0),
          (257, 256, 0.03, 100000), (5, 3, 0.5, 1), (96, 96, 0.02, 2047)]


class Robot:
    """A map driven twice: once by the plain calls, once inside batches."""

    def __init__(self, k, shape, dev, seed, extra=None):
        from paper_2204_12876_amd import ElevationMap
        nx, ny, r, n = shape
        self.params = dict(nx=nx, ny=ny, resolution=r, noise_alpha=1e-3, gate_k=3.0,
                           min_range=0.01, ray_step=r, clear_min_age_ms=300,
                           clear_normal_alpha=0.2, **(extra or {}))
        self.p = O.Params.from_dict(self.params)
        self.n = n
        self.rng = np.random.default_rng(seed)
        st = random_state(self.p, self.rng, valid_frac=0.8)
        st.h[:] = (0.3 * st.h - 0.9).astype(F32)
        self.plain = ElevationMap(self.params, 0.0, 0.0, 0, device=dev)
        self.batch = ElevationMap(self.params, 0.0, 0.0, 0, device=dev)
        load_state(self.plain, st)
        load_state(self.batch, st)
        self.dev = dev
        self.k = k
        self.cx = self.cy = 0.0

    def frame(self, it):
        n, r = self.n, self.p.resolution
        ext_x, ext_y = 0.55 * self.p.nx * r, 0.55 * self.p.ny * r
        xs = self.rng.uniform(-ext_x, ext_x, n).astype(F32)
        ys = self.rng.uniform(-ext_y, ext_y, n).astype(F32)
        zs = (0.15 * np.sin(2 * xs) - 1.0 + 0.02 * self.rng.normal(size=n)).astype(F32)
        zs[::17] += F32(0.5)                      # points above the ground: rays clear
        if n > 10:
            xs[3] = np.nan
        self.cx += float(self.rng.integers(-3, 4)) * r
        self.cy += float(self.rng.integers(-3, 4)) * r
        pose = _pose((self.cx, self.cy, 0.2 + 0.1 * it), yaw=float(self.rng.uniform(0, 6.28)))
        xyz = tuple(torch.from_numpy(a).to(self.dev) for a in (xs, ys, zs))
        return xyz, pose, 1000 + 100 * it

    def outputs(self):
        n = max(self.n, 1)
        C = self.p.nx * self.p.ny
        return (torch.full((n,), -7, dtype=torch.int32, device=self.dev),
                torch.full((n,), 7, dtype=torch.uint8, device=self.dev),
                torch.full((C,), 9, dtype=torch.uint8, device=self.dev))


def _plain(m, xyz, pose, t, center, w, stages, outs):
    from paper_2204_12876_amd import _emx
    cell, acc, clr = outs
    if stages & _emx.STAGE_MOVE:
        m.move_map(*center)
    if stages & _emx.STAGE_FUSE:
        m.fuse_points(*xyz, pose, t, out_cell=cell, out_accept=acc)
    if stages & _emx.STAGE_CLEAR:
        m.clear_visibility(*xyz, pose, t, out_cleared=clr)
    if stages & _emx.STAGE_NORMALS:
        m.compute_normals()
    if stages & _emx.STAGE_TRAV:
        m.traversability(w)


def _same(a, b, what):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    if not np.array_equal(a.view(np.uint8), b.view(np.uint8)):
        bad = np.nonzero(a.view(np.uint8) != b.view(np.uint8))[0]
        raise AssertionError(f"{what}: {bad.size} bytes differ, first at {bad[:8]}")


def _drive(robots, pb, w, frames, stages_of=None):
    """Run ``frames`` frames through plain calls and batches; compare all."""
    from paper_2204_12876_amd import BatchEntry, _emx
    for it in range(frames):
        entries, checks = [], []
        for rb in robots:
            st = _emx.STAGE_ALL if stages_of is None else stages_of(rb.k, it)
            xyz, pose, t = rb.frame(it)
            op, ob = rb.outputs(), rb.outputs()
            _plain(rb.plain, xyz, pose, t, (rb.cx, rb.cy), w, st, op)
            entries.append(BatchEntry(rb.batch, *xyz, pose=pose, t_ms=t, center=(rb.cx, rb.cy),
                                      weights=w, stages=st, out_cell=ob[0], out_accept=ob[1],
                                      out_cleared=ob[2]))
            checks.append((rb, op, ob, st, xyz))
        pb.run(entries)
        torch.cuda.synchronize()
        for rb, op, ob, st, xyz in checks:
            tag = f"frame {it} map {rb.k} ({rb.p.nx}x{rb.p.ny}, n={rb.n}, stages={st})"
            assert rb.plain.info() == rb.batch.info(), tag
            _same(rb.plain.export_state(), rb.batch.export_state(), tag + " state")
            if rb.params.get("upper_bound"):
                _same(rb.plain.upper_bound(), rb.batch.upper_bound(), tag + " upper bound")
            if st & _emx.STAGE_FUSE:
                _same(op[0], ob[0], tag + " out_cell")
                _same(op[1], ob[1], tag + " out_accept")
            if st & _emx.STAGE_CLEAR:
                _same(op[2], ob[2], tag + " out_cleared")
        del entries


def _robots(dev, shapes=SHAPES, seed=0):
    return [Robot(k, s, dev, 1000 * seed + k) for k, s in enumerate(shapes)]


# every fusion extension and the upper bound layer, alone and together,
# next to maps without them
EXTRAS = [
    {},
    dict(wall_min_count=2),
    dict(time_variance=0.003, upper_bound=1),      # this map's frames are empty
    dict(upper_bound=1),
    dict(excl_on=1, excl_theta=0.4, excl_b=0.3, excl_c=0.5, excl_d=0.9, outlier_variance=0.01),
    dict(time_variance=0.001, wall_min_count=3, upper_bound=1, excl_on=1, excl_theta=0.6,
         excl_b=0.2, excl_c=1.0, excl_d=0.7, outlier_variance=0.02),
]


def test_batch_with_every_extension(dev):
    from paper_2204_12876_amd import PipelineBatch
    _say("batch with every fusion extension")
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    robots = [Robot(k, s, dev, 7000 + k, extra=e) for k, (s, e) in enumerate(zip(SHAPES, EXTRAS))]
    assert robots[2].n == 0
    for graph in (1, 0):
        pb = PipelineBatch(json.dumps({"graph": graph}), device=dev)
        _drive(robots, pb, w, 4)
        pb.close()


def test_batch_equals_plain_calls_with_graph_replays(dev):
    """Six uneven maps, five frames: the captured graphs are replayed (two
    alternating host tables) and every replay is compared with the plain calls."""
    from paper_2204_12876_amd import PipelineBatch
    _say("batch vs plain, graph, 5 frames")
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    pb = PipelineBatch(device=dev)
    robots = _robots(dev)
    _drive(robots, pb, w, frames=5)
    pb.close()


@pytest.mark.parametrize("tuning", [
    '{"graph": 0}',
    # every key at an odd small value; unknown keys are ignored
    '{"grid_move": 1, "grid_chunk": 3, "grid_tile": 5, "grid_setup": 7, "grid_march": 9, '
    '"grid_cells": 1, "seg": 7, "no_such_key": 2}',
    '{"grid_chunk": 4096, "grid_tile": 4096, "grid_march": 8192, "seg": 128, "graph": 1}',
])
def test_batch_tuning_does_not_change_results(dev, tuning):
    from paper_2204_12876_amd import PipelineBatch
    _say("batch tuning", tuning)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    pb = PipelineBatch(tuning, device=dev)
    robots = _robots(dev, seed=1)
    _drive(robots, pb, w, frames=2)
    pb.close()


def test_batch_mixed_stages_and_wide_keys(dev):
    """Items with different stage sets in one batch, and a map wide enough for
    64-bit sort keys next to small ones."""
    from paper_2204_12876_amd import PipelineBatch, _emx
    _say("batch mixed stages + wide keys")
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    pb = PipelineBatch(device=dev)
    shapes = [(2080, 2100, 0.02, 60000), (64, 64, 0.05, 5000), (40, 70, 0.05, 3000),
              (128, 128, 0.04, 20000)]
    robots = _robots(dev, shapes, seed=2)
    sets = [_emx.STAGE_ALL, _emx.STAGE_FUSE, _emx.STAGE_NORMALS | _emx.STAGE_TRAV,
            _emx.STAGE_MOVE | _emx.STAGE_CLEAR]
    _drive(robots, pb, w, frames=2, stages_of=lambda k, it: sets[(k + it) % 4])
    pb.close()


def test_batch_item_matches_oracle(dev):
    """A batch of the 128x128 workload (fusion only) and a normals-only map,
    checked against the oracle directly."""
    from paper_2204_12876_amd import BatchEntry, ElevationMap, PipelineBatch, _emx
    _say("batch vs oracle")
    d = synth.cfg0(n_frames=1)
    p = O.Params.from_dict(d["params"])
    f = d["frames"][0]
    m = ElevationMap(d["params"], device=dev)
    st = O.init_map(p, 0.0, 0.0, 0)
    params2 = dict(nx=50, ny=41, resolution=0.05)
    p2 = O.Params.from_dict(params2)
    m2 = ElevationMap(params2, device=dev)
    st2 = random_state(p2, np.random.default_rng(77), valid_frac=0.95)
    load_state(m2, st2)
    xyz = tuple(t.to(dev).contiguous() for t in (f.x, f.y, f.z))
    cell = torch.full((f.n,), -7, dtype=torch.int32, device=dev)
    acc = torch.full((f.n,), 7, dtype=torch.uint8, device=dev)
    pb = PipelineBatch(device=dev)
    pb.run([BatchEntry(m, *xyz, pose=f.pose, t_ms=f.t_ms, stages=_emx.STAGE_FUSE,
                       out_cell=cell, out_accept=acc),
            BatchEntry(m2, stages=_emx.STAGE_NORMALS)])
    torch.cuda.synchronize()
    r = O.fuse(p, st, *f.numpy(), f.pose, f.t_ms)
    g = m.state_numpy()
    assert_fuse_parity(r, st, g, cell.cpu().numpy(), acc.cpu().numpy(), f.t_ms)
    assert_normals_parity(m2.state_numpy(), O.compute_normals(p2, st2.h, st2.valid))
    pb.close()
    m.close()
    m2.close()


def test_batch_rejects_bad_batches_without_touching_maps(dev):
    from paper_2204_12876_amd import BatchEntry, EmxError, ElevationMap, PipelineBatch, _emx
    _say("batch errors")
    params = dict(nx=32, ny=32, resolution=0.1)
    a = ElevationMap(params, device=dev)
    b = ElevationMap(params, device=dev)
    x = torch.zeros(100, device=dev)
    pose = _pose((0.0, 0.0, 1.0))
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    pb = PipelineBatch(device=dev)
    before = [a.export_state().cpu().numpy(), b.export_state().cpu().numpy(), a.info(), b.info()]

    def rejected(entries, status=_emx.EMX_EINVAL):
        with pytest.raises(EmxError) as e:
            pb.run(entries)
        assert e.value.status == status
        torch.cuda.synchronize()
        now = [a.export_state().cpu().numpy(), b.export_state().cpu().numpy(), a.info(), b.info()]
        assert np.array_equal(now[0], before[0]) and np.array_equal(now[1], before[1])
        assert now[2:] == before[2:]

    # the same map twice
    rejected([BatchEntry(a, x, x, x, pose, 10, center=(0.5, 0.5), weights=w),
              BatchEntry(a, x, x, x, pose, 10, stages=_emx.STAGE_FUSE)])
    # a valid move on a, then a frame older than b's start time
    rejected([BatchEntry(a, x, x, x, pose, 10, center=(0.5, 0.5), weights=w),
              BatchEntry(b, x, x, x, pose, -5, stages=_emx.STAGE_FUSE)])
    # a centre too far away to be a cell index
    rejected([BatchEntry(b, center=(1e30, 0.0), stages=_emx.STAGE_MOVE)])
    # traversability without weights
    rejected([BatchEntry(b, stages=_emx.STAGE_TRAV)])
    # a non-finite pose
    rejected([BatchEntry(a, x, x, x, np.full((3, 4), np.nan), 10, stages=_emx.STAGE_FUSE)])
    # scratch too small, through the C call
    items = _emx.make_batch_items([BatchEntry(a, x, x, x, pose, 10,
                                              stages=_emx.STAGE_FUSE).item()])
    from paper_2204_12876_amd import aligned_empty
    small = aligned_empty(4096, dev)
    with pytest.raises(EmxError) as e:
        _emx.pipeline_batch(pb.handle, items, 1, small.data_ptr(), 4096, 0)
    assert e.value.status == _emx.EMX_ENOMEM
    # more than the maximum number of items
    maps = [ElevationMap(dict(nx=4, ny=4, resolution=1.0), device=dev)
            for _ in range(_emx.BATCH_MAX_ITEMS + 1)]
    with pytest.raises(EmxError):
        pb.run([BatchEntry(mm, stages=_emx.STAGE_NORMALS) for mm in maps])
    # bad tuning
    with pytest.raises(EmxError):
        PipelineBatch('{"grid_tile": 0}', device=dev)
    with pytest.raises(EmxError):
        PipelineBatch('{"seg": 1000}', device=dev)
    # after all that, a good batch still runs and matches the plain calls
    c = ElevationMap(params, device=dev)
    for mm in (a, c):
        mm.move_map(0.35, -0.25)
        mm.fuse_points(x + 0.3, x - 0.2, x - 1.0, pose, 20)
    pb.run([BatchEntry(b, center=(0.35, -0.25), x=x + 0.3, y=x - 0.2, z=x - 1.0, pose=pose,
                       t_ms=20, stages=_emx.STAGE_MOVE | _emx.STAGE_FUSE)])
    torch.cuda.synchronize()
    _same(c.export_state(), b.export_state(), "after errors")
    for mm in [a, b, c] + maps:
        mm.close()
    pb.close()


def test_batch_stats_count_graph_captures(dev):
    """A repeated batch shape replays its cached graph; a new shape captures."""
    from paper_2204_12876_amd import BatchEntry, ElevationMap, PipelineBatch
    _say("batch stats")
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    pb = PipelineBatch('{"graph": 1}', device=dev)
    m = ElevationMap(dict(nx=64, ny=64, resolution=0.05), device=dev)
    x = torch.zeros(3000, device=dev)
    pose = _pose((0.0, 0.0, 1.0))
    for k in range(3):
        pb.run([BatchEntry(m, x + 0.01 * k, x, x - 1.0, pose, 100 * (k + 1), center=(0.0, 0.0),
                           weights=w)])
    torch.cuda.synchronize()
    assert pb.stats() == (3, 1)
    y = torch.zeros(300000, device=dev)  # many more chunks: other grid sizes
    pb.run([BatchEntry(m, y, y, y - 1.0, pose, 400, center=(0.0, 0.0), weights=w)])
    torch.cuda.synchronize()
    assert pb.stats() == (4, 2)
    pb.close()
    m.close()


def test_batch_scratch_bound_covers_every_batch(dev):
    from paper_2204_12876_amd import BatchEntry, ElevationMap, PipelineBatch, _emx
    _say("batch scratch bound")
    rng = np.random.default_rng(21)
    largest = dict(nx=300, ny=280, resolution=0.05)
    maps = [ElevationMap(dict(nx=int(rng.integers(3, 301)), ny=int(rng.integers(3, 281)),
                              resolution=0.05), device=dev) for _ in range(20)]
    x = torch.zeros(200000, device=dev)
    pose = _pose((0.0, 0.0, 1.0))
    for seg in (16, 32, 128):
        pb = PipelineBatch(json.dumps({"seg": seg}), device=dev)
        bound = pb.scratch_bound(largest, 20, 200000)
        for trial in range(5):
            n = int(rng.integers(1, 21))
            sizes = rng.multinomial(200000, np.ones(n) / n)
            entries = [BatchEntry(maps[i], x[:s], x[:s], x[:s], pose, 10,
                                  stages=int(rng.integers(0, 32)) | _emx.STAGE_FUSE,
                                  center=(0.0, 0.0), weights=torch.zeros(89, device=dev))
                       for i, s in enumerate(sizes)]
            arr = _emx.make_batch_items([e.item() for e in entries])
            need = _emx.batch_scratch_bytes(pb.handle, arr, n)
            assert 0 < need <= bound, (seg, n, need, bound)
        pb.close()
    for m in maps:
        m.close()


def test_kernel_timing_reports_each_kernel(dev):
    from paper_2204_12876_amd import ElevationMap, _emx
    _say("kernel timing")
    d = synth.cfg0(n_frames=2)
    m = ElevationMap(d["params"], device=dev)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    f0, f1 = d["frames"]
    xyz0 = tuple(t.to(dev).contiguous() for t in (f0.x, f0.y, f0.z))
    xyz1 = tuple(t.to(dev).contiguous() for t in (f1.x, f1.y, f1.z))
    m.fuse_points(*xyz0, f0.pose, 0)
    m.compute_normals()
    torch.cuda.synchronize()
    _emx.timing_begin()
    m.move_map(0.5, 0.0)
    m.fuse_points(*xyz1, f1.pose, 1000)
    m.clear_visibility(*xyz1, f1.pose, 1000)
    m.compute_normals()
    m.traversability(w)
    rep = _emx.timing_end()
    for k in ("k_move", "k_fuse_chunk", "k_fuse_tile", "k_clear_setup", "k_clear_march",
              "k_normals", "k_trav"):
        assert k in rep and rep[k][0] == 1 and rep[k][1] > 0.0, (k, rep)
    m.compute_normals()               # not timed once ended
    assert _emx.timing_end() == {}
    m.close()
