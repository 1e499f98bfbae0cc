"""Parity at the workloads' full sizes, in the launch configurations the
benchmark uses.

  * Stress workload: one 2000x2000 map at 0.02 m, two 4M-point frames from a
    128-beam LiDAR.  Fusion is compared with the oracle on every point and
    cell (the second frame is gated against the first).  Clearing runs on a
    seeded sample of the frame's rays over the full map, since the oracle
    cannot march four million 30 m rays in seconds.  Normals and
    traversability cover all four million cells.
  * 16 maps of uneven size in one batched call with the tuned geometry: each
    map against the oracle (fusion on every point, twice; normals and
    traversability; clearing on sampled rays).
  * The stress mix: the 2000x2000 map with a 4M-point frame and eight 400x400
    maps with 300k-point frames in one batched call, each map against the
    oracle in the same way.
  * 64 robots through the continuous-batching server: every map after a
    compressed trace equals, bit for bit, the map its frames give alone.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
import synth
from parity_util import (assert_fuse_parity, assert_normals_parity, assert_trav_parity,
                         load_state, state_from_gpu)

pytestmark = pytest.mark.gpu

F32 = np.float32
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_12876_amd import _emx
    _emx.lib()
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def _tuning():
    path = os.path.join(ROOT, "paper_2204_12876_amd", "tuning_mi355x.json")
    if os.path.exists(path):
        with open(path) as fh:
            return json.dumps(json.load(fh)["tuning"])
    return None


def _sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(k, n), replace=False))


def _check_clear_sampled(m, p, xs, ys, zs, pose, t_ms, dev, k=20000, seed=0):
    """Clearing from a seeded sample of the frame's rays, against the oracle."""
    idx = _sample(xs.size, k, seed)
    sx, sy, sz = (np.ascontiguousarray(a[idx]) for a in (xs, ys, zs))
    st, _ = state_from_gpu(m, *m.info())
    out = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
    xyz = tuple(torch.from_numpy(a).to(dev) for a in (sx, sy, sz))
    m.clear_visibility(*xyz, pose, t_ms, out_cleared=out)
    torch.cuda.synchronize()
    marks = O.clear_visibility(p, st, sx, sy, sz, pose, t_ms)
    got = out.cpu().numpy().reshape(p.ny, p.nx).astype(bool)
    assert np.array_equal(got, marks), f"marks differ at {np.argwhere(got != marks)[:10]}"
    g = m.state_numpy()
    exp = O.apply_clear(p, st, marks)
    for key in ("h", "v", "valid", "t_upd"):
        assert np.array_equal(g[key], getattr(exp, key)), key
    return int(marks.sum())


def test_stress_map_full_size(dev):
    from paper_2204_12876_amd import ElevationMap
    _say("stress 2000x2000, 2 x 4M points: generating")
    d = synth.cfg4(n_frames=2, device=dev)
    p = O.Params.from_dict(d["params"])
    cx, cy = d["centers"][0]
    m = ElevationMap(d["params"], cx, cy, 0, device=dev)
    st = O.init_map(p, cx, cy, 0)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    for k, f in enumerate(d["frames"]):
        cx, cy = d["centers"][k]
        m.move_map(cx, cy)
        st = O.move_map(p, st, cx, cy)
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        xs, ys, zs = f.numpy()
        n = xs.size
        cell = torch.full((n,), -7, dtype=torch.int32, device=dev)
        acc = torch.full((n,), 7, dtype=torch.uint8, device=dev)
        m.fuse_points(f.x.to(dev).contiguous(), f.y.to(dev).contiguous(),
                      f.z.to(dev).contiguous(), f.pose, f.t_ms, out_cell=cell, out_accept=acc)
        torch.cuda.synchronize()
        _say(f"stress frame {k}: {n} points fused; oracle")
        st_after, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        r = O.fuse(p, st, xs, ys, zs, f.pose, f.t_ms)
        errs = assert_fuse_parity(r, st, g, cell.cpu().numpy(), acc.cpu().numpy(),
                                  f.t_ms - st.t0)
        _say(f"stress frame {k}: accepted {int(r.accept.sum())}, rejected in map "
             f"{int((~r.accept & (r.cell >= 0)).sum())}, worst rel err v/h {errs}")
        st = st_after
        m.compute_normals()
        m.traversability(w)
        torch.cuda.synchronize()
    assert (~r.accept & (r.cell >= 0)).sum() > 0       # the second frame is gated
    g = m.state_numpy()
    assert_normals_parity(g, O.compute_normals(p, g["h"], g["valid"]))
    T, S = O.traversability(g["h"], g["valid"], synth.trav_weights())
    assert_trav_parity(g, T, S)
    f = d["frames"][1]
    xs, ys, zs = f.numpy()
    cleared = _check_clear_sampled(m, p, xs, ys, zs, f.pose, f.t_ms + 1000, dev)
    _say(f"stress: {cleared} cells cleared by 20000 sampled rays")
    m.close()


def test_sixteen_maps_batched_full_size(dev):
    from paper_2204_12876_amd import BatchEntry, ElevationMap, PipelineBatch, _emx
    _say("16 maps batched, full size: generating")
    d = synth.cfg2(device=dev)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    pb = PipelineBatch(_tuning(), device=dev)
    items = d["items"]
    ps = [O.Params.from_dict(it["params"]) for it in items]
    maps = [ElevationMap(it["params"], 0.0, 0.0, 0, device=dev) for it in items]
    frames = [it["frames"][0] for it in items]
    dev_xyz = [(f.x.to(dev).contiguous(), f.y.to(dev).contiguous(), f.z.to(dev).contiguous())
               for f in frames]
    host_xyz = [f.numpy() for f in frames]
    stages = _emx.STAGE_FUSE | _emx.STAGE_NORMALS | _emx.STAGE_TRAV
    for rep, t_ms in enumerate((100, 700)):
        before = [state_from_gpu(m, *m.info())[0] for m in maps]
        outs = [(torch.full((f.n,), -7, dtype=torch.int32, device=dev),
                 torch.full((f.n,), 7, dtype=torch.uint8, device=dev)) for f in frames]
        pb.run([BatchEntry(m, *xyz, f.pose, t_ms, weights=w, stages=stages, out_cell=c,
                           out_accept=a)
                for m, xyz, f, (c, a) in zip(maps, dev_xyz, frames, outs)])
        torch.cuda.synchronize()
        for i, (m, p, f) in enumerate(zip(maps, ps, frames)):
            _, g = state_from_gpu(m, *m.info())
            r = O.fuse(p, before[i], *host_xyz[i], f.pose, t_ms)
            assert_fuse_parity(r, before[i], g, outs[i][0].cpu().numpy(),
                               outs[i][1].cpu().numpy(), t_ms)
            assert_normals_parity(g, O.compute_normals(p, g["h"], g["valid"]))
            T, S = O.traversability(g["h"], g["valid"], synth.trav_weights())
            assert_trav_parity(g, T, S)
        _say(f"16 maps batched, pass {rep}: fusion, normals, traversability match")
    # clearing: one batched call on sampled rays of every map
    before = [state_from_gpu(m, *m.info())[0] for m in maps]
    picks, outs, entries = [], [], []
    for i, (m, p, f) in enumerate(zip(maps, ps, frames)):
        idx = _sample(f.n, 8000, i)
        s = tuple(np.ascontiguousarray(a[idx]) for a in host_xyz[i])
        picks.append(s)
        o = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
        outs.append(o)
        entries.append(BatchEntry(m, *(torch.from_numpy(a).to(dev) for a in s), f.pose, 1500,
                                  stages=_emx.STAGE_CLEAR, out_cleared=o))
    pb.run(entries)
    torch.cuda.synchronize()
    total = 0
    for i, (m, p, f) in enumerate(zip(maps, ps, frames)):
        marks = O.clear_visibility(p, before[i], *picks[i], f.pose, 1500)
        got = outs[i].cpu().numpy().reshape(p.ny, p.nx).astype(bool)
        assert np.array_equal(got, marks), f"map {i}: marks differ"
        total += int(marks.sum())
    _say(f"16 maps batched: clearing matches ({total} cells cleared)")
    pb.close()
    for m in maps:
        m.close()


def test_stress_mix_batched_full_size(dev):
    """The 2000x2000 map with a 4M-point frame and eight 400x400 maps with
    300k-point frames, in one batched call with the tuned geometry: every map
    against the oracle (fusion on every point, normals and traversability on
    every cell), then clearing on sampled rays of every map in one more
    batched call."""
    from paper_2204_12876_amd import BatchEntry, ElevationMap, PipelineBatch, _emx
    _say("stress mix batched, full size: generating")
    big = synth.cfg4(n_frames=1, device=dev)
    small = synth.cfg1(n_frames=8, device=dev)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    pb = PipelineBatch(_tuning(), device=dev)
    specs = [(big["params"], big["centers"][0], big["frames"][0])]
    specs += [(small["params"], small["centers"][k], small["frames"][k]) for k in range(8)]
    ps = [O.Params.from_dict(pr) for pr, _, _ in specs]
    maps = [ElevationMap(pr, *c, 0, device=dev) for pr, c, _ in specs]
    dev_xyz = [(f.x.to(dev).contiguous(), f.y.to(dev).contiguous(), f.z.to(dev).contiguous())
               for _, _, f in specs]
    host_xyz = [f.numpy() for _, _, f in specs]
    stages = _emx.STAGE_FUSE | _emx.STAGE_NORMALS | _emx.STAGE_TRAV
    t_ms = 100
    before = [state_from_gpu(m, *m.info())[0] for m in maps]
    outs = [(torch.full((f.n,), -7, dtype=torch.int32, device=dev),
             torch.full((f.n,), 7, dtype=torch.uint8, device=dev)) for _, _, f in specs]
    _say("stress mix batched: one call, 9 maps,",
         sum(f.n for _, _, f in specs), "points")
    pb.run([BatchEntry(m, *xyz, f.pose, t_ms, weights=w, stages=stages, out_cell=c, out_accept=a)
            for m, xyz, (_, _, f), (c, a) in zip(maps, dev_xyz, specs, outs)])
    torch.cuda.synchronize()
    for i, (m, p, (_, _, f)) in enumerate(zip(maps, ps, specs)):
        _, g = state_from_gpu(m, *m.info())
        r = O.fuse(p, before[i], *host_xyz[i], f.pose, t_ms)
        assert_fuse_parity(r, before[i], g, outs[i][0].cpu().numpy(),
                           outs[i][1].cpu().numpy(), t_ms)
        assert_normals_parity(g, O.compute_normals(p, g["h"], g["valid"]))
        T, S = O.traversability(g["h"], g["valid"], synth.trav_weights())
        assert_trav_parity(g, T, S)
        _say(f"stress mix batched: map {i} ({p.nx}x{p.ny}) fusion, normals, traversability match")
    # clearing: one batched call on sampled rays of every map
    before = [state_from_gpu(m, *m.info())[0] for m in maps]
    picks, couts, entries = [], [], []
    for i, (m, p, (_, _, f)) in enumerate(zip(maps, ps, specs)):
        idx = _sample(f.n, 20000 if i == 0 else 5000, 40 + i)
        sel = tuple(np.ascontiguousarray(a[idx]) for a in host_xyz[i])
        picks.append(sel)
        o = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
        couts.append(o)
        entries.append(BatchEntry(m, *(torch.from_numpy(a).to(dev) for a in sel), f.pose, 1500,
                                  stages=_emx.STAGE_CLEAR, out_cleared=o))
    pb.run(entries)
    torch.cuda.synchronize()
    total = 0
    for i, (m, p, (_, _, f)) in enumerate(zip(maps, ps, specs)):
        marks = O.clear_visibility(p, before[i], *picks[i], f.pose, 1500)
        got = couts[i].cpu().numpy().reshape(p.ny, p.nx).astype(bool)
        assert np.array_equal(got, marks), f"map {i}: marks differ"
        total += int(marks.sum())
    _say(f"stress mix batched: clearing matches ({total} cells cleared)")
    pb.close()
    for m in maps:
        m.close()


def test_sixty_four_robots_server_full_size(dev):
    from paper_2204_12876_amd import ElevationMap
    from paper_2204_12876_amd.server import GpuExecutor, Request, Server, run_trace
    _say("64 robots through the server: generating")
    d = synth.cfg3(device=dev, n_robots=64, n_frames=1)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    items = d["items"]
    rng = np.random.default_rng(64)
    reqs, seq = [], 0
    for k, it in enumerate(items):
        f = it["frames"][0]
        xyz = torch.empty((3, f.n), dtype=torch.float32, pin_memory=True)
        xyz[0].copy_(f.x)
        xyz[1].copy_(f.y)
        xyz[2].copy_(f.z)
        c = it["centers"][0]
        times = np.sort(rng.uniform(0.0, 0.03, 3))
        for j, t in enumerate(times):
            cx = c[0] + (it["params"]["resolution"] if j % 2 else 0.0)
            reqs.append(Request(robot=k, xyz=xyz, pose=f.pose, t_ms=300 * (j + 1),
                                center=(cx, c[1]), arrival=float(t), seq=seq))
            seq += 1
    largest = max((it["params"] for it in items), key=lambda q: q["nx"] * q["ny"])
    ex = GpuExecutor(largest, lanes=2, max_items=64, max_batch_points=8_000_000,
                     pool_points=24_000_000, weights=w, device=dev)
    srv = Server(ex, 32 << 30)
    for k, it in enumerate(items):
        srv.add_map(k, it["params"], *it["centers"][0])
    run_trace(srv, reqs, timeout_s=120)
    torch.cuda.synchronize()
    assert len(srv.completed) == len(reqs)
    _say(f"server: {len(reqs)} frames in {srv.batches} batches, largest {max(srv.batch_sizes)}")
    assert max(srv.batch_sizes) > 1
    for k, it in enumerate(items):
        alone = ElevationMap(it["params"], *it["centers"][0], 0, device=dev)
        for r in sorted((r for r in reqs if r.robot == k), key=lambda r: r.t_ms):
            x, y, z = (r.xyz[i].to(dev) for i in range(3))
            alone.move_map(*r.center)
            alone.fuse_points(x, y, z, r.pose, r.t_ms)
            alone.clear_visibility(x, y, z, r.pose, r.t_ms)
            alone.compute_normals()
            alone.traversability(w)
        torch.cuda.synchronize()
        a = alone.export_state().cpu().numpy()
        b = ex.maps[k].export_state().cpu().numpy()
        assert alone.info() == ex.maps[k].info(), f"robot {k}"
        assert np.array_equal(a, b), f"robot {k}: {(a != b).sum()} bytes differ"
        alone.close()
    _say("server: all 64 maps equal their frames run alone")
