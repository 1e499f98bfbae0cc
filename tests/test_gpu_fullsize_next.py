"""The next rows at the stress workload's full size: one 2000x2000 map at
0.02 m and two 4M-point frames of a 128-beam LiDAR, with time variance, the
wall/edge rule and the upper bound layer on.

  * fusion (wall rule, time variance) and drift compensation on every point
    and cell, against the oracle;
  * clearing with the upper bound on 20,000 seeded rays of the frame over the
    full map (the oracle cannot march four million 30 m rays in seconds);
  * overlap clearance and inpainting on all four million cells;
  * smoothing on a seeded sample of cells, each checked against the oracle run
    on the cell's own window (a crop holding the window, and the grid's edge
    where the window meets it, gives the same value as the whole grid).
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
import synth
from parity_util import assert_fuse_parity, state_from_gpu

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


def _bits(a):
    return np.ascontiguousarray(a, F32).view(np.uint32)


def _grown(r, before):
    b = dataclasses.replace(before)
    b.v = np.where(r.updated, before.v, r.state.v).astype(F32)
    return b


def _smooth_sampled(dev, x, kind, k, sigma, n=3000, seed=0):
    from paper_2204_12876_amd import smooth
    g = smooth(torch.from_numpy(x).to(dev), kind, k, sigma).cpu().numpy()
    ny, nx = x.shape
    r = k // 2
    rng = np.random.default_rng(seed)
    ys = np.concatenate([rng.integers(0, ny, n), [0, ny - 1, 0, ny - 1, r, ny - 1 - r]])
    xs = np.concatenate([rng.integers(0, nx, n), [0, nx - 1, nx - 1, 0, r, nx - 1 - r]])
    worst = 0.0
    for iy, ix in zip(ys, xs):
        y0, y1 = max(0, iy - r), min(ny, iy + r + 1)
        x0, x1 = max(0, ix - r), min(nx, ix + r + 1)
        # the crop must exceed the radius for the mirror; extend it inward
        y1 = max(y1, min(ny, y0 + r + 1))
        x1 = max(x1, min(nx, x0 + r + 1))
        crop = x[y0:y1, x0:x1]
        if kind == "median":
            e = O.smooth_median(crop, k)[iy - y0, ix - x0]
            got = g[iy, ix]
            assert (np.isnan(e) and np.isnan(got)) or _bits(got) == _bits(e), (iy, ix)
            continue
        if kind == "box":
            e, mag = O.smooth_box(crop, k), O.smooth_box(np.abs(crop), k)
        else:
            e, mag = O.smooth_gaussian(crop, k, sigma), O.smooth_gaussian(np.abs(crop), k, sigma)
        e, mag = e[iy - y0, ix - x0], mag[iy - y0, ix - x0]
        got = float(g[iy, ix])
        if np.isnan(e):
            assert np.isnan(got), (iy, ix)
            continue
        assert abs(got - e) <= 1e-5 * mag + 1e-30, (iy, ix, got, e)
        worst = max(worst, abs(got - e) / max(mag, 1e-30))
    return worst


def test_next_rows_on_the_stress_map(dev):
    from paper_2204_12876_amd import ElevationMap
    _say("next rows, 2000x2000, 2 x 4M points: generating")
    d = synth.cfg4(n_frames=2, device=dev)
    params = dict(d["params"], time_variance=1e-4, wall_min_count=8, upper_bound=1)
    p = O.Params.from_dict(params)
    cx, cy = d["centers"][0]
    m = ElevationMap(params, cx, cy, 0, device=dev)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    ub = np.full((p.ny, p.nx), np.inf, F32)
    st = O.init_map(p, cx, cy, 0)
    for k, f in enumerate(d["frames"]):
        cx, cy = d["centers"][k]
        m.move_map(cx, cy)
        ub = O.move_layer(p, st, ub, cx, cy, np.inf)
        st = O.move_map(p, st, cx, cy)
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        assert np.array_equal(_bits(m.upper_bound().cpu().numpy()), _bits(ub)), "moved bound"
        xs, ys, zs = f.numpy()
        xyz = (f.x.to(dev).contiguous(), f.y.to(dev).contiguous(), f.z.to(dev).contiguous())
        if k == 1:
            # drift compensation before the second frame's fusion
            trav_min = float(np.nanmedian(st.trav[st.valid == 1]))
            mean_d, cnt_d = m.compensate_drift(*xyz, f.pose, f.t_ms, trav_min)
            torch.cuda.synchronize()
            new, mean_o, cnt_o = O.compensate_drift(p, st, xs, ys, zs, f.pose, trav_min)
            assert int(cnt_d.item()) == cnt_o > 10000
            assert abs(float(mean_d.item()) - mean_o) <= 1e-12 * max(1.0, abs(mean_o))
            assert F32(float(mean_d.item())) == F32(mean_o)
            st, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
            assert np.array_equal(_bits(g["h"]), _bits(new.h))
            _say(f"drift: mean {mean_o:.6f} m over {cnt_o} points")
        n = xs.size
        cell = torch.full((n,), -7, dtype=torch.int32, device=dev)
        acc = torch.full((n,), 7, dtype=torch.uint8, device=dev)
        m.fuse_points(*xyz, f.pose, f.t_ms, out_cell=cell, out_accept=acc)
        torch.cuda.synchronize()
        _, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        r = O.fuse(p, st, xs, ys, zs, f.pose, f.t_ms)
        errs = assert_fuse_parity(r, _grown(r, st), g, cell.cpu().numpy(), acc.cpu().numpy(),
                                  f.t_ms)
        walled = int(O.point_decisions(p, st, xs, ys, zs, f.pose)["walled"].sum())
        _say(f"frame {k}: fused, {walled} points removed by the wall rule, worst rel err {errs}")
        if k == 1:
            assert walled > 0
        m.compute_normals()
        m.traversability(w)
        torch.cuda.synchronize()
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    # clearing with the bound, on sampled rays of the last frame
    f = d["frames"][1]
    xs, ys, zs = f.numpy()
    idx = np.sort(np.random.default_rng(5).choice(xs.size, 20000, replace=False))
    sx, sy, sz = (np.ascontiguousarray(a[idx]) for a in (xs, ys, zs))
    out = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
    m.clear_visibility(*(torch.from_numpy(a).to(dev) for a in (sx, sy, sz)), f.pose,
                       f.t_ms + 1000, out_cleared=out)
    torch.cuda.synchronize()
    marks = O.clear_visibility(p, st, sx, sy, sz, f.pose, f.t_ms + 1000)
    assert np.array_equal(out.cpu().numpy().reshape(p.ny, p.nx).astype(bool), marks)
    ub = O.upper_bound(p, st, ub, sx, sy, sz, f.pose)
    assert np.array_equal(_bits(m.upper_bound().cpu().numpy()), _bits(ub))
    _say(f"clearing: {int(marks.sum())} cells cleared, {int(np.isfinite(ub).sum())} bounded")
    st = O.apply_clear(p, st, marks)
    # overlap clearance around the robot
    robot = (f.pose[0, 3], f.pose[1, 3], f.pose[2, 3] - 0.5)
    out = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
    m.overlap_clear(robot, 3.0, 0.3, out_cleared=out)
    torch.cuda.synchronize()
    om = O.overlap_clear(p, st, robot, 3.0, 0.3)
    assert np.array_equal(out.cpu().numpy().reshape(p.ny, p.nx).astype(bool), om)
    st = O.apply_clear(p, st, om)
    g = m.state_numpy()
    for key in ("h", "v", "valid"):
        assert np.array_equal(g[key], getattr(st, key)), key
    _say(f"overlap: {int(om.sum())} cells removed")
    # inpainting of the whole map, then smoothing on sampled cells
    filled = m.inpaint_min().cpu().numpy()
    exp = O.inpaint_min(g["h"], g["valid"])
    assert np.array_equal(np.isnan(filled), np.isnan(exp))
    assert np.array_equal(_bits(filled)[~np.isnan(filled)], _bits(exp)[~np.isnan(exp)])
    _say(f"inpainting: {int((g['valid'] == 0).sum())} empty cells, "
         f"{int(np.isnan(exp).sum())} left without a border")
    for kind, k, s in (("box", 5, 0.0), ("gaussian", 7, 1.5), ("median", 5, 0.0)):
        worst = _smooth_sampled(dev, filled, kind, k, s)
        _say(f"smooth {kind} {k}: sampled cells match, worst rel err {worst:.3g}")
    m.close()
