"""GPU path against the oracle for the height-update extensions and drift
compensation (Sec. II-C: wall/edge rule, time variance; Sec. II-D: drift).

Stage-synchronised like test_gpu_parity: the oracle starts from the GPU's
float32 state.  Decisions (cells, accepts, the rule's removals, counts) are
compared bit for bit; fused heights and variances within parity_util's
tolerances; the time variance and the drift shift are single float32 additions
and are compared bit for bit.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
import synth
from parity_util import (assert_fuse_parity, gpu_fuse, load_state, random_state,
                         state_from_gpu)

pytestmark = pytest.mark.gpu

F32 = np.float32
F64 = np.float64


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_12876_amd import _emx
    _emx.lib()
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def _map(params, dev, cx=0.0, cy=0.0, t0=0):
    from paper_2204_12876_amd import ElevationMap
    return ElevationMap(params, cx, cy, t0, device=dev)


def _pose(t):
    P = np.zeros((3, 4))
    P[:, :3] = np.eye(3)
    P[:, 3] = t
    return P


def _dev(dev, *arrs):
    return tuple(torch.from_numpy(np.ascontiguousarray(a, F32)).to(dev) for a in arrs)


def _clustered_cloud(rng, n, nx, ny, res, pose_z, hot_cells=12):
    """Points over the map, a third of them piled into a few cells so that
    those cells exceed the rule's count threshold (map-local origin at the
    lower-left corner, the sensor at the map centre)."""
    xs = rng.uniform(-0.49 * nx * res, 0.49 * nx * res, n)
    ys = rng.uniform(-0.49 * ny * res, 0.49 * ny * res, n)
    k = n // 3
    hot = rng.integers(0, nx * ny, hot_cells)
    pick = hot[rng.integers(0, hot_cells, k)]
    xs[:k] = (pick % nx + rng.uniform(0.05, 0.95, k)) * res - 0.5 * nx * res
    ys[:k] = (pick // nx + rng.uniform(0.05, 0.95, k)) * res - 0.5 * ny * res
    zs = rng.uniform(-0.6, 0.9, n) - pose_z
    return xs.astype(F32), ys.astype(F32), zs.astype(F32)


# ------------------------------------------------------------------ wall rule
@pytest.mark.parametrize("thr,gate_k", [(1, 3.0), (4, 1e3), (16, 2.0)])
def test_wall_rule_fusion(dev, thr, gate_k):
    _say("wall rule", thr, gate_k)
    rng = np.random.default_rng(100 + thr)
    params = dict(nx=70, ny=45, resolution=0.1, noise_alpha=0.01, gate_k=gate_k,
                  min_range=0.05, wall_min_count=thr)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=0.8)
    load_state(m, st)
    n = 6 * 1024 + 37                                   # several chunks, ragged tail
    xs, ys, zs = _clustered_cloud(rng, n, p.nx, p.ny, p.resolution, 1.2)
    pose = _pose((0.0, 0.0, 1.2))
    cell, acc = gpu_fuse(m, _dev(dev, xs, ys, zs), pose, 40)
    _, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    r = O.fuse(p, st, xs, ys, zs, pose, 40)
    assert_fuse_parity(r, st, g, cell, acc, 40)
    walled = O.point_decisions(p, st, xs, ys, zs, pose)["walled"]
    _say(f"wall rule thr {thr}: {int(walled.sum())} points removed")
    assert walled.sum() > 20
    m.close()


def test_wall_rule_on_a_scene_over_two_frames(dev):
    _say("wall rule on the small scene")
    d = synth.cfg0(n_frames=2)
    params = dict(d["params"], wall_min_count=3)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = O.init_map(p, 0.0, 0.0, 0)
    removed = 0
    for f in d["frames"]:
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        xs, ys, zs = f.numpy()
        cell, acc = gpu_fuse(m, _dev(dev, xs, ys, zs), f.pose, f.t_ms)
        _, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        r = O.fuse(p, st, xs, ys, zs, f.pose, f.t_ms)
        assert_fuse_parity(r, st, g, cell, acc, f.t_ms)
        removed += int(O.point_decisions(p, st, xs, ys, zs, f.pose)["walled"].sum())
    assert removed > 0            # the second frame meets cells of the first
    m.close()


# -------------------------------------------------------------- time variance
def _grown(r, before):
    """The state the untouched cells must hold: the oracle's, bit for bit."""
    b = dataclasses.replace(before)
    b.v = np.where(r.updated, before.v, r.state.v).astype(F32)
    return b


def test_time_variance_fusion_then_clearing(dev):
    _say("time variance")
    rng = np.random.default_rng(7)
    params = dict(nx=50, ny=40, resolution=0.1, noise_alpha=0.01, gate_k=2.5,
                  min_range=0.05, time_variance=0.0025, ray_step=0.05)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=0.7)
    load_state(m, st)
    pose = _pose((0.0, 0.0, 1.0))
    for k, n in enumerate((700, 0, 2500)):
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        xs = rng.uniform(-2.4, 2.4, n).astype(F32)
        ys = rng.uniform(-1.9, 1.9, n).astype(F32)
        zs = (rng.uniform(-0.5, 0.8, n) - 1.0).astype(F32)
        t_ms = 100 * (k + 1)
        cell, acc = gpu_fuse(m, _dev(dev, xs, ys, zs), pose, t_ms)
        _, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        r = O.fuse(p, st, xs, ys, zs, pose, t_ms)
        grow = ~r.updated & (st.valid == 1)
        assert grow.sum() > 100
        assert np.array_equal(g["v"][~r.updated].view(np.uint32),
                              r.state.v[~r.updated].view(np.uint32)), "time variance"
        if n:
            assert_fuse_parity(r, _grown(r, st), g, cell, acc, t_ms)
        else:
            assert np.array_equal(g["h"], st.h) and not r.updated.any()
        _say(f"time variance frame {k}: {int(grow.sum())} cells grew, "
             f"{int(r.updated.sum())} updated")
    # the fusion's update flags share the clearing marks: they must be gone
    st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    xs = rng.uniform(-2.4, 2.4, 900).astype(F32)
    ys = rng.uniform(-1.9, 1.9, 900).astype(F32)
    zs = (rng.uniform(-2.0, -1.5, 900)).astype(F32)
    out = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
    m.clear_visibility(*_dev(dev, xs, ys, zs), pose, 900, out_cleared=out)
    torch.cuda.synchronize()
    marks = O.clear_visibility(p, st, xs, ys, zs, pose, 900)
    got = out.cpu().numpy().reshape(p.ny, p.nx).astype(bool)
    assert np.array_equal(got, marks)
    g = m.state_numpy()
    exp = O.apply_clear(p, st, marks)
    for key in ("h", "v", "valid", "t_upd"):
        assert np.array_equal(g[key], getattr(exp, key)), key
    m.close()


# ---------------------------------------------------------------------- drift
def _drift_check(m, p, st, xs, ys, zs, pose, t_ms, trav_min, dev):
    mean_d, cnt_d = m.compensate_drift(*_dev(dev, xs, ys, zs), pose, t_ms, trav_min)
    torch.cuda.synchronize()
    mean_g, cnt_g = float(mean_d.item()), int(cnt_d.item())
    g = m.state_numpy()
    new, mean_o, cnt_o = O.compensate_drift(p, st, xs, ys, zs, pose, trav_min)
    assert cnt_g == cnt_o
    if cnt_o:
        # both sides sum the same float64 errors in different orders: bound by
        # the summation error of a tree of depth <= 64 over the magnitudes
        d = O.point_decisions(p, st, xs, ys, zs, pose)
        c = d["cell"]
        cc = np.where(c >= 0, c, 0)
        tr = st.trav.reshape(-1)[cc]
        with np.errstate(invalid="ignore"):
            use = (c >= 0) & (st.valid.reshape(-1)[cc] != 0) & (tr > F32(trav_min))
        mag = np.abs(d["zm"][use].astype(F64) - st.h.reshape(-1)[cc[use]].astype(F64)).mean()
        assert abs(mean_g - mean_o) <= 64 * 2.0 ** -53 * mag
        assert F32(mean_g) == F32(mean_o)
    else:
        assert mean_g == 0.0
    exp_h = np.where(st.valid != 0, st.h + F32(mean_g), st.h).astype(F32) if cnt_o else st.h
    assert np.array_equal(g["h"].view(np.uint32), exp_h.view(np.uint32))
    assert np.array_equal(g["h"].view(np.uint32), new.h.view(np.uint32))
    for k in ("v", "valid", "t_upd"):
        assert np.array_equal(g[k], getattr(st, k)), k
    return mean_g, cnt_g


@pytest.mark.parametrize("n", [0, 1, 1023, 5 * 1024 + 37, 200_000])
def test_drift_random_state(dev, n):
    _say("drift random", n)
    rng = np.random.default_rng(50 + n % 97)
    params = dict(nx=64, ny=48, resolution=0.1, noise_alpha=0.01, gate_k=2.0, min_range=0.05)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=0.75)
    st.trav[rng.random(st.trav.shape) < 0.1] = np.nan
    load_state(m, st)
    xs = rng.uniform(-3.3, 3.3, n).astype(F32)            # some points off the map
    ys = rng.uniform(-2.5, 2.5, n).astype(F32)
    zs = (rng.uniform(-0.4, 0.9, n) - 1.1).astype(F32)
    xs[: min(n, 3)] = np.nan
    mean, cnt = _drift_check(m, p, st, xs, ys, zs, _pose((0.05, -0.02, 1.1)), 10, 0.2, dev)
    _say(f"drift n={n}: mean {mean:.6g} over {cnt} points")
    if n >= 1023:
        assert cnt > n // 10
    m.close()


def test_drift_without_contributing_points(dev):
    _say("drift none")
    rng = np.random.default_rng(9)
    params = dict(nx=32, ny=32, resolution=0.1, noise_alpha=0.01, gate_k=2.0, min_range=0.05)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng)
    st.trav[:] = np.nan
    load_state(m, st)
    xs, ys, zs = (rng.uniform(-1.5, 1.5, 3000).astype(F32) for _ in range(3))
    mean, cnt = _drift_check(m, p, st, xs, ys, zs, _pose((0.0, 0.0, 1.0)), 10, -1e9, dev)
    assert cnt == 0 and mean == 0.0
    m.close()


def test_drift_on_the_scene_recovers_a_height_offset(dev):
    """The small scene: fuse a frame, compute traversability, then hand the
    next frame with the robot's height estimate 4 cm off; the compensation
    moves the map by about that offset, as the oracle does."""
    _say("drift on the small scene")
    d = synth.cfg0(n_frames=2)
    p = O.Params.from_dict(d["params"])
    m = _map(d["params"], dev)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    f0, f1 = d["frames"]
    m.fuse_points(*_dev(dev, *f0.numpy()), f0.pose, f0.t_ms)
    m.compute_normals()
    m.traversability(w)
    torch.cuda.synchronize()
    st, g = state_from_gpu(m, *m.info())
    tr = g["trav"][g["valid"] == 1]
    trav_min = float(np.nanmedian(tr))
    pose = f1.pose.copy()
    pose[2, 3] += 0.04
    mean, cnt = _drift_check(m, p, st, *f1.numpy(), pose, f1.t_ms, trav_min, dev)
    _say(f"drift on the scene: mean {mean:.5f} m over {cnt} points")
    assert cnt > 1000 and abs(mean - 0.04) < 0.02
    m.close()


# ------------------------------------------------------------- batch refusal
def test_batch_runs_the_extensions_like_the_plain_calls(dev):
    """Each extension alone, one map, one fusion: the batched call gives the
    plain call's bits (the mixed, multi-frame case is in test_gpu_batch)."""
    from paper_2204_12876_amd import BatchEntry, PipelineBatch, _emx
    _say("batch with one extension each")
    pb = PipelineBatch(device=dev)
    rng = np.random.default_rng(9)
    xs, ys, zs = _clustered_cloud(rng, 3000, 16, 16, 0.1, 1.0)
    xyz = _dev(dev, xs, ys, zs)
    for extra in (dict(time_variance=0.001), dict(wall_min_count=2), dict(upper_bound=1),
                  dict(excl_on=1, excl_theta=0.3, excl_b=0.2, excl_c=0.3, excl_d=0.6),
                  dict(outlier_variance=0.01, gate_k=1.0)):
        params = dict(dict(nx=16, ny=16, resolution=0.1), **extra)
        p = O.Params.from_dict(params)
        st = random_state(p, rng, valid_frac=0.7)
        a, b = _map(params, dev), _map(params, dev)
        load_state(a, st)
        load_state(b, st)
        a.fuse_points(*xyz, _pose((0, 0, 1)), 10)
        pb.run([BatchEntry(b, *xyz, _pose((0, 0, 1)), 10, stages=_emx.STAGE_FUSE)])
        torch.cuda.synchronize()
        assert torch.equal(a.export_state(), b.export_state()), extra
        a.close()
        b.close()
    pb.close()


# ------------------------------------------------------ exclusion area (ramp)
@pytest.mark.parametrize("wall", [0, 3])
def test_exclusion_area_fusion(dev, wall):
    _say("exclusion area, wall rule", wall)
    rng = np.random.default_rng(200 + wall)
    params = dict(nx=70, ny=45, resolution=0.1, noise_alpha=0.01, gate_k=1e3, min_range=0.05,
                  wall_min_count=wall, excl_on=1, excl_theta=0.5, excl_b=0.1, excl_c=0.8,
                  excl_d=0.5)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=0.8)
    load_state(m, st)
    n = 6 * 1024 + 37
    xs, ys, zs = _clustered_cloud(rng, n, p.nx, p.ny, p.resolution, 0.3)
    pose = _pose((0.0, 0.0, 0.3))
    cell, acc = gpu_fuse(m, _dev(dev, xs, ys, zs), pose, 40)
    _, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    r = O.fuse(p, st, xs, ys, zs, pose, 40)
    assert_fuse_parity(r, st, g, cell, acc, 40)
    dd = O.point_decisions(p, st, xs, ys, zs, pose)
    _say(f"exclusion area: {int(dd['excluded'].sum())} points ignored, "
         f"{int(dd['walled'].sum())} by the wall rule")
    assert 500 < dd["excluded"].sum() < n - 500
    if wall:
        assert dd["walled"].sum() > 20
    m.close()


# ------------------------------------------------------------ outlier variance
def _assert_outlier_parity(r, before, g, cell, acc, t_now, p, dec):
    """As assert_fuse_parity, but cells that gain the outlier variance (and, with
    it, the time variance) without being updated hold the oracle's float32
    additions bit for bit."""
    assert np.array_equal(cell, r.cell.astype(np.int32))
    assert np.array_equal(acc.astype(bool), r.accept)
    u = r.updated
    changed = ~u & (r.state.v != before.v)
    for k in ("h", "t_upd", "valid"):
        assert np.array_equal(g[k][~u], getattr(before, k)[~u]), f"untouched {k} changed"
    assert np.array_equal(g["v"][~u].view(np.uint32), r.state.v[~u].view(np.uint32)), \
        "untouched variance differs from the oracle's float32 additions"
    dv = np.abs(g["v"][u].astype(np.float64) - r.v[u])
    assert np.all(dv <= 1e-5 * r.v[u])
    scale = np.maximum(np.abs(r.h[u]), r.h_scale[u])
    assert np.all(np.abs(g["h"][u].astype(np.float64) - r.h[u]) <= 1e-5 * scale)
    return int(changed.sum())


@pytest.mark.parametrize("var_t", [0.0, 0.002])
def test_outlier_variance_fusion(dev, var_t):
    _say("outlier variance, time variance", var_t)
    rng = np.random.default_rng(300 + int(var_t * 1e4))
    params = dict(nx=70, ny=45, resolution=0.1, noise_alpha=0.01, gate_k=2.0, min_range=0.05,
                  outlier_variance=0.0125, time_variance=var_t, wall_min_count=4)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=0.7)
    load_state(m, st)
    n = 5 * 1024 + 501
    xs, ys, zs = _clustered_cloud(rng, n, p.nx, p.ny, p.resolution, 1.2)
    pose = _pose((0.0, 0.0, 1.2))
    cell, acc = gpu_fuse(m, _dev(dev, xs, ys, zs), pose, 40)
    _, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    r = O.fuse(p, st, xs, ys, zs, pose, 40)
    dec = O.point_decisions(p, st, xs, ys, zs, pose)
    inflated = _assert_outlier_parity(r, st, g, cell, acc, 40, p, dec)
    rej_cells = np.unique(dec["cell"][dec["rejected"]])
    _say(f"outlier variance: {int(dec['rejected'].sum())} rejected points in "
         f"{rej_cells.size} cells; {inflated} cells changed without an update")
    assert dec["rejected"].sum() > 100
    # a second call: every mark was cleared, so only this frame's outliers count
    st2, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    xs2, ys2, zs2 = _clustered_cloud(rng, 3000, p.nx, p.ny, p.resolution, 1.2)
    cell, acc = gpu_fuse(m, _dev(dev, xs2, ys2, zs2), pose, 80)
    _, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    r = O.fuse(p, st2, xs2, ys2, zs2, pose, 80)
    _assert_outlier_parity(r, st2, g, cell, acc, 80, p,
                           O.point_decisions(p, st2, xs2, ys2, zs2, pose))
    m.close()
