"""GPU path (libemx.so through its C ABI) against the CPU oracle.

Stage-synchronised: before every call the oracle is handed the GPU's float32
state, so decisions are compared bit for bit and continuous values within the
tolerances stated in parity_util.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from parity_util import (assert_fuse_parity, assert_normals_parity, assert_trav_parity,
                         frame_dev, gpu_fuse, load_state, random_state, state_from_gpu)

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_12876_amd import _emx
    _emx.lib()
    return torch.device("cuda:0")


def _map(params, dev, cx=0.0, cy=0.0, t0=0):
    from paper_2204_12876_amd import ElevationMap
    return ElevationMap(params, cx, cy, t0, device=dev)


def _say(*a):
    print("[case]", *a, flush=True)


def _pose(t, R=None):
    P = np.zeros((3, 4))
    P[:, :3] = np.eye(3) if R is None else R
    P[:, 3] = t
    return P


def _fuse_check(m, p, st, xs, ys, zs, pose, t_ms, dev):
    xyz = tuple(torch.from_numpy(np.ascontiguousarray(a, F32)).to(dev) for a in (xs, ys, zs))
    cell, acc = gpu_fuse(m, xyz, pose, t_ms)
    st_after, g = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    r = O.fuse(p, st, xs, ys, zs, pose, t_ms)
    errs = assert_fuse_parity(r, st, g, cell, acc, t_ms - st.t0)
    return r, st_after, errs


# ------------------------------------------------------------------------ fusion
@pytest.mark.parametrize("seed", range(3))
def test_fuse_tiny_random_prior(dev, seed):
    _say("fuse tiny", seed)
    rng = np.random.default_rng(seed)
    params = dict(nx=9, ny=7, resolution=0.5, noise_alpha=0.01, gate_k=2.0, min_range=0.05,
                  init_variance=1e3)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng)
    st.v[:] = rng.uniform(0.01, 0.3, st.v.shape).astype(F32)
    load_state(m, st)
    n = 500
    xs = rng.uniform(-2.6, 2.4, n).astype(F32)
    ys = rng.uniform(-2.0, 2.0, n).astype(F32)
    zs = rng.uniform(-1.6, -0.2, n).astype(F32)
    xs[:5] = np.nan
    zs[5:8] = 0.0
    xs[5:8] = 0.0
    ys[5:8] = 0.001                       # below the minimum range
    pose = _pose((0.1, -0.2, 1.0))
    r, _, _ = _fuse_check(m, p, st, xs, ys, zs, pose, 250, dev)
    assert r.accept.sum() > 50 and (~r.accept & (r.cell >= 0)).sum() > 10
    m.close()


def test_fuse_cfg0_from_prior_and_gated_second_frame(dev):
    _say("fuse cfg0 two frames")
    d = synth.cfg0(n_frames=2)
    p = O.Params.from_dict(d["params"])
    m = _map(d["params"], dev)
    st = O.init_map(p, 0.0, 0.0, 0)
    for f in d["frames"]:
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        r, st, errs = _fuse_check(m, p, st, *f.numpy(), f.pose, f.t_ms, dev)
        print("cfg0 frame", f.t_ms, "accepted", int(r.accept.sum()), "cells", int(r.updated.sum()),
              "worst rel err v/h", errs, flush=True)
    # the second frame is gated against the first: some in-map points rejected
    assert (~r.accept & (r.cell >= 0)).sum() > 0
    m.close()


def test_fuse_heavy_cell_and_many_chunks(dev):
    """All points of several chunks in one cell, plus a ragged tail."""
    _say("fuse heavy cell")
    rng = np.random.default_rng(11)
    params = dict(nx=40, ny=33, resolution=0.1, noise_alpha=1e-3, gate_k=1e6, min_range=0.01)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = O.init_map(p, 0.0, 0.0, 0)
    n = 3 * 2048 + 37
    xs = rng.uniform(0.01, 0.09, n).astype(F32)    # one cell: local x in (2.01, 2.09)
    ys = rng.uniform(0.01, 0.09, n).astype(F32)
    zs = (rng.normal(size=n) * 0.01 - 1.0).astype(F32)
    pose = _pose((0.0, 0.0, 1.2))
    r, _, errs = _fuse_check(m, p, st, xs, ys, zs, pose, 10, dev)
    assert r.updated.sum() == 1 and r.n_acc.max() == n
    print("heavy cell worst rel err", errs, flush=True)
    m.close()


def test_fuse_ragged_tiles_spread(dev):
    """A map whose sides are not tile multiples, points spread over every tile."""
    _say("fuse ragged tiles")
    rng = np.random.default_rng(12)
    params = dict(nx=101, ny=67, resolution=0.05, noise_alpha=1e-3, gate_k=3.0, min_range=0.01)
    p = O.Params.from_dict(params)
    m = _map(params, dev, cx=0.3, cy=-0.2)
    st = O.init_map(p, 0.3, -0.2, 0)
    for it in range(3):
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        n = 20000 + 313 * it
        xs = rng.uniform(-2.7, 2.8, n).astype(F32)
        ys = rng.uniform(-1.8, 1.8, n).astype(F32)
        zs = (0.1 * np.sin(3 * xs) - 0.9 + 0.02 * rng.normal(size=n)).astype(F32)
        yaw = rng.uniform(0, 2 * math.pi)
        R = np.array([[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0],
                      [0, 0, 1]])
        pose = _pose((0.3, -0.2, 1.0), R)
        r, st, errs = _fuse_check(m, p, st, xs, ys, zs, pose, 100 * it, dev)
        print("ragged iter", it, "updated", int(r.updated.sum()), errs, flush=True)
    m.close()


def test_fuse_large_map_wide_keys(dev):
    """A map of more than 4096 fusion tiles, 2^22 cells (sort keys of 64 bits)."""
    _say("fuse large map")
    rng = np.random.default_rng(13)
    params = dict(nx=2080, ny=2100, resolution=0.02, noise_alpha=1e-3, gate_k=3.0, min_range=0.01)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = O.init_map(p, 0.0, 0.0, 0)
    n = 60000
    xs = rng.uniform(-20.7, 20.7, n).astype(F32)
    ys = rng.uniform(-20.9, 20.9, n).astype(F32)
    zs = (0.05 * np.cos(xs) - 1.0 + 0.01 * rng.normal(size=n)).astype(F32)
    xs[:3000] = rng.uniform(0.0, 0.1, 3000).astype(F32)      # a dense corner
    ys[:3000] = rng.uniform(0.0, 0.1, 3000).astype(F32)
    r, _, errs = _fuse_check(m, p, st, xs, ys, zs, _pose((0.0, 0.0, 1.0)), 10, dev)
    assert r.updated.sum() > 10000
    print("large map worst rel err", errs, flush=True)
    m.close()


def test_fuse_empty_and_all_dropped(dev):
    _say("fuse empty / all dropped")
    params = dict(nx=16, ny=16, resolution=0.1)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    rng = np.random.default_rng(3)
    st = random_state(p, rng)
    load_state(m, st)
    before = m.export_state().cpu().numpy()
    e = torch.empty(0, dtype=torch.float32, device=dev)
    m.fuse_points(e, e, e, _pose((0, 0, 1)), 5)
    torch.cuda.synchronize()
    assert np.array_equal(m.export_state().cpu().numpy(), before)
    nan = torch.full((1000,), float("nan"), device=dev)
    cell, acc = gpu_fuse(m, (nan, nan, nan), _pose((0, 0, 1)), 5)
    assert (cell == -1).all() and (acc == 0).all()
    assert np.array_equal(m.export_state().cpu().numpy(), before)
    far = torch.full((1000,), 100.0, device=dev)
    cell, acc = gpu_fuse(m, (far, far, far), _pose((0, 0, 1)), 5)
    assert (cell == -1).all() and (acc == 0).all()
    assert np.array_equal(m.export_state().cpu().numpy(), before)
    m.close()


def test_fuse_is_deterministic(dev):
    _say("fuse determinism")
    d = synth.cfg0(n_points=20000)
    f = d["frames"][0]
    outs = []
    for _ in range(2):
        m = _map(d["params"], dev)
        xyz = frame_dev(f, dev)
        gpu_fuse(m, xyz, f.pose, f.t_ms)
        outs.append(m.export_state().cpu().numpy())
        m.close()
    assert np.array_equal(outs[0], outs[1])


# ---------------------------------------------------------------------- clearing
def _clear_check(m, p, st, xs, ys, zs, pose, t_ms, dev):
    load_state(m, st)
    xyz = tuple(torch.from_numpy(np.ascontiguousarray(a, F32)).to(dev) for a in (xs, ys, zs))
    out = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
    m.clear_visibility(*xyz, pose, t_ms, out_cleared=out)
    torch.cuda.synchronize()
    marks = O.clear_visibility(p, st, xs, ys, zs, pose, t_ms)
    got = out.cpu().numpy().reshape(p.ny, p.nx).astype(bool)
    assert np.array_equal(got, marks), f"marks differ at {np.argwhere(got != marks)[:10]}"
    g = m.state_numpy()
    exp = O.apply_clear(p, st, marks)
    for k in ("h", "v", "valid", "t_upd"):
        assert np.array_equal(g[k], getattr(exp, k)), k
    return marks


def test_clear_hand_scenes(dev):
    _say("clear hand scenes")
    params = dict(nx=16, ny=16, resolution=1.0, ray_step=1.0, clear_normal_alpha=0.3,
                  clear_min_age_ms=500, min_range=0.05)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    pose = _pose((1.5 - 8.0, 8.5 - 8.0, 2.0))
    pt = (np.array([11.0, 19.0, 0.0], F32), np.array([0.0, 0.0, 0.0], F32),
          np.array([-2.0, -2.0, -2.0], F32))
    st = O.init_map(p, 0.0, 0.0, 0)
    for ix in range(16):
        st.h[8, ix] = 5.0
        st.v[8, ix] = 0.01
        st.valid[8, ix] = 1
        st.nrm[:, 8, ix] = (-1.0, 0.0, 0.0)
    st.t_upd[8, 7] = 900                 # recent: kept
    st.nrm[:, 8, 9] = (0.0, 1.0, 0.0)   # normal perpendicular to the ray: kept
    marks = _clear_check(m, p, st, *pt, pose, 1000, dev)
    assert sorted(np.nonzero(marks[8])[0].tolist()) == [2, 3, 4, 5, 6, 8, 10, 11, 12, 13, 14, 15]
    m.close()


@pytest.mark.parametrize("seed", range(3))
def test_clear_random_tiny(dev, seed):
    _say("clear tiny", seed)
    rng = np.random.default_rng(40 + seed)
    params = dict(nx=23, ny=17, resolution=0.25, ray_step=0.13, clear_normal_alpha=0.2,
                  clear_min_age_ms=100, min_range=0.05)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng)
    xs = rng.uniform(-5, 5, 3000).astype(F32)
    ys = rng.uniform(-4, 4, 3000).astype(F32)
    zs = rng.uniform(-2, 0.8, 3000).astype(F32)
    xs[:3] = np.inf
    marks = _clear_check(m, p, st, xs, ys, zs, _pose((0.1, -0.3, 1.1)), 450, dev)
    assert marks.sum() > 5
    m.close()


def test_clear_cfg0_after_fusion(dev):
    _say("clear cfg0")
    d = synth.cfg0(n_frames=2)
    p = O.Params.from_dict(d["params"])
    m = _map(d["params"], dev)
    f0, f1 = d["frames"]
    gpu_fuse(m, frame_dev(f0, dev), f0.pose, f0.t_ms)
    m.compute_normals()
    torch.cuda.synchronize()
    st, _ = state_from_gpu(m, 0, 0, 0)
    # plant ghost obstacles above the ground on valid cells
    rng = np.random.default_rng(5)
    ok = np.argwhere(st.valid == 1)
    pick = ok[rng.choice(len(ok), 300, replace=False)]
    st.h[pick[:, 0], pick[:, 1]] += F32(0.6)
    marks = _clear_check(m, p, st, *f1.numpy(), f1.pose, 1000, dev)
    print("cfg0 cleared", int(marks.sum()), flush=True)
    assert marks.sum() > 10
    m.close()


# ---------------------------------------------------------------- normals / conv
@pytest.mark.parametrize("shape", [(7, 5), (64, 64), (97, 45)])
def test_normals_and_traversability(dev, shape):
    _say("normals/trav", shape)
    ny, nx = shape
    rng = np.random.default_rng(nx * ny)
    params = dict(nx=nx, ny=ny, resolution=0.04)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=0.97)
    st.h[:] = (st.h + F32(3.0)).astype(F32)         # heights of a few metres
    load_state(m, st)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    m.compute_normals()
    m.traversability(w)
    torch.cuda.synchronize()
    g = m.state_numpy()
    assert_normals_parity(g, O.compute_normals(p, st.h, st.valid))
    T, S = O.traversability(st.h, st.valid, synth.trav_weights())
    assert_trav_parity(g, T, S)
    # the one-pass call gives the two calls' bits
    m2 = _map(params, dev)
    load_state(m2, st)
    m2.normals_traversability(w)
    g2 = m2.state_numpy()
    for k in ("nrm", "trav"):
        assert np.array_equal(g[k].view(np.uint32), g2[k].view(np.uint32)), k
    m.close()
    m2.close()


# --------------------------------------------------------------------------- move
@pytest.mark.parametrize("shift", [(3, -2), (-50, 7), (0, 1), (200, 0)])
def test_move_map_exact(dev, shift):
    _say("move", shift)
    params = dict(nx=61, ny=43, resolution=0.05)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    rng = np.random.default_rng(9)
    st = random_state(p, rng)
    load_state(m, st)
    cx = (shift[0] + 0.5) * 0.05
    cy = (shift[1] + 0.5) * 0.05
    m.move_map(cx, cy)
    torch.cuda.synchronize()
    exp = O.move_map(p, st, cx, cy)
    g = m.state_numpy()
    assert m.info()[:2] == (exp.cgx, exp.cgy)
    for k in ("h", "v", "t_upd", "valid", "trav"):
        assert np.array_equal(g[k].view(np.uint8), getattr(exp, k).view(np.uint8)), k
    assert np.array_equal(np.isnan(g["nrm"]), np.isnan(exp.nrm))
    assert np.array_equal(np.nan_to_num(g["nrm"]), np.nan_to_num(exp.nrm))
    m.close()


# ------------------------------------------------------------ full-size frames
def test_cfg1_frames_full_pipeline(dev):
    """Two 300k-point frames of the 400x400 workload, every stage checked."""
    _say("cfg1 full size")
    d = synth.cfg1(n_frames=2, device=dev)
    p = O.Params.from_dict(d["params"])
    cx, cy = d["centers"][0]
    m = _map(d["params"], dev, cx, cy)
    st = O.init_map(p, cx, cy, 0)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    for k, f in enumerate(d["frames"]):
        cx, cy = d["centers"][k]
        m.move_map(cx, cy)
        st = O.move_map(p, st, cx, cy)
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        xs, ys, zs = f.numpy()
        r, st, errs = _fuse_check(m, p, st, xs, ys, zs, f.pose, f.t_ms + 1000, dev)
        print("cfg1 frame", k, "accepted", int(r.accept.sum()), errs, flush=True)
        marks = _clear_check(m, p, st, xs, ys, zs, f.pose, f.t_ms + 1000, dev)
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        m.compute_normals()
        m.traversability(w)
        torch.cuda.synchronize()
        g = m.state_numpy()
        assert_normals_parity(g, O.compute_normals(p, st.h, st.valid))
        T, S = O.traversability(st.h, st.valid, synth.trav_weights())
        assert_trav_parity(g, T, S)
        print("cfg1 frame", k, "cleared", int(marks.sum()), flush=True)
    m.close()


# ---------------------------------------------------------------- ABI errors
def test_abi_rejects_bad_arguments(dev):
    _say("abi errors")
    from paper_2204_12876_amd import EmxError, _emx
    params = dict(nx=16, ny=16, resolution=0.1)
    m = _map(params, dev)
    x = torch.zeros(10, device=dev)
    with pytest.raises(EmxError) as e:
        m.fuse_points(x, x, x, np.full((3, 4), np.nan), 0)
    assert e.value.status == _emx.EMX_EINVAL
    with pytest.raises(EmxError):
        m.fuse_points(x, x, x, _pose((0, 0, 1)), -5)           # before t0
    f = _emx.make_frame(x.data_ptr(), x.data_ptr(), x.data_ptr(), 10, _pose((0, 0, 1)), 0)
    from paper_2204_12876_amd import aligned_empty
    small = aligned_empty(256, dev)
    # the fusion's only scratch is the wall rule's per-cell counts: none here
    _emx.fuse_points(m.handle, f, small.data_ptr(), 16, 0, 0, 0)
    with pytest.raises(EmxError):
        _emx.layer(m.handle, 99)
    m.close()
    mw = _map(dict(params, wall_min_count=2), dev)           # 4 bytes per cell
    with pytest.raises(EmxError) as e:
        _emx.fuse_points(mw.handle, f, small.data_ptr(), 16 * 16 * 4 - 1, 0, 0, 0)
    assert e.value.status == _emx.EMX_ENOMEM
    mw.close()
