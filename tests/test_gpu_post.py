"""GPU path against the oracle for the upper bound layer (Sec. II-H), overlap
clearance (Sec. II-F) and the locomotion filters (Sec. II-I).

Stage-synchronised: the oracle starts from the GPU's float32 state.
  * upper bound, overlap marks, inpainting and the median: bit for bit (a
    minimum, a mask and a selection involve no rounding);
  * box and Gaussian smoothing: |gpu - oracle| <= 1e-5 * sum_w |x| over the
    window (float32 sums of at most 2 x 31 terms against float64).
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from parity_util import load_state, random_state, state_from_gpu

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


def _bits(a):
    return np.ascontiguousarray(a, F32).view(np.uint32)


# -------------------------------------------------------------- upper bound
def _clear_with_bound(m, p, st, ub, xs, ys, zs, pose, t_ms, dev):
    out = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
    m.clear_visibility(*_dev(dev, xs, ys, zs), pose, t_ms, out_cleared=out)
    torch.cuda.synchronize()
    marks = O.clear_visibility(p, st, xs, ys, zs, pose, t_ms)
    got = out.cpu().numpy().reshape(p.ny, p.nx).astype(bool)
    assert np.array_equal(got, marks), "clearing marks"
    exp = O.upper_bound(p, st, ub, xs, ys, zs, pose)
    g = m.upper_bound().cpu().numpy()
    bad = _bits(g) != _bits(exp)
    assert not bad.any(), f"upper bound differs at {np.argwhere(bad)[:8]}"
    return exp, int(marks.sum())


@pytest.mark.parametrize("seed,valid_frac", [(0, 0.3), (1, 0.7), (2, 0.95)])
def test_upper_bound_random_state(dev, seed, valid_frac):
    _say("upper bound random", seed, valid_frac)
    rng = np.random.default_rng(300 + seed)
    params = dict(nx=120, ny=90, resolution=0.05, noise_alpha=0.01, gate_k=2.0, min_range=0.05,
                  ray_step=0.03, clear_normal_alpha=0.2, clear_min_age_ms=100, upper_bound=1)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=valid_frac)
    load_state(m, st)
    ub = np.full((p.ny, p.nx), np.inf, F32)
    assert np.all(np.isinf(m.upper_bound().cpu().numpy()))
    pose = _pose((0.1, -0.05, 1.0))
    for k in range(2):
        n = 3000 + 517 * k
        xs = rng.uniform(-4.0, 4.0, n).astype(F32)        # some rays leave the map
        ys = rng.uniform(-3.0, 3.0, n).astype(F32)
        zs = (rng.uniform(-0.8, 0.9, n) - 1.0).astype(F32)
        st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
        ub, cleared = _clear_with_bound(m, p, st, ub, xs, ys, zs, pose, 500 + 300 * k, dev)
        _say(f"upper bound frame {k}: {int(np.isfinite(ub).sum())} bounded cells, "
             f"{cleared} cleared")
    assert np.isfinite(ub).sum() > 100
    # the bound moves with the map; entering cells start unbounded
    st, _ = state_from_gpu(m, st.cgx, st.cgy, st.t0)
    m.move_map(0.37, -0.21)
    exp = O.move_layer(p, st, ub, 0.37, -0.21, np.inf)
    assert np.array_equal(_bits(m.upper_bound().cpu().numpy()), _bits(exp))
    m.close()


def test_upper_bound_does_not_change_clearing(dev):
    _say("upper bound vs plain clearing")
    d = synth.cfg0(n_frames=2)
    outs = []
    for ubf in (0, 1):
        params = dict(d["params"], upper_bound=ubf)
        m = _map(params, dev)
        f0, f1 = d["frames"]
        m.fuse_points(*_dev(dev, *f0.numpy()), f0.pose, f0.t_ms)
        m.compute_normals()
        out = torch.zeros(m.nx * m.ny, dtype=torch.uint8, device=dev)
        before, _ = state_from_gpu(m, *m.info())
        m.clear_visibility(*_dev(dev, *f1.numpy()), f1.pose, f1.t_ms + 2000, out_cleared=out)
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy(), m.state_numpy()))
        if ubf:
            p = O.Params.from_dict(params)
            ub0 = np.full((p.ny, p.nx), np.inf, F32)
            exp = O.upper_bound(p, before, ub0, *f1.numpy(), f1.pose)
            assert np.array_equal(_bits(m.upper_bound().cpu().numpy()), _bits(exp))
            _say(f"scene: {int(np.isfinite(exp).sum())} cells bounded")
        m.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    for k in ("h", "v", "valid", "t_upd"):
        assert np.array_equal(outs[0][1][k], outs[1][1][k])


# --------------------------------------------------------- overlap clearance
@pytest.mark.parametrize("seed", range(3))
def test_overlap_clear(dev, seed):
    _say("overlap", seed)
    rng = np.random.default_rng(400 + seed)
    params = dict(nx=97 + seed * 40, ny=61 + seed * 20, resolution=0.07, noise_alpha=0.01)
    p = O.Params.from_dict(params)
    m = _map(params, dev, cx=3.1, cy=-1.2)
    st = random_state(p, rng, valid_frac=0.8, cgx=m.info()[0], cgy=m.info()[1])
    st.h[:] = rng.uniform(-1.5, 3.0, st.h.shape).astype(F32)
    load_state(m, st)
    robot = (3.1 + rng.uniform(-1, 1), -1.2 + rng.uniform(-1, 1), rng.uniform(0, 1))
    R, thr = 1.2 + seed, 0.7
    out = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
    m.overlap_clear(robot, R, thr, out_cleared=out)
    torch.cuda.synchronize()
    marks = O.overlap_clear(p, st, robot, R, thr)
    got = out.cpu().numpy().reshape(p.ny, p.nx).astype(bool)
    assert np.array_equal(got, marks) and marks.sum() > 20
    g = m.state_numpy()
    exp = O.apply_clear(p, st, marks)
    for k in ("h", "v", "valid", "t_upd"):
        assert np.array_equal(g[k], getattr(exp, k)), k
    m.close()


# ---------------------------------------------------------------- inpainting
@pytest.mark.parametrize("shape,frac", [((7, 5), 0.5), ((90, 130), 0.35), ((300, 257), 0.6),
                                        ((64, 64), 0.0), ((33, 20), 1.0), ((517, 611), 0.45),
                                        ((260, 190), 0.03)])
def test_inpaint_min(dev, shape, frac):
    _say("inpaint", shape, frac)
    ny, nx = shape
    rng = np.random.default_rng(nx * 7 + ny)
    params = dict(nx=nx, ny=ny, resolution=0.1)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=frac)
    # blobs of empty cells on top of the scattered ones
    for _ in range(4):
        cy, cx = rng.integers(0, ny), rng.integers(0, nx)
        st.valid[max(cy - 6, 0):cy + 6, max(cx - 9, 0):cx + 9] = 0
    if frac == 1.0:
        st.valid[:] = 1
    load_state(m, st)
    out = m.inpaint_min()
    torch.cuda.synchronize()
    exp = O.inpaint_min(st.h, st.valid)
    g = out.cpu().numpy()
    assert np.array_equal(np.isnan(g), np.isnan(exp))
    assert np.array_equal(_bits(g)[~np.isnan(g)], _bits(exp)[~np.isnan(exp)])
    # the map itself is unchanged
    assert np.array_equal(m.state_numpy()["h"], st.h)
    m.close()


def test_inpaint_on_the_scene(dev):
    _say("inpaint on the small scene")
    d = synth.cfg0(n_frames=1)
    m = _map(d["params"], dev)
    f = d["frames"][0]
    m.fuse_points(*_dev(dev, *f.numpy()), f.pose, f.t_ms)
    g = m.state_numpy()
    out = m.inpaint_min().cpu().numpy()
    exp = O.inpaint_min(g["h"], g["valid"])
    assert (g["valid"] == 0).sum() > 100
    assert np.array_equal(np.isnan(out), np.isnan(exp))
    assert np.array_equal(_bits(out)[~np.isnan(out)], _bits(exp)[~np.isnan(exp)])
    m.close()


# ----------------------------------------------------------------- smoothing
def _smooth_case(dev, x, kind, k, sigma=0.0):
    from paper_2204_12876_amd import smooth
    xd = torch.from_numpy(x).to(dev)
    g = smooth(xd, kind, k, sigma).cpu().numpy()
    torch.cuda.synchronize()
    if kind == "median":
        exp = O.smooth_median(x, k)
        assert np.array_equal(np.isnan(g), np.isnan(exp))
        assert np.array_equal(_bits(g)[~np.isnan(g)], _bits(exp)[~np.isnan(exp)])
        return 0.0
    if kind == "box":
        exp, mag = O.smooth_box(x, k), O.smooth_box(np.abs(x), k)
    else:
        exp = O.smooth_gaussian(x, k, sigma)
        mag = O.smooth_gaussian(np.abs(x), k, sigma)
    assert np.array_equal(np.isnan(g), np.isnan(exp)), "NaN pattern"
    ok = ~np.isnan(exp)
    err = np.abs(g[ok].astype(np.float64) - exp[ok])
    assert np.all(err <= 1e-5 * mag[ok] + 1e-30), f"worst {np.max(err / mag[ok]):.3g}"
    return float(np.max(err / np.maximum(mag[ok], 1e-30), initial=0.0))


@pytest.mark.parametrize("kind,k,sigma", [("box", 1, 0), ("box", 3, 0), ("box", 7, 0),
                                          ("box", 31, 0), ("gaussian", 3, 0.8),
                                          ("gaussian", 9, 2.0), ("gaussian", 31, 6.0),
                                          ("median", 3, 0), ("median", 5, 0)])
@pytest.mark.parametrize("shape", [(37, 23), (16, 100), (129, 70)])
def test_smooth(dev, kind, k, sigma, shape):
    if min(shape) <= k // 2:
        pytest.skip("grid smaller than the radius")
    rng = np.random.default_rng(k * 1000 + shape[0])
    x = rng.normal(1.0, 2.0, shape).astype(F32)
    x[rng.random(shape) < 0.004] = np.nan
    worst = _smooth_case(dev, x, kind, k, sigma)
    _say(f"smooth {kind} k={k} {shape}: worst rel err {worst:.3g}")


def test_smooth_of_an_inpainted_map(dev):
    _say("inpaint then smooth")
    d = synth.cfg0(n_frames=1)
    m = _map(d["params"], dev)
    f = d["frames"][0]
    m.fuse_points(*_dev(dev, *f.numpy()), f.pose, f.t_ms)
    filled = m.inpaint_min().cpu().numpy()
    for kind, k, s in (("median", 5, 0), ("gaussian", 5, 1.0), ("box", 3, 0)):
        _smooth_case(dev, filled, kind, k, s)
    m.close()


def test_filters_reject_bad_arguments(dev):
    from paper_2204_12876_amd import EmxError, smooth
    x = torch.zeros((8, 8), dtype=torch.float32, device=dev)
    for kind, k, s in (("median", 7, 0), ("box", 4, 0), ("gaussian", 3, 0.0), ("box", 33, 0),
                       ("box", 17, 0)):
        with pytest.raises(EmxError):
            smooth(x, kind, k, s)
    with pytest.raises(EmxError):
        smooth(x, "box", 3, out=x)
    m = _map(dict(nx=8, ny=8, resolution=0.1), dev)
    with pytest.raises(EmxError):
        m.upper_bound()
    with pytest.raises(EmxError):
        m.overlap_clear((0, 0, 0), -1.0, 0.5)
    m.close()


def test_features_are_deterministic(dev):
    """Every feature gives the same bits on a second run of the same inputs
    (the upper bound and inpainting use integer atomics, drift a fixed-order
    float64 sum)."""
    from paper_2204_12876_amd import smooth
    _say("feature determinism")
    d = synth.cfg0(n_frames=2)
    params = dict(d["params"], upper_bound=1, wall_min_count=3, time_variance=0.001)
    outs = []
    for _ in range(2):
        m = _map(params, dev)
        w = torch.from_numpy(synth.trav_weights()).to(dev)
        res = []
        for k, f in enumerate(d["frames"]):
            xyz = _dev(dev, *f.numpy())
            mean, cnt = m.compensate_drift(*xyz, f.pose, f.t_ms, 0.0)
            m.move_fuse_points(0.04 * k, -0.04 * k, *xyz, f.pose, f.t_ms)
            m.clear_visibility(*xyz, f.pose, f.t_ms + 600)
            m.normals_traversability(w)
            m.overlap_clear((0.0, 0.0, 0.2), 0.8, 0.3)
            filled = m.inpaint_min()
            res += [mean.cpu(), cnt.cpu(), m.export_state().cpu(), m.upper_bound().cpu().clone(),
                    filled.cpu(), smooth(filled, "gaussian", 5, 1.0).cpu(),
                    smooth(filled, "median", 3).cpu()]
        torch.cuda.synchronize()
        outs.append(res)
        m.close()
    for a, b in zip(*outs):
        assert torch.equal(a.view(torch.uint8) if a.dtype != torch.uint8 else a,
                           b.view(torch.uint8) if b.dtype != torch.uint8 else b)


@pytest.mark.parametrize("ub", [0, 1])
def test_clearing_overflow_list(dev, ub):
    """Rays far longer than the queue's average budget (about 450 samples
    each against 128): whole workgroups of rays overflow their sub-queue and
    are marched from the overflow list.  Marks, state and bound as the oracle."""
    _say("clearing overflow", ub)
    rng = np.random.default_rng(77 + ub)
    params = dict(nx=1000, ny=1000, resolution=0.01, noise_alpha=0.01, gate_k=2.0,
                  min_range=0.05, ray_step=0.01, clear_normal_alpha=0.05, clear_min_age_ms=10,
                  upper_bound=ub)
    p = O.Params.from_dict(params)
    m = _map(params, dev)
    st = random_state(p, rng, valid_frac=0.6)
    st.h[:] = rng.uniform(-0.9, 0.2, st.h.shape).astype(F32)
    load_state(m, st)
    n = 2000
    ang = rng.uniform(0, 2 * np.pi, n)
    rad = rng.uniform(3.5, 4.9, n)
    xs = (rad * np.cos(ang)).astype(F32)
    ys = (rad * np.sin(ang)).astype(F32)
    zs = rng.uniform(-1.9, -1.2, n).astype(F32)
    pose = _pose((0.0, 0.0, 1.0))
    ub0 = np.full((p.ny, p.nx), np.inf, F32)
    new_ub, cleared = _clear_with_bound(m, p, st, ub0, xs, ys, zs, pose, 1000, dev) if ub else \
        (None, None)
    if not ub:
        out = torch.full((p.nx * p.ny,), 9, dtype=torch.uint8, device=dev)
        m.clear_visibility(*_dev(dev, xs, ys, zs), pose, 1000, out_cleared=out)
        torch.cuda.synchronize()
        marks = O.clear_visibility(p, st, xs, ys, zs, pose, 1000)
        assert np.array_equal(out.cpu().numpy().reshape(p.ny, p.nx).astype(bool), marks)
        cleared = int(marks.sum())
    else:
        marks = O.clear_visibility(p, st, xs, ys, zs, pose, 1000)
    g = m.state_numpy()
    exp = O.apply_clear(p, st, marks)
    for k in ("h", "v", "valid", "t_upd"):
        assert np.array_equal(g[k], getattr(exp, k)), k
    assert cleared > 50
    _say(f"overflow clearing: {cleared} cells removed")
    m.close()
