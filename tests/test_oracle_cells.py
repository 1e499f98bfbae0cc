"""Pins of the oracle's per-cell passes.

Each pass is checked against something other than the oracle itself:
  * clearing against hand-built scenes with known answers (Sec. II-E,
    Eq. 3 and 4);
  * normals against exact planes (Sec. II-A);
  * traversability against torch.nn.functional.conv2d in float64 (Sec. II-G);
  * move_map against shift identities.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O

F32 = np.float32


def _pose(t, R=None):
    P = np.zeros((3, 4))
    P[:, :3] = np.eye(3) if R is None else R
    P[:, 3] = t
    return P


# ----------------------------------------------------------------- clearing scenes
# 16x16 map at r = 1 centred on world (0, 0): local = world + 8.  Sensor at local
# (1.5, 8.5, 2.0).  The point at local (12.5, 8.5, 0.0) gives d = (11, 0, -2) and
# K = 11.  Samples k = 1..10 sit at local x = 1.5 + k, cells ix = 2..11, with
# z = 2 - 2k/11.  Cell (6, 8) is sampled at k = 5, z = 1.0909.
def _scene(**kw):
    p = O.Params(nx=16, ny=16, resolution=1.0, ray_step=1.0, clear_normal_alpha=0.3,
                 clear_min_age_ms=500, min_range=0.05)
    st = O.init_map(p, 0.0, 0.0, 0)
    pose = _pose((1.5 - 8.0, 8.5 - 8.0, 2.0))
    pt = (np.array([11.0], F32), np.array([0.0], F32), np.array([-2.0], F32))
    return p, st, pose, pt


def _ghost(st, ix, iy, h=1.5, v=0.01, t_upd=0, n=(-1.0, 0.0, 0.0)):
    st.h[iy, ix] = h
    st.v[iy, ix] = v
    st.valid[iy, ix] = 1
    st.t_upd[iy, ix] = t_upd
    st.nrm[:, iy, ix] = n


def test_clear_ghost_cell_below_ray_is_removed():
    p, st, pose, pt = _scene()
    _ghost(st, 6, 8)
    m = O.clear_visibility(p, st, *pt, pose, t_ms=1000)
    assert m.sum() == 1 and m[8, 6]
    st2 = O.apply_clear(p, st, m)
    assert st2.valid[8, 6] == 0 and st2.h[8, 6] == F32(0.0) and st2.v[8, 6] == F32(1e3)
    # idempotent: the removed cell is invalid, so a second pass marks nothing
    assert not O.clear_visibility(p, st2, *pt, pose, t_ms=1000).any()


def test_clear_recent_cell_kept():
    p, st, pose, pt = _scene()
    _ghost(st, 6, 8, t_upd=800)                    # age 200 <= 500
    assert not O.clear_visibility(p, st, *pt, pose, t_ms=1000).any()
    assert O.clear_visibility(p, st, *pt, pose, t_ms=1301).any()    # age 501 > 500
    assert not O.clear_visibility(p, st, *pt, pose, t_ms=1300).any()


def test_clear_ray_above_cell_kept():
    p, st, pose, pt = _scene()
    _ghost(st, 6, 8, h=0.5)                         # ray at z = 1.09 passes above
    assert not O.clear_visibility(p, st, *pt, pose, t_ms=1000).any()


def test_clear_eq3_uses_standard_deviation():
    p, st, pose, pt = _scene()
    zq = F32(2.0) + F32(F32(5) / F32(11)) * F32(-2.0)   # sample height at k = 5
    _ghost(st, 6, 8, h=float(zq + F32(0.25)), v=0.0625)  # hd = 0.25 = sigma: not below
    assert not O.clear_visibility(p, st, *pt, pose, t_ms=1000).any()
    _ghost(st, 6, 8, h=float(zq + F32(0.25)), v=0.0624)
    assert O.clear_visibility(p, st, *pt, pose, t_ms=1000).any()


def test_clear_normal_condition():
    p, st, pose, pt = _scene()
    _ghost(st, 6, 8, n=(0.0, 1.0, 0.0))             # normal perpendicular to the ray
    assert not O.clear_visibility(p, st, *pt, pose, t_ms=1000).any()
    _ghost(st, 6, 8, n=(0.0, 0.0, 1.0))             # (r.n)^2 = 4 < 0.09 * 125
    assert not O.clear_visibility(p, st, *pt, pose, t_ms=1000).any()
    _ghost(st, 6, 8, n=(np.nan, np.nan, np.nan))    # no normal yet
    assert not O.clear_visibility(p, st, *pt, pose, t_ms=1000).any()
    _ghost(st, 6, 8, n=(0.6, 0.0, 0.8))             # (6.6 - 1.6)^2 = 25 > 11.25
    assert O.clear_visibility(p, st, *pt, pose, t_ms=1000).any()


def test_clear_sample_set_excludes_sensor_and_end_cells():
    p, st, pose, pt = _scene()
    for ix in range(16):
        _ghost(st, ix, 8, h=5.0)
    m = O.clear_visibility(p, st, *pt, pose, t_ms=1000)
    assert sorted(np.nonzero(m[8])[0].tolist()) == list(range(2, 12))
    assert m.sum() == 10
    # an end point outside the map: every in-map sample counts, no end cell
    far = (np.array([19.0], F32), np.array([0.0], F32), np.array([-2.0], F32))
    m = O.clear_visibility(p, st, *far, pose, t_ms=1000)
    assert sorted(np.nonzero(m[8])[0].tolist()) == list(range(2, 16))
    # a vertical ray has no samples
    down = (np.array([0.0], F32), np.array([0.0], F32), np.array([-2.0], F32))
    assert not O.clear_visibility(p, st, *down, pose, t_ms=1000).any()


def test_clear_brute_force_tiny_map():
    """Random rays on a 6x6 map against a sample-by-sample Python loop."""
    rng = np.random.default_rng(7)
    p = O.Params(nx=6, ny=6, resolution=0.5, ray_step=0.3, clear_normal_alpha=0.2,
                 clear_min_age_ms=100, min_range=0.05)
    st = O.init_map(p, 0.0, 0.0, 0)
    st.valid[:] = (rng.random((6, 6)) < 0.8).astype(np.uint8)
    st.h[:] = rng.uniform(-0.5, 1.5, (6, 6)).astype(F32)
    st.v[:] = rng.uniform(0.0, 0.05, (6, 6)).astype(F32)
    st.t_upd[:] = rng.integers(0, 400, (6, 6)).astype(np.int32)
    n = rng.normal(size=(3, 6, 6))
    st.nrm[:] = (n / np.linalg.norm(n, axis=0)).astype(F32)
    pose = _pose((0.1, -0.2, 1.2))
    xs = rng.uniform(-2, 2, 40).astype(F32)
    ys = rng.uniform(-2, 2, 40).astype(F32)
    zs = rng.uniform(-2, 0.5, 40).astype(F32)
    m = O.clear_visibility(p, st, xs, ys, zs, pose, t_ms=500)
    # independent transcription, one sample at a time, float32 scalars
    ox, oy = F32(0.1 + 1.5), F32(-0.2 + 1.5)
    oz = F32(1.2)
    inv_r = F32(2.0)
    inv_step = F32(1.0 / float(F32(0.3)))
    an2 = F32(float(F32(0.2)) ** 2)
    exp = np.zeros((6, 6), bool)

    def cell(qx, qy):
        fx, fy = qx * inv_r, qy * inv_r
        if not (F32(0) <= fx < F32(6) and F32(0) <= fy < F32(6)):
            return None
        return int(math.floor(fy)), int(math.floor(fx))

    for i in range(40):
        x, y, z = xs[i], ys[i], zs[i]
        xm, ym, zm = x + ox, y + oy, z + oz
        dx, dy, dz = xm - ox, ym - oy, zm - oz
        K = int(math.ceil(max(abs(dx), abs(dy)) * inv_step))
        end = cell(xm, ym)
        for k in range(1, K):
            t = F32(k) / F32(K)
            qx, qy, qz = ox + t * dx, oy + t * dy, oz + t * dz
            c = cell(qx, qy)
            if c is None or c == end:
                continue
            iy, ix = c
            hd = st.h[iy, ix] - qz
            nn = st.nrm[:, iy, ix]
            dot = (dx * nn[0] + dy * nn[1]) + dz * nn[2]
            dd = (dx * dx + dy * dy) + dz * dz
            if (st.valid[iy, ix] and 500 - int(st.t_upd[iy, ix]) > 100 and hd > 0
                    and hd * hd > st.v[iy, ix] and dot * dot > an2 * dd):
                exp[iy, ix] = True
    assert exp.any()
    assert np.array_equal(m, exp)


# ---------------------------------------------------------------------- normals
def test_normals_exact_on_planes():
    p = O.Params(nx=9, ny=7, resolution=0.5)
    a, b, c = 0.25, -0.5, 1.0
    ix = np.arange(9) * 0.5
    iy = np.arange(7) * 0.5
    X, Y = np.meshgrid(ix, iy)
    h = (a * X + b * Y + c).astype(F32)
    valid = np.ones((7, 9), np.uint8)
    n = O.compute_normals(p, h, valid)
    s = math.sqrt(1 + a * a + b * b)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(n[0][inner], -a / s, atol=1e-15)
    assert np.allclose(n[1][inner], -b / s, atol=1e-15)
    assert np.allclose(n[2][inner], 1 / s, atol=1e-15)
    assert np.allclose(np.linalg.norm(n[:, 1:-1, 1:-1], axis=0), 1.0, atol=1e-15)
    border = np.ones((7, 9), bool)
    border[inner] = False
    assert np.isnan(n[:, border]).all()


def test_normals_nan_pattern_of_invalid_cell():
    p = O.Params(nx=8, ny=8, resolution=0.1)
    h = np.random.default_rng(0).uniform(-1, 1, (8, 8)).astype(F32)
    valid = np.ones((8, 8), np.uint8)
    valid[4, 3] = 0
    n = O.compute_normals(p, h, valid)
    nanm = np.isnan(n[2])
    exp = np.ones((8, 8), bool)
    exp[1:-1, 1:-1] = False
    exp[3:6, 2:5] = True
    assert np.array_equal(nanm, exp)
    assert (n[2][~nanm] > 0).all()


def test_normals_least_squares_fit_matches_lstsq():
    rng = np.random.default_rng(2)
    p = O.Params(nx=5, ny=5, resolution=0.2)
    h = rng.uniform(-0.3, 0.3, (5, 5)).astype(F32)
    n = O.compute_normals(p, h, np.ones((5, 5), np.uint8))
    iy, ix = 2, 3
    A, z = [], []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            A.append([dx * 0.2, dy * 0.2, 1.0])
            z.append(float(h[iy + dy, ix + dx]))
    (ga, gb, _), *_ = np.linalg.lstsq(np.array(A), np.array(z), rcond=None)
    s = math.sqrt(1 + ga * ga + gb * gb)
    assert np.allclose(n[:, iy, ix], [-ga / s, -gb / s, 1 / s], atol=1e-13)


# ------------------------------------------------------------------ traversability
def _torch_trav(h, w):
    w = torch.as_tensor(w, dtype=torch.float64)
    H = torch.as_tensor(h.astype(np.float64))[None, None]
    a = torch.nn.functional.conv2d(H, w[:72].view(8, 1, 3, 3), w[72:80])
    t = torch.nn.functional.conv2d(torch.relu(a), w[80:88].view(1, 8, 1, 1), w[88:89])
    return t[0, 0].numpy()


def test_traversability_matches_torch_conv2d():
    import synth
    rng = np.random.default_rng(4)
    h = rng.uniform(-0.5, 0.5, (20, 17)).astype(F32)
    w = synth.trav_weights()
    valid = np.ones((20, 17), np.uint8)
    T, S = O.traversability(h, valid, w)
    ref = _torch_trav(h, w)
    assert np.allclose(T[1:-1, 1:-1], ref, rtol=0, atol=1e-13)
    assert np.isnan(T[0]).all() and np.isnan(T[:, -1]).all()
    valid[5, 5] = 0
    T2, _ = O.traversability(h, valid, w)
    assert np.isnan(T2[4:7, 4:7]).all() and np.isfinite(T2[8, 8])


def test_traversability_delta_kernel_and_channel_select():
    rng = np.random.default_rng(5)
    h = rng.uniform(-1, 1, (6, 6)).astype(F32)
    valid = np.ones((6, 6), np.uint8)
    w = np.zeros(89, F32)
    w[72:80] = np.linspace(-0.3, 0.4, 8).astype(F32)
    for ch in range(8):
        w[ch * 9 + 4] = 1.0                          # centre tap: a_c = h + b1_c
    w[80 + 3] = 1.0                                  # select channel 3
    w[88] = 0.125
    T, _ = O.traversability(h, valid, w)
    exp = 0.125 + np.maximum(h.astype(float) + float(w[75]), 0.0)
    assert np.allclose(T[1:-1, 1:-1], exp[1:-1, 1:-1], atol=1e-15)


# ------------------------------------------------------------------------ move_map
def _rand_state(p, seed=0):
    rng = np.random.default_rng(seed)
    st = O.init_map(p, 0.0, 0.0, 0)
    st.h[:] = rng.normal(size=st.h.shape).astype(F32)
    st.v[:] = rng.uniform(0.1, 1, st.h.shape).astype(F32)
    st.valid[:] = 1
    st.t_upd[:] = rng.integers(0, 100, st.h.shape).astype(np.int32)
    st.nrm[:] = rng.normal(size=st.nrm.shape).astype(F32)
    st.trav[:] = rng.normal(size=st.h.shape).astype(F32)
    return st


def _layers(st):
    return [st.h, st.v, st.t_upd, st.valid, st.nrm[0], st.nrm[1], st.nrm[2], st.trav]


def test_move_shift_and_back_keeps_retained_region():
    p = O.Params(nx=12, ny=10, resolution=0.25)
    st = _rand_state(p)
    a = O.move_map(p, st, 3 * 0.25 + 0.1, -2 * 0.25 + 0.1)       # shift (3, -2)
    assert (a.cgx, a.cgy) == (3, -2)
    # new local (ix, iy) = old (ix + 3, iy - 2)
    assert np.array_equal(a.h[2:, :9], st.h[:8, 3:])
    assert (a.valid[:2] == 0).all() and (a.valid[:, 9:] == 0).all()
    assert np.isnan(a.nrm[:, :2]).all() and (a.v[:, 9:] == F32(1e3)).all()
    b = O.move_map(p, a, 0.1, 0.1)
    keep = (slice(0, 8), slice(3, 12))
    for x, y in zip(_layers(b), _layers(st)):
        np.testing.assert_array_equal(x[keep], y[keep])


def test_move_far_resets_everything_and_composes():
    p = O.Params(nx=8, ny=8, resolution=1.0)
    st = _rand_state(p, 1)
    far = O.move_map(p, st, 8.5, 0.5)
    assert (far.valid == 0).all() and (far.h == F32(0)).all()
    ab = O.move_map(p, O.move_map(p, st, 2.5, 1.5), 3.5, -0.5)
    direct = O.move_map(p, st, 3.5, -0.5)
    # cells kept through both steps (valid, since every old cell was valid) agree
    kept = ab.valid == 1
    assert kept.sum() == (8 - 3) * (8 - 2)      # |x| range 3..7 of old, |y| 2..7 via both
    for x, y in zip(_layers(ab), _layers(direct)):
        np.testing.assert_array_equal(x[kept], y[kept])
    assert (direct.valid == 1).sum() == (8 - 3) * (8 - 1)


# ---------------------------------------------------------------------- move_layer
# move_layer carries one extra layer (the upper bound) through the robot-centric
# move.  It is pinned by a per-cell brute force over the move's definition, by
# shift and inverse shift, by a shift past the map side and by agreement with
# move_map on the height layer.
def _brute_move(layer, sx, sy, fill):
    ny, nx = layer.shape
    out = np.empty_like(layer)
    for iy in range(ny):
        for ix in range(nx):
            jx, jy = ix + sx, iy + sy
            inside = 0 <= jx < nx and 0 <= jy < ny
            out[iy, ix] = layer[jy, jx] if inside else fill
    return out


@pytest.mark.parametrize("cx,cy", [(3 * 0.25 + 0.1, -2 * 0.25 + 0.1), (-1.3, 0.6), (0.0, 0.0),
                                   (0.1, -3 * 0.25 + 0.01)])
def test_move_layer_brute_force(cx, cy):
    p = O.Params(nx=9, ny=7, resolution=0.25)
    st = _rand_state(p, 3)
    lay = np.random.default_rng(4).normal(size=(7, 9)).astype(F32)
    sx = math.floor(cx / 0.25) - st.cgx
    sy = math.floor(cy / 0.25) - st.cgy
    out = O.move_layer(p, st, lay, cx, cy, np.inf)
    np.testing.assert_array_equal(out, _brute_move(lay, sx, sy, np.inf))


def test_move_layer_shift_back_far_and_move_map():
    p = O.Params(nx=12, ny=10, resolution=0.25)
    st = _rand_state(p, 5)
    lay = np.random.default_rng(6).normal(size=(10, 12)).astype(F32)
    a = O.move_layer(p, st, lay, 3 * 0.25 + 0.1, -2 * 0.25 + 0.1, np.inf)     # shift (3, -2)
    st_a = O.move_map(p, st, 3 * 0.25 + 0.1, -2 * 0.25 + 0.1)
    b = O.move_layer(p, st_a, a, 0.1, 0.1, np.inf)                           # and back
    keep = (slice(0, 8), slice(3, 12))
    np.testing.assert_array_equal(b[keep], lay[keep])
    assert np.isinf(b[8:]).all() and np.isinf(b[:, :3]).all()
    # a shift of at least the map side leaves only the fill
    assert (O.move_layer(p, st, lay, 12 * 0.25 + 0.1, 0.1, -7.0) == F32(-7.0)).all()
    assert (O.move_layer(p, st, lay, 0.1, -10 * 0.25 + 0.1, -7.0) == F32(-7.0)).all()
    # the height layer with the prior as fill is move_map's height layer
    for cx, cy in [(3 * 0.25 + 0.1, -2 * 0.25 + 0.1), (-0.9, 1.2), (5.0, 5.0)]:
        np.testing.assert_array_equal(O.move_layer(p, st, st.h, cx, cy, F32(0.0)),
                                      O.move_map(p, st, cx, cy).h)
