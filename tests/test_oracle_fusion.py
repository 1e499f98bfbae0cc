"""Pins of the CPU oracle's fusion against the paper and against mathematics.

Every check compares the oracle with something other than itself:
  * values worked by hand from Eq. 1 and 2 (golden fixture);
  * the textbook scalar Kalman gain form;
  * closed forms for noiseless planes;
  * exact float32 boundary cases;
  * invariants.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32


def _state(p, cx=0.0, cy=0.0):
    return O.init_map(p, cx, cy, 0)


def _pose(R=None, t=(0.0, 0.0, 0.0)):
    P = np.zeros((3, 4))
    P[:, :3] = np.eye(3) if R is None else R
    P[:, 3] = t
    return P


# ---------------------------------------------------------------- golden (Eq. 1, 2)
@pytest.mark.parametrize("case", ["gate_k_large", "gate_k_1"])
def test_hand_worked_kalman_example(case):
    g = json.load(open(os.path.join(GOLD, "kalman_three_points.json")))
    m = g["map"]
    p = O.Params(nx=m["nx"], ny=m["ny"], resolution=m["resolution"], noise_alpha=g["noise_alpha"],
                 gate_k=g[case]["gate_k"], min_range=0.01)
    st = _state(p, m["cx"], m["cy"])
    st.h[:] = g["prior"]["h"]
    st.v[:] = g["prior"]["v"]
    pts = np.array(g["points_sensor"], F32)
    P = np.array(g["pose"], float)
    r = O.fuse(p, st, pts[:, 0], pts[:, 1], pts[:, 2], P, t_ms=10)
    ix, iy = g["cell"]
    assert list(r.accept) == g[case]["accept"]
    assert set(r.cell[r.accept].tolist()) == {iy * p.nx + ix}
    assert r.h[iy, ix] == pytest.approx(g[case]["h"], rel=1e-14, abs=1e-15)
    assert r.v[iy, ix] == pytest.approx(g[case]["v"], rel=1e-14)
    hs, vs = O.fuse_sequential(p, st, pts[:, 0], pts[:, 1], pts[:, 2], P)
    assert hs[iy, ix] == pytest.approx(g[case]["h"], rel=1e-14, abs=1e-15)
    assert vs[iy, ix] == pytest.approx(g[case]["v"], rel=1e-14)
    # every other cell untouched
    mask = np.ones((p.ny, p.nx), bool)
    mask[iy, ix] = False
    assert np.array_equal(r.state.h[mask], st.h[mask])
    assert np.array_equal(r.state.v[mask], st.v[mask])
    assert r.state.valid[iy, ix] == 1 and r.state.t_upd[iy, ix] == 10
    if case == "gate_k_large":
        # intermediate values of the sequential update, point by point
        for k, (he, ve) in enumerate(g["sequential"]):
            hk, vk = O.fuse_sequential(p, st, pts[:k + 1, 0], pts[:k + 1, 1], pts[:k + 1, 2], P)
            assert hk[iy, ix] == pytest.approx(he, rel=1e-14)
            assert vk[iy, ix] == pytest.approx(ve, rel=1e-14)


# ------------------------------------------------ information form == sequential Eq. 1/2
@pytest.mark.parametrize("seed", range(6))
def test_information_form_equals_sequential_kalman(seed):
    rng = np.random.default_rng(seed)
    p = O.Params(nx=6, ny=5, resolution=0.5, noise_alpha=0.01, gate_k=1.0, min_range=0.05)
    st = _state(p)
    st.h[:] = rng.uniform(-0.5, 0.5, st.h.shape).astype(F32)
    st.v[:] = rng.uniform(0.01, 0.5, st.v.shape).astype(F32)
    n = 60
    # points clustered in a few cells so that cells receive several updates
    P = _pose(t=(0.1, -0.2, 1.0))
    xs = rng.uniform(-1.6, 1.4, n).astype(F32)
    ys = rng.uniform(-1.0, 1.2, n).astype(F32)
    zs = (rng.uniform(-1.6, -0.4, n)).astype(F32)
    r = O.fuse(p, st, xs, ys, zs, P, 5)
    hs, vs = O.fuse_sequential(p, st, xs, ys, zs, P)
    assert r.accept.sum() > 10 and (~r.accept & (r.cell >= 0)).sum() > 0
    assert np.allclose(r.v, vs, rtol=1e-12, atol=0)
    assert np.allclose(r.h, hs, rtol=1e-12, atol=1e-13)


# ------------------------------------------------------------ textbook scalar Kalman
@pytest.mark.parametrize("seed", range(5))
def test_single_point_is_textbook_kalman(seed):
    rng = np.random.default_rng(100 + seed)
    p = O.Params(nx=8, ny=8, resolution=0.25, noise_alpha=float(rng.uniform(1e-3, 1e-1)),
                 gate_k=1e6, min_range=0.01)
    st = _state(p)
    h0 = F32(rng.uniform(-1, 1))
    v0 = F32(rng.uniform(0.05, 2.0))
    st.h[:] = h0
    st.v[:] = v0
    xs, ys, zs = (np.array([rng.uniform(-0.4, 0.4)], F32) for _ in range(3))
    P = _pose(t=(0.0, 0.0, 0.8))
    r = O.fuse(p, st, xs, ys, zs, P, 1)
    (c,) = r.cell
    iy, ix = divmod(int(c), p.nx)
    z = float(np.float64(zs[0]) + np.float64(F32(0.8)))   # translation is carried in float32
    x64, y64, z64 = float(xs[0]), float(ys[0]), float(zs[0])
    s2 = float(np.float64(F32(p.noise_alpha))) * (x64 ** 2 + y64 ** 2 + z64 ** 2)
    gain = float(v0) / (float(v0) + s2)
    assert r.h[iy, ix] == pytest.approx(float(h0) + gain * (z - float(h0)), rel=1e-13, abs=1e-15)
    assert r.v[iy, ix] == pytest.approx((1 - gain) * float(v0), rel=1e-13)


# ------------------------------------------------------------- noiseless plane
def test_noiseless_plane_closed_form():
    """n points at equal range d on the plane z = c fall in one cell:
    v1 = 1/(1/v0 + n/(alpha d^2)) and h1 = c (1 - v1/v0) for h0 = 0."""
    p = O.Params(nx=4, ny=4, resolution=16.0, noise_alpha=0.01, gate_k=1e6, min_range=0.01,
                 init_variance=1e3)
    st = _state(p)
    pts = [(3, 4), (4, 3), (-3, 4), (-4, 3), (3, -4), (4, -3), (-3, -4), (-4, -3)]
    xs = np.array([a for a, _ in pts], F32)
    ys = np.array([b for _, b in pts], F32)
    zs = np.full(len(pts), -12.0, F32)          # d^2 = 9 + 16 + 144 = 169
    c = 0.5
    P = _pose(t=(8.0, 8.0, 12.5))
    r = O.fuse(p, st, xs, ys, zs, P, 1)
    assert r.accept.all() and len(set(r.cell.tolist())) == 1
    iy, ix = divmod(int(r.cell[0]), p.nx)
    n = len(pts)
    alpha = float(F32(0.01))
    v1 = 1.0 / (1.0 / 1e3 + n / (alpha * 169.0))
    assert r.v[iy, ix] == pytest.approx(v1, rel=1e-14)
    assert r.h[iy, ix] == pytest.approx(c * (1 - v1 / 1e3), rel=1e-14)
    assert r.v[iy, ix] < 1e3


# ------------------------------------------------------------------ invariants
def _cfg0_small(n=3000, seed=0):
    import synth
    d = synth.cfg0(seed_offset=seed, n_points=n, n_frames=2)
    p = O.Params.from_dict(d["params"])
    return p, d


def test_invariants_variance_never_increases_and_untouched_cells():
    p, d = _cfg0_small()
    st = O.init_map(p, 0.0, 0.0, 0)
    for f in d["frames"]:
        xs, ys, zs = f.numpy()
        r = O.fuse(p, st, xs, ys, zs, f.pose, f.t_ms)
        v0 = st.v.astype(float)
        assert np.all(r.v <= v0)
        assert np.all(r.v[r.updated] < v0[r.updated])
        assert np.array_equal(r.state.h[~r.updated], st.h[~r.updated])
        assert np.array_equal(r.state.v[~r.updated], st.v[~r.updated])
        assert np.array_equal(r.updated, r.n_acc > 0)
        st = r.state
    # the second frame is gated against a real prior: some in-map points rejected
    assert (~r.accept & (r.cell >= 0)).sum() > 0


def test_all_rejected_frame_leaves_state_bitwise():
    p, d = _cfg0_small()
    p.gate_k = 0.0
    st = O.init_map(p, 0.0, 0.0, 0)
    st.h[:] = F32(50.0)
    st.v[:] = F32(0.5)
    f = d["frames"][0]
    xs, ys, zs = f.numpy()
    r = O.fuse(p, st, xs, ys, zs, f.pose, f.t_ms)
    assert not r.accept.any() and (r.cell >= 0).any()
    for a, b in [(r.state.h, st.h), (r.state.v, st.v), (r.state.valid, st.valid),
                 (r.state.t_upd, st.t_upd)]:
        assert np.array_equal(a, b)


def test_permutation_invariance():
    p, d = _cfg0_small(n=2000)
    st = O.init_map(p, 0.0, 0.0, 0)
    f = d["frames"][0]
    xs, ys, zs = f.numpy()
    r1 = O.fuse(p, st, xs, ys, zs, f.pose, 0)
    perm = np.random.default_rng(3).permutation(len(xs))
    r2 = O.fuse(p, st, xs[perm], ys[perm], zs[perm], f.pose, 0)
    assert np.array_equal(r1.cell[perm], r2.cell)
    assert np.array_equal(r1.accept[perm], r2.accept)
    assert np.allclose(r1.h, r2.h, rtol=1e-12, atol=1e-14)
    assert np.allclose(r1.v, r2.v, rtol=1e-12, atol=0)


# -------------------------------------------------------------- binning / transform
def test_binning_identity_pose_cell_centres_and_ties():
    p = O.Params(nx=8, ny=6, resolution=0.5, min_range=0.01, gate_k=1e6)
    st = _state(p)              # centre cell 0 -> local origin (-2, -1.5)
    ix = np.arange(8)
    iy = np.arange(6)
    X, Y = np.meshgrid(ix, iy)
    # cell centres, sensor at world (0, 0, 1)
    xs = ((X.ravel() + 0.5) * 0.5 - 2.0).astype(F32)
    ys = ((Y.ravel() + 0.5) * 0.5 - 1.5).astype(F32)
    zs = np.full(xs.shape, -1.0, F32)
    dd = O.point_decisions(p, st, xs, ys, zs, _pose(t=(0, 0, 1)))
    assert np.array_equal(dd["cell"], Y.ravel() * 8 + X.ravel())
    # ties: a point on a cell boundary belongs to the higher cell; the upper map
    # edge is outside, the lower edge inside
    below_top = np.nextafter(F32(4.0), F32(0.0)) - F32(2.0)   # local x = 4 - ulp
    xs = np.array([-2.0, -1.5, 2.0, below_top, -2.0000002], F32)
    ys = np.zeros(5, F32)
    dd = O.point_decisions(p, st, xs, ys, np.full(5, -1.0, F32), _pose(t=(0, 0, 1)))
    assert dd["cell"].tolist() == [3 * 8 + 0, 3 * 8 + 1, -1, 3 * 8 + 7, -1]


def test_binning_quarter_turn_yaw_is_exact():
    p = O.Params(nx=10, ny=10, resolution=1.0, min_range=0.01, gate_k=1e6)
    st = _state(p)              # local origin (-5, -5)
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    xs = np.array([0.5, 2.5, -3.5, 4.5], F32)
    ys = np.array([1.5, -2.5, 0.5, 4.0], F32)
    zs = np.full(4, -1.0, F32)
    dd = O.point_decisions(p, st, xs, ys, zs, _pose(R, (0.0, 0.0, 1.0)))
    wx, wy = -ys, xs            # world = R @ sensor
    exp = [int(math.floor(b + 5)) * 10 + int(math.floor(a + 5)) for a, b in zip(wx, wy)]
    assert dd["cell"].tolist() == exp


def test_range_filter_and_non_finite_points_dropped():
    p = O.Params(nx=8, ny=8, resolution=0.5, min_range=0.5)
    st = _state(p)
    xs = np.array([0.1, 0.5, np.nan, np.inf, 0.3, 0.0], F32)
    ys = np.array([0.1, 0.0, 0.0, 0.0, 0.4, 0.0], F32)
    zs = np.array([0.1, 0.0, -1.0, -1.0, 0.0, -0.5], F32)
    dd = O.point_decisions(p, st, xs, ys, zs, _pose(t=(0, 0, 1)))
    # d2 = 0.03 < 0.25 dropped; 0.25 kept (>=); NaN, inf dropped; 0.25 kept; 0.25 kept
    assert dd["valid"].tolist() == [False, True, False, False, True, True]
    assert (dd["cell"][~dd["valid"]] == -1).all()


# -------------------------------------------------------------- gate boundary
def _gate_case(v0, k=1.0):
    p = O.Params(nx=4, ny=4, resolution=1.0, noise_alpha=0.25, gate_k=k, min_range=0.01)
    st = _state(p)
    st.h[:] = F32(0.0)
    st.v[:] = v0
    # sensor frame (0, 0, -2): d^2 = 4, sp2 = 1; map z = 4 - 2 = 2, e = 2, e^2 = 4
    dd = O.point_decisions(p, st, np.zeros(1, F32), np.zeros(1, F32), np.full(1, -2.0, F32),
                           _pose(t=(0.0, 0.0, 4.0)))
    return bool(dd["accept"][0])


def test_gate_boundary_is_inclusive():
    assert _gate_case(F32(3.0))                                 # 4 <= 1*(3+1)
    assert not _gate_case(np.nextafter(F32(3.0), F32(0.0)))     # 4 > 3.9999998
    assert _gate_case(F32(3.0), k=1e18)                         # k -> inf accepts
    assert not _gate_case(F32(3.0), k=0.0)                      # k = 0: only e = 0


def test_gate_k0_accepts_exact_match_only():
    p = O.Params(nx=4, ny=4, resolution=1.0, noise_alpha=0.25, gate_k=0.0, min_range=0.01)
    st = _state(p)
    st.h[:] = F32(2.0)
    dd = O.point_decisions(p, st, np.zeros(2, F32), np.zeros(2, F32),
                           np.array([-2.0, -1.0], F32), _pose(t=(0.0, 0.0, 4.0)))
    assert dd["accept"].tolist() == [True, False]
