"""Oracle pins for the rest of the height-update extensions (Sec. II-C):
the exclusion area (ramp) and the outlier variance.

The paper gives the exclusion area only by its parameters theta_a, b, c, d
and a figure that is not in the text, and says that the outlier check
increases the cell's variance without an amount.  Both are therefore pinned
on the stated reading (parity against the paper itself is unpinned):
  * ramp: around the sensor origin o, a point whose height above o exceeds
    the line b (horizontal distance rho <= c), b + tan(theta_a) (rho - c)
    beyond, at most d, is ignored.  Hand-built points on, just above and just
    below the line in each of its three parts; the rule off equals the
    default; ignoring means the same as leaving the points out of the frame
    (also for the wall rule's counts); raising b, d or theta_a, or lowering c,
    never ignores more points.
  * outlier variance: sigma_o^2 is added once per call to each cell that holds
    an estimate and receives at least one gate-rejected point, after the
    fusion and the time variance.  Hand-built cells with only rejected,
    rejected and accepted, only accepted, and many rejected points; invalid
    cells, wall-rule and ramp points do not count.
"""
import dataclasses
import math

import numpy as np

import oracle as O

F32 = np.float32


def _pose(t):
    P = np.zeros((3, 4))
    P[:, :3] = np.eye(3)
    P[:, 3] = t
    return P


# A 4 m x 4 m map at 0.1 m centred on the world origin; the sensor at
# (0, 0, 0.5), unrotated, so map-local x = xs + 2, y = ys + 2, z = zs + 0.5.
def _ramp_params(**kw):
    base = dict(nx=40, ny=40, resolution=0.1, noise_alpha=1e-4, gate_k=3.0, min_range=0.05,
                excl_on=1, excl_theta=math.pi / 4, excl_b=0.25, excl_c=1.0, excl_d=1.5)
    base.update(kw)
    return O.Params.from_dict(base)


POSE = _pose((0.0, 0.0, 0.5))


def test_ramp_slope_of_45_degrees_is_one():
    assert O.f32_constants(_ramp_params())["excl_slope"] == F32(1.0)


def test_ramp_hand_cases():
    p = _ramp_params()
    st = O.init_map(p, 0.0, 0.0, 0)   # prior variance 1e3: the gate takes every point
    # (xs, ys, zs, excluded): on the line (kept), above it, below it
    cases = [
        # rho = 0.5 <= c: the line is b = 0.25
        (0.5, 0.0, 0.25, False), (0.5, 0.0, 0.3, True), (0.5, 0.0, 0.2, False),
        (-0.5, 0.0, 0.26, True), (0.0, 0.5, 0.25, False), (0.0, -0.5, 0.3, True),
        # rho = 1.5: on the ramp, 0.25 + 1 * (1.5 - 1) = 0.75
        (1.5, 0.0, 0.75, False), (1.5, 0.0, 0.8, True), (1.5, 0.0, 0.7, False),
        (0.0, -1.5, 0.76, True),
        # rho = 1.75: 0.25 + 0.75 = 1.0
        (-1.75, 0.0, 1.0, False), (-1.75, 0.0, 1.05, True),
        # rho ~ 2.34: capped at d = 1.5
        (1.5, 1.8, 1.5, False), (1.5, 1.8, 1.6, True), (-1.5, -1.8, 1.4, False),
        # below the sensor: never
        (1.0, 1.0, -0.3, False), (0.1, 0.0, -0.45, False),
    ]
    xs = np.array([c[0] for c in cases], F32)
    ys = np.array([c[1] for c in cases], F32)
    zs = np.array([c[2] for c in cases], F32)
    want = np.array([c[3] for c in cases])
    d = O.point_decisions(p, st, xs, ys, zs, POSE)
    assert np.all(d["cell"] >= 0)
    assert np.array_equal(d["excluded"], want)
    assert np.array_equal(d["accept"], ~want)
    assert not d["rejected"].any()
    # out of the map: never excluded (and never accepted)
    d2 = O.point_decisions(p, st, np.array([2.5], F32), np.array([0.0], F32),
                           np.array([3.0], F32), POSE)
    assert d2["cell"][0] == -1 and not d2["excluded"][0] and not d2["accept"][0]


def test_ramp_around_the_sensor_not_the_map():
    # the same cases with the sensor moved by (0.6, -0.4) in the world (and
    # the points with it) give the same decisions
    p = _ramp_params()
    st = O.init_map(p, 0.0, 0.0, 0)
    xs = np.array([0.5, 0.5, 0.0, 0.0], F32)
    ys = np.array([0.0, 0.0, 1.5, 1.5], F32)
    zs = np.array([0.24, 0.26, 0.74, 0.76], F32)
    d = O.point_decisions(p, st, xs, ys, zs, _pose((0.6, -0.4, 0.5)))
    assert np.all(d["cell"] >= 0)
    assert np.array_equal(d["excluded"], [False, True, False, True])


def _cloud(rng, n):
    xs = rng.uniform(-1.95, 1.95, n).astype(F32)
    ys = rng.uniform(-1.95, 1.95, n).astype(F32)
    zs = rng.uniform(-0.5, 2.0, n).astype(F32)
    return xs, ys, zs


def _state(p, rng, valid_frac=0.7):
    st = O.init_map(p, 0.0, 0.0, 0)
    shp = (p.ny, p.nx)
    st.h[:] = rng.uniform(-0.3, 0.8, shp).astype(F32)
    st.v[:] = rng.uniform(0.5, 2.0, shp).astype(F32)
    st.valid[:] = (rng.random(shp) < valid_frac).astype(np.uint8)
    return st


def _same_state(a, b):
    for k in ("h", "v", "t_upd", "valid"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


def test_ramp_off_is_the_default():
    rng = np.random.default_rng(3)
    p = _ramp_params(excl_on=0)
    st = _state(p, rng)
    xs, ys, zs = _cloud(rng, 3000)
    plain = dataclasses.replace(p, excl_theta=0.0, excl_b=0.0, excl_c=0.0, excl_d=0.0)
    _same_state(O.fuse(p, st, xs, ys, zs, POSE, 10).state,
                O.fuse(plain, st, xs, ys, zs, POSE, 10).state)


def test_ramp_equals_leaving_the_points_out():
    rng = np.random.default_rng(4)
    for wall in (0, 3):
        p = _ramp_params(wall_min_count=wall, gate_k=1e3)
        st = _state(p, rng)
        xs, ys, zs = _cloud(rng, 4000)
        ex = O.point_decisions(p, st, xs, ys, zs, POSE)["excluded"]
        assert 0 < ex.sum() < ex.size
        on = O.fuse(p, st, xs, ys, zs, POSE, 10)
        off = O.fuse(dataclasses.replace(p, excl_on=0), st, xs[~ex], ys[~ex], zs[~ex], POSE, 10)
        _same_state(on.state, off.state)


def test_ramp_never_ignores_more_when_raised():
    # a higher, steeper or higher-capped line, or a ramp that starts nearer
    # the sensor, ignores a subset of the points
    rng = np.random.default_rng(5)
    p = _ramp_params()
    st = _state(p, rng)
    xs, ys, zs = _cloud(rng, 5000)
    base = O.point_decisions(p, st, xs, ys, zs, POSE)["excluded"]
    assert 0 < base.sum() < base.size
    for kw in (dict(excl_b=0.5), dict(excl_c=0.5), dict(excl_d=1.8), dict(excl_theta=1.0)):
        fewer = O.point_decisions(dataclasses.replace(p, **kw), st, xs, ys, zs, POSE)["excluded"]
        assert not (fewer & ~base).any(), kw
        assert fewer.sum() < base.sum(), kw


# ------------------------------------------------------------ outlier variance
def _ov_params(**kw):
    base = dict(nx=8, ny=8, resolution=0.5, noise_alpha=1e-4, gate_k=3.0, min_range=0.05,
                outlier_variance=0.125)
    base.update(kw)
    return O.Params.from_dict(base)


def _pt(ix, iy, z):
    # sensor frame point over cell (ix, iy) centre; map-local = sensor + (2, 2, 1)
    return (ix + 0.5) * 0.5 - 2.0, (iy + 0.5) * 0.5 - 2.0, z - 1.0


def _ov_scene():
    p = _ov_params()
    st = O.init_map(p, 0.0, 0.0, 0)
    st.h[:] = F32(0.2)
    st.v[:] = F32(1e-4)
    st.valid[:] = 1
    st.valid[0, 7] = 0          # cell (7, 0) has no estimate
    pts = [
        _pt(1, 1, 3.0),                                  # A: rejected only
        _pt(2, 1, 0.2), _pt(2, 1, 5.0),                  # B: accepted and rejected
        _pt(3, 1, 0.21), _pt(3, 1, 0.19),                # C: accepted only
        *[_pt(4, 1, 2.0 + k) for k in range(5)],          # E: five rejected
        _pt(7, 0, 500.0),                                # F: rejected, invalid cell
    ]
    xs, ys, zs = (np.array(c, F32) for c in zip(*pts))
    return p, st, xs, ys, zs, _pose((0.0, 0.0, 1.0))


def test_outlier_variance_hand_cases():
    p, st, xs, ys, zs, pose = _ov_scene()
    d = O.point_decisions(p, st, xs, ys, zs, pose)
    assert np.array_equal(d["rejected"], [1, 0, 1, 0, 0, 1, 1, 1, 1, 1, 1])
    on = O.fuse(p, st, xs, ys, zs, pose, 10).state
    off = O.fuse(dataclasses.replace(p, outlier_variance=0.0), st, xs, ys, zs, pose, 10).state
    vo = F32(0.125)
    # A: only rejected points: the prior plus sigma_o^2, nothing else changes
    assert on.v[1, 1] == st.v[1, 1] + vo and on.h[1, 1] == st.h[1, 1]
    assert on.t_upd[1, 1] == st.t_upd[1, 1]
    # B: the fused variance plus sigma_o^2; the height is the fused one
    assert off.v[1, 2] < st.v[1, 2]
    assert on.v[1, 2] == off.v[1, 2] + vo and on.h[1, 2] == off.h[1, 2]
    # C: nothing rejected
    assert on.v[1, 3] == off.v[1, 3]
    # E: five rejected points inflate once
    assert on.v[1, 4] == st.v[1, 4] + vo
    # F: no estimate, no inflation
    assert on.v[0, 7] == st.v[0, 7]
    # every other cell as without the rule
    other = np.ones((8, 8), bool)
    other[1, 1] = other[1, 2] = other[1, 4] = False
    assert np.array_equal(on.v[other], off.v[other])
    assert np.array_equal(on.h, off.h)


def test_outlier_variance_after_time_variance():
    p, st, xs, ys, zs, pose = _ov_scene()
    p = dataclasses.replace(p, time_variance=0.0625)
    on = O.fuse(p, st, xs, ys, zs, pose, 10).state
    assert on.v[1, 1] == (st.v[1, 1] + F32(0.0625)) + F32(0.125)
    assert on.v[5, 5] == st.v[5, 5] + F32(0.0625)        # untouched valid cell


def test_outlier_variance_off_is_the_default():
    p, st, xs, ys, zs, pose = _ov_scene()
    base = O.Params.from_dict({f.name: getattr(p, f.name) for f in dataclasses.fields(p)
                               if f.name != "outlier_variance"})
    _same_state(O.fuse(dataclasses.replace(p, outlier_variance=0.0), st, xs, ys, zs, pose, 10)
                .state, O.fuse(base, st, xs, ys, zs, pose, 10).state)


def test_outlier_variance_ignores_wall_and_ramp_points():
    # a crowded cell whose points lie far below its estimate: the wall rule
    # ignores them, so the gate never sees them and nothing inflates
    p, st, _, _, _, pose = _ov_scene()
    pts = [_pt(5, 5, -3.0 - 0.1 * k) for k in range(6)]
    xs, ys, zs = (np.array(c, F32) for c in zip(*pts))
    d0 = O.point_decisions(p, st, xs, ys, zs, pose)
    assert d0["rejected"].all()
    pw = dataclasses.replace(p, wall_min_count=3)
    dw = O.point_decisions(pw, st, xs, ys, zs, pose)
    assert dw["walled"].all() and not dw["rejected"].any()
    assert O.fuse(pw, st, xs, ys, zs, pose, 10).state.v[5, 5] == st.v[5, 5]
    # points high above the sensor: the ramp ignores them
    pts = [_pt(5, 5, 9.0 + 0.1 * k) for k in range(3)]
    xs, ys, zs = (np.array(c, F32) for c in zip(*pts))
    pr = dataclasses.replace(p, excl_on=1, excl_theta=0.3, excl_b=0.5, excl_c=0.5, excl_d=2.0)
    dr = O.point_decisions(pr, st, xs, ys, zs, pose)
    assert dr["excluded"].all() and not dr["rejected"].any()
    assert O.fuse(pr, st, xs, ys, zs, pose, 10).state.v[5, 5] == st.v[5, 5]
    assert O.fuse(p, st, xs, ys, zs, pose, 10).state.v[5, 5] == st.v[5, 5] + F32(0.125)
