"""Oracle pins for the height-update extensions and drift compensation
(Sec. II-C: time variance, wall/edge rule; Sec. II-D: drift compensation).

Each extension is pinned against the base fusion (whose own pins are in
test_oracle_fusion) or a closed form, never against its own code path:
  * wall rule: fusing a frame with the rule on equals fusing, with the rule
    off, the frame minus the points the rule removes (those below a valid
    cell's estimate in a cell that receives more than the threshold);
  * time variance: untouched valid cells grow by exactly sigma_t^2 per frame,
    in float32; updated and invalid cells are as without it;
  * drift: a noiseless flat scene gives the known offset; cells below the
    traversability threshold or without one do not contribute.
"""
import dataclasses

import numpy as np

import oracle as O

F32 = np.float32


def _pose(t):
    P = np.zeros((3, 4))
    P[:, :3] = np.eye(3)
    P[:, 3] = t
    return P


def _params(**kw):
    base = dict(nx=10, ny=8, resolution=0.5, noise_alpha=0.01, gate_k=3.0, min_range=0.05)
    base.update(kw)
    return O.Params.from_dict(base)


def _state(p, rng, valid_frac=0.7):
    st = O.init_map(p, 0.0, 0.0, 0)
    shp = (p.ny, p.nx)
    st.h[:] = rng.uniform(-0.3, 0.3, shp).astype(F32)
    st.v[:] = rng.uniform(0.001, 0.05, shp).astype(F32)
    st.valid[:] = (rng.random(shp) < valid_frac).astype(np.uint8)
    return st


def _cloud(rng, n, pose_z=1.5):
    # points in the sensor frame over the whole map (map-local x in [0, 5), y in [0, 4))
    xs = rng.uniform(-2.45, 2.45, n).astype(F32)
    ys = rng.uniform(-1.95, 1.95, n).astype(F32)
    zs = (rng.uniform(-0.4, 0.4, n) - pose_z).astype(F32)
    return xs, ys, zs


# ------------------------------------------------------------------ wall rule
def _removed_by_rule(p, st, xs, ys, zs, pose):
    """The rule's definition written out: per cell, count the valid in-map
    points; in valid cells with more than the threshold, the points whose
    map height is below the cell's estimate are the ones removed."""
    off = dataclasses.replace(p, wall_min_count=0)
    d = O.point_decisions(off, st, xs, ys, zs, pose)
    cell = d["cell"]
    rm = np.zeros(cell.size, bool)
    for c in np.unique(cell[cell >= 0]):
        mine = np.nonzero(cell == c)[0]
        iy, ix = divmod(int(c), p.nx)
        if mine.size > p.wall_min_count and st.valid[iy, ix]:
            rm[mine] = d["zm"][mine] < st.h[iy, ix]
    return rm


def test_wall_rule_equals_fusing_without_the_removed_points():
    rng = np.random.default_rng(1)
    for thr in (1, 3, 8):
        p = _params(wall_min_count=thr, gate_k=1e3)
        st = _state(p, rng)
        xs, ys, zs = _cloud(rng, 600)
        pose = _pose((0.0, 0.0, 1.5))
        rm = _removed_by_rule(p, st, xs, ys, zs, pose)
        assert 0 < rm.sum() < rm.size
        on = O.fuse(p, st, xs, ys, zs, pose, 10)
        off = O.fuse(dataclasses.replace(p, wall_min_count=0), st, xs[~rm], ys[~rm], zs[~rm],
                     pose, 10)
        assert np.array_equal(on.state.h, off.state.h)
        assert np.array_equal(on.state.v, off.state.v)
        assert np.array_equal(on.accept[~rm], off.accept) and not on.accept[rm].any()


def test_wall_rule_counts_before_the_gate_and_needs_an_estimate():
    p = _params(wall_min_count=3, gate_k=1.0, noise_alpha=1e-6)
    st = O.init_map(p, 0.0, 0.0, 0)
    st.h[:] = F32(0.2)
    st.v[:] = F32(1e-4)
    st.valid[:] = 1
    st.valid[0, 1] = 0                          # cell (ix=1, iy=0) holds no estimate
    pose = _pose((0.0, 0.0, 0.0))                 # identity rotation, no height offset:
    # zm equals zs exactly.  Cell (ix=0, iy=0): map-local x, y in [0, 0.5) with
    # the sensor at map-local (2.5, 2.0)
    xs = np.array([-2.3, -2.3, -2.3, -2.3, -2.3], F32)
    ys = np.array([-1.8, -1.8, -1.8, -1.8, -1.8], F32)
    zs = np.array([0.21, 0.2, 0.19, -0.3, 0.9], F32)
    d = O.point_decisions(p, st, xs, ys, zs, pose)
    # five points land (count 5 > 3) although the gate would reject two of them:
    # the rule removes the two below 0.2, the point at 0.2 stays
    assert list(d["walled"]) == [False, False, True, True, False]
    # the same points in the cell without an estimate: no rule
    d2 = O.point_decisions(p, st, xs + F32(0.5), ys, zs, pose)
    assert not d2["walled"].any()
    # three points only: at the threshold, no rule
    d3 = O.point_decisions(p, st, xs[:3], ys[:3], zs[:3], pose)
    assert not d3["walled"].any()


def test_wall_rule_off_is_the_base_fusion():
    rng = np.random.default_rng(2)
    p = _params()
    st = _state(p, rng)
    xs, ys, zs = _cloud(rng, 400)
    a = O.fuse(p, st, xs, ys, zs, _pose((0, 0, 1.5)), 5)
    b = O.fuse(dataclasses.replace(p, wall_min_count=0), st, xs, ys, zs, _pose((0, 0, 1.5)), 5)
    assert np.array_equal(a.state.h, b.state.h) and np.array_equal(a.accept, b.accept)


# -------------------------------------------------------------- time variance
def test_time_variance_grows_untouched_valid_cells_only():
    rng = np.random.default_rng(3)
    p0 = _params()
    p = dataclasses.replace(p0, time_variance=0.003)
    st = _state(p, rng)
    xs, ys, zs = _cloud(rng, 40)                  # leaves many cells untouched
    pose = _pose((0, 0, 1.5))
    a = O.fuse(p, st, xs, ys, zs, pose, 20)
    b = O.fuse(p0, st, xs, ys, zs, pose, 20)
    upd = b.updated
    grow = ~upd & (st.valid == 1)
    assert grow.sum() > 10 and upd.sum() > 5
    assert np.array_equal(a.state.v[grow], st.v[grow] + F32(0.003))
    assert np.array_equal(a.state.v[~grow], b.state.v[~grow])
    assert np.array_equal(a.state.h, b.state.h)


def test_time_variance_accumulates_per_frame():
    rng = np.random.default_rng(4)
    p = _params(time_variance=0.002)
    st = _state(p, rng, valid_frac=1.0)
    v = st.v.copy()
    far = (np.array([100.0], F32), np.array([0.0], F32), np.array([-1.0], F32))  # out of the map
    for k in range(5):
        st = O.fuse(p, st, *far, _pose((0, 0, 1.5)), 10 * (k + 1)).state
        v = v + F32(0.002)
    assert np.array_equal(st.v, v)


# ------------------------------------------------------------------- drift
def _flat_scene(trav_value=1.0):
    p = _params(nx=12, ny=12, resolution=0.25)
    st = O.init_map(p, 0.0, 0.0, 0)
    st.h[:] = F32(0.25)
    st.v[:] = F32(0.01)
    st.valid[:] = 1
    st.trav[:] = F32(trav_value)
    return p, st


def test_drift_closed_form_on_a_flat_scene():
    p, st = _flat_scene()
    rng = np.random.default_rng(5)
    n = 500
    xs = rng.uniform(-1.4, 1.4, n).astype(F32)
    ys = rng.uniform(-1.4, 1.4, n).astype(F32)
    zs = np.full(n, F32(0.375) - F32(1.0), F32)   # every point 0.125 m above the map
    new, mean, used = O.compensate_drift(p, st, xs, ys, zs, _pose((0, 0, 1.0)), 0.5)
    assert used == n and mean == 0.125
    assert np.array_equal(new.h, np.full_like(st.h, F32(0.375)))
    assert np.array_equal(new.v, st.v)


def test_drift_uses_only_flat_valid_cells():
    p, st = _flat_scene()
    st.trav[:, :6] = F32(0.1)                      # left half: not flat enough
    st.trav[0, 6:] = np.nan                        # one row without traversability
    st.valid[11, 11] = 0
    st.h[11, 11] = F32(-5.0)
    rng = np.random.default_rng(6)
    n = 2000
    xs = rng.uniform(-1.45, 1.45, n).astype(F32)
    ys = rng.uniform(-1.45, 1.45, n).astype(F32)
    zs = (rng.uniform(-0.1, 0.1, n) - 1.0).astype(F32)
    pose = _pose((0, 0, 1.0))
    new, mean, used = O.compensate_drift(p, st, xs, ys, zs, pose, 0.5)
    d = O.point_decisions(p, st, xs, ys, zs, pose)
    c = d["cell"]
    iy, ix = c // p.nx, c % p.nx
    ok = (c >= 0) & (ix >= 6) & (iy >= 1) & ~((iy == 11) & (ix == 11))
    assert used == ok.sum() > 100
    assert abs(mean - float(np.mean(d["zm"][ok].astype(np.float64) - 0.25))) < 1e-12
    assert new.h[11, 11] == F32(-5.0)              # invalid cells keep their value
    assert np.array_equal(new.h[0, :3], np.full(3, F32(0.25) + F32(mean)))


def test_drift_without_usable_points_changes_nothing():
    p, st = _flat_scene(trav_value=0.0)
    xs, ys, zs = (np.zeros(10, F32), np.zeros(10, F32), np.full(10, -1.0, F32))
    new, mean, used = O.compensate_drift(p, st, xs, ys, zs, _pose((0, 0, 1.0)), 0.5)
    assert used == 0 and mean == 0.0 and np.array_equal(new.h, st.h)
