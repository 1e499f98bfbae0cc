"""Oracle pins for the upper bound layer (Sec. II-H), overlap clearance
(Sec. II-F) and the locomotion filters (Sec. II-I).

Each is pinned against something other than its own code:
  * upper bound: closed forms of single rays (a level ray bounds every cell
    it crosses at its own height; a descending ray bounds a crossed cell
    between its exit height and one sample step above it), the running
    minimum over calls, and cells with an estimate left alone;
  * overlap clearance: the disc of cells in float64 away from its rim, and the
    strict height threshold on exactly representable values;
  * inpainting: scipy's connected-component labelling and dilation, plus hand
    cases;
  * smoothing: scipy.ndimage's uniform, Gaussian and median filters in
    'mirror' mode, which is the border rule used here.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle as O

F32 = np.float32
F64 = np.float64


def _pose(t):
    P = np.zeros((3, 4))
    P[:, :3] = np.eye(3)
    P[:, 3] = t
    return P


def _params(**kw):
    base = dict(nx=40, ny=10, resolution=0.25, ray_step=0.0625, noise_alpha=1e-4, gate_k=3.0,
                min_range=0.05)
    base.update(kw)
    return O.Params.from_dict(base)


# -------------------------------------------------------------- upper bound
def test_level_ray_bounds_every_crossed_cell_at_its_height():
    p = _params()
    st = O.init_map(p, 0.0, 0.0, 0)             # local origin at (-5, -1.25)
    ub = np.full((p.ny, p.nx), np.inf, F32)
    # sensor at the centre of cell (ix=4, iy=5); the point 20 cells along +x
    ox, oy, oz = -5.0 + 4.5 * 0.25, -1.25 + 5.5 * 0.25, 0.7
    pose = _pose((ox, oy, oz))
    new = O.upper_bound(p, st, ub, np.array([5.0], F32), np.array([0.0], F32),
                        np.array([0.0], F32), pose)
    crossed = np.zeros_like(new, bool)
    crossed[5, 4:24] = True                      # origin cell .. one before the end cell (24)
    assert np.all(new[crossed] == F32(oz))
    assert np.all(np.isinf(new[~crossed]))


def test_descending_ray_bound_sits_just_above_the_exit_height():
    p = _params()
    st = O.init_map(p, 0.0, 0.0, 0)
    ub = np.full((p.ny, p.nx), np.inf, F32)
    ox, oy, oz = -5.0 + 2.5 * 0.25, -1.25 + 5.5 * 0.25, 2.0
    L, drop = 7.0, 1.6                           # horizontal length and fall of the ray
    pose = _pose((ox, oy, oz))
    new = O.upper_bound(p, st, ub, np.array([L], F32), np.array([0.0], F32),
                        np.array([-drop], F32), pose)
    slope = drop / L
    end_ix = int(math.floor((2.5 * 0.25 + L) / 0.25))
    for ix in range(2, end_ix):
        x_exit = (ix + 1) * 0.25 - 2.5 * 0.25    # along-ray distance at the cell's far edge
        z_exit = oz - slope * x_exit
        b = float(new[5, ix])
        # the lowest sample in the cell is the last one before the edge: within
        # one sample spacing (<= ray_step) of the exit, so at most slope*step above
        assert z_exit - 1e-5 <= b <= z_exit + slope * p.ray_step + 1e-5, ix
    assert np.isinf(new[5, end_ix]) and np.isinf(new[4]).all()


def test_bound_is_a_running_minimum_and_skips_cells_with_an_estimate():
    p = _params()
    st = O.init_map(p, 0.0, 0.0, 0)
    st.valid[5, 10:14] = 1
    ub = np.full((p.ny, p.nx), np.inf, F32)
    pose = _pose((-5.0 + 4.5 * 0.25, -1.25 + 5.5 * 0.25, 0.9))
    a = (np.array([5.0], F32), np.array([0.0], F32), np.array([0.3], F32))     # rising
    b = (np.array([5.0], F32), np.array([0.0], F32), np.array([-0.4], F32))    # falling
    ab = O.upper_bound(p, st, O.upper_bound(p, st, ub, *a, pose), *b, pose)
    ba = O.upper_bound(p, st, O.upper_bound(p, st, ub, *b, pose), *a, pose)
    assert np.array_equal(ab, ba)
    assert np.array_equal(ab, np.minimum(O.upper_bound(p, st, ub, *a, pose),
                                         O.upper_bound(p, st, ub, *b, pose)))
    assert np.isinf(ab[5, 10:14]).all()          # cells with an estimate
    assert np.isfinite(ab[5, 5:10]).all()
    # a bound already below every ray stays
    low = np.full_like(ub, F32(-3.0))
    assert np.array_equal(O.upper_bound(p, st, low, *a, pose), low)


# ---------------------------------------------------------- overlap clearance
def test_overlap_clears_the_disc_away_from_its_rim():
    p = _params(nx=60, ny=50, resolution=0.1)
    st = O.init_map(p, 1.0, -2.0, 0)
    rng = np.random.default_rng(0)
    st.valid[:] = (rng.random(st.valid.shape) < 0.8).astype(np.uint8)
    st.h[:] = rng.uniform(-1.0, 3.0, st.h.shape).astype(F32)
    robot = (1.3, -1.7, 0.8)
    R, thr = 1.7, 0.6
    m = O.overlap_clear(p, st, robot, R, thr)
    ox = (st.cgx - p.nx // 2) * p.resolution
    oy = (st.cgy - p.ny // 2) * p.resolution
    cx = ox + (np.arange(p.nx) + 0.5) * p.resolution
    cy = oy + (np.arange(p.ny) + 0.5) * p.resolution
    dist = np.hypot(cx[None, :] - robot[0], cy[:, None] - robot[1])
    far = np.abs(st.h.astype(F64) - robot[2]) > thr
    exp = (st.valid == 1) & (dist <= R) & far
    sure = (np.abs(dist - R) > 1e-5) & (np.abs(np.abs(st.h.astype(F64) - robot[2]) - thr) > 1e-5)
    assert np.array_equal(m[sure], exp[sure])
    assert m.sum() > 50 and (~sure).sum() < 10
    st2 = O.apply_clear(p, st, m)
    assert not O.overlap_clear(p, st2, robot, R, thr).any()


def test_overlap_height_threshold_is_strict():
    p = _params(nx=8, ny=8, resolution=0.5)
    st = O.init_map(p, 0.0, 0.0, 0)
    st.valid[:] = 1
    st.h[:] = F32(1.5)
    st.h[0, 0] = np.nextafter(F32(1.5), F32(2.0))
    m = O.overlap_clear(p, st, (0.0, 0.0, 0.5), 100.0, 1.0)
    assert m[0, 0] and m.sum() == 1             # |1.5 - 0.5| == 1.0 is not "larger"
    st.valid[0, 0] = 0
    assert not O.overlap_clear(p, st, (0.0, 0.0, 0.5), 100.0, 1.0).any()


# ---------------------------------------------------------------- inpainting
def _inpaint_scipy(h, valid):
    hole = valid == 0
    cross = ndimage.generate_binary_structure(2, 1)
    lab, n = ndimage.label(hole, structure=cross)
    out = np.where(valid != 0, h, np.nan).astype(F32)
    for k in range(1, n + 1):
        reg = lab == k
        border = ndimage.binary_dilation(reg, structure=cross) & ~hole
        if border.any():
            out[reg] = h[border].min()
    return out


def test_inpaint_hand_cases():
    h = np.arange(25, dtype=F32).reshape(5, 5)
    v = np.ones((5, 5), np.uint8)
    assert np.array_equal(O.inpaint_min(h, v), h)
    assert np.isnan(O.inpaint_min(h, np.zeros_like(v))).all()
    v[2, 2] = 0                                  # one hole: min of 7, 11, 13, 17
    out = O.inpaint_min(h, v)
    assert out[2, 2] == F32(7) and np.array_equal(out[v == 1], h[v == 1])
    v[:] = 1
    v[0, 0] = v[0, 1] = 0                        # corner hole: border cells 2, 5, 6
    assert O.inpaint_min(h, v)[0, 1] == F32(2) and O.inpaint_min(h, v)[0, 0] == F32(2)
    v[:] = 1
    v[1, 1] = v[2, 2] = 0                        # diagonal cells are two regions
    out = O.inpaint_min(h, v)
    assert out[1, 1] == F32(1) and out[2, 2] == F32(7)


@pytest.mark.parametrize("seed", range(4))
def test_inpaint_matches_labelling(seed):
    rng = np.random.default_rng(seed)
    h = rng.normal(size=(23, 31)).astype(F32)
    v = (rng.random(h.shape) < (0.35 + 0.15 * seed)).astype(np.uint8)
    a = O.inpaint_min(h, v)
    b = _inpaint_scipy(h, v)
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


# ----------------------------------------------------------------- smoothing
@pytest.mark.parametrize("k", [1, 3, 5, 9])
def test_box_matches_uniform_filter(k):
    x = np.random.default_rng(k).normal(size=(17, 13)).astype(F32)
    ref = ndimage.uniform_filter(x.astype(F64), size=k, mode="mirror")
    assert np.allclose(O.smooth_box(x, k), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("k,sigma", [(3, 0.8), (5, 1.1), (7, 2.5), (11, 1.7)])
def test_gaussian_matches_gaussian_filter(k, sigma):
    x = np.random.default_rng(k).normal(size=(19, 14)).astype(F32)
    r = k // 2
    s = float(F32(sigma))
    ref = ndimage.gaussian_filter(x.astype(F64), s, mode="mirror", truncate=(r + 0.25) / s)
    assert np.allclose(O.smooth_gaussian(x, k, sigma), ref, rtol=0, atol=1e-12)
    assert abs(O.gaussian_weights(k, sigma).sum() - 1.0) < 1e-15


@pytest.mark.parametrize("k", [3, 5])
def test_median_matches_median_filter(k):
    x = np.random.default_rng(k).normal(size=(16, 21)).astype(F32)
    x[3, 4] = x[3, 5]                            # ties
    ref = ndimage.median_filter(x, size=k, mode="mirror")
    assert np.array_equal(O.smooth_median(x, k), ref)


def test_smoothing_nan_reach_and_constants():
    x = np.full((12, 12), F32(2.5))
    assert np.allclose(O.smooth_box(x, 5), 2.5) and np.allclose(O.smooth_gaussian(x, 7, 1.3), 2.5)
    x[6, 6] = np.nan
    for out in (O.smooth_box(x, 3), O.smooth_gaussian(x, 3, 1.0), O.smooth_median(x, 3)):
        nan = np.isnan(out)
        assert nan[5:8, 5:8].all() and nan.sum() == 9
    x[6, 6] = 2.5
    x[0, 0] = np.nan                             # a corner NaN is seen through the mirror
    assert np.isnan(O.smooth_box(x, 3)[:2, :2]).all() and np.isnan(O.smooth_box(x, 3)).sum() == 4
    with pytest.raises(ValueError):
        O.smooth_median(x, 7)
    with pytest.raises(ValueError):
        O.smooth_box(np.zeros((2, 9), F32), 5)
