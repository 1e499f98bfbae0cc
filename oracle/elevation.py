"""Plain CPU oracle of GPU elevation mapping: fusion, clearing, normals, conv.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import, call or execute this module.
It shares no code, headers, helpers, tables or constants with the GPU library.

The method (Miki et al., "Elevation Mapping for Locomotion and Navigation using
GPU", arXiv 2204.12876) keeps a robot-centric 2.5D grid.  Each cell holds a
height estimate h and its variance sigma_m^2.  Every point of a cloud updates
the cell it falls in with a scalar Kalman step:
  * Eq. 1 updates the height;
  * Eq. 2 updates the variance;
  * the point variance follows a range-quadratic noise model (Sec. II-C);
  * points beyond a Mahalanobis distance are rejected (Sec. II-C).
Visibility clean-up marches each sensor ray and removes cells the ray passes
below.  A cell is removed only if all of these hold (Sec. II-E):
  * the ray passes below the cell's height minus its standard deviation (Eq. 3);
  * the cell is older than a set age (no update within it);
  * the cell's normal is well aligned with the ray (Eq. 4).
Normals (Sec. II-A) and a small convolutional traversability filter
(Sec. II-G) run over the cells afterwards.

Precision.  The paper fixes none.
  * Continuous results are computed in float64: fused heights and variances,
    normals, traversability.
  * Decisions that decide an integer or a mask are emulated in float32, as the
    GPU path takes them.  These are the cell index, the range check, the gate,
    the ray samples and the clearing predicate.
  * The float32 emulation uses numpy element-wise float32 operations: IEEE
    round-to-nearest-even, one rounding per operation, no fused multiply-add,
    in the operand order written below.

Readings of points where the paper is silent or ambiguous (each one is also
listed with its reason in the design notes):
  * The gate tests the innovation e = z - h0 against k^2 * (sigma_m^2 + sigma_p^2),
    using the cell prior at frame start.  Accept iff e*e <= k2*(v0 + sp2).
  * d is the Euclidean range in the sensor frame; the model is applied as
    sp2 = alpha_d * d^2.
  * Rejected points leave their cell untouched (unless outlier_variance is set).
  * The first point of an empty cell is fused with the large-variance prior; it
    does not replace it.
  * In Eq. 3, sigma is the standard deviation.  The test is written as
    hd = h - q_z, with hd > 0 and hd*hd > v.
  * Ray samples are taken at t = k/K for k = 1..K-1, with
    K = ceil(max(|dx|, |dy|) / step).  A sample in the end point's own cell is
    skipped.  Every valid point casts a ray, including gated-out points and
    points whose end lies outside the map.
  * A removed cell returns to the prior (h_init, v_init) and becomes invalid.
  * The normal is the least-squares plane over the 3x3 window, i.e. Prewitt
    differences.  It is NaN on the border and where any of the 9 cells is
    invalid.
  * Traversability is a 3x3 conv (1->8 channels, with bias), then ReLU, then a
    1x1 conv (8->1, with bias); there is no output activation.  It is NaN where
    the normal would be.
  * Map geometry: cells are half-open and the map is robot-centric.  The centre
    cell is floor(c / r), computed in float64.  The translation is moved into
    map-local coordinates in float64 before rounding to float32.
  * Time variance sigma_t^2 is added once per fusion to every valid cell the
    fusion does not update.
  * The wall/edge rule counts a frame's valid in-map points per cell before
    any gate (points of the exclusion area are not counted); in cells that
    hold an estimate and receive more than the threshold, points below the
    estimate are ignored.
  * The exclusion area (Fig. 3 is missing from the text): around the sensor
    origin, a point higher above it than the line b, rising at tan(theta_a)
    from horizontal distance c on, at most d, is ignored by the fusion.
  * The outlier check increases the variance (the amount is not given): each
    cell that holds an estimate and gets at least one gate-rejected point has
    sigma_o^2 added to its variance once per call, after the fusion.
  * Drift compensation averages z - h over valid in-map points in valid cells
    whose traversability exceeds a threshold, and adds the mean to every valid
    cell's height before fusion.
  * The upper bound uses the clearing's ray samples.  A sample lowers the
    bound of its cell if that cell holds no estimate when the call starts;
    the bound is the running minimum over calls, +inf until a ray passes.
  * Overlap clearance takes the robot's position and height from the caller
    and removes valid cells whose centre is within a horizontal radius and
    whose height differs from the robot's by more than the threshold.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Params", "MapState", "init_map", "local_pose", "point_decisions", "fuse",
    "compensate_drift", "fuse_sequential", "clear_visibility", "apply_clear", "compute_normals",
    "traversability", "move_map", "f32_constants", "upper_bound", "overlap_clear", "move_layer",
]

F32 = np.float32
F64 = np.float64


@dataclasses.dataclass
class Params:
    nx: int
    ny: int
    resolution: float
    init_height: float = 0.0
    init_variance: float = 1e3
    noise_alpha: float = 1e-4
    gate_k: float = 3.0
    min_range: float = 0.05
    ray_step: float = None         # clearing ray step; None takes the resolution
    clear_normal_alpha: float = 0.3
    clear_min_age_ms: int = 500
    time_variance: float = 0.0     # sigma_t^2 added per fusion to cells it leaves alone
    wall_min_count: int = 0        # wall/edge rule threshold; 0 turns the rule off
    excl_on: int = 0               # 1: the exclusion area (ramp) drops points above its line
    excl_theta: float = 0.0        # theta_a, the ramp's angle (rad)
    excl_b: float = 0.0            # height of the line above the sensor near it (m)
    excl_c: float = 0.0            # horizontal distance at which the ramp starts (m)
    excl_d: float = 0.0            # the line's maximum height above the sensor (m)
    outlier_variance: float = 0.0  # sigma_o^2 added to a cell with gate-rejected points

    def __post_init__(self):
        if self.ray_step is None:
            self.ray_step = self.resolution

    @classmethod
    def from_dict(cls, d: dict) -> "Params":
        names = {f.name for f in dataclasses.fields(cls)}
        return cls(**{k: v for k, v in d.items() if k in names})


def f32_constants(p: Params) -> dict:
    """Float32 constants derived from the parameters.

    The float parameters other than the resolution are float32 values.  Each
    square or reciprocal is formed in float64 from those values and then
    rounded once to float32.
    """
    rmin = F64(F32(p.min_range))
    k = F64(F32(p.gate_k))
    an = F64(F32(p.clear_normal_alpha))
    step = F64(F32(p.ray_step))
    return dict(
        inv_r=F32(1.0 / F64(p.resolution)),
        rmin2=F32(rmin * rmin),
        k2=F32(k * k),
        an2=F32(an * an),
        inv_step=F32(1.0 / step),
        alpha=F32(p.noise_alpha),
        h_init=F32(p.init_height),
        v_init=F32(p.init_variance),
        var_t=F32(p.time_variance),
        # the ramp's slope: tan of the float32 angle in float64 (the C
        # library's tan, through the math module), rounded once to float32
        excl_slope=F32(math.tan(F64(F32(p.excl_theta)))),
        excl_b=F32(p.excl_b),
        excl_c=F32(p.excl_c),
        excl_d=F32(p.excl_d),
        var_o=F32(p.outlier_variance),
    )


@dataclasses.dataclass
class MapState:
    """Map layers as the GPU holds them: row-major [ny, nx], x = column."""
    h: np.ndarray        # float32 height
    v: np.ndarray        # float32 variance
    t_upd: np.ndarray    # int32 ms since t0 of the last fusion into the cell
    valid: np.ndarray    # uint8
    nrm: np.ndarray      # float32 [3, ny, nx]
    trav: np.ndarray     # float32
    cgx: int             # global index of the centre cell
    cgy: int
    t0: int              # ms

    def copy(self) -> "MapState":
        return MapState(self.h.copy(), self.v.copy(), self.t_upd.copy(), self.valid.copy(),
                        self.nrm.copy(), self.trav.copy(), self.cgx, self.cgy, self.t0)


def init_map(p: Params, cx: float, cy: float, t0_ms: int = 0) -> MapState:
    """Every cell starts at the prior: the height estimate h_init and a large
    variance (Sec. II-C starts the variance at a large value)."""
    c = f32_constants(p)
    shp = (p.ny, p.nx)
    return MapState(
        h=np.full(shp, c["h_init"], F32), v=np.full(shp, c["v_init"], F32),
        t_upd=np.zeros(shp, np.int32), valid=np.zeros(shp, np.uint8),
        nrm=np.full((3,) + shp, np.nan, F32), trav=np.full(shp, np.nan, F32),
        cgx=int(math.floor(cx / p.resolution)), cgy=int(math.floor(cy / p.resolution)),
        t0=int(t0_ms))


def local_pose(p: Params, st: MapState, pose: np.ndarray):
    """Sensor->map-local rigid transform (Sec. II-A: points are transformed into
    the map frame).  The map's local origin is the corner of cell
    (cg - n // 2), in float64.  Returns (R32 [3,3], t32 [3]) as float32."""
    pose = np.asarray(pose, F64).reshape(3, 4)
    ox = F64(st.cgx - p.nx // 2) * F64(p.resolution)
    oy = F64(st.cgy - p.ny // 2) * F64(p.resolution)
    R32 = pose[:, :3].astype(F32)
    t32 = np.array([pose[0, 3] - ox, pose[1, 3] - oy, pose[2, 3]], F64).astype(F32)
    return R32, t32


def _transform32(R, t, xs, ys, zs):
    xm = ((R[0, 0] * xs + R[0, 1] * ys) + R[0, 2] * zs) + t[0]
    ym = ((R[1, 0] * xs + R[1, 1] * ys) + R[1, 2] * zs) + t[1]
    zm = ((R[2, 0] * xs + R[2, 1] * ys) + R[2, 2] * zs) + t[2]
    return xm, ym, zm


def _bin32(xm, ym, inv_r, nx, ny):
    """Cell of map-local float32 coordinates; -1 outside.  Half-open cells."""
    fx = xm * inv_r
    fy = ym * inv_r
    inmap = (fx >= F32(0)) & (fx < F32(nx)) & (fy >= F32(0)) & (fy < F32(ny))
    ix = np.floor(np.where(inmap, fx, F32(0))).astype(np.int64)
    iy = np.floor(np.where(inmap, fy, F32(0))).astype(np.int64)
    return np.where(inmap, iy * nx + ix, -1)


def point_decisions(p: Params, st: MapState, xs, ys, zs, pose):
    """Per-point float32 decisions: range validity, cell, gate (Sec. II-C).

    Returns a dict with float32 arrays xm, ym, zm, d2, sp2 and the decisions:
      * valid: the coordinates are finite, d2 >= rmin^2 and sp2 is finite;
      * cell: iy*nx + ix for valid in-map points, else -1;
      * excluded: in the map but above the exclusion area's line (only with
        excl_on); such points are ignored by everything below;
      * walled: ignored by the wall/edge rule;
      * rejected: taken to the gate and outside it (outliers);
      * accept: valid, in the map, not excluded or walled, and inside the
        Mahalanobis gate against the cell's frame-start prior.
    """
    xs = np.asarray(xs, F32)
    ys = np.asarray(ys, F32)
    zs = np.asarray(zs, F32)
    c = f32_constants(p)
    R, t = local_pose(p, st, pose)
    with np.errstate(all="ignore"):
        xm, ym, zm = _transform32(R, t, xs, ys, zs)
        d2 = (xs * xs + ys * ys) + zs * zs
        sp2 = c["alpha"] * d2
        valid = (np.isfinite(xs) & np.isfinite(ys) & np.isfinite(zs) & np.isfinite(d2)
                 & (d2 >= c["rmin2"]) & np.isfinite(sp2))
        cell = np.where(valid, _bin32(xm, ym, c["inv_r"], p.nx, p.ny), -1)
        inmap = cell >= 0
        cc = np.where(inmap, cell, 0)
        h0 = st.h.reshape(-1)[cc]
        v0 = st.v.reshape(-1)[cc]
        # Exclusion area (Sec. II-C, Fig. 3; the figure is not in the text, so
        # this is a stated reading).  Around the sensor origin o = t, with
        # horizontal distance rho and height e_up above o, the line is
        #   b              for rho <= c,
        #   b + tan(theta_a) * (rho - c) beyond, up to at most d.
        # A point above the line (e_up > line) is ignored: it is neither
        # counted, gated nor fused.
        excluded = np.zeros_like(inmap)
        if p.excl_on:
            dxr = xm - t[0]
            dyr = ym - t[1]
            rho = np.sqrt(dxr * dxr + dyr * dyr)
            e_up = zm - t[2]
            line = np.minimum(c["excl_b"] + c["excl_slope"] * np.maximum(rho - c["excl_c"], F32(0)),
                              c["excl_d"])
            excluded = inmap & (e_up > line)
        kept = inmap & ~excluded
        e = zm - h0
        inside = (e * e) <= (c["k2"] * (v0 + sp2))
        # Wall/edge rule (Sec. II-C): where more than wall_min_count of the
        # frame's kept points fall into one cell that holds an estimate, the
        # points below that estimate are ignored.  It acts before the gate.
        walled = np.zeros_like(inmap)
        if p.wall_min_count > 0:
            count = np.bincount(cell[kept], minlength=p.nx * p.ny)
            crowded = (count[cc] > p.wall_min_count) & (st.valid.reshape(-1)[cc] != 0)
            walled = kept & crowded & (zm < h0)
        gated = kept & ~walled
        accept = gated & inside
        rejected = gated & ~inside
    return dict(xm=xm, ym=ym, zm=zm, d2=d2, sp2=sp2, valid=valid, cell=cell,
                accept=accept, walled=walled, excluded=excluded, rejected=rejected, R=R, t=t)


@dataclasses.dataclass
class FuseResult:
    cell: np.ndarray       # int64 [N], -1 if dropped or outside
    accept: np.ndarray     # bool [N]
    h: np.ndarray          # float64 [ny, nx] post-fusion heights (untouched cells = prior)
    v: np.ndarray          # float64 [ny, nx]
    updated: np.ndarray    # bool [ny, nx] cells with at least one accepted point
    n_acc: np.ndarray      # int64 [ny, nx] accepted points per cell
    h_scale: np.ndarray    # float64 [ny, nx] condition scale of h (tolerances)
    state: MapState        # post-fusion state, continuous values rounded to float32


def fuse(p: Params, st: MapState, xs, ys, zs, pose, t_ms: int) -> FuseResult:
    """One frame of height fusion, in information form (Sec. II-C, Eq. 1 and 2).

    Composing Eq. 1 and Eq. 2 over the accepted points of a cell, in any order,
    gives
        1/v1    = 1/v0 + sum_i 1/sp2_i
        h1 / v1 = h0/v0 + sum_i z_i/sp2_i.
    Eq. 2 is the harmonic combination v*s/(v+s) = 1/(1/v + 1/s).  Eq. 1 is the
    inverse-variance weighted mean of h and z.  The sums are evaluated here in
    float64, with heights and variances recomputed in float64 from the same
    float32 inputs.  Gate decisions come from ``point_decisions`` (float32).
    """
    d = point_decisions(p, st, xs, ys, zs, pose)
    c32 = f32_constants(p)
    C = p.nx * p.ny
    acc = d["accept"]
    cell = d["cell"]
    R = d["R"].astype(F64)
    t = d["t"].astype(F64)
    x64 = np.asarray(xs, F32).astype(F64)
    y64 = np.asarray(ys, F32).astype(F64)
    z64 = np.asarray(zs, F32).astype(F64)
    with np.errstate(all="ignore"):
        zm64 = R[2, 0] * x64 + R[2, 1] * y64 + R[2, 2] * z64 + t[2]
        zmag = np.abs(R[2, 0] * x64) + np.abs(R[2, 1] * y64) + np.abs(R[2, 2] * z64) + abs(t[2])
        sp2_64 = F64(F32(p.noise_alpha)) * (x64 * x64 + y64 * y64 + z64 * z64)
    a = np.nonzero(acc)[0]
    w = 1.0 / sp2_64[a]
    ca = cell[a]
    Sw = np.bincount(ca, weights=w, minlength=C)
    Swz = np.bincount(ca, weights=w * zm64[a], minlength=C)
    Swm = np.bincount(ca, weights=w * zmag[a], minlength=C)
    n_acc = np.bincount(ca, minlength=C)
    h0 = st.h.reshape(-1).astype(F64)
    v0 = st.v.reshape(-1).astype(F64)
    upd = n_acc > 0
    W = 1.0 / v0 + Sw
    v1 = np.where(upd, 1.0 / W, v0)
    h1 = np.where(upd, (h0 / v0 + Swz) / W, h0)
    hs = np.where(upd, (np.abs(h0) / v0 + Swm) / W, np.abs(h0))
    new = st.copy()
    t_now = int(t_ms) - st.t0
    new.h = np.where(upd, h1, st.h.reshape(-1)).astype(F32).reshape(p.ny, p.nx)
    # Time variance (Sec. II-C): every valid cell this fusion does not update
    # grows by sigma_t^2, once per fusion (the frame rate is the constant rate).
    # It is one float32 addition of two stored float32 values.
    v_keep = st.v.reshape(-1)
    if p.time_variance != 0.0:
        grow = ~upd & (st.valid.reshape(-1) != 0)
        v_keep = np.where(grow, v_keep + c32["var_t"], v_keep)
        v1 = np.where(grow, v_keep.astype(F64), v1)
    v_out = np.where(upd, v1, v_keep).astype(F32)
    # Outlier variance (Sec. II-C: the outlier check "increases the variance of
    # the cell"; the amount is not given, so this is a stated reading): a cell
    # that holds an estimate when the call starts and gets at least one
    # gate-rejected point in the frame has sigma_o^2 added to its variance,
    # once per call, after the fusion and the time variance (one float32
    # addition).
    if p.outlier_variance != 0.0:
        hit = np.bincount(cell[d["rejected"]], minlength=C) > 0
        inflate = hit & (st.valid.reshape(-1) != 0)
        v_out = np.where(inflate, v_out + c32["var_o"], v_out)
        v1 = np.where(inflate, v_out.astype(F64), v1)
    new.v = v_out.reshape(p.ny, p.nx)
    new.valid = np.where(upd, 1, st.valid.reshape(-1)).astype(np.uint8).reshape(p.ny, p.nx)
    new.t_upd = np.where(upd, t_now, st.t_upd.reshape(-1)).astype(np.int32).reshape(p.ny, p.nx)
    shp = (p.ny, p.nx)
    return FuseResult(cell=cell, accept=acc, h=h1.reshape(shp), v=v1.reshape(shp),
                      updated=upd.reshape(shp), n_acc=n_acc.reshape(shp),
                      h_scale=hs.reshape(shp), state=new)


def compensate_drift(p: Params, st: MapState, xs, ys, zs, pose, trav_min: float):
    """Height drift compensation (Sec. II-D).

    Each valid in-map point whose cell holds an estimate on flat ground
    (traversability defined and above trav_min) gives the error between its
    height and the map, e_i = zm_i - h[cell_i].  The mean error over those n
    points is added to the height of every valid cell; with n = 0 nothing
    changes.  Returns (new state, mean as float64, n).

    The error and the threshold test use the float32 values the map and the
    transform hold; the mean is formed in float64 and then added once, in
    float32, to each height.
    """
    d = point_decisions(p, st, xs, ys, zs, pose)
    cell = d["cell"]
    inmap = cell >= 0
    cc = np.where(inmap, cell, 0)
    trav = st.trav.reshape(-1)[cc]
    with np.errstate(invalid="ignore"):
        flat = ~np.isnan(trav) & (trav > F32(trav_min))
    use = inmap & (st.valid.reshape(-1)[cc] != 0) & flat
    n = int(use.sum())
    new = st.copy()
    if n == 0:
        return new, 0.0, 0
    err = d["zm"][use].astype(F64) - st.h.reshape(-1)[cc[use]].astype(F64)
    mean = float(err.sum() / n)
    keep = st.valid != 0
    new.h = np.where(keep, st.h + F32(mean), st.h).astype(F32)
    return new, mean, n


def fuse_sequential(p: Params, st: MapState, xs, ys, zs, pose):
    """Eq. 1 then Eq. 2 applied point by point in index order (tiny inputs only).

    The gate decisions are those of ``point_decisions``, taken against the
    frame-start prior.  Returns float64 (h, v) arrays [ny, nx].
    """
    d = point_decisions(p, st, xs, ys, zs, pose)
    R = d["R"].astype(F64)
    t = d["t"].astype(F64)
    h = st.h.astype(F64).reshape(-1).copy()
    v = st.v.astype(F64).reshape(-1).copy()
    alpha = F64(F32(p.noise_alpha))
    for i in range(len(d["cell"])):
        if not d["accept"][i]:
            continue
        c = d["cell"][i]
        x, y, z = F64(F32(xs[i])), F64(F32(ys[i])), F64(F32(zs[i]))
        pz = R[2, 0] * x + R[2, 1] * y + R[2, 2] * z + t[2]
        sp = alpha * (x * x + y * y + z * z)
        sm = v[c]
        h[c] = (sp * h[c] + sm * pz) / (sm + sp)          # Eq. 1
        v[c] = sm * sp / (sm + sp)                        # Eq. 2
    return h.reshape(p.ny, p.nx), v.reshape(p.ny, p.nx)


def _ray_samples(p: Params, st: MapState, xs, ys, zs, pose, chunk: int = 1 << 16):
    """The in-map ray samples of a frame (Sec. II-E), in chunks of rays.

    A ray runs from the sensor origin o to each valid point.  Let (dx, dy, dz)
    be the point minus o, and m = max(|dx|, |dy|).  K = ceil(m / step) and the
    samples are q_k = o + (k/K)(dx, dy, dz) for k = 1..K-1; if m/step is not
    below 2^24 the ray is not marched.  Samples outside the map and samples in
    the end point's own cell are left out.  All in float32.

    Yields (cs, qz, dx, dy, dz): the samples' cells and heights, and each
    sample's ray direction.
    """
    c = f32_constants(p)
    d = point_decisions(p, st, xs, ys, zs, pose)
    o = d["t"]
    idx_valid = np.nonzero(d["valid"])[0]
    for c0 in range(0, len(idx_valid), chunk):
        ii = idx_valid[c0:c0 + chunk]
        with np.errstate(all="ignore"):
            dx = d["xm"][ii] - o[0]
            dy = d["ym"][ii] - o[1]
            dz = d["zm"][ii] - o[2]
            m = np.maximum(np.abs(dx), np.abs(dy))
            ks = m * c["inv_step"]
        ok = ks < F32(16777216.0)
        K = np.where(ok, np.ceil(np.where(ok, ks, F32(0))), F32(0)).astype(np.int64)
        nsamp = np.maximum(K - 1, 0)
        if nsamp.sum() == 0:
            continue
        end_cell = _bin32(d["xm"][ii], d["ym"][ii], c["inv_r"], p.nx, p.ny)
        rep = np.repeat(np.arange(len(ii)), nsamp)
        starts = np.cumsum(nsamp) - nsamp
        k = np.arange(len(rep)) - np.repeat(starts, nsamp) + 1
        with np.errstate(all="ignore"):
            tt = k.astype(F32) / K[rep].astype(F32)
            qx = o[0] + tt * dx[rep]
            qy = o[1] + tt * dy[rep]
            qz = o[2] + tt * dz[rep]
        cs = _bin32(qx, qy, c["inv_r"], p.nx, p.ny)
        keep = (cs >= 0) & (cs != end_cell[rep])
        rk = rep[keep]
        yield cs[keep], qz[keep], dx[rk], dy[rk], dz[rk]


def clear_visibility(p: Params, st: MapState, xs, ys, zs, pose, t_ms: int,
                     chunk: int = 1 << 16) -> np.ndarray:
    """Visibility clean-up marks (Sec. II-E, Eq. 3 and Eq. 4), as bool [ny, nx].

    ``st`` is the snapshot the rays test against.  Its normals come from the
    last normal computation.  The samples are those of ``_ray_samples``.
    A sample in cell c marks c when all of the following hold:
      * c is valid (it is in the map and not the end point's own cell);
      * the age now - t_upd[c] exceeds the minimum age;
      * the sample passes below h[c] minus the standard deviation
        (hd = h[c] - q_z, with hd > 0 and hd*hd > v[c]);
      * the ray is aligned with the cell normal: (r.n)^2 > alpha_n^2 * |r|^2.
    All of it is evaluated in float32.
    """
    c = f32_constants(p)
    t_now = int(t_ms) - st.t0
    marks = np.zeros(p.nx * p.ny, bool)
    hf = st.h.reshape(-1)
    vf = st.v.reshape(-1)
    tf = st.t_upd.reshape(-1).astype(np.int64)
    validf = st.valid.reshape(-1)
    nxf = st.nrm[0].reshape(-1)
    nyf = st.nrm[1].reshape(-1)
    nzf = st.nrm[2].reshape(-1)
    tau = int(p.clear_min_age_ms)
    for cs, qz, dxk, dyk, dzk in _ray_samples(p, st, xs, ys, zs, pose, chunk):
        with np.errstate(all="ignore"):
            hd = hf[cs] - qz
            dot = (dxk * nxf[cs] + dyk * nyf[cs]) + dzk * nzf[cs]
            dd = (dxk * dxk + dyk * dyk) + dzk * dzk
            cond = ((validf[cs] != 0) & ((t_now - tf[cs]) > tau) & (hd > F32(0))
                    & ((hd * hd) > vf[cs]) & ~np.isnan(nzf[cs])
                    & ((dot * dot) > (c["an2"] * dd)))
        marks[cs[cond]] = True
    return marks.reshape(p.ny, p.nx)


def upper_bound(p: Params, st: MapState, ub: np.ndarray, xs, ys, zs, pose,
                chunk: int = 1 << 16) -> np.ndarray:
    """Height upper bound layer (Sec. II-H), float32 [ny, nx]; +inf = no bound.

    The ground under a ray cannot lie above the ray, or it would have been
    seen.  So every ray sample (those of ``_ray_samples``, the clearing's own)
    in a cell without an estimate (invalid in the snapshot ``st``) lowers that
    cell's bound to the sample height: the new bound is the minimum of the old
    one and the heights of all such samples.  Cells with an estimate keep
    their bound.
    """
    out = np.asarray(ub, F32).reshape(-1).copy()
    validf = st.valid.reshape(-1)
    for cs, qz, _, _, _ in _ray_samples(p, st, xs, ys, zs, pose, chunk):
        sel = validf[cs] == 0
        np.minimum.at(out, cs[sel], qz[sel])
    return out.reshape(p.ny, p.nx)


def overlap_clear(p: Params, st: MapState, robot_xyz, radius: float,
                  threshold: float) -> np.ndarray:
    """Overlap clearance marks (Sec. II-F), bool [ny, nx].

    A valid cell is removed when its centre lies within ``radius`` of the
    robot in the horizontal plane and its height differs from the robot's
    height by more than ``threshold``.  In float32, in map-local coordinates
    (the robot position is moved into them in float64, like the pose):
      * dx = (ix + 0.5) * r32 - rx,  dy = (iy + 0.5) * r32 - ry;
      * near iff dx*dx + dy*dy <= float32(radius^2);
      * far in height iff |h - rz| > threshold.
    The removed cells go back to the prior as in ``apply_clear``.
    """
    ox = F64(st.cgx - p.nx // 2) * F64(p.resolution)
    oy = F64(st.cgy - p.ny // 2) * F64(p.resolution)
    rx = F32(F64(robot_xyz[0]) - ox)
    ry = F32(F64(robot_xyz[1]) - oy)
    rz = F32(robot_xyz[2])
    r32 = F32(p.resolution)
    rad = F64(F32(radius))
    rad2 = F32(rad * rad)
    thr = F32(threshold)
    ix = np.arange(p.nx, dtype=F32)
    iy = np.arange(p.ny, dtype=F32)
    with np.errstate(all="ignore"):
        dx = (ix + F32(0.5)) * r32 - rx
        dy = (iy + F32(0.5)) * r32 - ry
        near = ((dx * dx)[None, :] + (dy * dy)[:, None]) <= rad2
        far = np.abs(st.h - rz) > thr
    return (st.valid != 0) & near & far


def move_layer(p: Params, st: MapState, layer: np.ndarray, cx: float, cy: float,
               fill) -> np.ndarray:
    """One extra layer through the robot-centric move of ``move_map``: cells
    that stay keep their value, cells that enter take ``fill``."""
    shift_x = int(math.floor(cx / p.resolution)) - st.cgx
    shift_y = int(math.floor(cy / p.resolution)) - st.cgy
    out = np.full_like(layer, fill)
    ny, nx = p.ny, p.nx
    # out local (ix, iy) <- layer local (ix + shift_x, iy + shift_y)
    x0, x1 = max(0, -shift_x), min(nx, nx - shift_x)
    y0, y1 = max(0, -shift_y), min(ny, ny - shift_y)
    if x0 < x1 and y0 < y1:
        out[y0:y1, x0:x1] = layer[y0 + shift_y:y1 + shift_y, x0 + shift_x:x1 + shift_x]
    return out


def apply_clear(p: Params, st: MapState, marks: np.ndarray) -> MapState:
    """A removed cell goes back to the prior and becomes invalid (Sec. II-E
    removes the cell's height).  Normals and traversability are left for the
    next per-cell pass."""
    c = f32_constants(p)
    new = st.copy()
    new.h = np.where(marks, c["h_init"], st.h).astype(F32)
    new.v = np.where(marks, c["v_init"], st.v).astype(F32)
    new.valid = np.where(marks, 0, st.valid).astype(np.uint8)
    return new


def _window_ok(valid: np.ndarray) -> np.ndarray:
    """True where the cell is interior and all 9 cells of its 3x3 window are valid."""
    ny, nx = valid.shape
    ok = np.zeros((ny, nx), bool)
    if ny < 3 or nx < 3:
        return ok
    v = valid != 0
    acc = np.ones((ny - 2, nx - 2), bool)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            acc &= v[1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx]
    ok[1:-1, 1:-1] = acc
    return ok


def compute_normals(p: Params, h: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """Surface normal per cell (Sec. II-A "normal calculation"), float64 [3, ny, nx].

    It is the least-squares plane z = a x + b y + c over the 3x3 window, with
    cell spacing r.  With x, y in {-r, 0, r} the normal equations decouple:
      a = sum_dy (h[y+dy, x+1] - h[y+dy, x-1]) / (6 r)
      b = sum_dx (h[y+1, x+dx] - h[y-1, x+dx]) / (6 r)
    The normal is n = (-a, -b, 1) / sqrt(a^2 + b^2 + 1).  It is NaN unless the
    cell is interior and all 9 cells are valid.
    """
    H = np.asarray(h, F32).astype(F64)
    ny, nx = H.shape
    out = np.full((3, ny, nx), np.nan)
    ok = _window_ok(valid)
    if ny < 3 or nx < 3:
        return out
    r = F64(p.resolution)
    a = np.zeros((ny - 2, nx - 2))
    b = np.zeros((ny - 2, nx - 2))
    for dy in (-1, 0, 1):
        a += H[1 + dy:ny - 1 + dy, 2:] - H[1 + dy:ny - 1 + dy, :-2]
    for dx in (-1, 0, 1):
        b += H[2:, 1 + dx:nx - 1 + dx] - H[:-2, 1 + dx:nx - 1 + dx]
    a /= 6.0 * r
    b /= 6.0 * r
    nrm = np.sqrt(a * a + b * b + 1.0)
    inner = ok[1:-1, 1:-1]
    out[0, 1:-1, 1:-1] = np.where(inner, -a / nrm, np.nan)
    out[1, 1:-1, 1:-1] = np.where(inner, -b / nrm, np.nan)
    out[2, 1:-1, 1:-1] = np.where(inner, 1.0 / nrm, np.nan)
    return out


def traversability(h: np.ndarray, valid: np.ndarray, weights: np.ndarray):
    """Traversability filter (Sec. II-G), float64 [ny, nx].

    The paper deploys a small trained CNN but gives neither its architecture nor
    its weights.  This is the fixed form it is read as:
      * a 3x3 cross-correlation, 1 -> 8 channels, with bias b1, over the raw
        heights;
      * ReLU;
      * a 1x1 convolution, 8 -> 1, with bias b2; no output activation.
    Weight layout (89 values): w1[8,1,3,3] (PyTorch conv layout), b1[8], w2[8],
    b2[1].  NaN where the 3x3 window is not interior and fully valid.

    Returns (T, scale); scale = |b2| + sum_c |w2_c| (|b1_c| + sum |w1||h|) is the
    error scale of the sum.
    """
    w = np.asarray(weights, F32).astype(F64)
    w1 = w[:72].reshape(8, 3, 3)
    b1 = w[72:80]
    w2 = w[80:88]
    b2 = w[88]
    H = np.asarray(h, F32).astype(F64)
    ny, nx = H.shape
    T = np.full((ny, nx), np.nan)
    S = np.full((ny, nx), np.nan)
    if ny < 3 or nx < 3:
        return T, S
    ok = _window_ok(valid)[1:-1, 1:-1]
    with np.errstate(all="ignore"):
        tot = np.full((ny - 2, nx - 2), b2)
        sc = np.full((ny - 2, nx - 2), abs(b2))
        for ch in range(8):
            act = np.full((ny - 2, nx - 2), b1[ch])
            mag = np.full((ny - 2, nx - 2), abs(b1[ch]))
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    win = H[1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx]
                    act = act + w1[ch, dy + 1, dx + 1] * win
                    mag = mag + abs(w1[ch, dy + 1, dx + 1]) * np.abs(win)
            tot = tot + w2[ch] * np.maximum(act, 0.0)
            sc = sc + abs(w2[ch]) * mag
    T[1:-1, 1:-1] = np.where(ok, tot, np.nan)
    S[1:-1, 1:-1] = np.where(ok, sc, np.nan)
    return T, S


def move_map(p: Params, st: MapState, cx: float, cy: float) -> MapState:
    """Re-centre the robot-centric map on (cx, cy) (Sec. I, robot-centric map).

    The centre cell becomes floor(c / r) and the map shifts by whole cells.
    Cells still inside keep all their layers.  Cells entering the map take the
    prior (h_init, v_init), invalid, t_upd 0, NaN normals and traversability.
    """
    c = f32_constants(p)
    ngx = int(math.floor(cx / p.resolution))
    ngy = int(math.floor(cy / p.resolution))
    sx, sy = ngx - st.cgx, ngy - st.cgy
    new = init_map(p, cx, cy, st.t0)
    new.h[:] = c["h_init"]
    ny, nx = p.ny, p.nx
    # new local (ix, iy) <- old local (ix + sx, iy + sy)
    x0, x1 = max(0, -sx), min(nx, nx - sx)
    y0, y1 = max(0, -sy), min(ny, ny - sy)
    if x0 < x1 and y0 < y1:
        src = (slice(y0 + sy, y1 + sy), slice(x0 + sx, x1 + sx))
        dst = (slice(y0, y1), slice(x0, x1))
        new.h[dst] = st.h[src]
        new.v[dst] = st.v[src]
        new.t_upd[dst] = st.t_upd[src]
        new.valid[dst] = st.valid[src]
        new.trav[dst] = st.trav[src]
        for k in range(3):
            new.nrm[k][dst] = st.nrm[k][src]
    return new
