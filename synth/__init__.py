"""Seeded synthetic workloads for GPU elevation-map fusion.

This module simulates the world the sensors observe and nothing else.
It builds:
  * terrains: a sum of sinusoids, one step edge and optional boxes;
  * sensor rigs: a dome LiDAR, pinhole depth frustums and a spinning LiDAR;
  * smooth robot trajectories;
  * ray-cast point clouds, expressed in the sensor frame, with range-dependent
    height noise and a fraction of gross outliers.

It holds none of the map-fusion arithmetic: no binning, gating, fusion,
clearing, normals or traversability.  Both the GPU path and the CPU oracle take
their inputs from here, so the two never differ in what they are fed.

All randomness comes from ``numpy.random.default_rng`` seeded by a
``SeedSequence``; ray casting runs in float64 with torch on the requested
device (deterministic arithmetic, no random draws on the device).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

SEED_BASE = 12876

__all__ = [
    "Terrain", "Frame", "MapSpec", "Rig", "make_terrain", "dome_lidar_dirs",
    "frustum_dirs", "spinning_lidar_dirs", "random_cone_dirs", "raycast",
    "pose_matrix", "Trajectory", "make_frame", "default_params", "trav_weights",
    "cfg0", "cfg1", "cfg2", "cfg3_rigs", "cfg4", "paper_analogue",
]


# --------------------------------------------------------------------------
# terrain
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Terrain:
    amp: np.ndarray        # [4] m
    lam: np.ndarray        # [4] m
    theta: np.ndarray      # [4] rad, wave direction
    phase: np.ndarray      # [4] rad
    step_dir: float        # rad, normal of the step line
    step_off: float        # m, signed offset of the step line from the origin
    step_h: float          # m
    boxes: np.ndarray      # [nb, 5]: cx, cy, half_x, half_y, height  (axis aligned)

    def height(self, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        """Ground height at world (x, y); float64 tensors of any shape."""
        z = torch.zeros_like(x)
        for k in range(len(self.amp)):
            arg = (x * math.cos(self.theta[k]) + y * math.sin(self.theta[k])) \
                * (2.0 * math.pi / self.lam[k]) + self.phase[k]
            z = z + self.amp[k] * torch.sin(arg)
        s = x * math.cos(self.step_dir) + y * math.sin(self.step_dir) - self.step_off
        z = z + self.step_h * (s > 0).to(x.dtype)
        if len(self.boxes):
            b = torch.as_tensor(self.boxes, dtype=x.dtype, device=x.device)
            xs = x.unsqueeze(-1)
            ys = y.unsqueeze(-1)
            inside = ((xs - b[:, 0]).abs() <= b[:, 2]) & ((ys - b[:, 1]).abs() <= b[:, 3])
            hb = torch.where(inside, b[:, 4], torch.zeros((), dtype=x.dtype, device=x.device))
            z = z + hb.amax(dim=-1)
        return z


def make_terrain(rng: np.random.Generator, n_boxes: int = 0, extent: float = 10.0,
                 step_h: float = 0.15) -> Terrain:
    """Four sinusoids (amplitude 0.05-0.2 m, wavelength 0.5-3 m), one step, boxes.

    Boxes are 0.1-0.5 m tall with sides 0.2-1.0 m, centred uniformly in
    [-extent, extent]^2.
    """
    amp = rng.uniform(0.05, 0.2, 4)
    lam = rng.uniform(0.5, 3.0, 4)
    theta = rng.uniform(0.0, 2 * math.pi, 4)
    phase = rng.uniform(0.0, 2 * math.pi, 4)
    step_dir = float(rng.uniform(0.0, 2 * math.pi))
    step_off = float(rng.uniform(-0.5 * extent, 0.5 * extent))
    boxes = np.zeros((n_boxes, 5))
    if n_boxes:
        boxes[:, 0] = rng.uniform(-extent, extent, n_boxes)
        boxes[:, 1] = rng.uniform(-extent, extent, n_boxes)
        boxes[:, 2] = 0.5 * rng.uniform(0.2, 1.0, n_boxes)
        boxes[:, 3] = 0.5 * rng.uniform(0.2, 1.0, n_boxes)
        boxes[:, 4] = rng.uniform(0.1, 0.5, n_boxes)
    return Terrain(amp, lam, theta, phase, step_dir, step_off, step_h, boxes)


# --------------------------------------------------------------------------
# sensor ray patterns (unit vectors in the sensor frame: x forward, z up)
# --------------------------------------------------------------------------
def _dirs(az: np.ndarray, el: np.ndarray) -> np.ndarray:
    ce = np.cos(el)
    return np.stack([ce * np.cos(az), ce * np.sin(az), np.sin(el)], axis=-1)


def random_cone_dirs(rng: np.random.Generator, n: int, el_lo_deg: float,
                     el_hi_deg: float) -> np.ndarray:
    """Azimuth U[0, 2pi), elevation U[lo, hi]; ordered by azimuth like a sweep."""
    az = rng.uniform(0.0, 2 * math.pi, n)
    el = np.deg2rad(rng.uniform(el_lo_deg, el_hi_deg, n))
    order = np.argsort(az, kind="stable")
    return _dirs(az[order], el[order])


def dome_lidar_dirs(rng: np.random.Generator, beams: int, per_beam: int,
                    el_lo_deg: float = -89.0, el_hi_deg: float = 0.0) -> np.ndarray:
    """Hemispherical (dome) LiDAR: ``beams`` rings, ring-major, azimuth sweep."""
    el = np.deg2rad(np.linspace(el_lo_deg, el_hi_deg, beams))
    phase = rng.uniform(0.0, 2 * math.pi)
    az = phase + np.arange(per_beam) * (2 * math.pi / per_beam)
    A, E = np.meshgrid(az, el)          # [beams, per_beam]
    return _dirs(A.ravel(), E.ravel())


def spinning_lidar_dirs(rng: np.random.Generator, beams: int, per_beam: int,
                        el_lo_deg: float, el_hi_deg: float) -> np.ndarray:
    """Spinning multi-beam LiDAR: seeded beam elevations, ring-major order."""
    el = np.sort(np.deg2rad(rng.uniform(el_lo_deg, el_hi_deg, beams)))
    phase = rng.uniform(0.0, 2 * math.pi)
    az = phase + np.arange(per_beam) * (2 * math.pi / per_beam)
    A, E = np.meshgrid(az, el)
    return _dirs(A.ravel(), E.ravel())


def frustum_dirs(width: int, height: int, hfov_deg: float, vfov_deg: float,
                 pitch_deg: float, yaw_deg: float) -> np.ndarray:
    """Pinhole depth camera, raster order, optical axis pitched then yawed."""
    fx = 0.5 * width / math.tan(math.radians(hfov_deg) / 2)
    fy = 0.5 * height / math.tan(math.radians(vfov_deg) / 2)
    u = (np.arange(width) + 0.5 - 0.5 * width) / fx
    v = (np.arange(height) + 0.5 - 0.5 * height) / fy
    U, V = np.meshgrid(u, v)            # [height, width]
    # camera frame expressed in the sensor frame: forward = x, left = y, up = z
    d = np.stack([np.ones_like(U), -U, -V], axis=-1).reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p = math.radians(pitch_deg)
    y = math.radians(yaw_deg)
    Ry = np.array([[math.cos(p), 0, -math.sin(p)], [0, 1, 0], [math.sin(p), 0, math.cos(p)]])
    Rz = np.array([[math.cos(y), -math.sin(y), 0], [math.sin(y), math.cos(y), 0], [0, 0, 1]])
    return d @ (Rz @ Ry).T


# --------------------------------------------------------------------------
# ray casting against the terrain
# --------------------------------------------------------------------------
def raycast(terrain: Terrain, origin: torch.Tensor, dirs: torch.Tensor, r_max: float,
            step: float = 0.05, bisect: int = 12, chunk: int = 1 << 19) -> torch.Tensor:
    """Distance along each ray to its first terrain crossing, NaN if none.

    ``origin``: [3] float64, ``dirs``: [M, 3] float64 unit vectors (world frame).
    Marches at ``step`` metres, then refines by bisection.
    """
    out = torch.full((dirs.shape[0],), float("nan"), dtype=torch.float64, device=dirs.device)
    n_steps = int(math.ceil(r_max / step))
    for c0 in range(0, dirs.shape[0], chunk):
        d = dirs[c0:c0 + chunk]
        m = d.shape[0]
        lo = torch.zeros(m, dtype=torch.float64, device=d.device)
        hit = torch.zeros(m, dtype=torch.bool, device=d.device)
        hi = torch.full((m,), float("nan"), dtype=torch.float64, device=d.device)
        for j in range(1, n_steps + 1):
            s = min(j * step, r_max)
            px = origin[0] + s * d[:, 0]
            py = origin[1] + s * d[:, 1]
            pz = origin[2] + s * d[:, 2]
            below = (pz <= terrain.height(px, py)) & ~hit
            hi = torch.where(below, torch.full_like(hi, s), hi)
            lo = torch.where(hit | below, lo, torch.full_like(lo, s))
            hit = hit | below
            if bool(hit.all()):
                break
        a, b = lo, torch.where(hit, hi, lo)
        for _ in range(bisect):
            mid = 0.5 * (a + b)
            px = origin[0] + mid * d[:, 0]
            py = origin[1] + mid * d[:, 1]
            pz = origin[2] + mid * d[:, 2]
            below = pz <= terrain.height(px, py)
            b = torch.where(below, mid, b)
            a = torch.where(below, a, mid)
        out[c0:c0 + m] = torch.where(hit, b, out[c0:c0 + m])
    return out


# --------------------------------------------------------------------------
# poses and trajectories
# --------------------------------------------------------------------------
def pose_matrix(x: float, y: float, z: float, yaw: float, pitch: float = 0.0,
                roll: float = 0.0) -> np.ndarray:
    """Row-major 3x4 sensor->world matrix, R = Rz(yaw) Ry(pitch) Rx(roll)."""
    cy, sy = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    cr, sr = math.cos(roll), math.sin(roll)
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1.0]])
    Ry = np.array([[cp, 0, sp], [0, 1.0, 0], [-sp, 0, cp]])
    Rx = np.array([[1.0, 0, 0], [0, cr, -sr], [0, sr, cr]])
    P = np.zeros((3, 4))
    P[:, :3] = Rz @ Ry @ Rx
    P[:, 3] = (x, y, z)
    return P


class Trajectory:
    """Smooth seeded path at ~1 m/s: heading = sum of 3 low-frequency sinusoids,
    roll/pitch <= 5 degrees, sensor held 0.5 m above the terrain."""

    def __init__(self, rng: np.random.Generator, terrain: Terrain, speed: float = 1.0,
                 height: float = 0.5):
        self.terrain = terrain
        self.speed = speed
        self.height = height
        self.psi0 = float(rng.uniform(0, 2 * math.pi))
        self.b = rng.uniform(0.2, 0.6, 3)
        self.w = rng.uniform(0.05, 0.4, 3)
        self.ph = rng.uniform(0, 2 * math.pi, 3)
        self.rp = rng.uniform(0, 2 * math.pi, 4)

    def heading(self, t):
        return self.psi0 + sum(self.b[k] * np.sin(self.w[k] * t + self.ph[k]) for k in range(3))

    def poses(self, n: int, hz: float = 10.0) -> List[np.ndarray]:
        sub = 20
        dt = 1.0 / (hz * sub)
        x = y = 0.0
        out = []
        t = 0.0
        for i in range(n):
            if i:
                for _ in range(sub):
                    psi = self.heading(t + 0.5 * dt)
                    x += self.speed * dt * math.cos(psi)
                    y += self.speed * dt * math.sin(psi)
                    t += dt
            g = float(self.terrain.height(torch.tensor([x], dtype=torch.float64),
                                          torch.tensor([y], dtype=torch.float64))[0])
            pitch = math.radians(5.0) * math.sin(0.7 * t + self.rp[0])
            roll = math.radians(5.0) * math.sin(0.9 * t + self.rp[1])
            out.append(pose_matrix(x, y, g + self.height, float(self.heading(t)), pitch, roll))
        return out


# --------------------------------------------------------------------------
# frames
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Frame:
    x: torch.Tensor          # [N] float32, sensor frame
    y: torch.Tensor
    z: torch.Tensor
    pose: np.ndarray         # [3, 4] float64 sensor->world
    t_ms: int

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def to(self, device) -> "Frame":
        return Frame(self.x.to(device), self.y.to(device), self.z.to(device), self.pose, self.t_ms)

    def numpy(self):
        return (self.x.cpu().numpy(), self.y.cpu().numpy(), self.z.cpu().numpy())


@dataclasses.dataclass
class Rig:
    """A set of ray patterns sharing one sensor origin, and the points each keeps."""
    patterns: Sequence[np.ndarray]      # each [M_k, 3] unit vectors, sensor frame
    counts: Sequence[int]               # points kept from each pattern
    r_max: Sequence[float]


def make_frame(rng: np.random.Generator, terrain: Terrain, pose: np.ndarray, rig: Rig,
               t_ms: int, outlier_frac: float, device="cpu", noise_k: float = 0.005,
               march_step: float = 0.05) -> Frame:
    """Ray-cast ``rig`` from ``pose``; add N(0, (noise_k d^2)^2) height noise and
    U(-1, 1) m outliers on a fraction of points; return sensor-frame points."""
    R = torch.as_tensor(pose[:, :3], dtype=torch.float64, device=device)
    o = torch.as_tensor(pose[:, 3], dtype=torch.float64, device=device)
    pts = []
    for pat, cnt, rmax in zip(rig.patterns, rig.counts, rig.r_max):
        if cnt == 0:
            continue
        ds = torch.as_tensor(pat, dtype=torch.float64, device=device)
        dw = ds @ R.T
        s = raycast(terrain, o, dw, rmax, step=march_step)
        ok = torch.nonzero(torch.isfinite(s)).squeeze(1).cpu().numpy()
        if len(ok) < cnt:
            raise ValueError(f"pattern yields {len(ok)} hits < {cnt} requested")
        keep = np.sort(rng.choice(ok, size=cnt, replace=False))
        keep_t = torch.as_tensor(keep, device=device)
        pw = o + s[keep_t, None] * dw[keep_t]
        d = s[keep_t]
        sigma = noise_k * d * d
        noise = torch.as_tensor(rng.standard_normal(cnt), dtype=torch.float64, device=device)
        z = pw[:, 2] + sigma * noise
        outl = torch.as_tensor(rng.random(cnt) < outlier_frac, device=device)
        jump = torch.as_tensor(rng.uniform(-1.0, 1.0, cnt), dtype=torch.float64, device=device)
        z = torch.where(outl, z + jump, z)
        pw = torch.stack([pw[:, 0], pw[:, 1], z], dim=1)
        pts.append((pw - o) @ R)        # R^T (p_w - o), row-vector form
    p = torch.cat(pts, 0).to(torch.float32)
    return Frame(p[:, 0].contiguous(), p[:, 1].contiguous(), p[:, 2].contiguous(),
                 pose.copy(), int(t_ms))


# --------------------------------------------------------------------------
# map specs, parameters, weights
# --------------------------------------------------------------------------
@dataclasses.dataclass
class MapSpec:
    nx: int
    ny: int
    resolution: float
    init_height: float = 0.0
    init_variance: float = 1e3


def default_params(spec: MapSpec) -> dict:
    """Per-map parameters of the synthetic workloads."""
    return dict(nx=spec.nx, ny=spec.ny, resolution=spec.resolution,
                init_height=spec.init_height, init_variance=spec.init_variance,
                noise_alpha=1e-4, gate_k=3.0, min_range=0.05, ray_step=spec.resolution,
                clear_normal_alpha=0.3, clear_min_age_ms=500)


def trav_weights(seed: int = SEED_BASE + 100) -> np.ndarray:
    """89 float32 values: w1[8,1,3,3], b1[8], w2[8], b2[1] (conv 3x3 1->8, ReLU, 1x1 8->1)."""
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(-1, 1, 72) / 3.0
    b1 = rng.uniform(-0.1, 0.1, 8)
    w2 = rng.uniform(-1, 1, 8) / math.sqrt(8.0)
    b2 = np.zeros(1)
    return np.concatenate([w1, b1, w2, b2]).astype(np.float32)


def _rng(cfg: int, *spawn_key) -> np.random.Generator:
    ss = np.random.SeedSequence(SEED_BASE + cfg, spawn_key=tuple(spawn_key))
    return np.random.default_rng(ss)


def _mixed_rig(rng, n: int, lidar_frac: float = 0.44, lidar_rmax: float = 12.0,
               cam_rmax: float = 4.0) -> Rig:
    """Dome LiDAR (64 beams) plus four depth frustums (87x58 deg, pitched -30 deg)."""
    n_l = int(round(lidar_frac * n))
    n_c = n - n_l
    per_cam = [n_c // 4 + (1 if k < n_c % 4 else 0) for k in range(4)]
    per_beam = max(64, int(math.ceil(1.6 * n_l / 64)))
    pats = [dome_lidar_dirs(rng, 64, per_beam)]
    counts = [n_l]
    rmax = [lidar_rmax]
    for k in range(4):
        px = max(1, per_cam[k])
        w = max(8, int(math.ceil(math.sqrt(1.6 * px * 87.0 / 58.0))))
        h = max(6, int(math.ceil(1.6 * px / w)))
        pats.append(frustum_dirs(w, h, 87.0, 58.0, -30.0, 90.0 * k))
        counts.append(per_cam[k])
        rmax.append(cam_rmax)
    return Rig(pats, counts, rmax)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
def cfg0(seed_offset: int = 0, device="cpu", n_points: int = 20000, n_frames: int = 1):
    """128x128 map at 0.04 m; 20k points from a sensor at (0, 0, 0.5) m with seeded
    yaw; elevations U[-60, -8] deg; sigma = 0.005 d^2; 2% outliers.
    ``n_frames`` > 1 repeats the sensor at the same pose with fresh draws (gating
    variant: frame 1 sets the prior, later frames are gated against it)."""
    rng = _rng(0, seed_offset)
    terrain = make_terrain(rng, n_boxes=0, extent=3.0)
    yaw = float(rng.uniform(0, 2 * math.pi))
    spec = MapSpec(128, 128, 0.04)
    g = float(terrain.height(torch.zeros(1, dtype=torch.float64),
                             torch.zeros(1, dtype=torch.float64))[0])
    pose = pose_matrix(0.0, 0.0, 0.5, yaw)
    del g
    frames = []
    for f in range(n_frames):
        dirs = random_cone_dirs(rng, int(n_points * 1.25) + 64, -60.0, -8.0)
        rig = Rig([dirs], [n_points], [8.0])
        frames.append(make_frame(rng, terrain, pose, rig, t_ms=100 * f, outlier_frac=0.02,
                                 device=device))
    return dict(spec=spec, params=default_params(spec), terrain=terrain, frames=frames,
                centers=[(0.0, 0.0)] * n_frames, weights=trav_weights())


def cfg1(n_frames: int = 100, device="cpu", n_points: int = 300000, seed_offset: int = 0):
    """400x400 map at 0.04 m; ``n_frames`` frames of 300k points (dome LiDAR + four
    depth frustums) along a seeded trajectory; 20 boxes; 3% outliers."""
    rng = _rng(1, seed_offset)
    terrain = make_terrain(rng, n_boxes=20, extent=8.0)
    traj = Trajectory(rng, terrain)
    spec = MapSpec(400, 400, 0.04)
    poses = traj.poses(n_frames)
    frames = []
    centers = []
    for f, P in enumerate(poses):
        rig = _mixed_rig(rng, n_points)
        frames.append(make_frame(rng, terrain, P, rig, t_ms=100 * f, outlier_frac=0.03,
                                 device=device))
        centers.append((float(P[0, 3]), float(P[1, 3])))
    return dict(spec=spec, params=default_params(spec), terrain=terrain, frames=frames,
                centers=centers, weights=trav_weights())


def paper_analogue(device="cpu"):
    """250x250 at 0.04 m (10 x 10 m) with one 43,017-point dome-LiDAR frame."""
    rng = _rng(5)
    terrain = make_terrain(rng, n_boxes=20, extent=5.0)
    spec = MapSpec(250, 250, 0.04)
    P = pose_matrix(0.0, 0.0, 0.5 + float(terrain.height(torch.zeros(1, dtype=torch.float64),
                                                           torch.zeros(1, dtype=torch.float64))[0]),
                    float(rng.uniform(0, 2 * math.pi)))
    n = 43017
    rig = Rig([dome_lidar_dirs(rng, 32, int(math.ceil(1.8 * n / 32)))], [n], [12.0])
    fr = make_frame(rng, terrain, P, rig, 0, 0.03, device=device)
    return dict(spec=spec, params=default_params(spec), terrain=terrain, frames=[fr],
                centers=[(float(P[0, 3]), float(P[1, 3]))], weights=trav_weights())


def cfg2(device="cpu", n_maps: int = 16, seed_offset: int = 0):
    """16 maps, side U{200..1000} cells at r ~ U[0.02, 0.1] m, each with one frame of
    N ~ logU[2e4, 1e6] points from the mixed rig; 3% outliers."""
    rng = _rng(2, seed_offset)
    items = []
    for m in range(n_maps):
        side = int(rng.integers(200, 1001))
        r = float(rng.uniform(0.02, 0.1))
        n = int(round(math.exp(rng.uniform(math.log(2e4), math.log(1e6)))))
        terrain = make_terrain(rng, n_boxes=20, extent=0.5 * side * r)
        spec = MapSpec(side, side, r)
        g = float(terrain.height(torch.zeros(1, dtype=torch.float64),
                                 torch.zeros(1, dtype=torch.float64))[0])
        P = pose_matrix(0.0, 0.0, g + 0.5, float(rng.uniform(0, 2 * math.pi)))
        rig = _mixed_rig(rng, n)
        fr = make_frame(rng, terrain, P, rig, 0, 0.03, device=device)
        items.append(dict(spec=spec, params=default_params(spec), terrain=terrain,
                          frames=[fr], centers=[(0.0, 0.0)]))
    return dict(items=items, weights=trav_weights())


def cfg3_rigs(n_robots: int = 64, seed_offset: int = 0):
    """64 simulated robots: map side U{256..800} at 0.04 m, frame size
    N ~ logU[5e4, 5e5] drawn once per robot, Poisson arrivals at 20 Hz each."""
    rng = _rng(3, seed_offset)
    robots = []
    for k in range(n_robots):
        side = int(rng.integers(256, 801))
        n = int(round(math.exp(rng.uniform(math.log(5e4), math.log(5e5)))))
        robots.append(dict(spec=MapSpec(side, side, 0.04), n_points=n, rate_hz=20.0,
                           seed=int(rng.integers(0, 2**31))))
    return robots


def cfg3(device="cpu", n_robots: int = 64, n_frames: int = 1, seed_offset: int = 0):
    """Frames for the robots of cfg3_rigs: each robot gets its own terrain
    (20 boxes), a seeded trajectory and ``n_frames`` frames of its drawn size
    from the mixed rig, 3% outliers.  Arrival times are drawn by the caller."""
    items = []
    for rb in cfg3_rigs(n_robots, seed_offset):
        rng = np.random.default_rng(rb["seed"])
        spec = rb["spec"]
        terrain = make_terrain(rng, n_boxes=20, extent=0.5 * spec.nx * spec.resolution)
        poses = Trajectory(rng, terrain).poses(n_frames)
        frames, centers = [], []
        for f, P in enumerate(poses):
            rig = _mixed_rig(rng, rb["n_points"])
            frames.append(make_frame(rng, terrain, P, rig, t_ms=100 * f, outlier_frac=0.03,
                                     device=device))
            centers.append((float(P[0, 3]), float(P[1, 3])))
        items.append(dict(spec=spec, params=default_params(spec), frames=frames,
                          centers=centers, rate_hz=rb["rate_hz"]))
    return dict(items=items, weights=trav_weights())


def cfg4(n_frames: int = 50, device="cpu", n_points: int = 4_000_000, seed_offset: int = 0):
    """2000x2000 map at 0.02 m; 4M-point frames from a 128-beam LiDAR (elevations
    U[-25, +15] deg, range 30 m); 10% outliers; 500 boxes."""
    rng = _rng(4, seed_offset)
    terrain = make_terrain(rng, n_boxes=500, extent=20.0)
    traj = Trajectory(rng, terrain)
    spec = MapSpec(2000, 2000, 0.02)
    poses = traj.poses(n_frames)
    frames, centers = [], []
    for f, P in enumerate(poses):
        per_beam = int(math.ceil(2.6 * n_points / 128))
        rig = Rig([spinning_lidar_dirs(rng, 128, per_beam, -25.0, 15.0)], [n_points], [30.0])
        frames.append(make_frame(rng, terrain, P, rig, 100 * f, 0.10, device=device,
                                 march_step=0.1))
        centers.append((float(P[0, 3]), float(P[1, 3])))
    return dict(spec=spec, params=default_params(spec), terrain=terrain, frames=frames,
                centers=centers, weights=trav_weights())
