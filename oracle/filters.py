"""Plain CPU oracle of the post-processing filters for legged locomotion
(Sec. II-I): minimum-filter inpainting and the smoothing filters.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.

The paper names the filters without formulas.  Readings (also listed with
their reasons in the design notes):
  * Inpainting: the empty cells (no estimate) form regions, connected through
    the four edge neighbours.  Each region takes the smallest height among the
    cells with an estimate that share an edge with it: the minimum along its
    occlusion border.  A region with no such cell stays NaN.  Cells with an
    estimate keep their height.
  * Smoothing works on a plain float32 grid (for instance an inpainted map).
    Border cells see the grid mirrored about the edge cell, without repeating
    it (index -1 reads index 1).  The window is ksize x ksize, ksize odd.
      - box: the mean of the window;
      - Gaussian: weights w_i proportional to exp(-i^2 / (2 sigma^2)) for
        i = -r..r, normalised to sum 1, applied along x and along y;
      - median: the middle value of the window (ksize 3 or 5).
    NaN anywhere in the window makes the output NaN (box and Gaussian by the
    arithmetic, median by rule).
Values are computed in float64 from the float32 inputs; the median is exact.
"""
from __future__ import annotations

import numpy as np

__all__ = ["inpaint_min", "gaussian_weights", "smooth_box", "smooth_gaussian", "smooth_median",
           "mirror_pad"]

F32 = np.float32
F64 = np.float64


def inpaint_min(h: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """Minimum-filter inpainting (Sec. II-I), float32 [ny, nx].

    Regions of empty cells are found by flood fill over edge neighbours; each
    is filled with the minimum height of the cells with an estimate on its
    border."""
    h = np.asarray(h, F32)
    ok = np.asarray(valid) != 0
    ny, nx = h.shape
    out = np.where(ok, h, F32(np.nan)).astype(F32)
    seen = ok.copy()
    steps = ((0, 1), (0, -1), (1, 0), (-1, 0))
    for sy in range(ny):
        for sx in range(nx):
            if seen[sy, sx]:
                continue
            region = [(sy, sx)]
            seen[sy, sx] = True
            best = np.inf
            k = 0
            while k < len(region):
                y, x = region[k]
                k += 1
                for ddy, ddx in steps:
                    yy, xx = y + ddy, x + ddx
                    if not (0 <= yy < ny and 0 <= xx < nx):
                        continue
                    if ok[yy, xx]:
                        best = min(best, float(h[yy, xx]))
                    elif not seen[yy, xx]:
                        seen[yy, xx] = True
                        region.append((yy, xx))
            if best < np.inf:
                ys, xs = zip(*region)
                out[list(ys), list(xs)] = F32(best)
    return out


def mirror_pad(x: np.ndarray, r: int) -> np.ndarray:
    """Pad by r on every side, mirrored about the edge cells (not repeated)."""
    ny, nx = x.shape
    if r >= nx or r >= ny:
        raise ValueError("grid smaller than the filter radius + 1")
    iy = np.abs(np.arange(-r, ny + r))
    iy = np.where(iy > ny - 1, 2 * (ny - 1) - iy, iy)
    ix = np.abs(np.arange(-r, nx + r))
    ix = np.where(ix > nx - 1, 2 * (nx - 1) - ix, ix)
    return x[np.ix_(iy, ix)]


def _windows(x: np.ndarray, ksize: int) -> np.ndarray:
    """[ny, nx, ksize, ksize] windows of the mirrored grid, as float64."""
    if ksize < 1 or ksize % 2 == 0:
        raise ValueError("ksize must be odd and positive")
    r = ksize // 2
    ny, nx = x.shape
    xp = mirror_pad(np.asarray(x, F32).astype(F64), r)
    w = np.empty((ny, nx, ksize, ksize), F64)
    for dy in range(ksize):
        for dx in range(ksize):
            w[:, :, dy, dx] = xp[dy:dy + ny, dx:dx + nx]
    return w


def smooth_box(x: np.ndarray, ksize: int) -> np.ndarray:
    """Box blur: the mean over the ksize x ksize window, float64 [ny, nx]."""
    return _windows(x, ksize).mean(axis=(2, 3))


def gaussian_weights(ksize: int, sigma: float) -> np.ndarray:
    """Normalised sampled Gaussian over i = -r..r (float64); sigma is float32."""
    if not sigma > 0:
        raise ValueError("sigma must be positive")
    r = ksize // 2
    s = F64(F32(sigma))
    i = np.arange(-r, r + 1, dtype=F64)
    w = np.exp(-(i * i) / (2.0 * s * s))
    return w / w.sum()


def smooth_gaussian(x: np.ndarray, ksize: int, sigma: float) -> np.ndarray:
    """Gaussian blur, float64 [ny, nx]: the window weighted by w_dy * w_dx."""
    w = gaussian_weights(ksize, sigma)
    return np.einsum("yxij,i,j->yx", _windows(x, ksize), w, w)


def smooth_median(x: np.ndarray, ksize: int) -> np.ndarray:
    """Median filter, float32 [ny, nx]; NaN if the window holds a NaN."""
    if ksize not in (3, 5):
        raise ValueError("the median takes ksize 3 or 5")
    w = _windows(x, ksize).reshape(x.shape + (ksize * ksize,))
    out = np.median(w, axis=2)
    out[np.isnan(w).any(axis=2)] = np.nan
    return out.astype(F32)
