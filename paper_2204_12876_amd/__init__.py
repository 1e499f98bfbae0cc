"""MI355X-native GPU elevation-map fusion (arXiv 2204.12876 hot path).

The library is ``libemx.so``, a C ABI over hand-written HIP kernels for gfx950;
its calls are declared in include/emx.h.  This package binds it with ctypes:
  * ``_emx`` mirrors the C calls one-to-one;
  * ``ElevationMap`` holds one map's device state in torch tensors and forwards
    each method to the C call of the same name, on torch's current stream.
Nothing here computes any part of the path.  Without the built library or a
GPU every call raises.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _emx
from ._emx import EmxError, make_params  # noqa: F401

__all__ = ["ElevationMap", "PipelineBatch", "BatchEntry", "EmxError", "make_params", "lib_path",
           "aligned_empty", "smooth"]

lib_path = _emx.LIB_PATH


def _require_gpu(device):
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2204_12876_amd needs a ROCm GPU; none is visible")
    _emx.lib()
    return torch.device(device if device is not None else "cuda")


def aligned_empty(nbytes: int, device, align: int = 256) -> torch.Tensor:
    """A uint8 device tensor of ``nbytes`` whose data pointer is ``align``-aligned."""
    raw = torch.empty(max(1, nbytes) + align, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % align
    return raw[off:off + max(1, nbytes)]


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _f32(t: torch.Tensor, device) -> torch.Tensor:
    if t.dtype != torch.float32 or t.device != device or not t.is_contiguous():
        raise ValueError("point arrays must be contiguous float32 tensors on the map's device")
    return t


class ElevationMap:
    """One robot-centric map.  Its state lives in a caller-side torch buffer."""

    def __init__(self, params: dict, cx: float = 0.0, cy: float = 0.0, t0_ms: int = 0,
                 device=None):
        self.device = _require_gpu(device)
        self.params = dict(params)
        self.p = make_params(params)
        self.nx, self.ny = self.p.nx, self.p.ny
        nbytes = _emx.state_bytes(self.p)
        if nbytes == 0:
            raise EmxError(_emx.EMX_EINVAL, _emx.last_error())
        self._state = aligned_empty(nbytes, self.device)
        self._scratch = None
        self._scratch_bytes = 0
        self.handle = _emx.init_map(self.p, float(cx), float(cy), int(t0_ms),
                                    self._state.data_ptr(), nbytes, _stream(self.device))

    def close(self):
        if getattr(self, "handle", None):
            _emx.free_map(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- calls
    def _frame(self, x, y, z, pose, t_ms):
        x, y, z = (_f32(t, self.device) for t in (x, y, z))
        n = x.numel()
        if y.numel() != n or z.numel() != n:
            raise ValueError("x, y, z differ in length")
        return _emx.make_frame(x.data_ptr(), y.data_ptr(), z.data_ptr(), n, pose, t_ms), n

    def scratch(self, n: int) -> torch.Tensor:
        need = max(_emx.scratch_bytes(self.p, n), _emx.drift_scratch_bytes(n))
        if self._scratch is None or self._scratch_bytes < need:
            self._scratch = aligned_empty(need, self.device)
            self._scratch_bytes = need
        return self._scratch

    def move_map(self, cx: float, cy: float):
        _emx.move_map(self.handle, float(cx), float(cy), _stream(self.device))

    def fuse_points(self, x, y, z, pose, t_ms: int, out_cell: torch.Tensor = None,
                    out_accept: torch.Tensor = None, scratch: torch.Tensor = None):
        f, n = self._frame(x, y, z, pose, t_ms)
        s = scratch if scratch is not None else self.scratch(n)
        if out_cell is not None and (out_cell.dtype != torch.int32 or out_cell.numel() < n):
            raise ValueError("out_cell must be int32 with n elements")
        if out_accept is not None and (out_accept.dtype != torch.uint8 or out_accept.numel() < n):
            raise ValueError("out_accept must be uint8 with n elements")
        _emx.fuse_points(self.handle, f, s.data_ptr(), s.numel(),
                         out_cell.data_ptr() if out_cell is not None else 0,
                         out_accept.data_ptr() if out_accept is not None else 0,
                         _stream(self.device))

    def fuse_points_noalloc(self, x, y, z, pose, t_ms: int, out_cell: torch.Tensor = None,
                            out_accept: torch.Tensor = None):
        """fuse_points on the library's built-in scratch: allocates nothing."""
        f, n = self._frame(x, y, z, pose, t_ms)
        if out_cell is not None and (out_cell.dtype != torch.int32 or out_cell.numel() < n):
            raise ValueError("out_cell must be int32 with n elements")
        if out_accept is not None and (out_accept.dtype != torch.uint8 or out_accept.numel() < n):
            raise ValueError("out_accept must be uint8 with n elements")
        _emx.fuse_points_noalloc(self.handle, f,
                                 out_cell.data_ptr() if out_cell is not None else 0,
                                 out_accept.data_ptr() if out_accept is not None else 0,
                                 _stream(self.device))

    def compensate_drift(self, x, y, z, pose, t_ms: int, trav_min: float,
                         scratch: torch.Tensor = None):
        """Shift the valid heights by the frame's mean error on flat ground
        (Sec. II-D); call before fuse_points with the same frame.  Returns
        device tensors (mean float64[1], count int64[1]) without waiting."""
        f, n = self._frame(x, y, z, pose, t_ms)
        s = scratch if scratch is not None else self.scratch(n)
        mean = torch.empty(1, dtype=torch.float64, device=self.device)
        count = torch.empty(1, dtype=torch.int64, device=self.device)
        _emx.compensate_drift(self.handle, f, float(trav_min), s.data_ptr(), s.numel(),
                              mean.data_ptr(), count.data_ptr(), _stream(self.device))
        return mean, count

    def move_fuse_points(self, cx: float, cy: float, x, y, z, pose, t_ms: int,
                         out_cell: torch.Tensor = None, out_accept: torch.Tensor = None,
                         scratch: torch.Tensor = None):
        """move_map(cx, cy) then fuse_points(...), bit for bit, in one pass."""
        f, n = self._frame(x, y, z, pose, t_ms)
        s = scratch if scratch is not None else self.scratch(n)
        if out_cell is not None and (out_cell.dtype != torch.int32 or out_cell.numel() < n):
            raise ValueError("out_cell must be int32 with n elements")
        if out_accept is not None and (out_accept.dtype != torch.uint8 or out_accept.numel() < n):
            raise ValueError("out_accept must be uint8 with n elements")
        _emx.move_fuse_points(self.handle, float(cx), float(cy), f, s.data_ptr(), s.numel(),
                              out_cell.data_ptr() if out_cell is not None else 0,
                              out_accept.data_ptr() if out_accept is not None else 0,
                              _stream(self.device))

    def clear_visibility(self, x, y, z, pose, t_ms: int, out_cleared: torch.Tensor = None,
                         scratch: torch.Tensor = None):
        f, n = self._frame(x, y, z, pose, t_ms)
        s = scratch if scratch is not None else self.scratch(n)
        if out_cleared is not None and (out_cleared.dtype != torch.uint8
                                        or out_cleared.numel() < self.nx * self.ny):
            raise ValueError("out_cleared must be uint8 with nx*ny elements")
        _emx.clear_visibility(self.handle, f, s.data_ptr(), s.numel(),
                              out_cleared.data_ptr() if out_cleared is not None else 0,
                              _stream(self.device))

    def overlap_clear(self, robot_xyz, radius: float, threshold: float,
                      out_cleared: torch.Tensor = None):
        """Remove valid cells within ``radius`` of the robot (horizontally) whose
        height differs from the robot's by more than ``threshold`` (Sec. II-F)."""
        if out_cleared is not None and (out_cleared.dtype != torch.uint8
                                        or out_cleared.numel() < self.nx * self.ny):
            raise ValueError("out_cleared must be uint8 with nx*ny elements")
        rx, ry, rz = (float(v) for v in robot_xyz)
        _emx.overlap_clear(self.handle, rx, ry, rz, radius, threshold,
                           out_cleared.data_ptr() if out_cleared is not None else 0,
                           _stream(self.device))

    def inpaint_min(self, out: torch.Tensor = None) -> torch.Tensor:
        """Minimum-filter inpainting (Sec. II-I) of the height layer into a new
        [ny, nx] float32 tensor (or ``out``); the map is not changed."""
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        elif (out.dtype != torch.float32 or out.numel() != self.nx * self.ny
              or not out.is_contiguous() or out.device != self.device):
            raise ValueError("out must be a contiguous float32 [ny, nx] tensor on the device")
        need = _emx.inpaint_scratch_bytes(self.p)
        if getattr(self, "_inpaint_scratch", None) is None:
            self._inpaint_scratch = aligned_empty(need, self.device)
        _emx.inpaint_min(self.handle, out.data_ptr(), self._inpaint_scratch.data_ptr(), need,
                         _stream(self.device))
        return out

    def upper_bound(self) -> torch.Tensor:
        """The upper bound layer (Sec. II-H) in local cell order, a [ny, nx]
        float32 copy; the map must have been created with upper_bound=1."""
        return self.local(_emx.LAYER_UPPER)

    def compute_normals(self):
        _emx.compute_normals(self.handle, _stream(self.device))

    def traversability(self, weights: torch.Tensor):
        if weights.dtype != torch.float32 or weights.numel() != 89 or weights.device != self.device:
            raise ValueError("weights must be 89 float32 values on the map's device")
        _emx.traversability(self.handle, weights.contiguous().data_ptr(), _stream(self.device))

    def normals_traversability(self, weights: torch.Tensor):
        """compute_normals then traversability, in one pass over the map."""
        if weights.dtype != torch.float32 or weights.numel() != 89 or weights.device != self.device:
            raise ValueError("weights must be 89 float32 values on the map's device")
        _emx.normals_traversability(self.handle, weights.contiguous().data_ptr(),
                                    _stream(self.device))

    # ----------------------------------------------------------------- state
    def layer(self, layer_id: int) -> torch.Tensor:
        """A [ny, nx] view of one layer as stored: a ring with origin
        ``origin()`` (local cell (ix, iy) at row (iy + oy) % ny, column
        (ix + ox) % nx)."""
        ptr = _emx.layer(self.handle, layer_id)
        off = ptr - self._state.data_ptr()
        C = self.nx * self.ny
        if layer_id == _emx.LAYER_VALID:
            return self._state[off:off + C].view(self.ny, self.nx)
        dt = torch.int32 if layer_id == _emx.LAYER_TIME else torch.float32
        return self._state[off:off + 4 * C].view(dt).view(self.ny, self.nx)

    def origin(self):
        """The ring origin (ox, oy) of the stored layers."""
        return _emx.map_origin(self.handle)

    def local(self, layer_id: int) -> torch.Tensor:
        """One layer in local cell order (a copy of the ring, unrolled)."""
        ox, oy = self.origin()
        return torch.roll(self.layer(layer_id), shifts=(-oy, -ox), dims=(0, 1)).contiguous()

    def info(self):
        return _emx.map_info(self.handle)

    def export_state(self) -> torch.Tensor:
        out = aligned_empty(_emx.export_bytes(self.p), self.device)
        _emx.export_state(self.handle, out.data_ptr(), _stream(self.device))
        return out

    def import_state(self, packed: torch.Tensor):
        if packed.numel() < _emx.export_bytes(self.p) or packed.device != self.device:
            raise ValueError("packed state too small or on the wrong device")
        packed = packed.contiguous()
        _emx.import_state(self.handle, packed.data_ptr(), _stream(self.device))
        torch.cuda.current_stream(self.device).synchronize()

    def state_numpy(self) -> dict:
        """Layers copied to host numpy arrays (synchronises the stream)."""
        b = self.export_state().cpu().numpy()
        return unpack_state(b, self.nx, self.ny)

    def load_numpy(self, h, v, t_upd, valid, nrm, trav):
        """Overwrite the layers from host arrays (stage-synchronised testing)."""
        self.import_state(torch.from_numpy(pack_state(h, v, t_upd, valid, nrm, trav)).to(
            self.device))


class BatchEntry:
    """One map and its frame for PipelineBatch.run (arguments as the plain calls)."""

    def __init__(self, emap: "ElevationMap", x=None, y=None, z=None, pose=None, t_ms: int = 0,
                 center=None, weights: torch.Tensor = None, stages: int = _emx.STAGE_ALL,
                 out_cell: torch.Tensor = None, out_accept: torch.Tensor = None,
                 out_cleared: torch.Tensor = None):
        self.map = emap
        self.x, self.y, self.z = x, y, z
        self.pose = pose
        self.t_ms = t_ms
        self.center = center
        self.weights = weights
        self.stages = stages
        self.out_cell, self.out_accept, self.out_cleared = out_cell, out_accept, out_cleared

    def item(self) -> "_emx.BatchItem":
        it = _emx.BatchItem()
        it.map = self.map.handle
        if self.x is not None:
            f, _ = self.map._frame(self.x, self.y, self.z, self.pose, self.t_ms)
            it.frame = f
        if self.center is not None:
            it.cx, it.cy = float(self.center[0]), float(self.center[1])
        elif self.stages & _emx.STAGE_MOVE:
            raise ValueError("a move needs a centre")
        if self.weights is not None:
            it.d_weights = self.weights.data_ptr()
        for name in ("out_cell", "out_accept", "out_cleared"):
            t = getattr(self, name)
            if t is not None:
                setattr(it, "d_" + name, t.data_ptr())
        it.stages = int(self.stages)
        return it


class PipelineBatch:
    """Batched executor: many maps and frames through the whole path in one
    graph launch (emx_pipeline_batch).  Owns its device scratch (torch)."""

    def __init__(self, tuning: str = None, device=None):
        self.device = _require_gpu(device)
        self.handle = _emx.batch_create(tuning)
        self._scratch = None
        self._scratch_bytes = 0

    @property
    def tuning(self) -> str:
        return _emx.batch_tuning(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            _emx.batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, nbytes: int):
        """Allocate the scratch buffer now (graphs are cached per address)."""
        if self._scratch is None or self._scratch_bytes < nbytes:
            self._scratch = aligned_empty(nbytes, self.device)
            self._scratch_bytes = int(nbytes)

    def stats(self):
        """(batches run, graphs captured)."""
        return _emx.batch_stats(self.handle)

    def scratch_buffer(self) -> torch.Tensor:
        """The executor's scratch buffer (None before the first reserve or run)."""
        return self._scratch

    def scratch_bound(self, largest_params: dict, max_items: int, max_points: int) -> int:
        return _emx.batch_scratch_bound(self.handle, make_params(largest_params), max_items,
                                        max_points)

    def run_items(self, arr, n: int, stream: int):
        """Run a ctypes array of emx_batch_item on ``stream``."""
        if self._scratch is not None:
            try:
                _emx.pipeline_batch(self.handle, arr, n, self._scratch.data_ptr(),
                                    self._scratch_bytes, stream)
                return
            except EmxError as e:
                if e.status != _emx.EMX_ENOMEM:
                    raise
        need = _emx.batch_scratch_bytes(self.handle, arr, n)
        if need == 0:
            raise EmxError(_emx.EMX_EINVAL, _emx.last_error())
        # keep one buffer, generously sized: graphs are cached per scratch address
        self.reserve(max(need, 2 * self._scratch_bytes))
        _emx.pipeline_batch(self.handle, arr, n, self._scratch.data_ptr(), self._scratch_bytes,
                            stream)

    def run(self, entries):
        arr = _emx.make_batch_items([e.item() for e in entries])
        self.run_items(arr, len(entries), _stream(self.device))


_SMOOTH_KINDS = {"box": _emx.SMOOTH_BOX, "gaussian": _emx.SMOOTH_GAUSSIAN,
                 "median": _emx.SMOOTH_MEDIAN}


def smooth(x: torch.Tensor, kind: str, ksize: int, sigma: float = 0.0,
           out: torch.Tensor = None) -> torch.Tensor:
    """Box, Gaussian or median smoothing of a [ny, nx] float32 grid on the GPU
    (Sec. II-I), with the border mirrored about the edge cells."""
    if kind not in _SMOOTH_KINDS:
        raise ValueError(f"kind must be one of {sorted(_SMOOTH_KINDS)}")
    if x.dim() != 2 or x.dtype != torch.float32 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("x must be a contiguous float32 [ny, nx] tensor on the GPU")
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must match x")
    ny, nx = x.shape
    _emx.smooth(x.data_ptr(), out.data_ptr(), nx, ny, _SMOOTH_KINDS[kind], ksize, sigma,
                _stream(x.device))
    return out


def pack_state(h, v, t_upd, valid, nrm, trav) -> np.ndarray:
    """Host packing in the export format: h, v, t, nx, ny, nz, trav, valid."""
    parts = [np.ascontiguousarray(h, np.float32).view(np.uint8).ravel(),
             np.ascontiguousarray(v, np.float32).view(np.uint8).ravel(),
             np.ascontiguousarray(t_upd, np.int32).view(np.uint8).ravel(),
             np.ascontiguousarray(nrm[0], np.float32).view(np.uint8).ravel(),
             np.ascontiguousarray(nrm[1], np.float32).view(np.uint8).ravel(),
             np.ascontiguousarray(nrm[2], np.float32).view(np.uint8).ravel(),
             np.ascontiguousarray(trav, np.float32).view(np.uint8).ravel(),
             np.ascontiguousarray(valid, np.uint8).ravel()]
    return np.concatenate(parts)


def unpack_state(b: np.ndarray, nx: int, ny: int) -> dict:
    C = nx * ny
    out = {}
    off = 0
    for name, dt in [("h", np.float32), ("v", np.float32), ("t_upd", np.int32),
                     ("nx", np.float32), ("ny", np.float32), ("nz", np.float32),
                     ("trav", np.float32)]:
        out[name] = b[off:off + 4 * C].view(dt).reshape(ny, nx).copy()
        off += 4 * C
    out["valid"] = b[off:off + C].reshape(ny, nx).copy()
    out["nrm"] = np.stack([out["nx"], out["ny"], out["nz"]])
    return out
