"""ctypes binding of libemx.so (argument marshalling only).

Every call forwards to the C ABI declared in include/emx.h under the same name.
PyTorch provides device memory and streams; no step of the path runs here.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_float, c_int32, c_int64,
                    c_size_t, c_uint32, c_void_p, create_string_buffer)

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libemx.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "emx.h")

EMX_OK = 0
EMX_EINVAL = -1
EMX_ENOMEM = -2
EMX_EHIP = -3
EMX_ESTATE = -5

LAYER_HEIGHT, LAYER_VARIANCE, LAYER_TIME = 0, 1, 2
LAYER_NORMAL_X, LAYER_NORMAL_Y, LAYER_NORMAL_Z = 3, 4, 5
LAYER_TRAV, LAYER_VALID, LAYER_UPPER = 6, 7, 8


class EmxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"emx status {status}: {msg}")
        self.status = status


class Params(Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("resolution", c_double),
                ("init_height", c_float), ("init_variance", c_float), ("noise_alpha", c_float),
                ("gate_k", c_float), ("min_range", c_float), ("ray_step", c_float),
                ("clear_normal_alpha", c_float), ("clear_min_age_ms", c_int32),
                ("time_variance", c_float), ("wall_min_count", c_int32),
                ("upper_bound", c_int32), ("excl_on", c_int32), ("excl_theta", c_float),
                ("excl_b", c_float), ("excl_c", c_float), ("excl_d", c_float),
                ("outlier_variance", c_float)]


class Frame(Structure):
    _fields_ = [("x", c_void_p), ("y", c_void_p), ("z", c_void_p), ("n", c_int64),
                ("pose", c_double * 12), ("t_ms", c_int64)]


class BatchItem(Structure):
    _fields_ = [("map", c_void_p), ("frame", Frame), ("cx", c_double), ("cy", c_double),
                ("d_weights", c_void_p), ("d_out_cell", c_void_p), ("d_out_accept", c_void_p),
                ("d_out_cleared", c_void_p), ("stages", c_uint32)]


STAGE_MOVE, STAGE_FUSE, STAGE_CLEAR, STAGE_NORMALS, STAGE_TRAV = 1, 2, 4, 8, 16
STAGE_ALL = 31
BATCH_MAX_ITEMS = 64


_SIGS = {
    "emx_version": (c_char_p, []),
    "emx_last_error": (c_char_p, []),
    "emx_params_check": (c_int32, [POINTER(Params)]),
    "emx_state_bytes": (c_size_t, [POINTER(Params)]),
    "emx_scratch_bytes": (c_size_t, [POINTER(Params), c_int64]),
    "emx_export_bytes": (c_size_t, [POINTER(Params)]),
    "emx_init_map": (c_int32, [POINTER(Params), c_double, c_double, c_int64, c_void_p, c_size_t,
                               c_void_p, POINTER(c_void_p)]),
    "emx_free_map": (c_int32, [c_void_p]),
    "emx_move_map": (c_int32, [c_void_p, c_double, c_double, c_void_p]),
    "emx_fuse_points": (c_int32, [c_void_p, POINTER(Frame), c_void_p, c_size_t, c_void_p,
                                  c_void_p, c_void_p]),
    "emx_noalloc_scratch_limit": (c_size_t, []),
    "emx_fuse_points_noalloc": (c_int32, [c_void_p, POINTER(Frame), c_void_p, c_void_p,
                                          c_void_p]),
    "emx_move_fuse_points": (c_int32, [c_void_p, c_double, c_double, POINTER(Frame), c_void_p,
                                       c_size_t, c_void_p, c_void_p, c_void_p]),
    "emx_clear_visibility": (c_int32, [c_void_p, POINTER(Frame), c_void_p, c_size_t, c_void_p,
                                       c_void_p]),
    "emx_drift_scratch_bytes": (c_size_t, [c_int64]),
    "emx_compensate_drift": (c_int32, [c_void_p, POINTER(Frame), c_float, c_void_p, c_size_t,
                                       c_void_p, c_void_p, c_void_p]),
    "emx_overlap_clear": (c_int32, [c_void_p, c_double, c_double, c_double, c_float, c_float,
                                    c_void_p, c_void_p]),
    "emx_inpaint_scratch_bytes": (c_size_t, [POINTER(Params)]),
    "emx_inpaint_min": (c_int32, [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "emx_smooth": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32, c_float,
                             c_void_p]),
    "emx_compute_normals": (c_int32, [c_void_p, c_void_p]),
    "emx_traversability": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "emx_normals_traversability": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "emx_layer": (c_int32, [c_void_p, c_int32, POINTER(c_void_p)]),
    "emx_map_info": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int64)]),
    "emx_map_origin": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "emx_export_state": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "emx_import_state": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "emx_batch_create": (c_int32, [c_char_p, POINTER(c_void_p)]),
    "emx_batch_destroy": (c_int32, [c_void_p]),
    "emx_batch_tuning": (c_int32, [c_void_p, c_char_p, c_size_t]),
    "emx_batch_scratch_bytes": (c_size_t, [c_void_p, POINTER(BatchItem), c_int32]),
    "emx_batch_stats": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64)]),
    "emx_batch_scratch_bound": (c_size_t, [c_void_p, POINTER(Params), c_int32, c_int64]),
    "emx_timing_begin": (c_int32, []),
    "emx_timing_end": (c_int32, [c_char_p, c_size_t]),
    "emx_pipeline_batch": (c_int32, [c_void_p, POINTER(BatchItem), c_int32, c_void_p, c_size_t,
                                     c_void_p]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libemx.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols(path: str = HEADER):
    """Function names declared in include/emx.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(emx_[a-z_]+)\s*\(", txt)))


def last_error() -> str:
    return lib().emx_last_error().decode()


def check(status: int):
    if status != EMX_OK:
        raise EmxError(status, last_error())


def make_params(d: dict) -> Params:
    p = Params()
    p.nx = int(d["nx"])
    p.ny = int(d["ny"])
    p.resolution = float(d["resolution"])
    p.init_height = float(d.get("init_height", 0.0))
    p.init_variance = float(d.get("init_variance", 1e3))
    p.noise_alpha = float(d.get("noise_alpha", 1e-4))
    p.gate_k = float(d.get("gate_k", 3.0))
    p.min_range = float(d.get("min_range", 0.05))
    p.ray_step = float(d.get("ray_step", d["resolution"]))
    p.clear_normal_alpha = float(d.get("clear_normal_alpha", 0.3))
    p.clear_min_age_ms = int(d.get("clear_min_age_ms", 500))
    p.time_variance = float(d.get("time_variance", 0.0))
    p.wall_min_count = int(d.get("wall_min_count", 0))
    p.upper_bound = int(d.get("upper_bound", 0))
    p.excl_on = int(d.get("excl_on", 0))
    p.excl_theta = float(d.get("excl_theta", 0.0))
    p.excl_b = float(d.get("excl_b", 0.0))
    p.excl_c = float(d.get("excl_c", 0.0))
    p.excl_d = float(d.get("excl_d", 0.0))
    p.outlier_variance = float(d.get("outlier_variance", 0.0))
    return p


def make_frame(x_ptr: int, y_ptr: int, z_ptr: int, n: int, pose, t_ms: int) -> Frame:
    f = Frame()
    f.x, f.y, f.z = c_void_p(x_ptr), c_void_p(y_ptr), c_void_p(z_ptr)
    f.n = int(n)
    P = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(12))
    for k in range(12):
        f.pose[k] = float(P[k])
    f.t_ms = int(t_ms)
    return f


# ------------------------------------------------------------ thin wrappers
def params_check(p: Params) -> int:
    return lib().emx_params_check(byref(p))


def state_bytes(p: Params) -> int:
    return lib().emx_state_bytes(byref(p))


def scratch_bytes(p: Params, max_points: int) -> int:
    return lib().emx_scratch_bytes(byref(p), int(max_points))


def export_bytes(p: Params) -> int:
    return lib().emx_export_bytes(byref(p))


def init_map(p: Params, cx: float, cy: float, t0_ms: int, d_state: int, state_bytes_: int,
             stream: int) -> int:
    h = c_void_p()
    check(lib().emx_init_map(byref(p), cx, cy, int(t0_ms), c_void_p(d_state), state_bytes_,
                             c_void_p(stream), byref(h)))
    return h.value


def free_map(h: int):
    check(lib().emx_free_map(c_void_p(h)))


def move_map(h: int, cx: float, cy: float, stream: int):
    check(lib().emx_move_map(c_void_p(h), cx, cy, c_void_p(stream)))


def fuse_points(h: int, f: Frame, d_scratch: int, nbytes: int, d_out_cell: int,
                d_out_accept: int, stream: int):
    check(lib().emx_fuse_points(c_void_p(h), byref(f), c_void_p(d_scratch), nbytes,
                                c_void_p(d_out_cell or None), c_void_p(d_out_accept or None),
                                c_void_p(stream)))


def noalloc_scratch_limit() -> int:
    return int(lib().emx_noalloc_scratch_limit())


def fuse_points_noalloc(h: int, f: Frame, d_out_cell: int, d_out_accept: int, stream: int):
    check(lib().emx_fuse_points_noalloc(c_void_p(h), byref(f), c_void_p(d_out_cell or None),
                                        c_void_p(d_out_accept or None), c_void_p(stream)))


SMOOTH_BOX, SMOOTH_GAUSSIAN, SMOOTH_MEDIAN = 0, 1, 2


def overlap_clear(h: int, rx: float, ry: float, rz: float, radius: float, threshold: float,
                  d_out_cleared: int, stream: int):
    check(lib().emx_overlap_clear(c_void_p(h), float(rx), float(ry), float(rz), float(radius),
                                  float(threshold), c_void_p(d_out_cleared or None),
                                  c_void_p(stream)))


def inpaint_scratch_bytes(p: Params) -> int:
    return lib().emx_inpaint_scratch_bytes(byref(p))


def inpaint_min(h: int, d_out: int, d_scratch: int, nbytes: int, stream: int):
    check(lib().emx_inpaint_min(c_void_p(h), c_void_p(d_out), c_void_p(d_scratch or None),
                                nbytes, c_void_p(stream)))


def smooth(d_in: int, d_out: int, nx: int, ny: int, kind: int, ksize: int, sigma: float,
           stream: int):
    check(lib().emx_smooth(c_void_p(d_in), c_void_p(d_out), int(nx), int(ny), int(kind),
                           int(ksize), float(sigma), c_void_p(stream)))


def drift_scratch_bytes(max_points: int) -> int:
    return lib().emx_drift_scratch_bytes(int(max_points))


def compensate_drift(h: int, f: Frame, trav_min: float, d_scratch: int, nbytes: int,
                     d_out_mean: int, d_out_count: int, stream: int):
    check(lib().emx_compensate_drift(c_void_p(h), byref(f), float(trav_min),
                                     c_void_p(d_scratch or None), nbytes,
                                     c_void_p(d_out_mean or None), c_void_p(d_out_count or None),
                                     c_void_p(stream)))


def move_fuse_points(h: int, cx: float, cy: float, f: Frame, d_scratch: int, nbytes: int,
                     d_out_cell: int, d_out_accept: int, stream: int):
    check(lib().emx_move_fuse_points(c_void_p(h), float(cx), float(cy), byref(f),
                                     c_void_p(d_scratch), nbytes, c_void_p(d_out_cell or None),
                                     c_void_p(d_out_accept or None), c_void_p(stream)))


def clear_visibility(h: int, f: Frame, d_scratch: int, nbytes: int, d_out_cleared: int,
                     stream: int):
    check(lib().emx_clear_visibility(c_void_p(h), byref(f), c_void_p(d_scratch or None), nbytes,
                                     c_void_p(d_out_cleared or None), c_void_p(stream)))


def compute_normals(h: int, stream: int):
    check(lib().emx_compute_normals(c_void_p(h), c_void_p(stream)))


def traversability(h: int, d_weights: int, stream: int):
    check(lib().emx_traversability(c_void_p(h), c_void_p(d_weights), c_void_p(stream)))


def normals_traversability(h: int, d_weights: int, stream: int):
    check(lib().emx_normals_traversability(c_void_p(h), c_void_p(d_weights), c_void_p(stream)))


def layer(h: int, layer_id: int) -> int:
    p = c_void_p()
    check(lib().emx_layer(c_void_p(h), int(layer_id), byref(p)))
    return p.value


def map_origin(h: int):
    ox, oy = c_int32(), c_int32()
    check(lib().emx_map_origin(c_void_p(h), byref(ox), byref(oy)))
    return ox.value, oy.value


def map_info(h: int):
    gx, gy, t0 = c_int32(), c_int32(), c_int64()
    check(lib().emx_map_info(c_void_p(h), byref(gx), byref(gy), byref(t0)))
    return gx.value, gy.value, t0.value


def export_state(h: int, d_dst: int, stream: int):
    check(lib().emx_export_state(c_void_p(h), c_void_p(d_dst), c_void_p(stream)))


def import_state(h: int, d_src: int, stream: int):
    check(lib().emx_import_state(c_void_p(h), c_void_p(d_src), c_void_p(stream)))


def batch_create(tuning_json: str = None) -> int:
    h = c_void_p()
    check(lib().emx_batch_create(tuning_json.encode() if tuning_json else None, byref(h)))
    return h.value


def batch_destroy(h: int):
    check(lib().emx_batch_destroy(c_void_p(h)))


def batch_tuning(h: int) -> str:
    buf = create_string_buffer(512)
    check(lib().emx_batch_tuning(c_void_p(h), buf, 512))
    return buf.value.decode()


def make_batch_items(items) -> "ctypes.Array":
    arr = (BatchItem * len(items))()
    for k, it in enumerate(items):
        arr[k] = it
    return arr


def batch_scratch_bytes(h: int, arr, n: int) -> int:
    return lib().emx_batch_scratch_bytes(c_void_p(h), arr, n)


def batch_stats(h: int):
    """(batches run, graphs captured) of a batch executor."""
    a, b = c_int64(), c_int64()
    check(lib().emx_batch_stats(c_void_p(h), byref(a), byref(b)))
    return a.value, b.value


def batch_scratch_bound(h: int, largest: Params, max_items: int, max_points: int) -> int:
    return lib().emx_batch_scratch_bound(c_void_p(h), byref(largest), int(max_items),
                                         int(max_points))


def timing_begin():
    check(lib().emx_timing_begin())


def timing_end() -> dict:
    """{kernel: (launches, total_ms)} since timing_begin (waits for the events)."""
    import json
    buf = create_string_buffer(1 << 14)
    check(lib().emx_timing_end(buf, 1 << 14))
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}


def pipeline_batch(h: int, arr, n: int, d_scratch: int, nbytes: int, stream: int):
    check(lib().emx_pipeline_batch(c_void_p(h), arr, n, c_void_p(d_scratch), nbytes,
                                   c_void_p(stream)))
