"""The C ABI on the host: the library loads, exports every declared symbol, and
rejects bad parameters before touching the GPU."""
import ctypes

import pytest

from paper_2204_12876_amd import _emx


@pytest.fixture(scope="module")
def L():
    return _emx.lib()


def test_every_header_symbol_is_exported(L):
    names = _emx.header_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_emx._SIGS), "binding and header disagree"


def test_version_and_sizes(L):
    assert L.emx_version().startswith(b"emx")
    p = _emx.make_params(dict(nx=400, ny=400, resolution=0.04))
    assert _emx.params_check(p) == 0
    C = 400 * 400
    sb = _emx.state_bytes(p)
    assert sb >= 30 * C and sb % 256 == 0
    assert _emx.export_bytes(p) == 29 * C
    assert _emx.scratch_bytes(p, 0) == 0
    s1 = _emx.scratch_bytes(p, 300000)
    assert s1 >= 300000 * 10
    assert _emx.scratch_bytes(p, 600000) > s1


@pytest.mark.parametrize("field,value", [
    ("nx", 2), ("ny", 16385), ("resolution", 0.0), ("resolution", float("nan")),
    ("init_variance", 0.0), ("noise_alpha", -1.0), ("min_range", 0.0), ("gate_k", -1.0),
    ("ray_step", 0.0), ("clear_normal_alpha", -0.1), ("clear_min_age_ms", -1),
])
def test_bad_params_rejected(L, field, value):
    d = dict(nx=64, ny=64, resolution=0.04)
    d[field] = value
    p = _emx.make_params(d)
    assert _emx.params_check(p) == _emx.EMX_EINVAL
    assert _emx.state_bytes(p) == 0
    assert len(_emx.last_error()) > 0


def test_init_map_argument_checks_need_no_gpu(L):
    p = _emx.make_params(dict(nx=64, ny=64, resolution=0.04))
    h = ctypes.c_void_p()
    assert L.emx_init_map(ctypes.byref(p), 0.0, 0.0, 0, None, 10**8, None, ctypes.byref(h)) \
        == _emx.EMX_EINVAL
    assert "d_state" in _emx.last_error()
    assert L.emx_init_map(ctypes.byref(p), 0.0, 0.0, 0, ctypes.c_void_p(4096), 16, None,
                          ctypes.byref(h)) == _emx.EMX_ENOMEM
    assert L.emx_init_map(ctypes.byref(p), 0.0, 0.0, 0, ctypes.c_void_p(4100), 10**8, None,
                          ctypes.byref(h)) == _emx.EMX_EINVAL          # misaligned
    assert L.emx_fuse_points(None, None, None, 0, None, None, None) == _emx.EMX_EINVAL
    assert L.emx_layer(None, 0, ctypes.byref(h)) == _emx.EMX_EINVAL


@pytest.mark.parametrize("field,value", [
    ("time_variance", -1e-3), ("time_variance", float("nan")), ("wall_min_count", -1),
    ("upper_bound", 2), ("upper_bound", -1), ("excl_on", 2), ("excl_on", -1),
    ("outlier_variance", -0.1), ("outlier_variance", float("inf")),
])
def test_bad_extension_params_rejected(L, field, value):
    d = dict(nx=64, ny=64, resolution=0.04)
    d[field] = value
    p = _emx.make_params(d)
    assert _emx.params_check(p) == _emx.EMX_EINVAL
    assert _emx.state_bytes(p) == 0 and _emx.inpaint_scratch_bytes(p) == 0


@pytest.mark.parametrize("extra", [dict(excl_theta=-0.1), dict(excl_theta=1.6),
                                   dict(excl_b=float("nan")), dict(excl_d=float("inf"))])
def test_bad_exclusion_area_rejected(L, extra):
    p = _emx.make_params(dict(nx=64, ny=64, resolution=0.04, excl_on=1, **extra))
    assert _emx.params_check(p) == _emx.EMX_EINVAL
    # with the area off its parameters are not looked at
    q = _emx.make_params(dict(nx=64, ny=64, resolution=0.04, excl_on=0, **extra))
    assert _emx.params_check(q) == _emx.EMX_OK


def test_extension_sizes(L):
    C = 64 * 48
    base = _emx.make_params(dict(nx=64, ny=48, resolution=0.04))
    ub = _emx.make_params(dict(nx=64, ny=48, resolution=0.04, upper_bound=1))
    # the bound layer: one float per cell
    assert _emx.state_bytes(ub) - _emx.state_bytes(base) >= 4 * C
    wall = _emx.make_params(dict(nx=64, ny=48, resolution=0.04, wall_min_count=3))
    # fusion's part grows by the per-cell counts (the buffer is the larger of
    # fusion's and clearing's needs)
    assert _emx.scratch_bytes(wall, 5000) >= _emx.scratch_bytes(base, 5000)
    assert _emx.inpaint_scratch_bytes(base) >= 8 * C
    assert _emx.drift_scratch_bytes(-1) == 0
    assert _emx.drift_scratch_bytes(0) > 0
    assert _emx.drift_scratch_bytes(300000) >= 293 * 12


def test_next_row_calls_check_arguments_without_a_gpu(L):
    none = ctypes.c_void_p()
    assert L.emx_overlap_clear(None, 0.0, 0.0, 0.0, 1.0, 0.5, None, None) == _emx.EMX_EINVAL
    assert L.emx_inpaint_min(None, None, None, 0, None) == _emx.EMX_EINVAL
    assert L.emx_compensate_drift(None, None, 0.0, None, 0, None, None, None) == _emx.EMX_EINVAL
    assert L.emx_move_fuse_points(None, 0.0, 0.0, None, None, 0, None, None, None) \
        == _emx.EMX_EINVAL
    assert L.emx_normals_traversability(None, None, None) == _emx.EMX_EINVAL
    # smoothing validates every argument on the host
    d_in, d_out = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 24)
    bad = [(None, d_out, 8, 8, 0, 3, 0.0), (d_in, d_out, 8, 8, 3, 3, 0.0),
           (d_in, d_out, 8, 8, 0, 4, 0.0), (d_in, d_out, 8, 8, 2, 7, 0.0),
           (d_in, d_out, 8, 8, 1, 3, 0.0), (d_in, d_out, 8, 8, 0, 33, 0.0),
           (d_in, d_out, 4, 8, 0, 9, 0.0), (d_in, d_in, 8, 8, 0, 3, 0.0),
           (d_in, ctypes.c_void_p((1 << 20) + 64), 8, 8, 0, 3, 0.0)]
    for args in bad:
        assert _emx.lib().emx_smooth(*args, none) == _emx.EMX_EINVAL, args
