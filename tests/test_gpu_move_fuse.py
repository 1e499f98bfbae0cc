"""emx_move_fuse_points against emx_move_map followed by emx_fuse_points: the
same state, outputs and upper bound layer, bit for bit, for small, zero and
far shifts, empty frames and every fusion extension.  (The two calls are
themselves checked against the oracle in test_gpu_parity and test_gpu_next.)
"""
import numpy as np
import pytest
import torch

import synth
from parity_util import load_state, random_state

import oracle as O

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_12876_amd import _emx
    _emx.lib()
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def _outputs(m, n, dev):
    cell = torch.full((max(n, 1),), -7, dtype=torch.int32, device=dev)
    acc = torch.full((max(n, 1),), 7, dtype=torch.uint8, device=dev)
    return cell, acc


@pytest.mark.parametrize("extra", [{}, {"wall_min_count": 4, "time_variance": 0.002},
                                   {"upper_bound": 1}])
def test_move_fuse_equals_move_then_fuse(dev, extra):
    from paper_2204_12876_amd import ElevationMap
    d = synth.cfg0(n_frames=2)
    params = dict(d["params"], **extra)
    p = O.Params.from_dict(params)
    r = p.resolution
    rng = np.random.default_rng(len(extra))
    st = random_state(p, rng, valid_frac=0.6)
    a = ElevationMap(params, 0.0, 0.0, 0, device=dev)
    b = ElevationMap(params, 0.0, 0.0, 0, device=dev)
    load_state(a, st)
    load_state(b, st)
    w = torch.from_numpy(synth.trav_weights()).to(dev)
    frames = d["frames"]
    # centres: a small shift, no shift, a far shift (every cell enters), back
    centres = [(3.2 * r, -2.1 * r), (3.2 * r, -2.1 * r), (500 * r, 7 * r), (0.5 * r, 0.5 * r)]
    for k, (cx, cy) in enumerate(centres):
        f = frames[k % 2]
        xyz = tuple(t.to(dev).contiguous() for t in (f.x, f.y, f.z))
        if k == 3:  # an empty frame with a shift
            xyz = tuple(t[:0] for t in xyz)
        n = xyz[0].numel()
        ca, aa = _outputs(a, n, dev)
        cb, ab = _outputs(b, n, dev)
        t_ms = 300 * (k + 1)
        a.move_map(cx, cy)
        a.fuse_points(*xyz, f.pose, t_ms, out_cell=ca, out_accept=aa)
        b.move_fuse_points(cx, cy, *xyz, f.pose, t_ms, out_cell=cb, out_accept=ab)
        torch.cuda.synchronize()
        assert a.info() == b.info()
        assert torch.equal(a.export_state(), b.export_state()), f"state differs at step {k}"
        assert torch.equal(ca, cb) and torch.equal(aa, ab), f"outputs differ at step {k}"
        if extra.get("upper_bound"):
            assert torch.equal(a.upper_bound().view(torch.int32), b.upper_bound().view(torch.int32))
        # the rest of the frame keeps both maps comparable
        for m in (a, b):
            m.clear_visibility(*xyz, f.pose, t_ms)
            m.normals_traversability(w)
        _say(f"move+fuse {extra} step {k}: {n} points, equal")
    a.close()
    b.close()


def test_move_fuse_refuses_like_the_two_calls(dev):
    from paper_2204_12876_amd import ElevationMap, EmxError
    m = ElevationMap(dict(nx=16, ny=16, resolution=0.1), 0.0, 0.0, 0, device=dev)
    before = m.export_state()
    x = torch.zeros(4, dtype=torch.float32, device=dev)
    bad = np.zeros((3, 4))
    bad[0, 0] = np.nan
    with pytest.raises(EmxError):
        m.move_fuse_points(1.0, 1.0, x, x, x, bad, 10)
    with pytest.raises(EmxError):
        m.move_fuse_points(1e300, 0.0, x, x, x, np.eye(3, 4), 10)
    assert m.info() == (0, 0, 0)
    assert torch.equal(before, m.export_state())
    m.close()


def test_ring_layout_after_moves(dev):
    """The layers are a ring: a move turns the origin by the shift and resets
    only the entering strips.  The stored layer unrolled from the origin is the
    exported (local order) layer, and the state equals the oracle's copy-based
    move after every shift, including shifts past a whole side."""
    from paper_2204_12876_amd import ElevationMap, _emx
    _say("ring layout")
    params = dict(nx=37, ny=23, resolution=0.1, upper_bound=1)
    p = O.Params.from_dict(params)
    rng = np.random.default_rng(17)
    st = random_state(p, rng, valid_frac=0.6)
    m = ElevationMap(params, 0.0, 0.0, 0, device=dev)
    load_state(m, st)
    r = p.resolution
    ox = oy = 0
    cx = cy = 0.0
    for dx, dy in [(3, 0), (0, -2), (-5, 4), (36, 1), (-40, -30), (1, 1), (0, 0)]:
        cx += dx * r
        cy += dy * r
        m.move_map(cx + 0.5 * r, cy + 0.5 * r)
        st = O.move_map(p, st, cx + 0.5 * r, cy + 0.5 * r)
        torch.cuda.synchronize()
        g = m.state_numpy()
        for k in ("h", "v", "t_upd", "valid", "trav"):
            assert np.array_equal(g[k].view(np.uint8), getattr(st, k).view(np.uint8)), (dx, dy, k)
        assert np.array_equal(g["nrm"].view(np.uint8), st.nrm.view(np.uint8)), (dx, dy)
        # the origin turns by the shift, modulo the sides
        ox, oy = (ox + dx) % p.nx, (oy + dy) % p.ny
        assert m.origin() == (ox, oy), (dx, dy)
        for lid, key in ((_emx.LAYER_HEIGHT, "h"), (_emx.LAYER_VARIANCE, "v"),
                         (_emx.LAYER_VALID, "valid")):
            assert np.array_equal(m.local(lid).cpu().numpy(), g[key]), (dx, dy, key)
        # the extra layer carries through the ring too
        assert np.array_equal(np.isinf(m.upper_bound().cpu().numpy()),
                              np.ones((p.ny, p.nx), bool)), (dx, dy)
    # import writes through the ring: a state loaded at a non-zero origin
    # exports unchanged
    st2 = random_state(p, rng, valid_frac=0.5)
    load_state(m, st2)
    g = m.state_numpy()
    for k in ("h", "v", "t_upd", "valid"):
        assert np.array_equal(g[k], getattr(st2, k)), k
    m.close()
