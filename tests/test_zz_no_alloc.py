"""emx_fuse_points_noalloc (the fusion on the library's built-in scratch)
against emx_fuse_points (the same kernels on a caller's scratch): the same
state layers and per-point outputs, bit for bit, over two calls in a row, the
second with a smaller frame; and the refusal of a map whose wall-rule counts
do not fit the built-in scratch, with nothing enqueued."""
import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import synth
from parity_util import load_state, random_state

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_12876_amd import _emx
    _emx.lib()
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def _state(m):
    g = m.state_numpy()
    return {k: g[k] for k in ("h", "v", "t_upd", "valid")}


@pytest.mark.parametrize("extra", [{}, {"wall_min_count": 4, "time_variance": 0.002}])
def test_noalloc_equals_scratch_call(dev, extra):
    from paper_2204_12876_amd import ElevationMap
    d = synth.cfg1(n_frames=2, n_points=120_000)
    params = dict(d["params"], **extra)
    p = O.Params.from_dict(params)
    st = random_state(p, np.random.default_rng(5), valid_frac=0.5)
    cx, cy = d["centers"][0]
    a = ElevationMap(params, cx, cy, 0, device=dev)
    b = ElevationMap(params, cx, cy, 0, device=dev)
    load_state(a, st)
    load_state(b, st)
    f0, f1 = d["frames"]
    # the second call takes a smaller frame: every third point of the next frame
    sizes = [f0.n, (f1.n + 2) // 3]
    for k, (f, n) in enumerate(zip((f0, f1), sizes)):
        _say("noalloc", extra, "call", k, "points", n)
        sl = slice(None) if k == 0 else slice(None, None, 3)
        xyz = tuple(t[sl].to(dev).contiguous() for t in (f.x, f.y, f.z))
        assert xyz[0].numel() == n
        ca = torch.full((n,), -7, dtype=torch.int32, device=dev)
        aa = torch.full((n,), 7, dtype=torch.uint8, device=dev)
        cb = torch.full((n,), -9, dtype=torch.int32, device=dev)
        ab = torch.full((n,), 9, dtype=torch.uint8, device=dev)
        a.fuse_points(*xyz, f.pose, f.t_ms, out_cell=ca, out_accept=aa)
        b.fuse_points_noalloc(*xyz, f.pose, f.t_ms, out_cell=cb, out_accept=ab)
        torch.cuda.synchronize()
        assert torch.equal(ca, cb), "cell outputs differ"
        assert torch.equal(aa, ab), "accept outputs differ"
        assert int((aa == 1).sum()) > 0
        sa, sb = _state(a), _state(b)
        for key in sa:
            assert np.array_equal(sa[key].view(np.uint8), sb[key].view(np.uint8)), key
    a.close()
    b.close()


def test_noalloc_limit_is_the_wall_counts(dev):
    """The fusion's only scratch is the wall rule's per-cell counts (4 bytes a
    cell): the largest map they fit in the built-in scratch is served, one row
    more is refused with nothing enqueued, and without the rule any size is."""
    from paper_2204_12876_amd import ElevationMap, _emx
    limit = _emx.noalloc_scratch_limit()
    assert limit == 16 << 20
    d = synth.cfg0(n_frames=1)
    f = d["frames"][0]
    side = 2048                                   # 2048 * 2048 * 4 bytes = 16 MiB
    assert side * side * 4 == limit
    for ny, wall, ok in ((side, 4, True), (side + 1, 4, False), (side + 1, 0, True)):
        params = dict(d["params"], nx=side, ny=ny, wall_min_count=wall)
        _say("noalloc limit, map", side, "x", ny, "wall", wall)
        m = ElevationMap(params, 0.0, 0.0, 0, device=dev)
        xyz = tuple(t.to(dev).contiguous() for t in (f.x, f.y, f.z))
        before = _state(m)
        if ok:
            acc = torch.full((f.n,), 7, dtype=torch.uint8, device=dev)
            m.fuse_points_noalloc(*xyz, f.pose, f.t_ms, out_accept=acc)
            torch.cuda.synchronize()
            assert int((acc == 1).sum()) > 0
        else:
            with pytest.raises(_emx.EmxError) as ei:
                m.fuse_points_noalloc(*xyz, f.pose, f.t_ms)
            assert ei.value.status == _emx.EMX_ENOMEM
            assert "built-in scratch" in str(ei.value)
            torch.cuda.synchronize()
            after = _state(m)
            for key in before:
                assert np.array_equal(before[key], after[key]), key
        m.close()
