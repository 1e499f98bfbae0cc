"""The seeded input generator: determinism, exact sizes, and separation from
the oracle and the GPU package."""
import ast
import os

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cfg0_is_deterministic_and_exact_size():
    a = synth.cfg0(n_points=3000)
    b = synth.cfg0(n_points=3000)
    fa, fb = a["frames"][0], b["frames"][0]
    assert fa.n == 3000
    for u, v in zip(fa.numpy(), fb.numpy()):
        assert u.dtype == np.float32 and np.array_equal(u, v)
    assert np.array_equal(fa.pose, fb.pose)
    c = synth.cfg0(n_points=3000, seed_offset=1)
    assert not np.array_equal(c["frames"][0].numpy()[0], fa.numpy()[0])


def test_points_lie_near_terrain_and_include_outliers():
    d = synth.cfg0(n_points=4000)
    f = d["frames"][0]
    x, y, z = (t.double() for t in (f.x, f.y, f.z))
    import torch
    P = torch.as_tensor(f.pose)
    pw = torch.stack([x, y, z], 1) @ P[:, :3].T + P[:, 3]
    g = d["terrain"].height(pw[:, 0], pw[:, 1])
    err = (pw[:, 2] - g).abs()
    assert (err < 0.05).float().mean() > 0.95           # inliers on the surface
    assert ((err > 0.1).float().mean() > 0.005)          # ~2% gross outliers


def test_trav_weights_layout():
    w = synth.trav_weights()
    assert w.shape == (89,) and w.dtype == np.float32 and w[88] == 0


def _imports(path):
    tree = ast.parse(open(path).read())
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom) and node.module:
            out.add(node.module.split(".")[0])
    return out


def test_oracle_gpu_package_and_generator_are_separate():
    pkg = "paper_2204_12876_amd"
    for d in ("oracle", "synth"):
        for fn in os.listdir(os.path.join(ROOT, d)):
            if fn.endswith(".py"):
                imps = _imports(os.path.join(ROOT, d, fn))
                assert pkg not in imps, (d, fn)
                assert ("oracle" not in imps) or d == "oracle", (d, fn)
    pdir = os.path.join(ROOT, pkg)
    if os.path.isdir(pdir):
        for fn in os.listdir(pdir):
            if fn.endswith(".py"):
                imps = _imports(os.path.join(pdir, fn))
                assert "oracle" not in imps and "synth" not in imps, fn
