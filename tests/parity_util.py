"""Helpers of the GPU-vs-oracle parity tests.

Tolerances (float32 GPU against float64 oracle):
  * cell, accept, clear marks, validity, t_upd and NaN patterns: bit-exact.
  * variance: |dv| <= 1e-5 * v_oracle.  All terms are positive.
  * height: |dh| <= 1e-5 * max(|h_oracle|, a_c).  a_c is the weighted mean of
    the magnitudes entering the height: |h0|/v0 and each point's
    |R20 xs| + |R21 ys| + |R22 zs| + |tz|, weighted by 1/sp2.  The float32
    transform rounds relative to those terms, not to the result.
  * normals: |dn| <= 1e-5 per component (unit vectors).
  * traversability: |dT| <= 1e-5 * (|b2| + sum_c |w2_c| (|b1_c| + sum |w1||h|)).
"""
import numpy as np
import torch

import oracle as O

REL = 1e-5


def state_from_gpu(m, cgx, cgy, t0):
    g = m.state_numpy()
    return O.MapState(g["h"], g["v"], g["t_upd"], g["valid"], g["nrm"], g["trav"], cgx, cgy, t0), g


def load_state(m, st: O.MapState):
    m.load_numpy(st.h, st.v, st.t_upd, st.valid, st.nrm, st.trav)


def frame_dev(f, dev):
    return tuple(t.to(dev).contiguous() for t in (f.x, f.y, f.z))


def gpu_fuse(m, xyz, pose, t_ms):
    n = xyz[0].numel()
    cell = torch.full((max(n, 1),), -7, dtype=torch.int32, device=xyz[0].device)
    acc = torch.full((max(n, 1),), 7, dtype=torch.uint8, device=xyz[0].device)
    m.fuse_points(*xyz, pose, t_ms, out_cell=cell, out_accept=acc)
    torch.cuda.synchronize()
    return cell[:n].cpu().numpy(), acc[:n].cpu().numpy()


def assert_fuse_parity(r: "O.FuseResult", before: O.MapState, g: dict, cell, acc, t_now):
    assert np.array_equal(cell, r.cell.astype(np.int32)), \
        f"cell mismatch at {np.nonzero(cell != r.cell)[0][:10]}"
    assert np.array_equal(acc.astype(bool), r.accept), \
        f"accept mismatch at {np.nonzero(acc.astype(bool) != r.accept)[0][:10]}"
    u = r.updated
    # untouched cells bitwise
    for k in ("h", "v", "t_upd", "valid"):
        a = g[k][~u]
        b = getattr(before, k)[~u]
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"untouched {k} changed"
    assert (g["valid"][u] == 1).all() and (g["t_upd"][u] == t_now).all()
    dv = np.abs(g["v"][u].astype(np.float64) - r.v[u])
    assert np.all(dv <= REL * r.v[u]), f"variance: worst rel {np.max(dv / r.v[u]):.3g}"
    scale = np.maximum(np.abs(r.h[u]), r.h_scale[u])
    dh = np.abs(g["h"][u].astype(np.float64) - r.h[u])
    assert np.all(dh <= REL * scale), f"height: worst rel {np.max(dh / scale):.3g}"
    return float(np.max(dv / r.v[u], initial=0)), float(np.max(dh / scale, initial=0))


def assert_normals_parity(g: dict, ref: np.ndarray):
    assert np.array_equal(np.isnan(g["nrm"]), np.isnan(ref)), "normal NaN pattern"
    ok = ~np.isnan(ref)
    err = np.abs(g["nrm"][ok].astype(np.float64) - ref[ok])
    assert np.all(err <= REL), f"normal error {err.max():.3g}"


def assert_trav_parity(g: dict, T: np.ndarray, S: np.ndarray):
    assert np.array_equal(np.isnan(g["trav"]), np.isnan(T)), "trav NaN pattern"
    ok = ~np.isnan(T)
    err = np.abs(g["trav"][ok].astype(np.float64) - T[ok])
    assert np.all(err <= REL * S[ok]), f"trav error {np.max(err / S[ok]):.3g}"


def random_state(p: O.Params, rng, valid_frac=0.9, cgx=0, cgy=0):
    st = O.init_map(p, 0.0, 0.0, 0)
    st.cgx, st.cgy = cgx, cgy
    shp = (p.ny, p.nx)
    st.h[:] = rng.uniform(-0.5, 0.8, shp).astype(np.float32)
    st.v[:] = rng.uniform(1e-4, 0.05, shp).astype(np.float32)
    st.valid[:] = (rng.random(shp) < valid_frac).astype(np.uint8)
    st.t_upd[:] = rng.integers(0, 400, shp).astype(np.int32)
    n = rng.normal(size=(3,) + shp)
    n[2] = np.abs(n[2])
    st.nrm[:] = (n / np.linalg.norm(n, axis=0)).astype(np.float32)
    st.trav[:] = rng.normal(size=shp).astype(np.float32)
    return st
