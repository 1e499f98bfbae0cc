"""The oracle's pins catch plausible mistakes.

Each case below plants one mistake in a copy of the oracle: a transposed
operand, a dropped term, a wrong sign or index, a wrong rounding.  The oracle's
own CPU tests then run against that copy in a fresh process and must fail.  An
unmodified copy must pass, so a failure means the mistake was seen.  Every
mistake is planted on the CPU, in the oracle only.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["test_oracle_fusion.py", "test_oracle_cells.py", "test_oracle_next.py",
                "test_oracle_post.py", "test_oracle_ramp.py"]

# (name, file in oracle/, text, replacement[, times the text occurs])
MUTANTS = [
    ("rotation transposed in x", "elevation.py",
     "xm = ((R[0, 0] * xs + R[0, 1] * ys) + R[0, 2] * zs) + t[0]",
     "xm = ((R[0, 0] * xs + R[1, 0] * ys) + R[0, 2] * zs) + t[0]"),
    ("noise linear in range", "elevation.py",
     'sp2 = c["alpha"] * d2', 'sp2 = c["alpha"] * np.sqrt(d2)'),
    ("gate without the point's noise", "elevation.py",
     '(c["k2"] * (v0 + sp2))', '(c["k2"] * v0)'),
    ("binning rounds", "elevation.py",
     "ix = np.floor(np.where(inmap, fx, F32(0))).astype(np.int64)",
     "ix = np.round(np.where(inmap, fx, F32(0))).astype(np.int64)"),
    ("height update drops the prior", "elevation.py",
     "h1 = np.where(upd, (h0 / v0 + Swz) / W, h0)", "h1 = np.where(upd, Swz / W, h0)"),
    ("variance update drops the prior", "elevation.py",
     "W = 1.0 / v0 + Sw", "W = Sw"),
    ("time variance on updated cells too", "elevation.py",
     "grow = ~upd & (st.valid.reshape(-1) != 0)", "grow = st.valid.reshape(-1) != 0"),
    ("wall rule keeps points above", "elevation.py",
     "walled = kept & crowded & (zm < h0)", "walled = kept & crowded & (zm > h0)"),
    ("ray end cell not skipped", "elevation.py",
     "keep = (cs >= 0) & (cs != end_cell[rep])", "keep = cs >= 0"),
    ("clearing ignores the variance", "elevation.py",
     "& ((hd * hd) > vf[cs])", ""),
    ("clearing ignores the age", "elevation.py",
     "& ((t_now - tf[cs]) > tau)", ""),
    ("upper bound on valid cells", "elevation.py",
     "sel = validf[cs] == 0", "sel = validf[cs] >= 0"),
    ("normal x sign", "elevation.py",
     "out[0, 1:-1, 1:-1] = np.where(inner, -a / nrm, np.nan)",
     "out[0, 1:-1, 1:-1] = np.where(inner, a / nrm, np.nan)"),
    ("normal slope over 2r", "elevation.py", "a /= 6.0 * r", "a /= 2.0 * r"),
    ("traversability without ReLU", "elevation.py",
     "tot = tot + w2[ch] * np.maximum(act, 0.0)", "tot = tot + w2[ch] * act"),
    ("traversability kernel flipped", "elevation.py",
     "act = act + w1[ch, dy + 1, dx + 1] * win", "act = act + w1[ch, 1 - dy, 1 - dx] * win"),
    ("move in the wrong direction", "elevation.py",
     "sx, sy = ngx - st.cgx, ngy - st.cgy", "sx, sy = st.cgx - ngx, st.cgy - ngy"),
    ("extra layer moved in the wrong direction", "elevation.py",
     "shift_x = int(math.floor(cx / p.resolution)) - st.cgx",
     "shift_x = st.cgx - int(math.floor(cx / p.resolution))"),
    ("extra layer filled with zero", "elevation.py",
     "out = np.full_like(layer, fill)", "out = np.zeros_like(layer)"),
    ("extra layer rows and columns swapped", "elevation.py",
     "out[y0:y1, x0:x1] = layer[y0 + shift_y:y1 + shift_y, x0 + shift_x:x1 + shift_x]",
     "out[y0:y1, x0:x1] = layer[y0 + shift_x:y1 + shift_x, x0 + shift_y:x1 + shift_y]"),
    ("drift error sign", "elevation.py",
     'err = d["zm"][use].astype(F64) - st.h.reshape(-1)[cc[use]].astype(F64)',
     'err = st.h.reshape(-1)[cc[use]].astype(F64) - d["zm"][use].astype(F64)'),
    ("overlap on cell corners", "elevation.py",
     "dx = (ix + F32(0.5)) * r32 - rx", "dx = ix * r32 - rx"),
    ("inpainting takes the maximum", "filters.py",
     "best = min(best, float(h[yy, xx]))", "best = max(best if best < np.inf else -np.inf, float(h[yy, xx]))"),
    ("mirror repeats the edge", "filters.py",
     "iy = np.where(iy > ny - 1, 2 * (ny - 1) - iy, iy)", "iy = np.where(iy > ny - 1, 2 * ny - 1 - iy, iy)"),
    ("Gaussian with sigma, not sigma squared", "filters.py",
     "w = np.exp(-(i * i) / (2.0 * s * s))", "w = np.exp(-(i * i) / (2.0 * s))"),
    ("gate boundary exclusive", "elevation.py",
     'inside = (e * e) <= (c["k2"] * (v0 + sp2))',
     'inside = (e * e) < (c["k2"] * (v0 + sp2))'),
    ("fused height from the x row", "elevation.py",
     "zm64 = R[2, 0] * x64 + R[2, 1] * y64 + R[2, 2] * z64 + t[2]",
     "zm64 = R[0, 0] * x64 + R[2, 1] * y64 + R[2, 2] * z64 + t[2]"),
    ("ray step count from |dx| + |dy|", "elevation.py",
     "m = np.maximum(np.abs(dx), np.abs(dy))", "m = np.abs(dx) + np.abs(dy)"),
    ("ray samples from k = 0", "elevation.py",
     "k = np.arange(len(rep)) - np.repeat(starts, nsamp) + 1",
     "k = np.arange(len(rep)) - np.repeat(starts, nsamp)"),
    ("upper bound takes the maximum", "elevation.py",
     "np.minimum.at(out, cs[sel], qz[sel])", "np.maximum.at(out, cs[sel], qz[sel])"),
    ("overlap threshold inclusive", "elevation.py",
     "far = np.abs(st.h - rz) > thr", "far = np.abs(st.h - rz) >= thr"),
    ("normal window without its corners", "elevation.py",
     "acc &= v[1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx]",
     "acc &= v[1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx] if dx * dy == 0 else True"),
    ("normal z not normalised", "elevation.py",
     "out[2, 1:-1, 1:-1] = np.where(inner, 1.0 / nrm, np.nan)",
     "out[2, 1:-1, 1:-1] = np.where(inner, 1.0, np.nan)"),
    ("inpainting over 8 neighbours", "filters.py",
     "steps = ((0, 1), (0, -1), (1, 0), (-1, 0))",
     "steps = ((0, 1), (0, -1), (1, 0), (-1, 0), (1, 1), (1, -1), (-1, 1), (-1, -1))"),
    ("box blur over one row", "filters.py",
     "return _windows(x, ksize).mean(axis=(2, 3))",
     "return _windows(x, ksize)[:, :, ksize // 2, :].mean(axis=2)"),
    ("median by mean", "filters.py",
     "out = np.median(w, axis=2)", "out = np.mean(w, axis=2)"),
    ("exclusion line inclusive", "elevation.py",
     "excluded = inmap & (e_up > line)", "excluded = inmap & (e_up >= line)"),
    ("ramp without its start", "elevation.py",
     'np.maximum(rho - c["excl_c"], F32(0))', '(rho - c["excl_c"])'),
    ("ramp without its cap", "elevation.py",
     'c["excl_d"])', "F32(np.inf))"),
    ("ramp distance in 3-D", "elevation.py",
     "rho = np.sqrt(dxr * dxr + dyr * dyr)",
     "rho = np.sqrt(dxr * dxr + dyr * dyr + (zm - t[2]) * (zm - t[2]))"),
    ("ramp around the map corner", "elevation.py", "dxr = xm - t[0]", "dxr = xm"),
    ("ramp points counted by the wall rule", "elevation.py",
     "count = np.bincount(cell[kept], minlength=p.nx * p.ny)",
     "count = np.bincount(cell[inmap], minlength=p.nx * p.ny)"),
    ("outlier variance per rejected point", "elevation.py",
     'v_out = np.where(inflate, v_out + c32["var_o"], v_out)',
     'v_out = np.where(inflate, v_out + c32["var_o"] * np.bincount(cell[d["rejected"]], '
     'minlength=C).astype(F32), v_out)'),
    ("outlier variance on cells without an estimate", "elevation.py",
     "inflate = hit & (st.valid.reshape(-1) != 0)", "inflate = hit"),
    ("wall-rule points count as outliers", "elevation.py",
     "rejected = gated & ~inside", "rejected = kept & ~inside"),
]


def _copy_with(tmp, name, fname, old, new, times=1):
    root = os.path.join(tmp, name.replace(" ", "_").replace(",", ""))
    dst = os.path.join(root, "oracle")
    shutil.copytree(os.path.join(ROOT, "oracle"), dst,
                    ignore=shutil.ignore_patterns("__pycache__", "*.so", "*.o"))
    if fname is not None:
        path = os.path.join(dst, fname)
        with open(path) as fh:
            src = fh.read()
        assert src.count(old) == times, f"{name}: the text must occur {times} time(s) in {fname}"
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))
    return root


def _run(root):
    # one thread each: several of these processes run at once
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([root, ROOT]), PYTHONDONTWRITEBYTECODE="1",
               OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    which = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.__file__)"],
                           cwd=root, env=env, capture_output=True, text=True, timeout=300)
    files = [os.path.join(ROOT, "tests", f) for f in ORACLE_TESTS]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *files],
                       cwd=root, env=env, capture_output=True, text=True, timeout=600)
    return which.stdout.strip(), r.returncode, r.stdout[-2000:]


def test_oracle_mutants_are_caught(tmp_path):
    tmp = str(tmp_path)
    control = _copy_with(tmp, "control", None, None, None)
    roots = [_copy_with(tmp, *m) for m in MUTANTS]
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(_run, [control] + roots))
    where, rc, out = results[0]
    assert where.startswith(control), f"the copy was not the oracle imported: {where}"
    assert rc == 0, "the unmodified copy must pass its tests:\n" + out
    missed = []
    for (name, *_), root, (where, rc, out) in zip(MUTANTS, roots, results[1:]):
        assert where.startswith(root), f"{name}: imported {where}"
        # 1 = tests failed; anything else (collection error, crash) is not a catch
        if rc != 1:
            missed.append(f"{name} (exit {rc})")
    assert not missed, "mistakes no pin caught: " + ", ".join(missed)
