"""bench.py's command line on the CPU: more than one GPU is refused with a
message before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


# --------------------------------------------------------------------------
# the host-side parts of bench.py that run after the GPU legs, on stubs
# --------------------------------------------------------------------------
import math  # noqa: E402

import numpy as np  # noqa: E402
import torch  # noqa: E402

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_driver_arguments_parse():
    a = bench.parse(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.gpus, a.steps, a.warmup) == (1, 20, 5)
    d = bench.parse([])
    assert d.steps >= 1 and d.warmup >= 1 and d.gpus == 1


def _stub_ctx(n_robots=3, n=1500):
    """A serving context in bench.py's layout: small maps and pinned-free host
    frames (the CPU baseline reads them as numpy)."""
    rng = np.random.default_rng(1)
    items, host = [], []
    for k in range(n_robots):
        params = dict(nx=24 + 4 * k, ny=20, resolution=0.1, noise_alpha=1e-4, gate_k=3.0,
                      min_range=0.05, ray_step=0.1, clear_normal_alpha=0.3,
                      clear_min_age_ms=500)
        xs = rng.uniform(0.2, 1.0, n).astype(np.float32)
        ys = rng.uniform(-0.8, 0.8, n).astype(np.float32)
        zs = (-0.5 + 0.01 * rng.normal(size=n)).astype(np.float32)
        P = np.zeros((3, 4))
        P[:, :3] = np.eye(3)
        P[:, 3] = (0.0, 0.0, 0.5)
        items.append(dict(params=params, rate_hz=20.0))
        host.append((torch.from_numpy(np.stack([xs, ys, zs])), P, (0.0, 0.0)))
    return dict(items=items, host=host,
                stats=[dict(n=n, C=p["params"]["nx"] * 20, touched=10, updated=9) for p in items])


def test_cpu_baseline_runs_on_a_stub_workload():
    args = bench.parse(["--steps", "20", "--warmup", "5", "--cpu-seconds", "0.3",
                        "--cpu-procs", "2"])
    pool, procs = bench.cpu_pool(args)
    ctx = _stub_ctx()
    # two small maps stand in for a multi-map workload (one map per process)
    bench.HOST_SPECS.clear()
    bench.HOST_SPECS["batched"] = [
        (it["params"], c, *(a.numpy() for a in xyz), pose)
        for it, (xyz, pose, c) in zip(ctx["items"][:2], ctx["host"][:2])]
    try:
        out = bench.cpu_baseline(args, ctx, pool, procs)
    finally:
        pool.shutdown()
        bench.HOST_SPECS.clear()
    b = out["per_workload"]["batched"]
    assert b["maps"] == 2 and b["cores"] == 2 and b["points_per_s"] > 0
    assert b["points"] == 2 * 1500
    assert out["kind"] == "oracle" and out["unit"] == "points/s"
    assert out["cores"] == 2 and out["value"] > 0
    assert out["single_core"]["cores"] == 1 and out["single_core"]["value"] > 0
    assert out["fusion_128x128_20k"]["reps"] == 20
    assert "processes" in out["sample"]


class _R:
    def __init__(self, arrival, done, n, robot=0):
        self.arrival, self.done, self.n, self.robot = arrival, done, n, robot

    @property
    def latency(self):
        return self.done - self.arrival


def test_window_summary_counts_only_the_window():
    reqs = [_R(0.5, 0.6, 10), _R(1.0, 1.01, 100), _R(1.5, 1.52, 100), _R(2.0, 2.5, 999)]
    s = bench.window_summary(reqs, 1.0, 2.0)
    assert s["frames"] == 2 and s["points"] == 200
    assert math.isclose(s["offered_points_per_s"], 200.0)
    assert math.isclose(s["points_per_s"], 200 / 0.52)
    assert math.isclose(s["p99_ms"], 1e3 * (0.01 + 0.99 * 0.01), rel_tol=1e-9)


def test_poisson_trace_is_seeded_and_sorted():
    ctx = _stub_ctx()
    a = bench.poisson_trace(ctx, 2.0)
    b = bench.poisson_trace(ctx, 2.0)
    assert a == b and len(a) > 60
    assert all(x[2] <= y[2] for x, y in zip(a, a[1:]))
    assert all(0 <= t < 2.0 for _, _, t in a)
    # per robot, frame indices count up in time order
    for k in range(3):
        js = [j for r, j, _ in a if r == k]
        assert js == list(range(len(js)))


def test_roofline_takes_the_kernel_with_the_most_time():
    kt = {"k_a": [10, 1.0], "k_b": [5, 3.0], "k_c": [1, 9.0]}
    alg = {"k_a": 1e9, "k_b": 6e9}
    k = bench.kernel_table(kt, alg)
    r = bench.roofline(k)
    assert r["kernel"] == "k_b"                   # k_c has no algorithmic bytes
    assert math.isclose(r["achieved"], 6e9 / 3e-3 / 1e9)
    assert math.isclose(r["frac"], r["achieved"] / 8000.0)
    assert math.isclose(r["alg_bytes_per_launch"], 6e9 / 5)
    fb = bench.frame_bytes(100, 50, 7, 5, 10)
    assert fb["fuse_chunk"] == 1200 + 56 and fb["fuse_tile"] == 105
    assert fb["move"] == 29 * 10 and bench.frame_bytes(100, 50, 7, 5, 0)["move"] == 0


def test_source_hash_ignores_comments_but_not_code():
    src = ('#include "a.h"  // header\n'
           '/* a block\n   comment */\n'
           'const char* s = "// not a comment";\n'
           "int f(int x) { return x + '/'; }  // tail\n")
    code = bench.code_only(src)
    assert code == ('#include "a.h"\n'
                    'const char* s = "// not a comment";\n'
                    "int f(int x) { return x + '/'; }")
    # a comment edit keeps the code; a code edit does not
    assert bench.code_only(src.replace("// tail", "// other words")) == code
    assert bench.code_only(src.replace("x + ", "x - ")) != code


def test_traffic_is_read_only_for_the_kernels_it_was_taken_on(tmp_path, monkeypatch):
    """A summary whose hash is the kernel's current code gives bytes per
    launch (counters scaled by the calibration factors); another hash, or no
    summary, gives None."""
    k = "k_fuse_chunk_b"
    f = tmp_path / "traffic.txt"
    f.write_text("# comment: ignored\nfetch_factor: 2.0\nwrite_factor: 1.0\n"
                 f"{k}.source_sha256_16: {bench.kernel_source_hash(k)}\n"
                 f"{k}.fetch_kib: 10\n{k}.write_kib: 3\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic(k) == 1024.0 * (10 * 2.0 + 3 * 1.0)
    f.write_text(f.read_text().replace(bench.kernel_source_hash(k), "0" * 16))
    assert bench.measured_traffic(k) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.txt"))
    assert bench.measured_traffic(k) is None


def test_ray_samples_hand_cases():
    eye = np.eye(4)[:3]
    step = 0.125                                  # exact in binary: K is exact
    # (1, 0.25, 0): the ray's major axis spans 1 m = 8 steps, samples k = 1..7
    assert bench.ray_samples([1.0], [0.25], [0.0], eye, 0.05, step) == 7
    # a 90-degree yaw swaps the axes, the count stays
    yaw = np.array([[0.0, -1.0, 0.0, 5.0], [1.0, 0.0, 0.0, -3.0], [0.0, 0.0, 1.0, 0.2]])
    assert bench.ray_samples([1.0], [0.25], [0.0], yaw, 0.05, step) == 7
    # the vertical part never counts; a ray shorter than one step has none
    assert bench.ray_samples([0.5], [0.0], [3.0], eye, 0.05, step) == 3
    assert bench.ray_samples([0.1], [0.0], [0.0], eye, 0.05, step) == 0
    # points inside the minimum range and non-finite points cast no ray
    assert bench.ray_samples([0.01, np.nan], [0.0, 0.0], [0.0, 0.0], eye, 0.05, step) == 0
    # rays of 2^24 steps or more are skipped
    assert bench.ray_samples([2.0 ** 21], [0.0], [0.0], eye, 0.05, step) == 0
    # a frame is the sum of its rays
    xs, ys, zs = [1.0, 0.5, 0.1], [0.25, 0.0, 0.0], [0.0, 3.0, 0.0]
    assert bench.ray_samples(xs, ys, zs, eye, 0.05, step) == 7 + 3 + 0


def test_sample_rate_per_march_launch():
    k = bench.kernel_table({"k_clear_march_b": [4, 2.0], "k_cells_b": [4, 1.0]}, {})
    bench.add_sample_rate(k, {"k_clear_march_b": 8e9, "k_clear_march": 5})
    assert k["k_clear_march_b"]["samples_per_launch"] == 2e9
    assert math.isclose(k["k_clear_march_b"]["G_samples_per_s"], 8e9 / 2e-3 / 1e9)
    assert "samples_per_launch" not in k["k_cells_b"]
    assert "k_clear_march" not in k                # a kernel that did not run stays absent
