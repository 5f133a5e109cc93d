"""bench.py's contract on the host: one GPU only, a clear exit without a GPU, and the traffic
lookup that ties a profile summary to the kernel source it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=600, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_no_gpu_exits_with_a_message():
    import torch
    if torch.cuda.is_available():
        return
    r = _run("--steps", "1")
    assert r.returncode == 1 and "needs a GPU" in r.stderr


def test_traffic_is_read_only_for_the_profiled_kernel_source(tmp_path):
    src = os.path.join(ROOT, "paper_1707_00198_amd", "csrc", "lbm_kernels.hip")
    import hashlib
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()

    def summary(sha, workload="sweep", storage="c16"):
        p = tmp_path / f"{sha[:6]}_{workload}_{storage}.md"
        body = {"workload": workload, "storage": storage, "kernel_source_sha256": sha,
                "bytes_per_launch": 123456}
        p.write_text("# traffic\n\n```json\n" + json.dumps(body) + "\n```\n")
        return str(p)

    assert bench.measured_traffic(summary(h), "sweep", "c16") == 123456
    assert bench.measured_traffic(summary("0" * 64), "sweep", "c16") is None
    assert bench.measured_traffic(summary(h), "x9", "c16") is None
    assert bench.measured_traffic(summary(h, storage="f64"), "sweep", "c16") is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), "sweep", "c16") is None


def test_traffic_is_read_only_for_the_profiled_tile_shape(tmp_path):
    """A summary measured on one tile shape is not reported for a run on another (the autotuner
    may pick a different chunk height or the two-column kernel); the kernel name follows the
    shape."""
    src = os.path.join(ROOT, "paper_1707_00198_amd", "csrc", "lbm_kernels.hip")
    import hashlib
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    shape = {"chunk_rows": 64, "waves": 4, "cols": 1, "cols_per_lane": 1}
    p = tmp_path / "t.md"
    p.write_text("```json\n" + json.dumps({"workload": "sweep", "storage": "c16", "kernel_source_sha256": h,
                                            "bytes_per_launch": 7, "tile": shape}) + "\n```\n")
    assert bench.measured_traffic(str(p), "sweep", "c16", dict(shape, items=31744, rule="autotuned")) == 7
    assert bench.measured_traffic(str(p), "sweep", "c16", dict(shape, chunk_rows=48)) is None
    assert bench.measured_traffic(str(p), "sweep", "c16", dict(shape, cols_per_lane=2)) is None
    assert bench.measured_traffic(str(p), "sweep", "c16") == 7
    r = bench.roofline_of("c16", 1000, 1.0, "sweep", str(p), dict(shape, cols_per_lane=2))
    assert r["traffic"] is None and r["kernel"] == "pair_kernel<lbmcg::C16>"
    r = bench.roofline_of("c16", 1000, 1.0, "sweep", str(p), shape)
    assert r["traffic"] == 7 and r["kernel"] == "step_kernel<lbmcg::C16>"

