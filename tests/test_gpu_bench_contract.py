"""GPU: one short bench.py run in a child process, its JSON line against the contract the
benchmark reports on (keys, units, the roofline and CPU-baseline objects)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_keeps_the_contract(cuda):
    # the 16^4 workload keeps this run short; the default (32^3 x 64) has the same keys
    print("[gpu] bench.py --workload c1 --steps 2 --warmup 1 (child process)", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "c1", "--steps", "2",
           "--warmup", "1", "--fp64-steps", "2", "--no-batch", "--no-paper-workload",
           "--cpu-sample-iters", "10"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["unit"] == "shifted-solves/s" and d["higher_is_better"] is True
    assert d["value"] > 0 and d["converged"] is True
    assert d["max_true_rel_res"] <= 1e-10
    assert d["config"]["workload"].startswith("c1:")
    assert d["fp64_plain"]["steps"] == 2
    # the headline is quoted on the matrix-free operator; the stored matrix's lines
    # stand beside it
    assert d["config"]["operator"] == "matrix_free"
    st = d["stored_matrix"]
    assert st["mixed"]["converged"] is True and st["fp64"]["converged"] is True
    assert st["mixed"]["max_true_rel_res"] <= 1e-10
    assert d["roofline"]["kernel_name"] in ("k1_site<double, 2, true, false>",
                                            "k1_site<double, 2, true, true>",
                                            "k2_site<double, 2, true>", "k2_site<double, 2, false>",
                                            "k1_site<float, 2, false, true>",
                                            "k1_site<float, 2, false, false>",
                                            "k2_site<float, 2, true>", "k2_site<float, 2, false>")
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], abs=1e-4)
    assert 0 < rf["frac"] < 1
    assert rf["kernel"] in d["kernels"]
    assert rf["copy_ceiling"]["same_bytes_gbs"] > 0
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
    assert cb["unit"] == d["unit"]
    assert cb["cpu_model"] and cb["s_per_iter"] > 0
