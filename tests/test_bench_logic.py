"""Host logic of bench.py (no GPU): the roofline kernel's choice, the digest that keeps
counter traffic tied to the kernel sources it was measured on, and the one-GPU limit."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_dominant_kernel_is_the_most_time_per_step():
    # the complex64 head is the slowest launch, but the FP64 head runs more of them
    kernels = {
        "FP64 head": {"avg_us": 23.8, "ms_per_step": 6.96},
        "FP64 K2": {"avg_us": 17.3, "ms_per_step": 5.06},
        "complex64 head": {"avg_us": 30.0, "ms_per_step": 5.90},
        "complex64 K2": {"avg_us": 11.9, "ms_per_step": 4.09},
    }
    assert bench.dominant_kernel(kernels) == "FP64 head"
    kernels["complex64 head"]["ms_per_step"] = 7.5
    assert bench.dominant_kernel(kernels) == "complex64 head"


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    import hashlib
    data = json.load(open(bench.TRAFFIC_FILE))
    wl = sorted(data["workloads"])[0]
    name = sorted(data["workloads"][wl])[0]
    names = [(k, False) for k, v in bench.KERNEL_NAMES.items() if v == name] + \
            [(k, True) for k, v in bench.KERNEL_NAMES_MF.items() if name in v]
    (prec, kern), mf = names[0]
    ent = data["workloads"][wl][name]
    want = 1024.0 * (ent["fetch_kib"] * data["fetch_scale"] + ent["write_kib"] * data["write_scale"])
    # a summary whose digest matches the kernel sources as they are gives the figure
    h = hashlib.sha256()
    for rel in data["kernel_sources"]:
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    data["kernel_source_sha256"] = h.hexdigest()
    fresh = tmp_path / "fresh.json"
    fresh.write_text(json.dumps(data))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(fresh))
    got, kname = bench.measured_traffic(wl, prec, kern, matrix_free=mf)
    assert kname == name and got == pytest.approx(want)
    # a digest that no longer matches the kernel sources turns the figure off
    data["kernel_source_sha256"] = "0" * 64
    stale = tmp_path / "hbm_traffic.json"
    stale.write_text(json.dumps(data))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    got, kname = bench.measured_traffic(wl, prec, kern, matrix_free=mf)
    assert got is None and kname == (bench.KERNEL_NAMES_MF[(prec, kern)][0] if mf else name)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_default_workload_is_the_largest_single_gpu_configuration():
    # 32^3 x 64 is the headline; 16^4 is reported beside it as cache-resident
    import argparse
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--workload", default="c2"' in src
    assert bench.WORKLOAD_NAMES["c2"].startswith("32^3x64")


def test_cpu_model_is_read_from_the_host():
    name = bench.cpu_model()
    assert isinstance(name, str) and name and name != "x86_64"
