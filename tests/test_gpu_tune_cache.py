"""GPU: the batched solve's launch choices cached on disk (MSC_TUNE_CACHE).

The first batched solve of a shape measures its candidates (SpMV layout x grid) and,
with MSC_TUNE_CACHE naming a file, appends one line for that shape; a fresh process with
the same file takes the stored choice without measuring again (no new line) and gives
the same bits.  Shapes are keyed by systems, right-hand sides, rows, entries, format,
lanes, grid and the row-length histogram.
"""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import sys
    import numpy as np
    import torch
    sys.path.insert(0, {root!r})
    import workloads as W
    from paper_1102_2143_amd import Operator, solve_batched
    dev = torch.device("cuda:0")
    ops, bs = [], []
    for i, dims in enumerate([(4, 4, 4, 6), (4, 6, 4, 4)]):
        p = W.staggered_problem(dims, 0.1, 7100 + i, 7200 + i, (1e-3, 1.0, 5), nrhs=2)
        op = Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind="mhm", device=dev)
        op.set_shifts(p["sigma"])
        ops.append(op)
        bs.append(p["b"])
    xs, infos, status = solve_batched(ops, bs, tol=1e-10, prec="fp64")
    assert status == "ok"
    np.save({out!r}, np.concatenate([x.cpu().numpy().ravel() for x in xs]))
    print("[tune-cache] solved", flush=True)
""")


def _run(cache, out):
    env = dict(os.environ, MSC_TUNE_CACHE=str(cache))
    code = SCRIPT.format(root=ROOT, out=str(out))
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=240)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]


def test_tune_cache_written_then_used(tmp_path, cuda):
    print("[gpu] tune cache: two processes", flush=True)
    cache = tmp_path / "tune.txt"
    _run(cache, tmp_path / "a.npy")
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("batch sys 2 rhs 2 ")
    sell, lanes, grid = (int(v) for v in lines[0].split("=")[1].split())
    assert sell in (0, 1) and lanes in (4, 8, 16) and 8 <= grid <= 2048
    _run(cache, tmp_path / "b.npy")
    assert cache.read_text().splitlines() == lines  # taken from the file, not re-measured
    assert np.array_equal(np.load(tmp_path / "a.npy"), np.load(tmp_path / "b.npy"))


def test_malformed_lines_are_ignored(tmp_path, cuda):
    cache = tmp_path / "tune.txt"
    cache.write_text("garbage\nbatch sys 2 = 1 99 64\n")
    _run(cache, tmp_path / "c.npy")
    lines = cache.read_text().splitlines()
    assert lines[:2] == ["garbage", "batch sys 2 = 1 99 64"] and len(lines) == 3
