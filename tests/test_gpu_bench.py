"""bench.py end to end on the GPU, on a small workload: one JSON line on stdout
with the contract's fields, a roofline block whose fraction is achieved / peak,
and a refined solve block."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "noisy_dnn", "--steps", "3", "--warmup", "1",
           "--skip-cpu-baseline", "--skip-faces", "--skip-periodic-z", "--skip-pcr"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=110, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["unit"] == "Mpts/s" and d["dtype"] == "f64" and d["higher_is_better"] is True
    assert d["config"]["workload"] == "noisy_dnn"
    npts = 256 ** 3
    assert d["value"] == pytest.approx(npts / d["ms_per_step"] / 1e3, rel=1e-3)
    rb = d["roofline"]
    assert rb["bound"] == "hbm" and rb["unit"] == "GB/s" and rb["peak"] == 8000.0
    assert rb["frac"] == pytest.approx(rb["achieved"] / rb["peak"], rel=1e-3)
    assert 0.0 < rb["frac"] < 1.0
    assert d["f64_backward_error"] < 1e-14
    ref = d["fp32_refined"]
    assert ref["max_rel_diff_vs_f64"] < 1e-12 and ref["refinement_steps"] >= 1
