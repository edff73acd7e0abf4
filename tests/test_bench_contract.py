"""CPU checks of bench.py's contract: one GPU only, the algorithmic byte counts
behind the roofline figure, and the fields of the roofline block."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_512_f64():
    # 512^3, periodic x (256 slots of packed spectra): 8 B per real value
    ab = bench.algorithmic_bytes((512, 512, 512), 1, 256, 8, 16)
    n = 512 ** 3
    assert ab["x_forward"] == 16 * n            # read f, write S
    assert ab["z_march"] == 32 * n              # S read and written on the way up and down
    assert ab["x_inverse"] == 16 * n            # read S, write u
    assert sum(ab.values()) == 64 * n


def test_algorithmic_bytes_batch_and_float_spectra():
    ab = bench.algorithmic_bytes((8, 16, 32), 3, 16, 8, 8)
    n = 8 * 16 * 32 * 3
    assert ab["x_forward"] == 8 * n + 4 * n
    assert ab["z_march"] == 16 * n


def _per(xf, zm, xi):
    return {"x_forward": dict(total_ms=20 * xf, launches=20, avg_ms=xf),
            "z_march": dict(total_ms=20 * zm, launches=20, avg_ms=zm),
            "x_inverse": dict(total_ms=20 * xi, launches=20, avg_ms=xi),
            "other": dict(total_ms=0.1, launches=20, avg_ms=0.005)}


def test_roofline_block_picks_dominant_kernel():
    ab = bench.algorithmic_bytes((512, 512, 512), 1, 256, 8, 16)
    rb = bench.roofline_block(_per(0.4, 0.9, 0.45), ab, "no_such_workload", "f64", 512)
    assert rb["kernel"] == "k_zpipe" and rb["bound"] == "hbm" and rb["unit"] == "GB/s"
    assert rb["peak"] == 8000.0
    assert rb["achieved"] == pytest.approx(ab["z_march"] / 0.9e-3 / 1e9, rel=1e-3)
    assert rb["frac"] == pytest.approx(rb["achieved"] / 8000.0, rel=1e-3)
    assert rb["traffic"] is None            # no counters for this workload
    rb = bench.roofline_block(_per(1.0, 0.9, 0.45), ab, "no_such_workload", "f64", 512)
    assert rb["kernel"] == "k_xfwd"
    rb = bench.roofline_block(_per(0.4, 0.9, 0.45), ab, "no_such_workload", "f64", 2048)
    assert rb["kernel"] == "k_zmarch"        # the older march takes y lines over 1024


def test_traffic_needs_counters_of_the_current_kernels(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    entry = {"entries": {"w/f64/z_march": {"bytes_per_launch": 123}}}
    f.write_text(json.dumps(dict(entry, kernel_source_hash="0000")))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_for("z_march", "w", "f64") is None
    f.write_text(json.dumps(dict(entry, kernel_source_hash=bench.kernel_source_hash())))
    assert bench.traffic_for("z_march", "w", "f64") == 123
    assert bench.traffic_for("x_forward", "w", "f64") is None


def test_refined_bytes_512_one_correction():
    # first solve 8 + 4 (x), 16 (z), 4 + 4 (x inverse to float u0); first
    # correction 8 + 4 + 4 (fused residual), 16, 4 + 4 + 8: 84 B per point
    n = 512 ** 3
    rb = bench.refined_bytes((512, 512, 512), 1, 256, 1)
    assert rb["x_forward"] == 28 * n
    assert rb["z_march"] == 32 * n
    assert rb["x_inverse"] == 24 * n
    assert sum(rb.values()) == 84 * n
    # each later correction: residual 24 B/pt + x transform 4 B/pt, march 16, update 20
    rb2 = bench.refined_bytes((512, 512, 512), 1, 256, 2)
    assert sum(rb2.values()) - sum(rb.values()) == (24 + 4 + 16 + 20) * n
