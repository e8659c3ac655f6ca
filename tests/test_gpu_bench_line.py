"""bench.py's output line on the GPU: one JSON object with the benchmark's
metric, the roofline of the step kernel (algorithmic bytes over the live
kernel time) and the fields the line promises."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_roofline():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "32",
                        "--warmup", "4", "--no-extras", "--no-cpu"],
                       capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    out = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in out, k
    assert out["n_gpus"] == 1 and out["steps"] == 32 and out["warmup"] == 4
    assert out["unit"] == "MLUPS" and out["dtype"] == "f32" and out["higher_is_better"] is True
    assert out["config"]["workload"] == "cavity128_Ra1e5_Pr0.02_Ste0.1"
    cells = 128 ** 3
    # MLUPS and ms_per_step describe the same timed steps
    assert abs(out["value"] - cells / (out["ms_per_step"] * 1e3)) < 0.01 * out["value"]
    rf = out["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["bytes_per_cell"] == 208 and rf["bytes_per_launch"] == 208 * cells
    achieved = rf["bytes_per_launch"] / (rf["kernel_ms"] * 1e-3) / 1e9
    assert abs(rf["achieved"] - achieved) < 0.01 * achieved
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    # the step kernel fits inside the step, and the kernel runs near its byte rate
    assert rf["kernel_ms"] <= out["ms_per_step"] * 1.05
    assert 0.4 < rf["frac"] < 1.2
    assert out["cpu_baseline"] is None      # --no-cpu
