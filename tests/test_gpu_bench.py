"""bench.py's one JSON line on the GPU: the keys its readers rely on and the
consistency of value, time and roofline."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_nine_colours():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--only", "nine", "--steps", "3",
                        "--warmup", "1", "--no-cpu-baseline"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads([ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["value"] > 0
    assert abs(d["value"] * d["ms_per_step"] * 1e-3 - d["config"]["pairs_per_step"]) < 1e-6 * d["value"]
    rf = d["roofline"]
    assert rf["bound"] in ("alu", "hbm", "mfma") and 0 < rf["frac"] < 1
    assert abs(rf["achieved"] / rf["peak"] - rf["frac"]) < 1e-9
    assert d["config"]["survivors_per_step"] > 0
    # the published FP32 peak; evaluated pairs are a subset of the decided ones
    assert rf["peak"] == 157.3 and rf["unit"] == "TFLOP/s"
    assert abs(rf["flops_per_launch"] - 85 * rf["evaluated_pairs"]) == 0
    assert 0 < d["evaluated_pairs_per_s"] <= d["decided_pairs_per_s"] == d["value"]
