"""The benchmark's output contract: one JSON line with the required fields, on
one GPU; more than one GPU is refused with a message."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.gpu
def test_bench_line_has_the_contract_fields():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--config", "small", "--steps", "2", "--warmup", "1",
           "--no-cpu-baseline", "--surfaces", "0", "--requests", "0"]
    print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["unit"] == "pair-evals/s" and d["higher_is_better"] is True and d["dtype"] == "f64"
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert "workload" in d["config"] and d["config"]["nc"] > 3
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert (rf["bound"], rf["unit"]) in (("alu", "TFLOP/s"), ("hbm", "GB/s"))
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    # one roofline per kernel of the step; the headline one is the kernel with the most device time per step
    names = [e["kernel"] for e in d["rooflines"]]
    assert names == ["k_volume64", "k_sweep", "k_factor_l", "k_factor_u", "k_certify"]
    assert rf["kernel"] == max(d["rooflines"], key=lambda e: e.get("rocprof_ms_per_step", e["ms_per_step"]))["kernel"]
    for e in d["rooflines"]:
        assert e["launches_per_step"] >= 1 and e["avg_launch_ms"] > 0 and e["frac"] > 0
    assert d["kernel_timing_run"]["same_result_as_timed_steps"]
    # pair-evaluations per step times steps per second equals the value
    pairs = d["pairs"]["group"] + d["pairs"]["append"] + d["pairs"]["volume"]
    assert abs(pairs / (d["ms_per_step"] * 1e-3) - d["value"]) <= 1e-6 * d["value"]
    assert d["greedy_iteration"]["bound"] == "latency"
    assert d["host_buffers"]["ms_per_step"] > 0
