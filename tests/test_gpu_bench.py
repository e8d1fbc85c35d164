"""bench.py's JSON line on the GPU: one short run of the uniform batch with
the documented fields, a roofline whose fraction is its achieved rate over
the published peak and whose achieved rate is the algorithmic flops of a
launch over the event-timed launch, and the uneven batch's balanced windows
named in its config."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*extra):
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1", "--no-cpu",
           "--no-legs"] + list(extra)
    print("bench:", " ".join(cmd[2:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    return json.loads(lines[0])


def test_bench_line_contract():
    out = run_bench("--workload", "uniform8")
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in out, k
    assert out["n_gpus"] == 1 and out["steps"] == 2 and out["warmup"] == 1
    assert out["higher_is_better"] is True and out["scaling"] == "weak" and out["dtype"] == "f64"
    assert out["vs_baseline"] is None
    assert out["config"]["workload"].startswith("uniform8")
    assert out["config"]["systems"] == 4096 and out["config"]["wh_steps_per_step"] == 4096
    rf = out["roofline"]
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == 78.6
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    assert abs(rf["achieved"] - rf["algorithmic_flops_per_launch"] / (rf["avg_launch_ms"] * 1e-3) / 1e12) \
        < 1e-9 * rf["achieved"]
    assert rf["algorithmic_flops_per_launch"] == 2893 * 4096 * 4096
    # whole-job throughput over the same timed launches
    assert abs(out["value"] - 4096 * 4096 / (out["ms_per_step"] * 1e-3)) < 1e-9 * out["value"]
    assert 0.05 < rf["frac"] < 1.0


def test_bench_uneven_runs_in_windows():
    out = run_bench("--workload", "uneven2to8")
    cfg = out["config"]
    assert cfg["packing"] == "mixed" and cfg["balance"] == 1
    assert cfg["launches_per_chunk"] > 1 and cfg["wavefronts_per_window"] >= 256
    assert cfg["flagged_systems"] == 0


def test_bench_by_planet_count():
    """--planets N: the workload's recipe with N planets per system, its own
    flop count in the roofline, no counter-derived traffic (the committed
    counters are for the workload's own count)."""
    out = run_bench("--workload", "uniform8", "--planets", "3")
    assert out["metric"] == "system-steps/s (3-planet FP64)"
    assert "with 3 planets per system" in out["config"]["workload"]
    assert out["config"]["planets_total"] == 3 * 4096
    rf = out["roofline"]
    assert rf["algorithmic_flops_per_launch"] == 898 * 4096 * 4096
    assert rf["traffic"] is None
