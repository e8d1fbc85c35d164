"""bench.py's host-side contract: the one-GPU refusal, the CPU baseline's
fields (the oracle timed on a tiny sample), and the algorithmic flop count
the roofline divides by."""
import argparse
import json
import os
import subprocess
import sys

import numpy as np

import bench
from paper_2307_05683_amd import inputs
from paper_2307_05683_amd.flops import ALGO_FLOPS, ALGO_FLOPS_GR, ALGO_FLOPS_KC1

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_systems_subset_is_bounded():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "uniform8", "--systems",
                        "5000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "--systems must be in 1..4096" in r.stderr


def test_planet_count_option_is_bounded():
    for argv in (["--planets", "9"], ["--planets", "3", "--workload", "uneven2to8"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 2 and "--planets must be in 1..8" in r.stderr, argv


def test_cpu_baseline_fields():
    s = inputs.make_systems(8, 3, n_planets=8)
    args = argparse.Namespace(cpu_systems=4, cpu_steps=40, coords="dhc", no_legs=True)
    out = bench.cpu_baseline(s, args, 10065.0)
    json.dumps(out)
    assert out["kind"] == "oracle" and out["unit"] == "system-steps/s"
    assert out["value"] > 0 and out["value_1core"] > 0
    assert out["cores"] >= 1
    assert "4 systems" in out["sample"] and "GR" in out["sample"]
    assert isinstance(out["cpu"], dict)


def test_cpu_baseline_legs():
    """With the legs: the uniform and uneven batches' samples, the one-system
    configuration in full and the long-double reference, on tiny samples."""
    s = inputs.make_systems(8, 3, n_planets=8)
    args = argparse.Namespace(cpu_systems=8, cpu_steps=400, coords="dhc", no_legs=False)
    out = bench.cpu_baseline(s, args, 0.0)
    for k in ("uniform8", "uneven2to8", "single8", "long_double_1core"):
        assert out[k]["value"] > 0, k
    assert "1e5 steps" in out["single8"]["sample"]


def test_algorithmic_flops_of_a_batch():
    n = np.array([2, 3, 8, 8, 5])
    assert bench.flops_per_system_step(n, False) == sum(ALGO_FLOPS[k] for k in n)
    assert bench.flops_per_system_step(n, True) == sum(ALGO_FLOPS_GR[k] for k in n)
    assert bench.flops_per_system_step(n, False, kepler_counts=1) == sum(ALGO_FLOPS_KC1[k] for k in n)
    # a SABA_n step is n drifts and n kicks
    assert bench.flops_per_system_step(n, False, scheme="saba3") == 3 * sum(ALGO_FLOPS[k] for k in n)
    # the headline launch: 65536 GR systems x 4096 steps
    assert bench.flops_per_system_step(np.full(65536, 8), True) * 4096 == 3124 * 65536 * 4096
