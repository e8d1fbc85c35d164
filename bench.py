"""Benchmark: Wisdom-Holman ensemble throughput on one MI355X.

Headline workload (the largest single-GPU configuration): 65536 independent
systems of 8 planets with the GR potential (c = 10065), star mass 1, planet
masses log-uniform in [1e-7, 1e-3], semi-major axes log-uniform in [0.4, 30]
with >= 10 mutual Hill radii spacing, e and i uniform in [0, 0.05],
dt = P_inner/20, drift-kick-drift; seeded and synthetic.

A bench "step" is one launch of the persistent step kernel: every system of
the batch advances by --chunk (4096) Wisdom-Holman timesteps (Kepler drift,
interaction kick, jumps and GR kick of every planet, 4096 times) with the
state held in registers.  --steps K times K such launches back to back on
the stream the kernel runs on; the metric counts Wisdom-Holman
system-steps per second.  The state is resident in device memory before the
timed region starts.

Printed: one JSON line with the metric, a roofline object for the dominant
kernel (algorithmic FP64 flops per launch / average launch duration, against
the 78.6 TFLOP/s FP64 vector peak), a CPU baseline (the oracle timed on the
host's cores on bounded samples) and, measured in the same run, the other
parts of the metric:
  legs.uniform8   -- 4096 x 8 planets, no GR: system-steps/s and frac;
  legs.uneven2to8 -- 16384 systems of 2..8 planets with per-system dt: the
                     fused persistent kernel against the plain per-size-launch
                     kernel (ratio) and its frac;
  legs.adjoint8   -- 1024 x 8 planets, 2e4 steps, checkpoints every 1000:
                     reverse-mode cost over the plain forward of the same run;
  legs.single8    -- the one-system configuration (1 x 8 planets, 1e5 steps,
                     kick-drift-kick): steps/s on one 16-lane group;
  legs.explorer_counts -- the headline batch with the Kepler iteration
                     counts the autotuner picks after validating the cheaper
                     compiled set with the envelope explorer (App. A).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk

WORKLOAD_TEXT = {
    "large8gr": "65536 systems x 8 planets, GR (c = 10065), dt = P_inner/20, drift-kick-drift",
    "uniform8": "4096 systems x 8 planets, dt = P_inner/20, drift-kick-drift, no GR",
    "uneven2to8": "16384 systems x 2..8 planets (uniform), dt uniform in [P_inner/30, P_inner/15], drift-kick-drift",
    "single8": "1 system x 8 planets, dt = P_inner/20, kick-drift-kick",
    "adjoint8": "1024 systems x 8 planets, dt = P_inner/20, drift-kick-drift; reverse mode with checkpoints "
                "every 1000 steps, loss sum |Q(T)|^2",
}

# Lane packing per workload.  Two planets per lane pays once the one-planet
# layout has more wavefronts than the chip has SIMDs (fewer, heavier waves
# with more independent work); two lanes per planet pays when it has fewer.
DEFAULT_PACKING = {"large8gr": "pair", "uneven2to8": "mixed", "uniform8": "split", "single8": "split",
                   "adjoint8": "split"}
# Wavefronts per workgroup: four-wave workgroups put one wave of each
# workgroup on each SIMD of a CU.
DEFAULT_BLOCK_WAVES = {"large8gr": 1, "uneven2to8": 4, "uniform8": 4, "single8": 1, "adjoint8": 4}
# Balanced launch windows (wh_config.balance) for the uneven batch: its
# one-planet-per-lane wavefronts of several costs (1315 with two systems
# sharing the 8-lane groups of 5+3 and 6+2 planets, 1535 without) run in
# windows of 1024 equal-work wavefronts (+15% over two planets per lane,
# whose 769 heavy wavefronts leave a quarter of the SIMDs idle; the shared
# groups add 6%).  The GR batch's 4096 pair wavefronts of one cost measured
# the same with and without windows.
DEFAULT_BALANCE = {"large8gr": 0, "uneven2to8": 1, "uniform8": 0, "single8": 0, "adjoint8": 0}
KERNEL_NAME = {"pair": "k_step_pair (persistent step kernel, two planets per lane)",
               "split": "k_step_split (persistent step kernel, two lanes per planet)",
               "serial": "k_step_serial (persistent step kernel, one lane per system)",
               "mixed": "k_step_mixed (persistent step kernel, one planet per lane, two systems in some 8-lane "
                        "groups)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60,
                    help="timed bench steps; one bench step = one launch of --chunk Wisdom-Holman steps of the batch")
    ap.add_argument("--warmup", type=int, default=4, help="untimed bench steps before the timed region")
    ap.add_argument("--workload", default="large8gr", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--packing", default=None, help="auto|pow2|g8|pair|split|serial (default: per workload)")
    ap.add_argument("--block-waves", type=int, default=None)
    ap.add_argument("--balance", type=int, default=None, choices=[0, 1],
                    help="balanced launch windows (default: per workload)")
    ap.add_argument("--chunk", type=int, default=4096, help="Wisdom-Holman steps per launch")
    ap.add_argument("--planets", type=int, default=0,
                    help="draw the workload's systems with N planets each instead of its own count (1..8; the "
                         "uniform-count workloads only): throughput by planet count, not the headline")
    ap.add_argument("--systems", type=int, default=0,
                    help="run only the workload's first N systems (0: all; an occupancy scan, not the headline)")
    ap.add_argument("--exchange", default="auto", choices=["auto", "dpp", "lds"])
    ap.add_argument("--scheme", default=None, choices=["dkd", "kdk", "saba2", "saba3", "saba4"],
                    help="step composition (default: the workload's, drift-kick-drift)")
    ap.add_argument("--coords", default="dhc", choices=["dhc", "jacobi"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-legs", action="store_true", help="skip the uniform, uneven, adjoint and single legs")
    ap.add_argument("--cpu-steps", type=int, default=40000, help="steps of the oracle's multi-thread sample")
    ap.add_argument("--cpu-systems", type=int, default=256)
    ap.add_argument("--save-state", default=None,
                    help="write the final synchronized states and per-system energy errors to this .npz file")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates memory counters)")
    return ap.parse_args()


def measured_counters(workload: str, chunk: int, coords: str = "dhc", packing: str = "auto", windows: int = 1):
    """HBM bytes and hardware FP64 flops per launch (per chunk of balanced
    windows when windows > 1) from the committed counter summary, if the
    kernel and host-planner sources are still the ones it was taken on (else
    None)."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", "k_step_hbm_traffic.md")).read()
        rec = json.loads(re.search(r"```json\n(.*?)```", text, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    for name, digest in rec["sources"].items():
        try:
            with open(os.path.join(ROOT, "paper_2307_05683_amd", "csrc", name), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    if chunk != rec["chunk_steps"] or coords != "dhc":
        return None
    key = "%s/%s%s" % (workload, "pow2" if packing == "auto" else packing, "+windows" if windows > 1 else "")
    if key not in rec["bytes_per_launch"]:
        return None
    return {"traffic": rec["bytes_per_launch"][key], "hw_flops": rec.get("hw_flops_per_launch", {}).get(key)}


def fp64_issue_probe() -> dict | None:
    """Run the standalone FP64 issue-rate probe (built beside the library) as
    a child process: the rate of independent FMA chains at 8 wavefronts per
    SIMD and the issue cost of a reciprocal seed, context for the roofline
    fractions.  None if the probe is not built or fails."""
    exe = os.path.join(ROOT, "paper_2307_05683_amd", "fp64_issue_probe")
    if not os.access(exe, os.X_OK):
        return None
    try:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    except (OSError, subprocess.SubprocessError):
        return None
    if r.returncode != 0:
        return None
    try:
        return json.loads(r.stdout.strip().splitlines()[-1])
    except (ValueError, IndexError):
        return None


def flops_per_system_step(n_planets: np.ndarray, gr: bool, coords: str = "dhc", scheme: str = "dkd",
                          kepler_counts: int = 0) -> float:
    """Algorithmic FP64 operations of one step of the batch (the oracle's count
    of the fixed-iteration step with the count set that ran: the paper's, or
    kepler_counts = 1); a SABA_n step is n drifts and n kicks: n times the
    counted step."""
    from paper_2307_05683_amd.flops import (ALGO_FLOPS, ALGO_FLOPS_GR, ALGO_FLOPS_GR_KC1, ALGO_FLOPS_JACOBI,
                                            ALGO_FLOPS_JACOBI_GR, ALGO_FLOPS_KC1)
    if coords == "jacobi":
        table = ALGO_FLOPS_JACOBI_GR if gr else ALGO_FLOPS_JACOBI
    elif kepler_counts == 1:
        table = ALGO_FLOPS_GR_KC1 if gr else ALGO_FLOPS_KC1
    else:
        table = ALGO_FLOPS_GR if gr else ALGO_FLOPS
    stages = int(scheme[4:]) if scheme.startswith("saba") else 1
    return float(stages * sum(table[int(n)] for n in n_planets))


def _cpu_model() -> dict:
    """CPU model and topology as the host reports them (/proc/cpuinfo, lscpu)."""
    out = {"model": "unknown"}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                out["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)",
                     "CPU max MHz", "Vendor ID", "CPU family", "Model"):
                out["lscpu " + k] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        out["affinity_cpus"] = len(os.sched_getaffinity(0))
    except OSError:
        pass
    return out


def cpu_baseline(systems, args, gr_c, scheme="dkd"):
    """The oracle as it stands (double precision, Kepler solved to
    convergence, OpenMP over systems) on bounded samples: the headline
    workload on all host threads and on one, the uniform and uneven
    batches, the one-system configuration in full, and the long-double
    parity reference."""
    import oracle
    from paper_2307_05683_amd import inputs
    threads = oracle.max_threads()

    def run(s, n, nthreads, precision="d", sch=scheme, gr=gr_c):
        t0 = time.perf_counter()
        if args.coords == "jacobi":
            oracle.jacobi_integrate(s, n, scheme=sch, precision=precision, nthreads=nthreads, gr_c=gr)
        else:
            oracle.integrate(s, n, scheme=sch, gr_c=gr, precision=precision, nthreads=nthreads)
        return time.perf_counter() - t0

    sub = systems.subset(np.arange(min(args.cpu_systems, systems.S)))
    dt = run(sub, args.cpu_steps, threads)
    one = sub.subset(np.arange(min(16, sub.S)))
    n1 = max(1, args.cpu_steps // 8)
    dt1 = run(one, n1, 1)
    out = {
        "value": sub.S * args.cpu_steps / dt,
        "unit": "system-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d systems of the headline workload (%s) x %d steps, FP64, converged Kepler solves, OpenMP "
                  "over systems on %d threads (%.1f s wall)" % (sub.S, "GR" if gr_c > 0 else "no GR",
                                                                 args.cpu_steps, threads, dt),
        "value_1core": one.S * n1 / dt1,
        "sample_1core": "%d systems x %d steps on one thread (%.1f s wall)" % (one.S, n1, dt1),
        "cpu": _cpu_model(),
    }
    if not args.no_legs and args.coords == "dhc":
        uni = inputs.workload("uniform8").subset(np.arange(args.cpu_systems))
        n_uni = args.cpu_steps // 4
        t_uni = run(uni, n_uni, threads, gr=0.0)
        out["uniform8"] = {"value": uni.S * n_uni / t_uni, "sample": "%d systems x %d steps, %d threads (%.1f s)"
                           % (uni.S, n_uni, threads, t_uni)}
        unev = inputs.workload("uneven2to8").subset(np.arange(args.cpu_systems))
        n_u = args.cpu_steps // 4
        t_u = run(unev, n_u, threads, gr=0.0)
        out["uneven2to8"] = {"value": unev.S * n_u / t_u, "sample": "%d systems x %d steps, %d threads (%.1f s)"
                             % (unev.S, n_u, threads, t_u)}
        single = inputs.workload("single8")
        t_s = run(single, 100_000, 1, sch="kdk", gr=0.0)
        out["single8"] = {"value": 1e5 / t_s, "sample": "1 system x 1e5 steps (the whole configuration), "
                          "kick-drift-kick, one thread (%.2f s)" % t_s}
        ld = sub.subset(np.arange(min(16, sub.S)))
        t_ld = run(ld, 2000, 1, precision="ld")
        out["long_double_1core"] = {"value": ld.S * 2000 / t_ld,
                                    "sample": "%d systems x 2000 steps in long double on one thread (the parity "
                                              "reference, not the baseline; %.1f s)" % (ld.S, t_ld)}
    return out


def warm(ens, n_launch, chunk):
    """Untimed launches; at least one graph's worth, so that the HIP graph of
    the step loop is captured before any timed region.  Returns the count."""
    n = max(n_launch, int(ens.cfg.graph_launches))
    ens.step(n * chunk)
    return n


def timed_chunks(ens, n_launch, chunk, stream):
    """Run n_launch launches of chunk steps; seconds between events recorded
    on the kernels' stream."""
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    ens.step(n_launch * chunk)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / 1e3


def leg_uniform(dev, stream, chunk):
    from paper_2307_05683_amd import inputs
    from paper_2307_05683_amd.ensemble import Ensemble
    s = inputs.workload("uniform8")
    e = Ensemble.from_systems(s, device=dev, packing="split", block_waves=4, chunk_steps=chunk)
    warm(e, 1, chunk)
    n = 8
    t = timed_chunks(e, n, chunk, stream)
    e.close()
    fl = flops_per_system_step(s.n_planets, False)
    return {"workload": WORKLOAD_TEXT["uniform8"], "packing": "split", "value": s.S * n * chunk / t,
            "unit": "system-steps/s", "steps": n * chunk, "avg_launch_ms": t * 1e3 / n,
            "frac": fl * chunk / (t / n) / 1e12 / FP64_PEAK_TFLOPS,
            "kernel": KERNEL_NAME["split"]}


def leg_uneven(dev, stream, chunk):
    """Fused persistent launch (fixed packing) vs the plain per-size-launch
    kernel (one 8-lane group per system, one launch per planet count per step,
    state through HBM every step, no graph) and vs one persistent context per
    planet count run one after the other."""
    import torch
    from paper_2307_05683_amd import inputs
    from paper_2307_05683_amd.ensemble import Ensemble
    s = inputs.workload("uneven2to8")
    pk, bw, bal = DEFAULT_PACKING["uneven2to8"], DEFAULT_BLOCK_WAVES["uneven2to8"], DEFAULT_BALANCE["uneven2to8"]
    e = Ensemble.from_systems(s, device=dev, packing=pk, block_waves=bw, chunk_steps=chunk, balance=bal)
    windows = e.launch_windows[0]
    warm(e, 1, chunk)
    n = 8
    t = timed_chunks(e, n, chunk, stream)
    e.close()
    fused = s.S * n * chunk / t
    fl = flops_per_system_step(s.n_planets, False)
    plain = Ensemble.from_systems(s, device=dev, packing="g8")
    plain.step_plain(10)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_plain = 512
    torch.cuda.synchronize()
    ev0.record(stream)
    plain.step_plain(n_plain)
    ev1.record(stream)
    torch.cuda.synchronize()
    tp = ev0.elapsed_time(ev1) / 1e3
    plain.close()
    subs = [Ensemble.from_systems(s.subset(np.flatnonzero(s.n_planets == k)), packing="g8", device=dev,
                                  chunk_steps=chunk)
            for k in range(1, 9) if (s.n_planets == k).any()]
    for sub in subs:
        sub.step(64)
    torch.cuda.synchronize()
    ev0.record(stream)
    for sub in subs:
        sub.step(chunk)
    ev1.record(stream)
    torch.cuda.synchronize()
    ts = ev0.elapsed_time(ev1) / 1e3
    for sub in subs:
        sub.close()
    return {"workload": WORKLOAD_TEXT["uneven2to8"], "packing": pk, "block_waves": bw, "balance": bal,
            "launches_per_chunk": windows, "value": fused,
            "unit": "system-steps/s", "steps": n * chunk, "avg_launch_ms": t * 1e3 / n,
            "frac": fl * chunk / (t / n) / 1e12 / FP64_PEAK_TFLOPS, "kernel": KERNEL_NAME.get(pk, "k_step"),
            "plain_per_size": {"value": s.S * n_plain / tp, "steps": n_plain},
            "speedup_fused_over_plain": fused / (s.S * n_plain / tp),
            "per_size_persistent": {"value": s.S * chunk / ts, "steps": chunk},
            "speedup_fused_over_per_size_persistent": fused / (s.S * chunk / ts)}


def leg_adjoint(dev, stream, workload="adjoint8", n_steps=20000, every=1000):
    """Reverse-mode cost: (forward with checkpoints + adjoint) over the plain
    forward of the same steps, all in the workload's packing (the one that
    fills the most SIMDs for it).  The adjoint configuration's batch (1024 x
    8) fills a quarter of the SIMDs; the uniform batch (4096 x 8, two lanes
    per planet) fills all of them.  A short run first loads every kernel
    involved; the loss seed dL/dQ_T = 2 Q_T is formed outside the timed
    intervals."""
    import torch
    from paper_2307_05683_amd import inputs
    from paper_2307_05683_amd.ensemble import Ensemble
    s = inputs.workload(workload)
    opts = dict(packing=DEFAULT_PACKING[workload], block_waves=DEFAULT_BLOCK_WAVES[workload])
    w = Ensemble.from_systems(s.subset(np.arange(64)), device=dev, **opts)
    w.forward_ckpt(4, 2)
    QT, VT = w.state()
    w.adjoint(2 * QT, torch.zeros_like(VT))
    w.step(64)
    torch.cuda.synchronize()
    w.close()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    f = Ensemble.from_systems(s, device=dev, **opts)
    torch.cuda.synchronize()
    ev[4].record(stream)
    f.step(n_steps)
    ev[5].record(stream)
    torch.cuda.synchronize()
    f.close()
    e = Ensemble.from_systems(s, device=dev, **opts)
    torch.cuda.synchronize()
    ev[0].record(stream)
    e.forward_ckpt(n_steps, every)
    ev[1].record(stream)
    QT, VT = e.state()
    gQ, gV = 2 * QT, torch.zeros_like(VT)
    torch.cuda.synchronize()
    ev[2].record(stream)
    g = e.adjoint(gQ, gV)
    ev[3].record(stream)
    torch.cuda.synchronize()
    t_plain = ev[4].elapsed_time(ev[5]) / 1e3
    t_ckpt = ev[0].elapsed_time(ev[1]) / 1e3
    t_adj = ev[2].elapsed_time(ev[3]) / 1e3
    finite = bool(all(torch.isfinite(x).all().item() for x in g))
    e.close()
    fl = flops_per_system_step(s.n_planets, False)
    text = WORKLOAD_TEXT[workload]
    if workload != "adjoint8":
        text += "; reverse mode with checkpoints every %d steps, loss sum |Q(T)|^2" % every
    return {"workload": text, "packing": opts["packing"], "steps": n_steps,
            "ckpt_every": every, "forward_s": t_plain, "forward_frac": fl * n_steps / t_plain / 1e12 / FP64_PEAK_TFLOPS,
            "forward_ckpt_s": t_ckpt, "adjoint_s": t_adj, "cost_ratio": (t_ckpt + t_adj) / t_plain,
            "backward_over_forward": t_adj / t_plain, "gradients_finite": finite}


def leg_counts(systems, dev, stream, chunk):
    """The headline batch with the Kepler count set the autotuner picks: the
    cheaper compiled set (one Halley step with 3 terms, two Newton steps)
    after the envelope explorer has validated it on the batch's own orbits
    within App. A's bound, else the paper's.  Its frac counts the flops of
    the set that ran."""
    from paper_2307_05683_amd import inputs
    from paper_2307_05683_amd.autotune import choose_kepler_counts
    from paper_2307_05683_amd.envelope import INTEGRATOR_COUNTS
    from paper_2307_05683_amd.ensemble import Ensemble
    opts = dict(packing=DEFAULT_PACKING["large8gr"], block_waves=DEFAULT_BLOCK_WAVES["large8gr"])
    kc, worst, z = choose_kepler_counts(systems, opts, "dkd", "dhc", dev)
    e = Ensemble.from_systems(systems, device=dev, gr_c=inputs.GR_C, chunk_steps=chunk, kepler_counts=kc, **opts)
    warm(e, 1, chunk)
    n = 8
    t = timed_chunks(e, n, chunk, stream)
    flags = int((e.flags().cpu().numpy() != 0).sum())
    e.close()
    fl = flops_per_system_step(systems.n_planets, True, kepler_counts=kc)
    return {"workload": WORKLOAD_TEXT["large8gr"], "packing": opts["packing"],
            "kepler_counts": list(INTEGRATOR_COUNTS[kc]), "validation_worst_da_over_a": worst,
            "validation_max_z": z, "value": systems.S * n * chunk / t, "unit": "system-steps/s",
            "steps": n * chunk, "avg_launch_ms": t * 1e3 / n,
            "frac": fl * chunk / (t / n) / 1e12 / FP64_PEAK_TFLOPS, "flagged_systems": flags}


def leg_single(dev, stream):
    import torch
    from paper_2307_05683_amd import inputs
    from paper_2307_05683_amd.ensemble import Ensemble
    s = inputs.workload("single8")
    e = Ensemble.from_systems(s, device=dev, packing="split", scheme="kdk")
    e.step(4096)
    E0 = e.energy()
    n = 100_000
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    e.step(n)
    ev1.record(stream)
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) / 1e3
    dE = float(((e.energy() - E0) / E0).abs().item())
    e.close()
    return {"workload": WORKLOAD_TEXT["single8"], "packing": "split", "steps": n, "value": n / t,
            "unit": "steps/s", "rel_energy_error": dE}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (systems are independent; "
              "see the sharding design notes). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0 or args.chunk < 1:
        print("--steps must be >= 1, --warmup >= 0 and --chunk >= 1", file=sys.stderr)
        sys.exit(2)
    packing = args.packing or DEFAULT_PACKING.get(args.workload, "auto")
    block_waves = args.block_waves or DEFAULT_BLOCK_WAVES.get(args.workload, 1)
    balance = DEFAULT_BALANCE.get(args.workload, 0) if args.balance is None else args.balance
    import torch
    from paper_2307_05683_amd import inputs
    from paper_2307_05683_amd.ensemble import Ensemble

    gr_c = inputs.GR_C if args.workload == "large8gr" else 0.0
    scheme = args.scheme or ("kdk" if args.workload == "single8" else "dkd")
    if args.planets:
        kw = dict(inputs.WORKLOADS[args.workload])
        if not 1 <= args.planets <= 8 or kw.get("n_planets") is None:
            print("--planets must be in 1..8, for a workload with one planet count per system", file=sys.stderr)
            sys.exit(2)
        kw["n_planets"] = args.planets
        systems = inputs.make_systems(**kw)
    else:
        systems = inputs.workload(args.workload)
    full_S = systems.S
    if args.systems:
        if not 1 <= args.systems <= full_S:
            print("--systems must be in 1..%d for %s" % (full_S, args.workload), file=sys.stderr)
            sys.exit(2)
        systems = systems.subset(np.arange(args.systems))
    dev = torch.device("cuda:0")
    chunk = args.chunk
    opts = dict(packing=packing, block_waves=block_waves, chunk_steps=chunk, exchange=args.exchange,
                coords=args.coords, balance=balance)
    ens = Ensemble.from_systems(systems, gr_c=gr_c, scheme=scheme, device=dev, **opts)
    windows, window_slots = ens.launch_windows
    E0 = ens.energy()        # initial energy of every system (outside the timed region)
    print("[bench] %s: S=%d, packing %s, warmup %d x %d steps" % (args.workload, systems.S, packing, args.warmup,
                                                                  chunk), file=sys.stderr, flush=True)
    if args.copy_probe_mb:
        x = torch.ones(args.copy_probe_mb << 17, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    warm_run = warm(ens, args.warmup, chunk)
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    gpu_s = timed_chunks(ens, args.steps, chunk, stream)
    wall = time.perf_counter() - t0
    print("[bench] timed %d launches x %d steps: %.3f s (events), %.3f s (wall)" % (args.steps, chunk, gpu_s, wall),
          file=sys.stderr, flush=True)
    flags = ens.flags().cpu().numpy()
    E1 = ens.energy()
    dE = ((E1 - E0) / E0).abs().cpu().numpy()
    ok = flags == 0
    if args.save_state:
        Q, V = ens.state()
        np.savez(args.save_state, Q=Q.cpu().numpy(), V=V.cpu().numpy(), rel_energy_error=dE, flags=flags,
                 n_planets=systems.n_planets, steps=(warm_run + args.steps) * chunk)
    ens.close()
    wh_steps = args.steps * chunk
    value = systems.S * wh_steps / gpu_s
    avg_launch = gpu_s / args.steps
    flops_step = flops_per_system_step(systems.n_planets, gr_c > 0, args.coords, scheme)
    achieved = flops_step * chunk / avg_launch / 1e12
    out = {
        "metric": ("system-steps/s (%d-planet FP64)" % args.planets if args.planets
                   else "system-steps/s (8-planet FP64)" if "8" in args.workload else "system-steps/s (FP64)"),
        "value": value,
        "unit": "system-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": avg_launch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: %s%s%s" % (args.workload, WORKLOAD_TEXT[args.workload],
                                        " (with %d planets per system)" % args.planets if args.planets else "",
                                        "" if systems.S == full_S else " (first %d systems only)" % systems.S),
            "wh_steps_per_step": chunk,
            "warmup_launches_run": warm_run,
            "systems": systems.S,
            "planets_total": int(systems.n_planets.sum()),
            "packing": packing,
            "block_waves": block_waves,
            "balance": balance,
            "launches_per_chunk": windows,
            "wavefronts_per_window": window_slots,
            "exchange": args.exchange,
            "coords": args.coords,
            "scheme": scheme,
            "kepler_counts": [2, 2, 4, 8],
            "flagged_systems": int((flags != 0).sum()),
        },
        # relative energy error |E(T) - E(0)| / |E(0)| per system after the warmup and timed steps (unflagged)
        "energy_error": {
            "steps": (warm_run + args.steps) * chunk,
            "median": float(np.median(dE[ok])) if ok.any() else None,
            "p90": float(np.percentile(dE[ok], 90)) if ok.any() else None,
            "p99": float(np.percentile(dE[ok], 99)) if ok.any() else None,
            "max": float(dE[ok].max()) if ok.any() else None,
            "flagged_fraction": float(1.0 - ok.mean()),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": None,
            "traffic_unit": "HBM bytes per bench step: one launch, or one chunk of balanced windows "
                            "(rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
            "kernel": KERNEL_NAME.get(packing, "k_step (persistent step kernel)"),
            "algorithmic_flops_per_launch": flops_step * chunk,
            "avg_launch_ms": avg_launch * 1e3,
            "launches": args.steps,
        },
    }
    # the committed counters describe the whole batch
    counters = (measured_counters(args.workload, chunk, args.coords, packing, windows)
                if systems.S == full_S and not args.planets else None)
    if counters and scheme == "dkd":
        out["roofline"]["traffic"] = counters["traffic"]
        if counters["hw_flops"]:
            # FP64 flops the hardware executed per launch (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes, FMA = 2)
            # over the measured launch: the kernel's issue efficiency, beside the algorithmic fraction
            hw = counters["hw_flops"] / avg_launch / 1e12
            out["roofline"]["achieved_hardware"] = hw
            out["roofline"]["frac_hardware"] = hw / FP64_PEAK_TFLOPS
    probe = fp64_issue_probe()
    if probe:
        # what a plain stream of independent FP64 FMAs reaches on this GPU in
        # the same run (a reference for the box, not a ceiling), beside the
        # published peak that `frac` is taken against
        out["roofline"]["fma_stream_tflops"] = probe["fma_tflops"]
        out["roofline"]["frac_of_fma_stream"] = achieved / probe["fma_tflops"]
        out["roofline"]["issue_probe"] = probe
    if not args.no_legs:
        legs = {}
        todo = [("uniform8", lambda: leg_uniform(dev, stream, chunk)),
                ("uneven2to8", lambda: leg_uneven(dev, stream, chunk)),
                ("adjoint8", lambda: leg_adjoint(dev, stream)),
                ("adjoint_uniform8", lambda: leg_adjoint(dev, stream, "uniform8")),
                ("single8", lambda: leg_single(dev, stream))]
        if args.workload == "large8gr" and args.coords == "dhc" and scheme == "dkd":
            todo.append(("explorer_counts", lambda: leg_counts(systems, dev, stream, chunk)))
        for name, fn in todo:
            print("[bench] leg %s ..." % name, file=sys.stderr, flush=True)
            legs[name] = fn()
        out["legs"] = legs
    if not args.no_cpu:
        print("[bench] CPU baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(systems, args, gr_c, scheme)
    # the paper's own figures (AVX512 CPU, real Solar System, 5-day step):
    # context only, not this metric's baseline
    out["context"] = {
        "paper_steps_per_s_per_core": 3.02e6,
        "paper_note": "WHFast512, 8 planets with GR, one AVX512 core (5 Gyr in 1.40 d); 80-thread node ~1.6e8 "
                      "system-steps/s; different hardware and workload, so vs_baseline stays null",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
