"""Benchmark: Wisdom-Holman ensemble throughput on one MI355X.

Default workload: 4096 independent systems of 8 planets (star mass 1,
planet masses log-uniform in [1e-7, 1e-3], semi-major axes log-uniform in
[0.4, 30] with >= 10 mutual Hill radii spacing, e and i uniform in
[0, 0.05], dt = P_inner/20, drift-kick-drift, no GR), seeded and synthetic.
A "step" is one Wisdom-Holman timestep of every system of the batch (the
Kepler drift, interaction kick and jump of every planet); the metric is
system-steps per second.  The state is resident in device memory before
the timed region starts.

Printed: one JSON line with the metric, a roofline object for the step
kernel (algorithmic FP64 flops per launch / average launch time, against
the 78.6 TFLOP/s FP64 vector peak) and a CPU baseline (the oracle timed on
the host's cores on a bounded sample of the same workload).

Other workloads: --workload uneven2to8 (16384 systems, 2..8 planets,
per-system dt) also times the per-size reference path; --workload large8gr
(65536 systems with GR).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk

WORKLOAD_TEXT = {
    "uniform8": "4096 systems x 8 planets, dt = P_inner/20, drift-kick-drift, no GR",
    "uneven2to8": "16384 systems x 2..8 planets (uniform), dt uniform in [P_inner/30, P_inner/15], drift-kick-drift",
    "large8gr": "65536 systems x 8 planets, GR (c = 10065), dt = P_inner/20, drift-kick-drift",
    "single8": "1 system x 8 planets, dt = P_inner/20, kick-drift-kick",
    "adjoint8": "1024 systems x 8 planets, dt = P_inner/20, drift-kick-drift; reverse mode with checkpoints "
                "every 1000 steps, loss sum |Q(T)|^2",
}


# Steps of each workload's run; large8gr's 1e7-step run is timed over 1e6
# steps to keep the GPU held for seconds, not a minute.
DEFAULT_STEPS = {"uniform8": 1_000_000, "uneven2to8": 1_000_000, "large8gr": 1_000_000, "single8": 100_000,
                 "adjoint8": 100_000}


# Two planets per lane pays once the one-planet layout has more wavefronts
# than the chip has SIMDs (fewer, heavier waves with more independent work);
# two lanes per planet pays when it has fewer (more, lighter waves).
# The uneven batch is run as its workload states, with the autotuned packing
# (which picks two planets per lane).
DEFAULT_PACKING = {"uneven2to8": "tuned", "large8gr": "pair", "uniform8": "split", "single8": "split"}
KERNEL_NAME = {"pair": "k_step_pair (persistent step kernel, two planets per lane)",
               "split": "k_step_split (persistent step kernel, two lanes per planet)",
               "serial": "k_step_serial (persistent step kernel, one lane per system)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed Wisdom-Holman steps (default: 1e5 for adjoint8 and single8, 1e6 otherwise)")
    ap.add_argument("--warmup", type=int, default=4096, help="untimed steps before the timed region")
    ap.add_argument("--workload", default="uniform8", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--packing", default=None,
                    help="auto|pow2|g8|pair|split|serial|tuned (default: tuned for uneven2to8, pair for large8gr, whose "
                         "batch fills more wavefronts than the chip has SIMDs, split for uniform8 and single8, which "
                         "fill fewer; auto otherwise)")
    ap.add_argument("--block-waves", type=int, default=None,
                    help="wavefronts per workgroup (default 4 for uniform8: one four-wave workgroup per CU puts "
                         "exactly one of its 1024 wavefronts on each SIMD; 1 otherwise)")
    ap.add_argument("--chunk", type=int, default=4096)
    ap.add_argument("--exchange", default="auto", choices=["auto", "dpp", "lds"])
    ap.add_argument("--scheme", default=None, choices=["dkd", "kdk", "saba2", "saba3", "saba4"],
                    help="step composition (default: the workload's, drift-kick-drift)")
    ap.add_argument("--coords", default="dhc", choices=["dhc", "jacobi"],
                    help="splitting coordinates: democratic heliocentric (the paper's) or Jacobi")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--cpu-steps", type=int, default=80000)
    ap.add_argument("--cpu-systems", type=int, default=256)
    ap.add_argument("--plain-steps", type=int, default=2000, help="steps of the per-size reference path")
    ap.add_argument("--ckpt-every", type=int, default=1000, help="checkpoint interval of the adjoint workload")
    ap.add_argument("--save-state", default=None,
                    help="write the final synchronized states and per-system energy errors to this .npz file")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates memory counters)")
    return ap.parse_args()


def measured_counters(workload: str, chunk: int, coords: str = "dhc", packing: str = "auto"):
    """HBM bytes and hardware FP64 flops per launch from the committed counter
    summary, if the kernel sources are still the ones it was taken on (else
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
    key = "%s/%s" % (workload, "pow2" if packing == "auto" else packing)
    if key not in rec["bytes_per_launch"]:
        return None
    return {"traffic": rec["bytes_per_launch"][key], "hw_flops": rec.get("hw_flops_per_launch", {}).get(key)}


def flops_per_system_step(n_planets: np.ndarray, gr: bool, coords: str = "dhc", scheme: str = "dkd") -> float:
    """A SABA_n step is n drifts and n kicks: n times the counted step."""
    from paper_2307_05683_amd.flops import ALGO_FLOPS, ALGO_FLOPS_GR, ALGO_FLOPS_JACOBI, ALGO_FLOPS_JACOBI_GR
    if coords == "jacobi":
        table = ALGO_FLOPS_JACOBI_GR if gr else ALGO_FLOPS_JACOBI
    else:
        table = ALGO_FLOPS_GR if gr else ALGO_FLOPS
    stages = int(scheme[4:]) if scheme.startswith("saba") else 1
    return float(stages * sum(table[int(n)] for n in n_planets))


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(systems, args, gr_c, scheme="dkd"):
    """The oracle (double, converged Kepler solves) on a bounded sample of the
    same workload, on all host threads and on one."""
    import oracle
    sub = systems.subset(np.arange(min(args.cpu_systems, systems.S)))
    threads = oracle.max_threads()

    def run(s, n, nthreads):
        t0 = time.perf_counter()
        if args.coords == "jacobi":
            oracle.jacobi_integrate(s, n, scheme=scheme, precision="d", nthreads=nthreads, gr_c=gr_c)
        else:
            oracle.integrate(s, n, scheme=scheme, gr_c=gr_c, precision="d", nthreads=nthreads)
        return time.perf_counter() - t0

    dt = run(sub, args.cpu_steps, threads)
    one = sub.subset(np.arange(min(16, sub.S)))
    n1 = max(1, args.cpu_steps // 8)
    dt1 = run(one, n1, 1)
    return {
        "value": sub.S * args.cpu_steps / dt,
        "unit": "system-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d systems of the same workload x %d steps, FP64, converged Kepler solves, OpenMP over systems "
                  "(%.1f s wall)" % (sub.S, args.cpu_steps, dt),
        "value_1core": one.S * n1 / dt1,
        "sample_1core": "%d systems x %d steps on one thread (%.1f s wall)" % (one.S, n1, dt1),
        "cpu_model": _cpu_model(),
    }


def adjoint_cost(systems, args, dev, stream, t_plain, gr_c, scheme, opts):
    """Forward with checkpoints + adjoint, against the plain forward of the
    same steps (the cost ratio of reverse mode), with the scheme and packing
    of the forward run.  A short run first loads every kernel involved; the
    loss seed dL/dQ_T = 2 Q_T is formed outside the timed intervals."""
    import torch
    from paper_2307_05683_amd.ensemble import Ensemble
    w = Ensemble.from_systems(systems.subset(np.arange(min(64, systems.S))), device=dev, gr_c=gr_c, scheme=scheme,
                              **opts)
    w.forward_ckpt(4, 2)
    QT, VT = w.state()
    w.adjoint(2 * QT, torch.zeros_like(VT))
    torch.cuda.synchronize()
    w.close()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e = Ensemble.from_systems(systems, device=dev, gr_c=gr_c, scheme=scheme, **opts)
    ev[0].record(stream)
    e.forward_ckpt(args.steps, args.ckpt_every)
    ev[1].record(stream)
    QT, VT = e.state()
    gQ, gV = 2 * QT, torch.zeros_like(VT)
    torch.cuda.synchronize()
    ev[2].record(stream)
    g = e.adjoint(gQ, gV)
    ev[3].record(stream)
    torch.cuda.synchronize()
    t_ckpt = ev[0].elapsed_time(ev[1]) / 1e3
    t_adj = ev[2].elapsed_time(ev[3]) / 1e3
    finite = bool(all(torch.isfinite(x).all().item() for x in g))
    e.close()
    return {"steps": args.steps, "ckpt_every": args.ckpt_every, "forward_s": t_plain, "forward_ckpt_s": t_ckpt,
            "adjoint_s": t_adj, "cost_ratio": (t_ckpt + t_adj) / t_plain, "backward_over_forward": t_adj / t_plain,
            "gradients_finite": finite}


def main():
    args = parse()
    if args.packing is None:
        args.packing = DEFAULT_PACKING.get(args.workload, "auto")
    if args.block_waves is None:
        args.block_waves = 4 if args.workload == "uniform8" else 1
    if args.steps is None:
        args.steps = DEFAULT_STEPS.get(args.workload, 1_000_000)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (systems are independent; "
              "see the sharding design notes). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2307_05683_amd import inputs
    from paper_2307_05683_amd.ensemble import Ensemble

    gr_c = inputs.GR_C if args.workload == "large8gr" else 0.0
    scheme = args.scheme or ("kdk" if args.workload == "single8" else "dkd")
    systems = inputs.workload(args.workload)
    dev = torch.device("cuda:0")
    opts = dict(packing=args.packing, block_waves=args.block_waves, chunk_steps=args.chunk, exchange=args.exchange,
                coords=args.coords)
    tune_table = None
    if args.packing == "tuned":
        from paper_2307_05683_amd.autotune import autotune
        print("[bench] autotuning the lane packing ...", file=sys.stderr, flush=True)
        best, tune_table = autotune(systems, gr_c=gr_c, scheme=scheme, device=dev, coords=args.coords)
        opts.update(best)
        print("[bench] chosen: %s" % best, file=sys.stderr, flush=True)
    ens = Ensemble.from_systems(systems, gr_c=gr_c, scheme=scheme, device=dev, **opts)
    E0 = ens.energy()        # initial energy of every system (outside the timed region)
    print("[bench] %s: S=%d, warmup %d steps" % (args.workload, systems.S, args.warmup), file=sys.stderr, flush=True)
    if args.copy_probe_mb:
        x = torch.ones(args.copy_probe_mb << 17, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.warmup:
        ens.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    ens.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    print("[bench] timed %d steps: %.3f s (events), %.3f s (wall)" % (args.steps, gpu_s, wall), file=sys.stderr,
          flush=True)
    flags = ens.flags().cpu().numpy()
    E1 = ens.energy()
    dE = ((E1 - E0) / E0).abs().cpu().numpy()
    ok = flags == 0
    if args.save_state:
        Q, V = ens.state()
        np.savez(args.save_state, Q=Q.cpu().numpy(), V=V.cpu().numpy(), rel_energy_error=dE, flags=flags,
                 n_planets=systems.n_planets, steps=args.warmup + args.steps)
    sys_steps = systems.S * args.steps
    value = sys_steps / gpu_s
    n_launch = -(-args.steps // opts["chunk_steps"])
    flops_step = flops_per_system_step(systems.n_planets, gr_c > 0, args.coords, scheme)
    achieved = flops_step * args.steps / gpu_s / 1e12
    out = {
        "metric": "system-steps/s (8-planet FP64)" if "8" in args.workload else "system-steps/s (FP64)",
        "value": value,
        "unit": "system-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: %s" % (args.workload, WORKLOAD_TEXT[args.workload]),
            "systems": systems.S,
            "planets_total": int(systems.n_planets.sum()),
            "packing": opts["packing"],
            "chunk_steps": opts["chunk_steps"],
            "block_waves": opts["block_waves"],
            "exchange": opts["exchange"],
            "coords": args.coords,
            "scheme": scheme,
            "flagged_systems": int((flags != 0).sum()),
        },
        # relative energy error |E(T) - E(0)| / |E(0)| per system after the warmup and timed steps (unflagged)
        "energy_error": {
            "steps": args.warmup + args.steps,
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
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
            "kernel": KERNEL_NAME.get(opts["packing"], "k_step (persistent step kernel)"),
            "algorithmic_flops_per_step": flops_step,
            "avg_launch_ms": gpu_s * 1e3 / n_launch,
            "launches": n_launch,
        },
    }
    counters = measured_counters(args.workload, opts["chunk_steps"], args.coords, opts["packing"])
    if counters and scheme == "dkd":
        out["roofline"]["traffic"] = counters["traffic"]
        if counters["hw_flops"]:
            # FP64 flops the hardware executed (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes, FMA = 2, per step of a
            # counted launch) over the timed steps: the kernel's own issue efficiency, beside the
            # algorithmic fraction
            hw = counters["hw_flops"] / opts["chunk_steps"] * args.steps / gpu_s / 1e12
            out["roofline"]["achieved_hardware"] = hw
            out["roofline"]["frac_hardware"] = hw / FP64_PEAK_TFLOPS
    if tune_table is not None:
        out["config"]["autotune"] = [dict(r["opts"], rate=r["system_steps_per_s"]) for r in tune_table]
    if args.workload == "adjoint8":
        out["adjoint"] = adjoint_cost(systems, args, dev, stream, gpu_s, gr_c, scheme, opts)
    if args.workload == "uneven2to8" and args.plain_steps > 0:
        plain = Ensemble.from_systems(systems, gr_c=gr_c, scheme=scheme, packing="g8", coords=args.coords,
                                      device=dev)
        plain.step_plain(10)
        torch.cuda.synchronize()
        ev0.record(stream)
        plain.step_plain(args.plain_steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ps = ev0.elapsed_time(ev1) / 1e3
        out["plain_per_size"] = {"value": systems.S * args.plain_steps / ps, "steps": args.plain_steps,
                                 "speedup_fused_over_plain": value / (systems.S * args.plain_steps / ps)}
        plain.close()
        # the stronger variant: one persistent context per planet count (the
        # same 8-lane groups, each size's steps in chunked launches), run one
        # after the other -- separates the gain of packing from that of
        # persistence
        subs = [Ensemble.from_systems(systems.subset(np.flatnonzero(systems.n_planets == n)), gr_c=gr_c,
                                      scheme=scheme, packing="g8", coords=args.coords, device=dev)
                for n in range(1, 9) if (systems.n_planets == n).any()]
        n_sub = 8 * args.plain_steps
        for sub in subs:
            sub.step(64)
        torch.cuda.synchronize()
        ev0.record(stream)
        for sub in subs:
            sub.step(n_sub)
        ev1.record(stream)
        torch.cuda.synchronize()
        ts = ev0.elapsed_time(ev1) / 1e3
        out["per_size_persistent"] = {"value": systems.S * n_sub / ts, "steps": n_sub,
                                      "speedup_fused_over_it": value / (systems.S * n_sub / ts)}
        for sub in subs:
            sub.close()
    ens.close()
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
