"""Autotuner for the lane packing of an ensemble.

Candidates: packing (1/2/4/8-lane groups, always 8 lanes, two planets per
lane in 1/2/4-lane groups, two lanes per planet in 16-lane groups, one
lane per system, or 1/2/4/8-lane groups with two systems sharing some 8-lane
groups), partner exchange (DPP or LDS crossbar; the last three
layouts have a single schedule), wavefronts per workgroup, steps per
launch and balanced launch windows (on or off) (the splitting coordinates are the caller's choice, not a candidate:
they change the results, not just the speed).  Each candidate integrates the real batch for a short run; the
fastest (system-steps per second, GPU event time) wins.  Results are cached
in a JSON file keyed by GPU architecture, coordinates, scheme, GR on/off, the batch size
bucket and the planet-count histogram bucket, so a repeated shape reuses
the choice without timing again.

Probe runs start from a copy of the caller's initial state and are
discarded, so tuning never changes the caller's results.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import torch

from . import _lib
from .ensemble import Ensemble

CANDIDATES = {
    "packing": ["pow2", "g8", "pair", "split", "serial", "mixed"],
    "exchange": ["dpp", "lds"],
    "block_waves": [1, 4],
    "chunk_steps": [1024, 4096],
    "balance": [0, 1],
}


def cache_path() -> str:
    return os.environ.get("WH_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "wh_autotune.json"))


def shape_key(n_planets, gr: bool, scheme: str, coords: str = "dhc") -> str:
    n = np.asarray(n_planets)
    S = len(n)
    s_bucket = 1 << int(np.ceil(np.log2(max(S, 1))))
    hist = np.bincount(n, minlength=9)[1:] / max(S, 1)
    h_bucket = ",".join("%d" % round(10 * x) for x in hist)     # tenths of the batch per planet count
    try:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        arch = "unknown"
    return "%s|%s|%s|gr%d|S%d|%s" % (arch, coords, scheme, int(gr), s_bucket, h_bucket)


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def time_candidate(systems, opts, gr_c, scheme, steps, warmup, device, coords="dhc") -> float:
    """System-steps per second of one configuration on a short run."""
    e = Ensemble.from_systems(systems, gr_c=gr_c, scheme=scheme, device=device, graph_launches=-1, coords=coords,
                              **opts)
    try:
        e.step(warmup)
        stream = torch.cuda.current_stream(device)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        e.step(steps)
        b.record(stream)
        torch.cuda.synchronize(device)
        return systems.S * steps / (a.elapsed_time(b) / 1e3)
    finally:
        e.close()


def choose_kepler_counts(systems, opts, scheme: str = "dkd", coords: str = "dhc", device="cuda"):
    """The cheaper compiled count set (wh_config.kepler_counts = 1) if the
    layout can run it and the envelope explorer validates it on this batch's
    own orbits within App. A's bound (envelope.validate_counts), else the
    paper's (0).  Returns (kepler_counts, worst |da/a| of set 1, its largest z)."""
    from .envelope import INTEGRATOR_COUNTS, validate_counts
    runs_it = (coords == "dhc" and scheme in ("dkd", "kdk") and opts.get("packing") != "serial"
               and opts.get("exchange", "auto") != "lds")
    if not runs_it:
        return 0, None, None
    ok, worst, z = validate_counts(systems, INTEGRATOR_COUNTS[1], device=device)
    return (1 if ok else 0), worst, z


def autotune(systems, gr_c: float = 0.0, scheme: str = "dkd", steps: int = 1024, warmup: int = 64,
             device="cuda", use_cache: bool = True, candidates=None, verbose: bool = False, coords: str = "dhc",
             counts: bool = False):
    """Return (best_options, table) for this batch; best_options can be passed
    to Ensemble(...) as keyword arguments.  counts=True also picks the Kepler
    count set (choose_kepler_counts) for the winning layout."""
    key = shape_key(systems.n_planets, gr_c > 0, scheme, coords) + ("|counts" if counts else "")
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        return cache[key]["best"], cache[key]["table"]
    cands = candidates or CANDIDATES
    names = list(cands)
    table = []
    for values in itertools.product(*(cands[n] for n in names)):
        opts = dict(zip(names, values))
        if opts.get("packing") in ("pair", "split", "serial") and opts.get("exchange") == "lds":
            continue              # same kernel as the DPP candidate
        if opts.get("packing") == "mixed" and opts.get("exchange") == "lds":
            continue              # shared groups run the DPP rounds only
        if opts.get("packing") == "serial" and opts.get("balance"):
            continue              # the serial layout ignores the launch plan
        # the steps of a probe must cover a few launches of the candidate's chunk
        n = max(steps, 2 * opts.get("chunk_steps", 0)) if "chunk_steps" in opts else steps
        try:
            rate = time_candidate(systems, opts, gr_c, scheme, n, warmup, device, coords)
        except _lib.WHError:      # a combination the library does not run (e.g. pair packing with SABA_n)
            continue
        table.append({"opts": opts, "system_steps_per_s": rate})
        if verbose:
            print("autotune %s: %.4g system-steps/s" % (opts, rate), flush=True)
    best = dict(max(table, key=lambda r: r["system_steps_per_s"])["opts"])
    if counts:
        kc, worst, z = choose_kepler_counts(systems, best, scheme, coords, device)
        best["kepler_counts"] = kc
        if verbose:
            print("autotune: kepler_counts %d (set 1: worst |da/a| %s, largest z %s)" % (kc, worst, z), flush=True)
    if use_cache:
        cache[key] = {"best": best, "table": table}
        _save(cache)
    return best, table
