"""Balanced launch windows (wh_config.balance).

A window boundary only stores the state and reloads it, so a run cut into
windows must equal the one-launch-per-chunk run bit for bit, whatever the
packing, scheme or GR, and for step counts that are and are not multiples of
the chunk.  The batches here have more wavefronts than one launch gives the
GPU's SIMDs, so a plan with several windows is actually built (checked).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_05683_amd import inputs
from paper_2307_05683_amd.ensemble import Ensemble

pytestmark = pytest.mark.gpu


def run(s, n_steps, chunk=1024, **kw):
    e = Ensemble.from_systems(s, chunk_steps=chunk, **kw)
    windows = e.launch_windows
    e.step(n_steps)
    Q, V = e.state()
    flags = e.flags().cpu().numpy()
    E = e.energy().cpu().numpy()
    out = Q.cpu().numpy(), V.cpu().numpy(), flags, E
    e.close()
    return out, windows


CASES = [("auto", "dkd", 0.0, 1), ("auto", "kdk", 10065.0, 4), ("pair", "dkd", 0.0, 1), ("pair", "dkd", 10065.0, 4),
         ("auto", "saba2", 0.0, 1), ("pair", "kdk", 0.0, 1), ("split", "dkd", 0.0, 4)]


@pytest.mark.parametrize("packing,scheme,gr_c,bw", CASES)
def test_windows_are_bitwise_one_launch_per_chunk(packing, scheme, gr_c, bw):
    # the uneven batch (16384 systems of 2..8 planets: 1536 one-planet-per-lane
    # wavefronts) or, for the pair and split layouts, 40960 / 10000 eight-planet
    # systems (2560 pair / 2500 split wavefronts): more than a whole number of
    # wavefronts per SIMD, so the plan has several windows
    if packing in ("pair", "split"):
        base = inputs.workload("uniform8")
        reps = 10 if packing == "pair" else 3
        s = inputs.Systems(np.tile(base.n_planets, reps), np.tile(base.m0, reps), np.tile(base.m, (reps, 1)),
                           np.tile(base.Q, (reps, 1, 1)), np.tile(base.V, (reps, 1, 1)), np.tile(base.dt, reps))
        if packing == "split":
            s = s.subset(np.arange(10000))
    else:
        s = inputs.workload("uneven2to8")
    n = 2 * 1024 + 333
    print("case: %s %s gr_c=%g bw=%d S=%d n=%d" % (packing, scheme, gr_c, bw, s.S, n), flush=True)
    (Qa, Va, fa, Ea), wa = run(s, n, packing=packing, scheme=scheme, gr_c=gr_c, block_waves=bw, balance=1)
    (Qb, Vb, fb, Eb), wb = run(s, n, packing=packing, scheme=scheme, gr_c=gr_c, block_waves=bw, balance=0)
    print("windows per chunk: %d (%d wavefronts each) vs %d" % (wa[0], wa[1], wb[0]), flush=True)
    assert wb == (1, 0)
    assert wa[0] > 1 and wa[1] >= 1024
    assert np.array_equal(Qa, Qb) and np.array_equal(Va, Vb)
    assert np.array_equal(fa, fb) and np.array_equal(Ea, Eb)


def test_windows_match_the_oracle_on_sampled_systems():
    """The uneven batch in balanced windows, 1000 steps (not a multiple of the
    4096-step chunk: the tail runs as one launch), sampled systems against
    the oracle to 1e-12."""
    s = inputs.workload("uneven2to8")
    e = Ensemble.from_systems(s, balance=1, block_waves=4)
    assert e.launch_windows[0] > 1
    e.step(4096 + 1000)
    Q, V = e.state()
    Q = Q.cpu().numpy(); V = V.cpu().numpy()
    e.close()
    idx = np.random.default_rng(5).choice(s.S, 24, replace=False)
    sub = s.subset(idx)
    Qo, Vo = oracle.integrate(sub, 5096)
    lm = np.arange(8)[None, :] < sub.n_planets[:, None]
    Qo = Qo.astype(float)
    err = np.linalg.norm(Q[idx] - Qo, axis=2)[lm] / np.linalg.norm(Qo, axis=2)[lm]
    print("max relative position error %.2e" % err.max(), flush=True)
    assert err.max() < 1e-11


def test_no_plan_when_the_batch_fits():
    s = inputs.workload("uniform8", S=512)
    e = Ensemble.from_systems(s, balance=1)
    assert e.launch_windows == (1, 0)
    e.step(100)
    torch.cuda.synchronize()
    e.close()


def test_short_chunks_fit_the_plan():
    """A chunk of 31 steps (one step per window for the heaviest waves: each
    appears in 31 windows of a chunk) plans within the workspace and equals
    one launch per chunk bit for bit."""
    s = inputs.workload("uneven2to8")
    n = 2 * 31 + 7
    (Qa, Va, fa, Ea), wa = run(s, n, chunk=31, balance=1, block_waves=4)
    (Qb, Vb, fb, Eb), wb = run(s, n, chunk=31, balance=0, block_waves=4)
    print("windows per chunk: %d" % wa[0], flush=True)
    assert wa[0] >= 31 and wb == (1, 0)
    assert np.array_equal(Qa, Qb) and np.array_equal(Va, Vb)
    assert np.array_equal(fa, fb) and np.array_equal(Ea, Eb)
