"""Autotuner of the lane packing (GPU)."""
import numpy as np
import pytest
import torch

from paper_2307_05683_amd import inputs
from paper_2307_05683_amd.autotune import autotune, shape_key
from paper_2307_05683_amd.ensemble import Ensemble

pytestmark = pytest.mark.gpu


def test_autotune_choice_cache_and_results(tmp_path, monkeypatch):
    monkeypatch.setenv("WH_TUNE_CACHE", str(tmp_path / "tune.json"))
    s = inputs.make_systems(300, 41, n_planets=None, n_range=(2, 8), dt_mode="u15_30")
    cands = {"packing": ["pow2", "g8"], "exchange": ["dpp", "lds"], "block_waves": [1], "chunk_steps": [256]}
    best, table = autotune(s, steps=256, warmup=16, candidates=cands)
    assert len(table) == 4 and all(r["system_steps_per_s"] > 0 for r in table)
    assert best == max(table, key=lambda r: r["system_steps_per_s"])["opts"]
    again, _ = autotune(s, steps=256, warmup=16, candidates=cands)      # served from the cache
    assert again == best
    assert (tmp_path / "tune.json").exists()
    assert shape_key(s.n_planets, False, "dkd") in (tmp_path / "tune.json").read_text()
    # tuning never changes the physics beyond rounding
    a = Ensemble.from_systems(s, **best); a.step(200); Qa, _ = a.state(); a.close()
    b = Ensemble.from_systems(s); b.step(200); Qb, _ = b.state(); b.close()
    live = torch.tensor(np.arange(8)[None, :] < s.n_planets[:, None], device=Qa.device)
    d = (Qa - Qb).abs()[live].max().item()
    assert d < 1e-13 * Qb.abs().max().item()


def test_autotune_times_every_packing(tmp_path, monkeypatch):
    """Every lane packing is a candidate (the exchange only varies where a
    layout has two schedules), and each candidate's run agrees with the
    default packing to rounding."""
    monkeypatch.setenv("WH_TUNE_CACHE", str(tmp_path / "tune.json"))
    s = inputs.make_systems(200, 42, n_planets=None, n_range=(1, 8))
    cands = {"packing": ["pow2", "g8", "pair", "split", "serial"], "exchange": ["dpp", "lds"], "block_waves": [1],
             "chunk_steps": [256]}
    best, table = autotune(s, steps=256, warmup=16, candidates=cands, use_cache=False)
    packings = sorted(r["opts"]["packing"] for r in table)
    assert packings == ["g8", "g8", "pair", "pow2", "pow2", "serial", "split"], packings
    b = Ensemble.from_systems(s); b.step(200); Qb, _ = b.state(); b.close()
    live = torch.tensor(np.arange(8)[None, :] < s.n_planets[:, None], device=Qb.device)
    for r in table:
        a = Ensemble.from_systems(s, **r["opts"]); a.step(200); Qa, _ = a.state(); a.close()
        assert (Qa - Qb).abs()[live].max().item() < 1e-13 * Qb.abs().max().item(), r["opts"]
