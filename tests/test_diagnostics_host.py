"""Host logic of the long-run diagnostics on a scripted stand-in ensemble."""
import numpy as np
import pytest
import torch

from paper_2307_05683_amd.diagnostics import scan


class Scripted:
    """Replays given per-sample eccentricities and energies."""

    def __init__(self, n_planets, e_seq, E_seq):
        self.n_planets = np.asarray(n_planets, dtype=np.int32)
        self.e_seq, self.E_seq = e_seq, E_seq
        self.k = 0
        self.steps_done = 0

    def step(self, n):
        self.k += 1
        self.steps_done += n

    def elements(self):
        e = torch.as_tensor(self.e_seq[self.k])
        return torch.zeros_like(e), e

    def energy(self):
        return torch.as_tensor(self.E_seq[self.k])

    def flags(self):
        return torch.zeros(len(self.n_planets), dtype=torch.int32)


def test_first_crossing_and_fraction():
    S, n = 3, 4
    e = np.zeros((n + 1, S, 8))
    e[:, :, 0] = 0.1
    e[2:, 1, 0] = 0.7          # system 1 crosses at sample 2
    e[3, 2, 0] = 0.66          # system 2 crosses at sample 3 only (then recovers)
    e[:, 0, 1] = 0.9           # planet 1 of system 0: ignored when watching planet 0
    E = -np.ones((n + 1, S))
    s = scan(Scripted([2, 1, 1], e, E), n, 10)
    assert list(s["steps"]) == [0, 10, 20, 30, 40]
    assert list(s["first_unstable"]) == [-1, 20, 30]
    assert np.allclose(s["unstable_fraction"], [0, 0, 1 / 3, 2 / 3, 2 / 3])
    # watching every planet picks up system 0's second planet from the start
    s = scan(Scripted([2, 1, 1], e, E), n, 10, planet=None)
    assert s["first_unstable"][0] == 0


def test_energy_criterion_and_missing_planet():
    S, n = 2, 3
    e = np.zeros((n + 1, S, 8))
    E = -np.ones((n + 1, S))
    E[2, 0] = -1 + 5e-7        # relative error 5e-7 at sample 2
    E[3, 1] = np.nan           # a broken-down system counts as unstable
    s = scan(Scripted([1, 1], e, E), n, 5, dE_crit=1e-7)
    assert list(s["first_unstable"]) == [10, 15]
    assert np.isclose(s["dE"][2, 0], 5e-7)
    # a watched slot beyond the system's planets never triggers
    s = scan(Scripted([1, 1], np.full((n + 1, S, 8), 0.9), -np.ones((n + 1, S))), n, 5, planet=3)
    assert list(s["first_unstable"]) == [-1, -1]
    with pytest.raises(ValueError):
        scan(Scripted([1], e[:, :1], E[:, :1]), 1, 1, planet=8)
