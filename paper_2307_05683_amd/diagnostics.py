"""Long-run ensemble diagnostics (Sec. 5, long-term integrations).

The paper follows an ensemble of Solar-System integrations and calls a run
unstable once Mercury's osculating eccentricity exceeds 0.65 (other criteria,
e > 0.55, e > 0.6 or a relative energy error above 1e-7, gave similar
statistics), and plots each run's relative energy error over time.  scan()
does the same for any ensemble: it integrates in blocks of steps and, at
every sample point, reads the osculating eccentricities (wh_elements), the
energies (wh_energy) and the status flags of a synchronized copy, so the
integration itself is never perturbed.  The per-sample arrays are small
(S x 8 doubles) and are copied to the host, where the thresholds are applied.
"""
from __future__ import annotations

import numpy as np


def scan(ens, n_samples: int, steps_per_sample: int, e_crit: float = 0.65, planet: int | None = 0,
         dE_crit: float | None = None):
    """Integrate n_samples * steps_per_sample steps, sampling after every block.

    planet: the watched planet slot (0 = innermost), or None for the largest
    eccentricity of any planet of the system.  Returns a dict of numpy arrays:
      steps [n_samples+1]          step count at each sample (first = start)
      e [n_samples+1, S]           watched eccentricity
      dE [n_samples+1, S]          relative energy error (E - E_0) / |E_0|
      first_unstable [S]           first sampled step with e > e_crit (or, if
                                   dE_crit is given, |dE| > dE_crit), -1 if none
      flags [S]                    sticky WH_F_* bits at the end
      unstable_fraction [n_samples+1]  fraction of systems flagged by then
    """
    if n_samples < 0 or steps_per_sample < 0:
        raise ValueError("n_samples and steps_per_sample must be >= 0")
    n_planets = np.asarray(ens.n_planets)
    live = np.arange(8)[None, :] < n_planets[:, None]
    if planet is not None and not (0 <= planet < 8):
        raise ValueError("planet must be a slot in 0..7 or None")

    def sample():
        _, e = ens.elements()
        e = e.cpu().numpy()
        if planet is None:
            w = np.where(live, e, -np.inf).max(axis=1)
        else:
            w = np.where(n_planets > planet, e[:, planet], np.nan)
        return w, ens.energy().cpu().numpy()

    e0, E0 = sample()
    steps = [ens.steps_done]
    es, dEs = [e0], [np.zeros_like(E0)]
    for _ in range(n_samples):
        ens.step(steps_per_sample)
        w, E = sample()
        steps.append(ens.steps_done)
        es.append(w)
        dEs.append((E - E0) / np.abs(E0))
    steps = np.asarray(steps, dtype=np.int64)
    es = np.asarray(es)
    dEs = np.asarray(dEs)
    hit = es > e_crit                       # NaN (no such planet) compares False
    if dE_crit is not None:
        hit |= np.abs(dEs) > dE_crit
    hit |= ~np.isfinite(dEs)                # a broken-down system counts as unstable
    first_idx = np.where(hit.any(axis=0), hit.argmax(axis=0), -1)
    first = np.where(first_idx >= 0, steps[np.maximum(first_idx, 0)], -1)
    frac = np.cumsum(hit, axis=0).astype(bool).mean(axis=1)
    return dict(steps=steps, e=es, dE=dEs, first_unstable=first, flags=ens.flags().cpu().numpy(),
                unstable_fraction=frac)
