"""Kepler-solver envelope explorer on the GPU (Sec. 3.2, Fig. 1; App. A).

The integrator's Kepler drift runs a fixed number of Halley and Newton steps
with truncated Stumpff series and no convergence test, so it is exact only
where the step resolves the pericentre passage.  This module maps where that
holds and searches the iteration counts, with batches of massless test
particles advanced by wh_kepler_envelope:

* kepler_envelope -- relative semi-major-axis change of each particle;
* envelope_map    -- the Fig. 1 map: worst |da/a| per (a, e) cell over random
                     phases, next to the pericentre timescale T_f;
* search_counts   -- the App. A search: every (Halley steps, Newton steps,
                     Halley terms, Newton terms) combination that keeps
                     |da/a| under a bound for all e <= e_max at one a, and
                     the cheapest of them by FP64 operation count.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

from . import _lib
from .ensemble import _stream
from .inputs import DT_5_DAYS, make_test_particles

PAPER_COUNTS = (2, 2, 4, 8)      # Halley steps, Newton steps, Halley terms, Newton terms (Sec. 3.2)
# The integrator's compiled count sets (wh_config.kepler_counts): 0 the
# paper's, 1 the cheapest set the App. A search finds for e <= 0.6.
INTEGRATOR_COUNTS = {0: PAPER_COUNTS, 1: (1, 2, 3, 8)}


def kepler_envelope(Q, V, mu, tau, n_steps: int, counts=PAPER_COUNTS, device="cuda", return_state=False):
    """Advance test particles n_steps drifts; returns da/a (torch, on device).

    Q, V: [n, 3] float64 (numpy or torch); mu, tau: scalars or [n]."""
    dev = torch.device(device)
    Qt = torch.as_tensor(np.asarray(Q, dtype=np.float64) if not torch.is_tensor(Q) else Q,
                         dtype=torch.float64, device=dev).reshape(-1, 3).contiguous()
    Vt = torch.as_tensor(np.asarray(V, dtype=np.float64) if not torch.is_tensor(V) else V,
                         dtype=torch.float64, device=dev).reshape(-1, 3).contiguous()
    n = Qt.shape[0]
    mut = torch.as_tensor(mu, dtype=torch.float64, device=dev).expand(n).contiguous()
    taut = torch.as_tensor(tau, dtype=torch.float64, device=dev).expand(n).contiguous()
    err = torch.empty(n, dtype=torch.float64, device=dev)
    zmax = torch.empty(n, dtype=torch.float64, device=dev)
    Qo = torch.empty_like(Qt) if return_state else None
    Vo = torch.empty_like(Vt) if return_state else None
    nh, nn, kh, kn = (int(c) for c in counts)
    _lib.check(_lib.load().wh_kepler_envelope(
        n, Qt.data_ptr(), Vt.data_ptr(), mut.data_ptr(), taut.data_ptr(), int(n_steps), nh, nn, kh, kn,
        Qo.data_ptr() if return_state else None, Vo.data_ptr() if return_state else None,
        err.data_ptr(), zmax.data_ptr(), _stream(dev)))
    if return_state:
        return err, zmax, Qo, Vo
    return err, zmax


def pericentre_timescale(a, e, mu=1.0):
    """T_f = (2 pi / n) (1 - e)^2 / sqrt(1 - e^2) (Sec. 3.2, pericentre equation)."""
    a = np.asarray(a, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = np.sqrt(mu / a ** 3)
    return 2 * np.pi / n * (1 - e) ** 2 / np.sqrt(1 - e * e)


def envelope_map(a_values, e_values, n_phase=8, dt=DT_5_DAYS, years=10.0, counts=PAPER_COUNTS, seed=7,
                 device="cuda"):
    """Fig. 1: worst relative a-error per (a, e) cell after `years`.

    Returns dict(err [n_a, n_e] signed error of largest magnitude (NaN if any
    phase broke down), steps_per_Tf [n_a, n_e], n_steps)."""
    Q, V, A, E = make_test_particles(a_values, e_values, n_phase, seed)
    n_steps = int(round(years * 2 * np.pi / dt))
    err, zmax = kepler_envelope(Q.reshape(-1, 3), V.reshape(-1, 3), 1.0, dt, n_steps, counts, device)
    err = err.cpu().numpy().reshape(A.shape)
    bad = ~np.isfinite(err).all(axis=-1)
    idx = np.nanargmax(np.where(np.isfinite(err), np.abs(err), -1.0), axis=-1)
    worst = np.take_along_axis(err, idx[..., None], axis=-1)[..., 0]
    worst = np.where(bad, np.nan, worst)
    tf = pericentre_timescale(np.asarray(a_values)[:, None], np.asarray(e_values)[None, :])
    return dict(err=worst, steps_per_Tf=tf / dt, n_steps=n_steps,
                zmax=zmax.cpu().numpy().reshape(A.shape).max(axis=-1))


def solve_cost(counts) -> int:
    """FP64 operations of one fixed Kepler solve with these counts, as the
    integrator's solver spends them: 23 to set up, 2(K-1) + 21 per Halley
    step and 2(K-1) + 15 per Newton step with K series terms, 4 more for the
    first-order update after the last Newton step (or 2(K-1) + 7 for a fresh
    evaluation when there is none), and 20 for the Lagrange coefficients."""
    nh, nn, kh, kn = (int(c) for c in counts)
    c = 23 + nh * (2 * (kh - 1) + 21) + nn * (2 * (kn - 1) + 15) + 20
    c += 4 if nn > 0 else 2 * (kn - 1) + 7
    return c


def all_counts(halley=range(0, 4), newton=range(0, 7), terms_halley=range(2, 7), terms_newton=range(4, 10)):
    """The search space: every combination with at least one iteration
    (810 by default; App. A searched 700)."""
    return [c for c in itertools.product(halley, newton, terms_halley, terms_newton) if c[0] + c[1] >= 1]


def search_counts(a=0.387, e_max=0.7, n_e=15, n_phase=8, dt=DT_5_DAYS, years=10.0, bound=1e-13, candidates=None,
                  seed=7, device="cuda"):
    """App. A: combinations whose worst |da/a| stays below `bound` for every
    e in [0, e_max] at semi-major axis a; returns (passing, best, table),
    passing sorted by cost, best = the cheapest."""
    cands = candidates if candidates is not None else all_counts()
    e_values = np.linspace(0.0, e_max, n_e)
    Q, V, _, _ = make_test_particles([a], e_values, n_phase, seed)
    Q = Q.reshape(-1, 3); V = V.reshape(-1, 3)
    n_steps = int(round(years * 2 * np.pi / dt))
    table = []
    for c in cands:
        err, _ = kepler_envelope(Q, V, 1.0, dt, n_steps, c, device)
        e = err.abs().max().item() if torch.isfinite(err).all() else float("nan")
        table.append(dict(counts=tuple(int(x) for x in c), worst=e, cost=solve_cost(c)))
    passing = sorted((r for r in table if np.isfinite(r["worst"]) and r["worst"] < bound), key=lambda r: r["cost"])
    best = passing[0]["counts"] if passing else None
    return passing, best, table


def validate_counts(systems, counts, n_steps=1000, bound=1e-13, z_max=1.0, device="cuda"):
    """Whether a count set solves every Kepler drift of this batch within
    App. A's accuracy bound: each planet of each system, taken as a test
    particle about its star (its own Q, V, mu = m0 and step dt, the drift the
    integrator applies), runs n_steps fixed-count drifts; the set passes if
    every |da/a| < bound, every state stays finite and the largest Stumpff
    argument stays within z_max (the integrator's WH_F_ZMAX guard).  The
    interaction kicks move the planets between drifts, so this checks the
    solver on the batch's own orbits, not the whole map.  Returns
    (ok, worst |da/a|, largest z)."""
    live = np.arange(8)[None, :] < systems.n_planets[:, None]
    Q = systems.Q[live]
    V = systems.V[live]
    mu = np.repeat(systems.m0, systems.n_planets)
    tau = np.repeat(systems.dt, systems.n_planets)
    err, zmax = kepler_envelope(Q, V, mu, tau, n_steps, counts, device)
    ok_finite = bool(torch.isfinite(err).all().item())
    worst = float(err.abs().max().item()) if ok_finite else float("nan")
    z = float(zmax.max().item())
    return ok_finite and worst < bound and z <= z_max, worst, z
