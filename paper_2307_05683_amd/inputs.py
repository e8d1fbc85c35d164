"""Seeded synthetic planetary systems (input generator only).

This module draws initial conditions; it holds none of the integrator's
arithmetic.  Both the GPU path and the CPU oracle take their inputs from here.

Workload recipe (stand-in for the present-day Solar System used in the
paper's performance and long-term tests, Sec. 4-5, which is not available):

* star mass m0 = 1, G = 1 (units AU, yr/2pi);
* N planets (fixed, or uniform in {n_min..n_max} for uneven batches);
* masses log-uniform in [1e-7, 1e-3], semi-major axes log-uniform in
  [0.4, 30], sorted inward-out, the k-th drawn mass given to the k-th
  innermost planet; the whole (masses, a) draw is rejected and redrawn until
  every adjacent pair is at least 10 mutual Hill radii apart,
  R_H = ((m_k + m_k+1) / (3 m0))^(1/3) (a_k + a_k+1) / 2;
* eccentricity U[0, 0.05], inclination U[0, 0.05] rad, node, argument of
  pericentre and mean anomaly U[0, 2pi);
* heliocentric elements with mu_k = G (m0 + m_k), converted to democratic
  heliocentric coordinates: Q_k = heliocentric position,
  V_k = u_k - sum_j m_j u_j / M_tot (barycentric velocity);
* dt = P_inner / 20 with P_inner = 2 pi sqrt(a_1^3 / (m0 + m_1)), or, for
  uneven batches, dt uniform in [P_inner/30, P_inner/15].

Kepler-envelope test particles (Sec. 3.2, Fig. 1): massless particles about
a unit-mass star (mu = 1) on a grid of semi-major axis and eccentricity, in
the reference plane (i = node = pericentre argument = 0), with mean anomalies
uniform in [0, 2pi) from domain 4 of a per-cell key; the step is 5 days,
dt = 2pi * 5 / 365.25 in these units.

Randomness: a counter-based SplitMix64.  System i of base seed s owns the
stream key = mix((s << 32) | i); draw k of domain d is
mix(mix(key + d * 0x632BE59BD9B4E019) + (k + 1) * 0x9E3779B97F4A7C15) and its
top 53 bits give a uniform double in [0, 1).  Domains: 0 planet count,
1 masses and semi-major axes (16 draws per rejection attempt), 2 angles and
shape, 3 timestep, 4 test-particle phases (keyed by grid cell instead of
system).  A system's values therefore do not depend on how many
systems are drawn with it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

NMAX = 8
_GOLD = np.uint64(0x9E3779B97F4A7C15)
_DOM = np.uint64(0x632BE59BD9B4E019)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea & Flood 2014)."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _keys(base_seed: int, idx: np.ndarray) -> np.ndarray:
    x = (np.uint64(base_seed) << np.uint64(32)) | idx.astype(np.uint64)
    return _mix(x)


def uniform(keys: np.ndarray, domain: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0,1); keys [S], counters broadcastable to [S, k]."""
    with np.errstate(over="ignore"):
        dk = _mix(keys + np.uint64(domain) * _DOM)
        z = dk[:, None] + (np.asarray(counters, dtype=np.uint64) + np.uint64(1)) * _GOLD
    return (_mix(z) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclass
class Systems:
    """A batch of S planetary systems in democratic heliocentric coordinates.

    Arrays (float64 unless noted); planet slots >= n_planets[s] are zero.
      n_planets int32 [S]; m0 [S]; m [S, 8]; Q [S, 8, 3] (heliocentric
      positions); V [S, 8, 3] (barycentric velocities); dt [S].
    """

    n_planets: np.ndarray
    m0: np.ndarray
    m: np.ndarray
    Q: np.ndarray
    V: np.ndarray
    dt: np.ndarray

    @property
    def S(self) -> int:
        return int(self.n_planets.shape[0])

    def copy(self) -> "Systems":
        return Systems(*(a.copy() for a in (self.n_planets, self.m0, self.m, self.Q, self.V, self.dt)))

    def subset(self, idx) -> "Systems":
        idx = np.asarray(idx)
        return Systems(self.n_planets[idx].copy(), self.m0[idx].copy(), self.m[idx].copy(),
                       self.Q[idx].copy(), self.V[idx].copy(), self.dt[idx].copy())


def _solve_kepler_E(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly from mean anomaly (elliptic, e < 1), Newton to convergence."""
    E = M + e * np.sin(M)
    for _ in range(50):
        dE = (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        E = E - dE
        if np.max(np.abs(dE)) < 1e-16:
            break
    return E


def elements_to_cartesian(mu, a, e, inc, Om, om, M):
    """Heliocentric position/velocity from classical elements (elliptic)."""
    E = _solve_kepler_E(np.mod(M, 2 * np.pi), e)
    cE, sE = np.cos(E), np.sin(E)
    sq = np.sqrt(1.0 - e * e)
    n = np.sqrt(mu / a ** 3)
    x = a * (cE - e)
    y = a * sq * sE
    den = 1.0 - e * cE
    vx = -a * n * sE / den
    vy = a * n * sq * cE / den
    cO, sO, co, so, ci, si = np.cos(Om), np.sin(Om), np.cos(om), np.sin(om), np.cos(inc), np.sin(inc)
    # rotation R3(Om) R1(inc) R3(om) applied to the perifocal vector
    r11 = cO * co - sO * so * ci
    r12 = -cO * so - sO * co * ci
    r21 = sO * co + cO * so * ci
    r22 = -sO * so + cO * co * ci
    r31 = so * si
    r32 = co * si
    pos = np.stack([r11 * x + r12 * y, r21 * x + r22 * y, r31 * x + r32 * y], axis=-1)
    vel = np.stack([r11 * vx + r12 * vy, r21 * vx + r22 * vy, r31 * vx + r32 * vy], axis=-1)
    return pos, vel


def _draw_mass_a(keys: np.ndarray, nplan: np.ndarray, m0: float, max_attempts: int):
    """Rejection-sample (masses, a) per system; returns sorted a and masses."""
    S = keys.shape[0]
    masses = np.zeros((S, NMAX))
    axes = np.zeros((S, NMAX))
    done = np.zeros(S, dtype=bool)
    attempt0 = 0
    chunk = 32
    slot = np.arange(NMAX)
    while not done.all():
        if attempt0 >= max_attempts:
            raise RuntimeError("Hill-spacing rejection did not accept within %d attempts" % max_attempts)
        pend = np.nonzero(~done)[0]
        kp = keys[pend]
        ctr = (attempt0 + np.arange(chunk))[:, None] * 16 + np.arange(16)[None, :]
        u = uniform(kp, 1, ctr.reshape(1, -1)).reshape(len(pend), chunk, 16)
        mm = 10.0 ** (-7.0 + 4.0 * u[:, :, :NMAX])
        aa = np.exp(np.log(0.4) + u[:, :, NMAX:] * np.log(30.0 / 0.4))
        npl = nplan[pend][:, None, None]
        live = slot[None, None, :] < npl
        aa_s = np.where(live, aa, np.inf)
        order = np.argsort(aa_s, axis=-1, kind="stable")
        a_sorted = np.take_along_axis(aa_s, order, axis=-1)
        m_in = np.where(live, mm, 0.0)
        # k-th drawn mass goes to the k-th innermost planet: masses stay in draw order
        ok = np.ones(a_sorted.shape[:2], dtype=bool)
        for k in range(NMAX - 1):
            pair = (k + 1) < npl[:, :, 0]
            a1, a2 = a_sorted[:, :, k], a_sorted[:, :, k + 1]
            m1, m2 = m_in[:, :, k], m_in[:, :, k + 1]
            with np.errstate(invalid="ignore"):
                rh = np.cbrt((m1 + m2) / (3.0 * m0)) * 0.5 * (a1 + a2)
                good = (a2 - a1) >= 10.0 * rh
            ok &= np.where(pair, good, True)
        first = np.where(ok.any(axis=1), ok.argmax(axis=1), -1)
        hit = first >= 0
        rows = pend[hit]
        fa = first[hit]
        masses[rows] = m_in[hit, fa]
        axes[rows] = np.where(np.isfinite(a_sorted[hit, fa]), a_sorted[hit, fa], 0.0)
        done[rows] = True
        attempt0 += chunk
    return masses, axes


def make_systems(S: int, base_seed: int, n_planets: int | None = 8, n_range: tuple[int, int] | None = None,
                 dt_mode: str = "p20", start: int = 0, max_attempts: int = 1 << 16) -> Systems:
    """Draw systems start..start+S-1 of stream `base_seed`.

    n_planets fixes N for every system; n_range=(lo, hi) draws N uniformly in
    {lo..hi} instead.  dt_mode "p20" gives dt = P_inner/20, "u15_30" gives dt
    uniform in [P_inner/30, P_inner/15].
    """
    m0 = 1.0
    idx = np.arange(start, start + S, dtype=np.int64)
    keys = _keys(base_seed, idx)
    if n_range is not None:
        lo, hi = n_range
        u = uniform(keys, 0, np.zeros((1, 1)))[:, 0]
        nplan = (lo + np.floor(u * (hi - lo + 1))).astype(np.int32)
        nplan = np.minimum(nplan, hi)
    else:
        nplan = np.full(S, int(n_planets), dtype=np.int32)
    if nplan.min() < 1 or nplan.max() > NMAX:
        raise ValueError("planet count must be in 1..8")
    masses, axes = _draw_mass_a(keys, nplan, m0, max_attempts)
    u = uniform(keys, 2, np.arange(5 * NMAX)[None, :]).reshape(S, 5, NMAX)
    ecc = 0.05 * u[:, 0]
    inc = 0.05 * u[:, 1]
    Om = 2 * np.pi * u[:, 2]
    om = 2 * np.pi * u[:, 3]
    Mm = 2 * np.pi * u[:, 4]
    live = np.arange(NMAX)[None, :] < nplan[:, None]
    a_safe = np.where(live, axes, 1.0)
    mu = m0 + masses
    pos, vel = elements_to_cartesian(mu, a_safe, ecc, inc, Om, om, Mm)
    pos = np.where(live[:, :, None], pos, 0.0)
    vel = np.where(live[:, :, None], vel, 0.0)
    mtot = m0 + masses.sum(axis=1)
    vcm = (masses[:, :, None] * vel).sum(axis=1) / mtot[:, None]
    V = np.where(live[:, :, None], vel - vcm[:, None, :], 0.0)
    p_in = 2 * np.pi * np.sqrt(axes[:, 0] ** 3 / (m0 + masses[:, 0]))
    if dt_mode == "p20":
        dt = p_in / 20.0
    elif dt_mode == "u15_30":
        ud = uniform(keys, 3, np.zeros((1, 1)))[:, 0]
        dt = p_in * (1.0 / 30.0 + ud * (1.0 / 15.0 - 1.0 / 30.0))
    else:
        raise ValueError(dt_mode)
    return Systems(nplan, np.full(S, m0), masses, np.ascontiguousarray(pos), np.ascontiguousarray(V), dt)


# Named workloads (planet count, timestep rule, GR speed of light).
WORKLOADS = {
    "single8": dict(S=1, base_seed=0, n_planets=8, dt_mode="p20"),
    "uniform8": dict(S=4096, base_seed=1, n_planets=8, dt_mode="p20"),
    "uneven2to8": dict(S=16384, base_seed=2, n_planets=None, n_range=(2, 8), dt_mode="u15_30"),
    "adjoint8": dict(S=1024, base_seed=3, n_planets=8, dt_mode="p20"),
    "large8gr": dict(S=65536, base_seed=4, n_planets=8, dt_mode="p20"),
}
GR_C = 10065.0   # speed of light in AU / (yr/2pi)


def workload(name: str, S: int | None = None) -> Systems:
    kw = dict(WORKLOADS[name])
    if S is not None:
        kw["S"] = S
    return make_systems(**kw)


DT_5_DAYS = 2.0 * np.pi * 5.0 / 365.25


def make_test_particles(a_values, e_values, n_phase: int, base_seed: int = 7):
    """Test particles on the (a, e) grid, n_phase random phases per cell.

    Returns (Q, V, a, e) with Q, V [n_a, n_e, n_phase, 3] and the per-particle
    a, e [n_a, n_e, n_phase] (heliocentric, mu = 1)."""
    a_values = np.asarray(a_values, dtype=np.float64)
    e_values = np.asarray(e_values, dtype=np.float64)
    na, ne = len(a_values), len(e_values)
    cells = np.arange(na * ne, dtype=np.int64)
    M = 2.0 * np.pi * uniform(_keys(base_seed, cells), 4, np.arange(n_phase)[None, :])
    A = np.broadcast_to(a_values[:, None, None], (na, ne, n_phase)).reshape(-1)
    E = np.broadcast_to(e_values[None, :, None], (na, ne, n_phase)).reshape(-1)
    z = np.zeros_like(A)
    Q, V = elements_to_cartesian(1.0, A, E, z, z, z, M.reshape(-1))
    shp = (na, ne, n_phase)
    return Q.reshape(shp + (3,)), V.reshape(shp + (3,)), A.reshape(shp), E.reshape(shp)
