"""The seeded input generator: determinism, stream independence, recipe."""
import numpy as np

from paper_2307_05683_amd import inputs


def test_splitmix64_known_answer():
    # SplitMix64 seeded with 0: first two outputs of the reference generator
    g = np.uint64(0x9E3779B97F4A7C15)
    out = inputs._mix(np.array([g, g * np.uint64(2)], dtype=np.uint64))
    assert [hex(int(x)) for x in out] == ["0xe220a8397b1dcdaf", "0x6e789e6aa1b965f4"]


def test_deterministic_and_independent_of_batch():
    a = inputs.make_systems(12, 5, n_planets=None, n_range=(2, 8), dt_mode="u15_30")
    b = inputs.make_systems(12, 5, n_planets=None, n_range=(2, 8), dt_mode="u15_30")
    c = inputs.make_systems(3, 5, n_planets=None, n_range=(2, 8), dt_mode="u15_30", start=7)
    for x, y in [(a.Q, b.Q), (a.V, b.V), (a.m, b.m), (a.dt, b.dt)]:
        assert np.array_equal(x, y)
    assert np.array_equal(a.Q[7:10], c.Q) and np.array_equal(a.n_planets[7:10], c.n_planets)
    d = inputs.make_systems(12, 6, n_planets=None, n_range=(2, 8))
    assert not np.array_equal(a.Q, d.Q)


def _helio_elements(s):
    mtot = s.m0 + s.m.sum(1)
    vs = -(s.m[:, :, None] * s.V).sum(1) / s.m0[:, None]      # star velocity
    u = s.V - vs[:, None, :]                                   # heliocentric velocity
    mu = s.m0[:, None] + s.m
    r = np.linalg.norm(s.Q, axis=2)
    v2 = (u * u).sum(2)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = 1 / (2 / r - v2 / mu)
        h = np.cross(s.Q, u)
        evec = np.cross(u, h) / mu[:, :, None] - s.Q / r[:, :, None]
    e = np.linalg.norm(evec, axis=2)
    inc = np.arccos(np.clip(h[:, :, 2] / np.linalg.norm(h, axis=2), -1, 1))
    return a, e, inc, mtot


def test_recipe_ranges_and_spacing():
    s = inputs.make_systems(64, 9, n_planets=8)
    live = np.arange(8)[None, :] < s.n_planets[:, None]
    a, e, inc, _ = _helio_elements(s)
    assert np.all((a[live] > 0.4 * (1 - 1e-12)) & (a[live] < 30 * (1 + 1e-12)))
    assert np.all(e[live] <= 0.05 + 1e-12) and np.all(inc[live] <= 0.05 + 1e-12)
    mm = s.m[live]
    assert np.all((mm >= 1e-7) & (mm <= 1e-3))
    assert np.all(np.diff(a, axis=1) > 0)
    rh = np.cbrt((s.m[:, :-1] + s.m[:, 1:]) / 3.0) * 0.5 * (a[:, :-1] + a[:, 1:])
    assert np.all(np.diff(a, axis=1) >= 10 * rh * (1 - 1e-9))
    p_in = 2 * np.pi * np.sqrt(a[:, 0] ** 3 / (s.m0 + s.m[:, 0]))
    assert np.allclose(s.dt, p_in / 20, rtol=1e-12)
    # democratic heliocentric: V is barycentric, so total momentum of planets + star is zero by construction
    assert np.all(s.Q[~live] == 0) and np.all(s.V[~live] == 0)


def test_uneven_batch_recipe():
    s = inputs.make_systems(2000, 10, n_planets=None, n_range=(2, 8), dt_mode="u15_30")
    counts = np.bincount(s.n_planets, minlength=9)[2:]
    assert counts.min() > 200 and counts.max() < 380
    a, _, _, _ = _helio_elements(s)
    p_in = 2 * np.pi * np.sqrt(a[:, 0] ** 3 / (s.m0 + s.m[:, 0]))
    ratio = p_in / s.dt
    assert ratio.min() >= 15 - 1e-9 and ratio.max() <= 30 + 1e-9
