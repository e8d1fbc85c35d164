"""Host-side parts of the envelope explorer (no GPU)."""
import numpy as np

from paper_2307_05683_amd import envelope as env
from paper_2307_05683_amd.inputs import DT_5_DAYS, make_test_particles


def test_pericentre_timescale_closed_forms():
    # circular orbit: the orbital period 2 pi a^(3/2)
    assert np.isclose(env.pericentre_timescale(2.0, 0.0), 2 * np.pi * 2.0 ** 1.5, rtol=1e-15)
    # (1 - e)^2 / sqrt(1 - e^2) at e = 0.6: 0.16 / 0.8 = 0.2
    assert np.isclose(env.pericentre_timescale(1.0, 0.6), 2 * np.pi * 0.2, rtol=1e-15)


def test_solve_cost_slopes():
    base = env.solve_cost((2, 2, 4, 8))
    assert env.solve_cost((2, 2, 5, 8)) - base == 4      # one more term in each of 2 Halley steps
    assert env.solve_cost((2, 2, 4, 9)) - base == 4
    assert env.solve_cost((3, 2, 4, 8)) - base == 2 * 3 + 21
    assert env.solve_cost((2, 3, 4, 8)) - base == 2 * 7 + 15


def test_search_space():
    c = env.all_counts()
    assert len(c) == 810 and len(set(c)) == 810
    assert env.PAPER_COUNTS in c
    assert all(h + n >= 1 for h, n, _, _ in c)


def test_test_particles_grid():
    Q, V, A, E = make_test_particles([0.4, 1.0], [0.0, 0.3], 5, 9)
    assert Q.shape == (2, 2, 5, 3) and A.shape == (2, 2, 5)
    r = np.linalg.norm(Q, axis=-1)
    # r stays within [a(1-e), a(1+e)]; z = 0 in the reference plane
    assert np.all(r >= A * (1 - E) * (1 - 1e-14)) and np.all(r <= A * (1 + E) * (1 + 1e-14))
    assert np.all(Q[..., 2] == 0) and np.all(V[..., 2] == 0)
    # vis-viva fixes |V| from r and a (mu = 1)
    v2 = (V * V).sum(-1)
    assert np.allclose(v2, 2 / r - 1 / A, rtol=1e-13)
    # phases differ between cells and particles; the same seed repeats them
    Q2, _, _, _ = make_test_particles([0.4, 1.0], [0.0, 0.3], 5, 9)
    assert np.array_equal(Q, Q2)
    assert DT_5_DAYS == 2 * np.pi * 5 / 365.25
