"""Pins for the oracle's SABA_n splittings (Laskar & Robutel 2001).

SABA_n composes n+1 Kepler drifts and n kicks with Gauss-Legendre
coefficients; for a perturbation of relative size eps its error is
O(eps dt^(2n) + eps^2 dt^2).  Pins: the coefficients' closed forms for
n = 2 and 3 (textbook Gauss-Legendre nodes and weights), symmetry and sums;
the energy error falls 16x per halving of dt for SABA_2 (fourth order) and
about 64x for SABA_3 until the eps^2 dt^2 term takes over; time reversal;
angular momentum.  Both in democratic heliocentric and Jacobi coordinates.
"""
import numpy as np
import pytest

import oracle
from paper_2307_05683_amd import inputs

LD = np.longdouble


def test_coefficients():
    c, d = oracle.saba_coeffs(2)
    assert np.allclose(c.astype(float), [0.5 - np.sqrt(3) / 6, np.sqrt(3) / 3, 0.5 - np.sqrt(3) / 6], rtol=0, atol=1e-16)
    assert np.allclose(d.astype(float), [0.5, 0.5], rtol=0, atol=1e-16)
    c, d = oracle.saba_coeffs(3)
    r = np.sqrt(15) / 10
    assert np.allclose(c.astype(float), [0.5 - r, r, r, 0.5 - r], rtol=0, atol=1e-16)
    assert np.allclose(d.astype(float), [5 / 18, 4 / 9, 5 / 18], rtol=0, atol=1e-16)
    for n in (1, 2, 3, 4):
        c, d = oracle.saba_coeffs(n)
        assert abs(float(c.sum() - 1)) < 1e-18 and abs(float(d.sum() - 1)) < 1e-18
        assert np.allclose(c.astype(float), c[::-1].astype(float), atol=1e-18)
        assert np.allclose(d.astype(float), d[::-1].astype(float), atol=1e-18)
        # Gauss quadrature of degree 2n-1 is exact: sum d_k t_k^j = 1/(j+1)
        t = np.cumsum(c[:-1])
        for j in range(2 * n):
            assert abs(float((d * t ** j).sum() - LD(1) / (j + 1))) < 1e-17


def heavy(n, seed, mass):
    s = inputs.make_systems(1, seed, n_planets=n)
    s.m[0, :n] = mass * np.linspace(1.0, 0.5, n)
    return s


def energy_error(s, dt, n_steps, scheme, jacobi):
    E0 = oracle.energy(s)[0]
    Q, V = s.Q.astype(LD), s.V.astype(LD)
    f = oracle.jacobi_integrate if jacobi else oracle.integrate
    per = max(1, n_steps // 50)
    worst = 0.0
    for _ in range(n_steps // per):
        Q, V = f(s, per, scheme=scheme, Q=Q, V=V, dt=np.array([dt]))
        worst = max(worst, abs(float((oracle.energy(s, Q, V)[0] - E0) / E0)))
    return worst


@pytest.mark.parametrize("jacobi", [False, True])
def test_saba2_is_fourth_order(jacobi):
    s = heavy(2, 44, 1e-5)
    p_in = 2 * np.pi * np.sqrt(np.linalg.norm(s.Q[0, 0]) ** 3)
    e = [energy_error(s, p_in / k, 10 * k, "saba2", jacobi) for k in (10, 20, 40)]
    assert 13 < e[0] / e[1] < 20 and 13 < e[1] / e[2] < 20, e
    dkd = energy_error(s, p_in / 20, 200, "dkd", jacobi)
    assert e[1] < dkd / 100


def test_saba3_higher_order_then_eps_squared_floor():
    """Jacobi, eps = 1e-5: ~64x per halving (sixth order).  DHC at the same
    eps: the eps^2 dt^2 term of its larger perturbation shows up as a ratio of
    about 4 at the smallest step."""
    s = heavy(2, 44, 1e-5)
    p_in = 2 * np.pi * np.sqrt(np.linalg.norm(s.Q[0, 0]) ** 3)
    ej = [energy_error(s, p_in / k, 10 * k, "saba3", True) for k in (10, 20)]
    assert ej[0] / ej[1] > 40, ej
    ed = [energy_error(s, p_in / k, 10 * k, "saba3", False) for k in (20, 40)]
    assert 3 < ed[0] / ed[1] < 5, ed


@pytest.mark.parametrize("jacobi", [False, True])
@pytest.mark.parametrize("scheme", ["saba2", "saba3", "saba4"])
def test_time_reversible_and_angular_momentum(scheme, jacobi):
    s = heavy(3, 45, 1e-3)
    f = oracle.jacobi_integrate if jacobi else oracle.integrate
    Q, V = f(s, 40, scheme=scheme)
    Qb, Vb = f(s, 40, scheme=scheme, Q=Q, V=-V)
    assert np.abs((Qb - s.Q.astype(LD))[0, :3].astype(float)).max() < 1e-15
    assert np.abs((-Vb - s.V.astype(LD))[0, :3].astype(float)).max() < 1e-15
    L0 = oracle.angmom(s); L1 = oracle.angmom(s, Q, V)
    assert np.abs((L1 - L0).astype(float)).max() < 1e-16 * np.abs(L0.astype(float)).max()
