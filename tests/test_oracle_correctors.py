"""Pins of the oracle's symplectic correctors for the Jacobi map (Wisdom,
Holman & Touma 1996), and of the backward Kepler drift they use.

What fixes them independently of the oracle's code:
  * the series F(x) of the map's first-order modified Hamiltonian against
    the closed forms (x/2)/sinh(x/2) (drift-kick-drift) and (x/2)coth(x/2)
    (kick-drift-kick) evaluated by numpy;
  * the stage coefficients against the conditions they must meet,
    sum_i 2 b_i sinh(a_i x) = (1 - F(x))/x to order x^(2n-1);
  * C^-1(C(x)) = x;  C(x) - x = O(eps dt^2) (scaling in dt and in the masses);
  * the corrected map's energy error falls with the corrector's order: its
    dt-scaling exponent rises from 2 to 4 (one stage) and towards 6 (two
    stages), and the opposite direction of the change doubles the error
    instead (which pins the direction);
  * the exact Kepler flow run backwards undoes it (negative time).
"""
import numpy as np
import pytest

import oracle
from paper_2307_05683_amd import inputs


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
def test_first_order_series_matches_the_closed_form(scheme):
    f = oracle.corrector_F_series(scheme, 6).astype(float)
    x = np.array([0.05, 0.2, 0.5])
    series = sum(f[k] * x ** (2 * k) for k in range(7))
    closed = (x / 2) / np.sinh(x / 2) if scheme == "dkd" else (x / 2) / np.tanh(x / 2)
    assert np.allclose(series, closed, rtol=1e-13, atol=0)


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
@pytest.mark.parametrize("stages", [1, 2, 3])
def test_stage_coefficients_meet_their_conditions(scheme, stages):
    a, b = (v.astype(float) for v in oracle.corrector_coeffs(stages, scheme))
    assert np.allclose(a, np.arange(1, stages + 1) / (2.0 * stages))
    x = np.array([0.16, 0.32])       # large enough that (1 - F)/x carries no cancellation noise
    F = (x / 2) / np.sinh(x / 2) if scheme == "dkd" else (x / 2) / np.tanh(x / 2)
    psi = (1 - F) / x
    gen = sum(2 * b[i] * np.sinh(a[i] * x) for i in range(stages))
    # the difference starts at order x^(2 stages + 1): doubling x multiplies
    # it by 2^(2 stages + 1)
    d = np.abs(gen - psi)
    ratio = d[1] / d[0]
    assert 2 ** (2 * stages + 1) * 0.7 < ratio < 2 ** (2 * stages + 1) * 1.3, ratio


def test_backward_drift_undoes_the_forward_drift():
    s = inputs.make_systems(6, 5, n_planets=3)
    Q = s.Q[:, :3].reshape(-1, 3)
    V = s.V[:, :3].reshape(-1, 3)
    mu = np.ones(len(Q))
    for tau in (0.3, 2.0, 30.0):
        Q1, V1 = oracle.kepler(Q, V, mu, np.full(len(Q), tau))[:2]
        Q0, V0 = oracle.kepler(Q1, V1, mu, np.full(len(Q), -tau))[:2]
        assert np.abs(Q0.astype(float) - Q).max() < 1e-15 * np.abs(Q).max()
        assert np.abs(V0.astype(float) - V).max() < 1e-15 * np.abs(V).max()
        # and equals the forward drift of the velocity-reversed state, reversed
        Qr, Vr = oracle.kepler(Q1, -V1.astype(float), mu, np.full(len(Q), tau))[:2]
        assert np.abs(Qr.astype(float) - Q0.astype(float)).max() < 1e-14 * np.abs(Q).max()


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
def test_corrector_is_a_near_identity_change_of_variables(scheme):
    s = inputs.make_systems(4, 5, n_planets=3)
    Qc, Vc = oracle.jacobi_corrector(s, 2, scheme)
    Qb, Vb = oracle.jacobi_corrector(s, 2, scheme, inverse=True, Q=Qc, V=Vc)
    assert np.abs(Qb.astype(float) - s.Q).max() < 1e-16 * 30
    assert np.abs(Vb.astype(float) - s.V).max() < 1e-16 * 30

    def size(sys):
        Q, V = oracle.jacobi_corrector(sys, 1, scheme)
        return np.abs(Q.astype(float) - sys.Q).max()
    d0 = size(s)
    half = s.copy(); half.dt[:] *= 0.5
    light = s.copy(); light.m[:] *= 0.5
    assert 3.5 < d0 / size(half) < 4.5          # O(dt^2)
    assert 1.8 < d0 / size(light) < 2.2         # O(eps)


def max_energy_error(s, scheme, stages, n_steps, blocks=20, sign=None):
    E0 = oracle.energy(s).astype(float)
    if stages:
        Q, V = oracle.jacobi_corrector(s, stages, scheme, inverse=True, sign=sign)
    else:
        Q, V = s.Q.astype(np.longdouble), s.V.astype(np.longdouble)
    w = np.zeros(s.S)
    for _ in range(blocks):
        Q, V = oracle.jacobi_integrate(s, n_steps // blocks, scheme=scheme, Q=Q, V=V)
        Qr, Vr = oracle.jacobi_corrector(s, stages, scheme, Q=Q, V=V, sign=sign) if stages else (Q, V)
        E = oracle.energy(s, Qr, Vr).astype(float)
        w = np.maximum(w, np.abs((E - E0) / E0))
    return np.median(w)


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
def test_corrected_energy_error_falls_with_the_order(scheme):
    s = inputs.make_systems(4, 5, n_planets=2)
    e0 = max_energy_error(s, scheme, 0, 500)
    e1 = max_energy_error(s, scheme, 1, 500)
    e2 = max_energy_error(s, scheme, 2, 500)
    assert e1 < e0 / 5 and e2 < e1 / 3
    # the change applied the other way round adds the error instead
    assert max_energy_error(s, scheme, 1, 500, sign=-1) > 1.5 * e0


def test_corrected_error_scales_with_the_corrector_order():
    """Small masses (the eps^2 dt^2 terms out of the way): halving dt divides
    the energy error by ~4 uncorrected, ~16 with one stage, ~64 with two."""
    base = inputs.make_systems(4, 5, n_planets=2)
    base.m[:] *= 1e-3

    def err(stages, f):
        s = base.copy(); s.dt[:] *= f
        return max_energy_error(s, "dkd", stages, int(400 / f))
    r0 = err(0, 1.0) / err(0, 0.5)
    r1 = err(1, 1.0) / err(1, 0.5)
    r2 = err(2, 1.0) / err(2, 0.5)
    assert 3.5 < r0 < 4.6
    assert 13 < r1 < 20
    assert r2 > 40
