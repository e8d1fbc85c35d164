"""Pins for the oracle's whole step map (paper Sec. 3.1).

The composition is pinned by properties any correct Wisdom-Holman map in
democratic heliocentric coordinates has, and by brute force:
  * total angular momentum is conserved to rounding (every sub-flow conserves
    it exactly);
  * the energy error stays bounded and scales as dt^2 (Sec. 3.1);
  * the map is time-reversible under a velocity flip (Sec. 3.5 assumptions);
  * the map is symplectic: M^T Omega M = Omega in canonical (Q, P = m V);
  * as dt -> 0 the trajectory converges at second order to a
    Gragg-Bulirsch-Stoer solution of the full Newtonian problem;
  * the tangent map agrees with central differences;
  * the 1/r^2 GR term reproduces the closed-form pericentre precession.
"""
import numpy as np
import pytest

import oracle
from paper_2307_05683_amd import inputs

LD = np.longdouble


def heavy_system(n=3, seed=21, mass=1e-3):
    s = inputs.make_systems(1, seed, n_planets=n)
    s.m[0, :n] = mass * np.linspace(1.0, 0.5, n)
    return s


def sampled_energy_error(s, dt, n_steps, scheme="dkd", gr_c=0.0):
    E0 = oracle.energy(s, gr_c=gr_c)[0]
    Q, V = s.Q.astype(LD), s.V.astype(LD)
    worst = 0.0
    for _ in range(n_steps):
        Q, V = oracle.integrate(s, 1, scheme=scheme, gr_c=gr_c, Q=Q, V=V, dt=np.array([dt]))
        E = oracle.energy(s, Q, V, gr_c=gr_c)[0]
        worst = max(worst, abs(float((E - E0) / E0)))
    return worst


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 0.0), ("dkd", 10065.0), ("kdk", 30.0)])
def test_angular_momentum_conserved(scheme, gr_c):
    s = inputs.make_systems(8, 22, n_planets=None, n_range=(2, 8))
    L0 = oracle.angmom(s)
    Q, V = oracle.integrate(s, 500, scheme=scheme, gr_c=gr_c)
    L1 = oracle.angmom(s, Q, V)
    rel = np.linalg.norm((L1 - L0).astype(float), axis=1) / np.linalg.norm(L0.astype(float), axis=1)
    assert rel.max() < 1e-16


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 0.0), ("dkd", 30.0)])
def test_energy_error_second_order(scheme, gr_c):
    s = heavy_system()
    p_in = 2 * np.pi * np.sqrt(np.linalg.norm(s.Q[0, 0]) ** 3)
    errs = []
    for k in range(3):
        dt = p_in / (20 * 2 ** k)
        errs.append(sampled_energy_error(s, dt, int(3 * p_in / dt), scheme, gr_c))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs
    assert errs[0] < 1e-4


def test_energy_error_bounded_no_drift():
    s = inputs.workload("single8")
    E0 = oracle.energy(s)[0]
    Q, V = s.Q.astype(LD), s.V.astype(LD)
    errs = []
    for _ in range(20):
        Q, V = oracle.integrate(s, 500, Q=Q, V=V)
        errs.append(float((oracle.energy(s, Q, V)[0] - E0) / E0))
    errs = np.abs(errs)
    # bounded: the second half is no worse than a small multiple of the first half
    assert errs[10:].max() < 3 * errs[:10].max()
    assert errs.max() < 1e-5


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 0.0), ("dkd", 30.0), ("kdk", 30.0)])
def test_time_reversible(scheme, gr_c):
    s = inputs.make_systems(4, 23, n_planets=None, n_range=(2, 8))
    Q, V = oracle.integrate(s, 300, scheme=scheme, gr_c=gr_c)
    Qb, Vb = oracle.integrate(s, 300, scheme=scheme, gr_c=gr_c, Q=Q, V=-V)
    lm = (np.arange(8)[None, :] < s.n_planets[:, None])
    dq = np.abs((Qb - s.Q.astype(LD)).astype(float))[lm].max()
    dv = np.abs((-Vb - s.V.astype(LD)).astype(float))[lm].max()
    assert dq < 1e-15 * np.abs(s.Q).max() and dv < 1e-15 * np.abs(s.V).max()


@pytest.mark.parametrize("gr_c", [0.0, 30.0])
def test_kdk_is_dkd_conjugated_by_a_half_step(gr_c):
    """With U = I(h), J(h), K(h) (in the order they act; I includes GR), one
    drift-kick-drift step is U^R U and one kick-drift-kick step U U^R (U^R the
    same operators in reverse order), so n kick-drift-kick steps followed by
    U equal U followed by n drift-kick-drift steps.  With GR the jump and the
    kick do not commute, so a kick-drift-kick step that ordered them
    differently would fail this."""
    s = inputs.make_systems(5, 29, n_planets=None, n_range=(2, 8))
    h = 0.5 * s.dt

    def U(Q, V):
        Q, V = oracle.substep("interaction", s, h, Q=Q, V=V)
        if gr_c > 0:
            Q, V = oracle.substep("gr", s, h, gr_c=gr_c, Q=Q, V=V)
        Q, V = oracle.substep("jump", s, h, Q=Q, V=V)
        return oracle.substep("kepler", s, h, Q=Q, V=V)

    Qa, Va = oracle.integrate(s, 200, scheme="kdk", gr_c=gr_c)
    Qa, Va = U(Qa, Va)
    Qb, Vb = U(s.Q, s.V)
    Qb, Vb = oracle.integrate(s, 200, scheme="dkd", gr_c=gr_c, Q=Qb, V=Vb)
    lm = (np.arange(8)[None, :] < s.n_planets[:, None])
    dq = np.abs((Qa - Qb).astype(float))[lm].max()
    dv = np.abs((Va - Vb).astype(float))[lm].max()
    assert dq < 1e-15 * np.abs(s.Q).max() and dv < 1e-15 * np.abs(s.V).max(), (dq, dv)


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 30.0)])
def test_symplectic(scheme, gr_c):
    """M^T Omega M = Omega for the Jacobian in canonical (Q, P = m V)."""
    n = 2
    base = heavy_system(n=n, seed=24)
    dim = 6 * n
    S = dim
    rep = base.subset(np.zeros(S, dtype=int))
    dQ = np.zeros((S, 8, 3)); dV = np.zeros((S, 8, 3))
    for k in range(S):
        if k < 3 * n:
            dQ[k, k // 3, k % 3] = 1.0
        else:
            j = k - 3 * n
            dV[k, j // 3, j % 3] = 1.0
    _, _, tQ, tV = oracle.tangent(rep, 60, dQ, dV, np.zeros((S, 8)), np.zeros(S), scheme=scheme, gr_c=gr_c)
    M = np.zeros((dim, dim), dtype=LD)
    for k in range(S):
        M[:3 * n, k] = tQ[k, :n].reshape(-1)
        M[3 * n:, k] = tV[k, :n].reshape(-1)
    m = np.repeat(base.m[0, :n], 3).astype(LD)
    D = np.diag(np.concatenate([np.ones(3 * n, dtype=LD), m]))
    Dinv = np.diag(np.concatenate([np.ones(3 * n, dtype=LD), 1 / m]))
    J = (D @ M @ Dinv).astype(float)
    Om = np.block([[np.zeros((3 * n, 3 * n)), np.eye(3 * n)], [-np.eye(3 * n), np.zeros((3 * n, 3 * n))]])
    R = J.T @ Om @ J - Om
    assert np.abs(R).max() < 1e-9 * np.abs(J).max() ** 2
    assert abs(np.linalg.det(J) - 1) < 1e-9


def test_converges_to_brute_force_at_second_order():
    """Sec. 3.1: second order.  Error vs a Gragg-Bulirsch-Stoer solution of
    the full problem drops by ~4 per halving of dt."""
    s = heavy_system(n=3, seed=25)
    p_in = 2 * np.pi * np.sqrt(np.linalg.norm(s.Q[0, 0]) ** 3)
    T = 4 * p_in
    Qg, Vg, err = oracle.gbs(s, T, 400)
    Qg2, Vg2, _ = oracle.gbs(s, T, 800)
    assert np.abs((Qg - Qg2).astype(float)).max() < 1e-12     # reference converged far below the WH error
    errs = []
    for k in range(3):
        nst = 40 * 2 ** k
        dt = T / nst
        Q, V = oracle.integrate(s, nst, dt=np.array([dt]))
        errs.append(np.abs((Q - Qg).astype(float)).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 0.0), ("kdk", 40.0), ("saba2", 0.0), ("saba3", 0.0)])
def test_tangent_matches_central_differences(scheme, gr_c):
    """The dual-number tangent of each scheme's step, along state and mass
    directions, against central differences of the same long-double map."""
    s = heavy_system(n=3, seed=26)
    rng = np.random.default_rng(7)
    dQ = np.zeros((1, 8, 3)); dV = np.zeros((1, 8, 3)); dm = np.zeros((1, 8))
    dQ[0, :3] = rng.normal(size=(3, 3)) * 0.1
    dV[0, :3] = rng.normal(size=(3, 3)) * 0.1
    dm[0, :3] = rng.normal(size=3) * 1e-4
    dm0 = np.array([0.01])
    n_steps = 80
    _, _, tQ, tV = oracle.tangent(s, n_steps, dQ, dV, dm, dm0, scheme=scheme, gr_c=gr_c)
    h = LD(1e-7)

    def run(sign):
        t = s.copy()
        Q = s.Q.astype(LD) + sign * h * dQ.astype(LD)
        V = s.V.astype(LD) + sign * h * dV.astype(LD)
        m = s.m.astype(LD) + sign * h * dm.astype(LD)
        m0 = s.m0.astype(LD) + sign * h * dm0.astype(LD)
        S = t.S
        Qa, Va = Q.copy(), V.copy()
        oracle.lib().or_integrate_ld(S, 8, t.n_planets.astype(np.int32), m0, m, Qa, Va, s.dt.astype(LD),
                                     n_steps, oracle.SCHEMES[scheme], LD(gr_c), 1)
        return Qa, Va

    Qp, Vp = run(1)
    Qm, Vm = run(-1)
    fQ = ((Qp - Qm) / (2 * h)).astype(float)
    fV = ((Vp - Vm) / (2 * h)).astype(float)
    assert np.abs(fQ - tQ.astype(float)).max() < 1e-7 * np.abs(fQ).max()
    assert np.abs(fV - tV.astype(float)).max() < 1e-7 * np.abs(fV).max()


def _pericentre_angles(s, dt, n_steps, gr_c):
    Q, V = s.Q.astype(LD), s.V.astype(LD)
    out = []
    prev = None
    for _ in range(n_steps):
        Qn, Vn = oracle.integrate(s, 1, scheme="dkd", gr_c=gr_c, Q=Q, V=V, dt=np.array([dt]))
        eta0 = float((Q[0, 0] * V[0, 0]).sum())
        eta1 = float((Qn[0, 0] * Vn[0, 0]).sum())
        if eta0 < 0 <= eta1:
            f = -eta0 / (eta1 - eta0)
            th0 = np.arctan2(float(Q[0, 0, 1]), float(Q[0, 0, 0]))
            th1 = np.arctan2(float(Qn[0, 0, 1]), float(Qn[0, 0, 0]))
            d = np.angle(np.exp(1j * (th1 - th0)))
            out.append(th0 + f * d)
        Q, V = Qn, Vn
        prev = eta1
    return np.unwrap(np.array(out)), prev


def test_gr_pericentre_precession_closed_form():
    """The -k/r^2 potential with k = 3 mu^2/c^2 precesses the pericentre by
    2 pi (1/sqrt(1 - 2k/h^2) - 1) per radial period, h^2 = mu a (1 - e^2);
    to first order 6 pi mu / (c^2 a (1-e^2)), the relativistic value."""
    a, e, c = 1.0, 0.3, 20.0
    pos, vel = inputs.elements_to_cartesian(1.0, np.array([a]), np.array([e]), np.zeros(1), np.zeros(1),
                                            np.zeros(1), np.array([np.pi]))
    s = inputs.Systems(np.array([1], np.int32), np.array([1.0]), np.zeros((1, 8)), np.zeros((1, 8, 3)),
                       np.zeros((1, 8, 3)), np.array([0.0]))
    s.m[0, 0] = 1e-14
    s.Q[0, 0] = pos[0]
    s.V[0, 0] = vel[0]
    P = 2 * np.pi * a ** 1.5
    ang, _ = _pericentre_angles(s, P / 2000, 2 * 2000 + 200, c)
    assert len(ang) >= 2
    prec = np.diff(ang)
    k = 3.0 / c ** 2
    h2 = a * (1 - e * e)
    exact = 2 * np.pi * (1 / np.sqrt(1 - 2 * k / h2) - 1)
    first = 6 * np.pi / (c ** 2 * a * (1 - e * e))
    assert np.all(np.abs(prec - exact) < 2e-3 * exact), (prec, exact)
    assert abs(first - exact) > 5e-3 * exact      # the test resolves the difference
    # without GR the orbit does not precess
    ang0, _ = _pericentre_angles(s, P / 2000, 2 * 2000 + 200, 0.0)
    assert np.all(np.abs(np.diff(ang0)) < 1e-4)


def test_operation_count_structure():
    """Third-law pairing (Sec. 3.3): one square root per planet pair plus one
    per planet's Kepler solve; the Kepler part grows linearly with N."""
    c8 = oracle.count_ops(8)
    c4 = oracle.count_ops(4)
    c2 = oracle.count_ops(2)
    assert c8["sqrt"] == 28 + 8 and c4["sqrt"] == 6 + 4 and c2["sqrt"] == 1 + 2
    # second difference in N isolates the quadratic pair term
    c6 = oracle.count_ops(6)
    pair_flops = ((c8["flops"] - c6["flops"]) - (c4["flops"] - c2["flops"])) / 8.0
    assert 15 < pair_flops < 40
    assert oracle.count_ops(8, gr=True)["flops"] > c8["flops"]


def test_osculating_elements_recover_drawn_elements():
    """The oracle's osculating (a, e) invert the generator's element-to-
    Cartesian conversion (an independent construction: Kepler's equation
    and rotations, then V = u - sum_j m_j u_j / M_tot)."""
    rng = np.random.default_rng(3)
    S, n = 6, 5
    m = np.zeros((S, 8)); m[:, :n] = 10 ** rng.uniform(-7, -3, (S, n))
    a = rng.uniform(0.3, 20, (S, n)); e = rng.uniform(0, 0.9, (S, n))
    inc = rng.uniform(0, 1.0, (S, n)); ang = rng.uniform(0, 2 * np.pi, (3, S, n))
    mu = 1.0 + m[:, :n]
    pos, vel = inputs.elements_to_cartesian(mu, a, e, inc, ang[0], ang[1], ang[2])
    Q = np.zeros((S, 8, 3)); U = np.zeros((S, 8, 3))
    Q[:, :n] = pos; U[:, :n] = vel
    Mtot = 1.0 + m.sum(1)
    V = U - ((m[..., None] * U).sum(1) / Mtot[:, None])[:, None, :]
    sysm = inputs.Systems(np.full(S, n, dtype=np.int32), np.ones(S), m, Q, V, np.full(S, 0.01))
    ao, eo = oracle.elements(sysm)
    assert np.allclose(ao[:, :n].astype(float), a, rtol=1e-12, atol=0)
    assert np.allclose(eo[:, :n].astype(float), e, rtol=0, atol=1e-12)
    assert np.all(np.isnan(ao[:, n:].astype(float)))


def test_osculating_elements_closed_forms():
    """Circular orbit: a = r, e = 0; at pericentre with speed
    sqrt(mu (1 + e) / (a (1 - e))): the given a and e."""
    m = np.zeros((1, 8)); m[0, :2] = [1e-9, 1e-9]
    Q = np.zeros((1, 8, 3)); V = np.zeros((1, 8, 3))
    a1, e1 = 2.0, 0.0
    a2, e2 = 3.0, 0.4
    mu1, mu2 = 1 + 1e-9, 1 + 1e-9
    Q[0, 0] = [a1, 0, 0]; V[0, 0] = [0, np.sqrt(mu1 / a1), 0]
    rp = a2 * (1 - e2)
    Q[0, 1] = [0, 0, rp]; V[0, 1] = [np.sqrt(mu2 * (1 + e2) / rp), 0, 0]
    # barycentric velocities of these heliocentric ones (star mass 1)
    U = V.copy()
    V = U - ((m[..., None] * U).sum(1) / (1 + m.sum()))[:, None, :]
    sysm = inputs.Systems(np.array([2], dtype=np.int32), np.ones(1), m, Q, V, np.ones(1))
    ao, eo = oracle.elements(sysm)
    assert abs(float(ao[0, 0]) - a1) < 1e-14 and float(eo[0, 0]) < 1e-14
    assert abs(float(ao[0, 1]) - a2) < 1e-14 and abs(float(eo[0, 1]) - e2) < 1e-14
