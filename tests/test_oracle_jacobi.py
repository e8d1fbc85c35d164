"""Pins for the oracle's Wisdom-Holman map in Jacobi coordinates.

The Jacobi splitting (Wisdom & Holman 1991) is the alternative the paper
names for systems of two or four planets.  Its pins:
  * the coordinate change: an exact round trip, the barycentric kinetic
    energy equals sum m'|v'|^2/2, and H_K + H_I equals the energy of the
    democratic-heliocentric state (an independently written function);
  * one planet: H_I vanishes identically, so the map is the exact two-body
    Kepler flow with mu = G (m0 + m1);
  * the kick equals -tau grad H_I / m', with the gradient of an H_I written
    here in 40-digit mpmath by central differences;
  * the map: angular momentum to rounding, bounded second-order energy error,
    time reversal, symplecticity in canonical Jacobi coordinates, and second-
    order convergence to a Gragg-Bulirsch-Stoer solution of the full problem.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2307_05683_amd import inputs

LD = np.longdouble


def live(s):
    return np.arange(8)[None, :] < s.n_planets[:, None]


def heavy_system(n=2, seed=41, mass=1e-3):
    s = inputs.make_systems(1, seed, n_planets=n)
    s.m[0, :n] = mass * np.linspace(1.0, 0.5, n)
    return s


def test_coordinate_change_identities():
    s = inputs.make_systems(12, 5, n_planets=None, n_range=(1, 8))
    lm = live(s)
    xp, vp = oracle.jacobi_from_dhc(s)
    Q, V = oracle.jacobi_to_dhc(s, xp, vp)
    assert np.abs((Q - s.Q.astype(LD))[lm]).max() < 1e-17
    assert np.abs((V - s.V.astype(LD))[lm]).max() < 1e-18
    T, HK, HI = oracle.jacobi_parts(s)
    m = s.m.astype(LD); Vb = s.V.astype(LD); m0 = s.m0.astype(LD)
    P = (m[..., None] * Vb).sum(1)
    Tdhc = 0.5 * (m[..., None] * Vb ** 2).sum((1, 2)) + (P ** 2).sum(1) / (2 * m0)
    assert np.abs((T - Tdhc) / Tdhc).max() < 1e-17
    E = oracle.energy(s)
    assert np.abs((HK + HI - E) / E).max() < 1e-17


def test_first_jacobi_coordinate_is_heliocentric():
    """x'_1 = Q_1 and v'_1 = heliocentric velocity of the innermost planet;
    the last one is measured from the centre of mass of everything inside."""
    s = inputs.make_systems(4, 6, n_planets=3)
    xp, vp = oracle.jacobi_from_dhc(s)
    m, Q, V, m0 = s.m.astype(LD), s.Q.astype(LD), s.V.astype(LD), s.m0.astype(LD)
    u = V + ((m[..., None] * V).sum(1) / m0[:, None])[:, None, :]
    assert np.abs(xp[:, 0] - Q[:, 0]).max() < 1e-18
    assert np.abs(vp[:, 0] - u[:, 0]).max() < 1e-18
    com = (m[:, 0, None] * Q[:, 0] + m[:, 1, None] * Q[:, 1]) / (m0 + m[:, 0] + m[:, 1])[:, None]
    assert np.abs(xp[:, 2] - (Q[:, 2] - com)).max() < 1e-17


def test_single_planet_is_exact_two_body_flow():
    s = inputs.make_systems(6, 7, n_planets=1)
    s.m[:, 0] = np.array([1e-3, 3e-4, 1e-5, 1e-7, 2e-3, 5e-4])
    n = 37
    Qj, Vj = oracle.jacobi_integrate(s, n)
    m, V, m0 = s.m[:, 0].astype(LD), s.V[:, 0].astype(LD), s.m0.astype(LD)
    u = V + (m / m0)[:, None] * V                     # heliocentric velocity
    Qe, ue = oracle.kepler(s.Q[:, 0], u, m0 + m, n * s.dt.astype(LD))
    Ve = ue - (m / (m0 + m))[:, None] * ue            # back to barycentric
    assert np.abs((Qj[:, 0] - Qe) / np.linalg.norm(Qe.astype(float), axis=1)[:, None]).max() < 1e-16
    assert np.abs((Vj[:, 0] - Ve) / np.linalg.norm(Ve.astype(float), axis=1)[:, None]).max() < 1e-16


def _hint_mp(m0, m, xp):
    """H_I written from its definition in mpmath: heliocentric positions from
    the Jacobi ones, U, plus sum G M_i m'_i / |x'_i|."""
    n = len(m)
    M = [m0]
    for k in range(n):
        M.append(M[-1] + m[k])
    Q = []
    acc = [mp.mpf(0)] * 3
    for k in range(n):
        q = [xp[k][a] + acc[a] / M[k] for a in range(3)]
        Q.append(q)
        acc = [acc[a] + m[k] * q[a] for a in range(3)]
    H = mp.mpf(0)
    for i in range(n):
        H -= m0 * m[i] / mp.sqrt(sum(c * c for c in Q[i]))
        for j in range(i + 1, n):
            H -= m[i] * m[j] / mp.sqrt(sum((Q[i][a] - Q[j][a]) ** 2 for a in range(3)))
        mred = m[i] * M[i] / M[i + 1]
        H += M[i + 1] * mred / mp.sqrt(sum(c * c for c in xp[i]))
    return H


def test_kick_is_gradient_of_hint():
    mp.mp.dps = 40
    s = heavy_system(n=3, seed=42, mass=2e-3)
    n = 3
    tau = 0.05
    xp, vp = oracle.jacobi_from_dhc(s)
    Qk, Vk = oracle.jacobi_kick(s, tau)
    xk, vk = oracle.jacobi_from_dhc(s, Qk, Vk)
    assert np.abs((xk - xp)[0, :n].astype(float)).max() < 1e-17          # positions unchanged
    m0 = mp.mpf(float(s.m0[0])); m = [mp.mpf(float(x)) for x in s.m[0, :n]]
    M = [m0]
    for k in range(n):
        M.append(M[-1] + m[k])
    base = [[mp.mpf(float(xp[0, k, a])) for a in range(3)] for k in range(n)]
    h = mp.mpf("1e-15")
    for i in range(n):
        mred = m[i] * M[i] / M[i + 1]
        for a in range(3):
            up = [row[:] for row in base]; dn = [row[:] for row in base]
            up[i][a] += h; dn[i][a] -= h
            g = (_hint_mp(m0, m, up) - _hint_mp(m0, m, dn)) / (2 * h)
            want = -tau * g / mred
            got = float(vk[0, i, a] - vp[0, i, a])
            assert abs(got - float(want)) < 1e-15 * max(abs(float(want)), 1e-3), (i, a, got, float(want))


def test_angular_momentum_conserved():
    s = inputs.make_systems(6, 43, n_planets=None, n_range=(2, 5))
    L0 = oracle.angmom(s)
    Q, V = oracle.jacobi_integrate(s, 200)
    L1 = oracle.angmom(s, Q, V)
    assert np.abs(((L1 - L0) / np.linalg.norm(L0.astype(float), axis=1)[:, None]).astype(float)).max() < 1e-16


def _energy_error(s, dt, n_steps, scheme="dkd"):
    E0 = oracle.energy(s)[0]
    Q, V = s.Q.astype(LD), s.V.astype(LD)
    worst = 0.0
    for _ in range(n_steps):
        Q, V = oracle.jacobi_integrate(s, 1, scheme=scheme, Q=Q, V=V, dt=np.array([dt]))
        worst = max(worst, abs(float((oracle.energy(s, Q, V)[0] - E0) / E0)))
    return worst


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
def test_energy_error_second_order_and_bounded(scheme):
    s = heavy_system(n=2, seed=44)
    p_in = 2 * np.pi * np.sqrt(np.linalg.norm(s.Q[0, 0]) ** 3)
    e1 = _energy_error(s, p_in / 20, 400, scheme)
    e2 = _energy_error(s, p_in / 40, 800, scheme)
    assert e1 < 1e-5
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
def test_time_reversible(scheme):
    s = heavy_system(n=3, seed=45)
    n = 50
    Q, V = oracle.jacobi_integrate(s, n, scheme=scheme)
    Qb, Vb = oracle.jacobi_integrate(s, n, scheme=scheme, Q=Q, V=-V)
    assert np.abs((Qb - s.Q.astype(LD))[0, :3].astype(float)).max() < 1e-15
    assert np.abs((-Vb - s.V.astype(LD))[0, :3].astype(float)).max() < 1e-15


def test_symplectic_in_canonical_jacobi_coordinates():
    """M^T Omega M = Omega for the Jacobian of the map in (x', p' = m' v'),
    by central differences in long double."""
    s = heavy_system(n=2, seed=46, mass=3e-3)
    n = 2
    dim = 6 * n
    xp0, vp0 = oracle.jacobi_from_dhc(s)
    m = s.m[0, :n].astype(LD)
    M = np.cumsum(np.concatenate([[LD(s.m0[0])], m]))
    mred = m * M[:-1] / M[1:]

    def to_z(xp, vp):
        return np.concatenate([xp[0, :n].reshape(-1), (vp[0, :n] * mred[:, None]).reshape(-1)])

    def run(z):
        xp = np.zeros((1, 8, 3), dtype=LD); vp = np.zeros((1, 8, 3), dtype=LD)
        xp[0, :n] = z[:3 * n].reshape(n, 3)
        vp[0, :n] = (z[3 * n:].reshape(n, 3)) / mred[:, None]
        Q, V = oracle.jacobi_to_dhc(s, xp, vp)
        Q, V = oracle.jacobi_integrate(s, 8, Q=Q, V=V)
        return to_z(*oracle.jacobi_from_dhc(s, Q, V))

    z0 = to_z(xp0, vp0)
    J = np.zeros((dim, dim))
    for k in range(dim):
        h = LD(1e-7) * max(abs(z0[k]), LD(1e-6))
        zp = z0.copy(); zm = z0.copy()
        zp[k] += h; zm[k] -= h
        J[:, k] = ((run(zp) - run(zm)) / (2 * h)).astype(float)
    Om = np.block([[np.zeros((3 * n, 3 * n)), np.eye(3 * n)], [-np.eye(3 * n), np.zeros((3 * n, 3 * n))]])
    # scale rows/columns so every block is O(1) before comparing
    d = np.concatenate([np.ones(3 * n), 1 / mred.astype(float).repeat(3)])
    Js = np.diag(d) @ J @ np.diag(1 / d)
    R = Js.T @ (np.diag(1 / d) @ Om @ np.diag(1 / d)) @ Js - np.diag(1 / d) @ Om @ np.diag(1 / d)
    scale = np.abs(np.diag(1 / d) @ Om @ np.diag(1 / d)).max() * np.abs(Js).max() ** 2
    assert np.abs(R).max() < 1e-8 * scale
    assert abs(np.linalg.det(J) - 1) < 1e-7


def test_converges_to_brute_force_at_second_order():
    s = heavy_system(n=2, seed=47)
    p_in = 2 * np.pi * np.sqrt(np.linalg.norm(s.Q[0, 0]) ** 3)
    T = 4 * p_in
    Qg, Vg, _ = oracle.gbs(s, T, 400)
    errs = []
    for k in range(3):
        nst = 40 * 2 ** k
        Q, V = oracle.jacobi_integrate(s, nst, dt=np.array([T / nst]))
        errs.append(np.abs((Q - Qg)[0, :2].astype(float)).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_closed_form_kick_equals_gradient_kick():
    """The closed-form Jacobi acceleration a_i - A_{i-1} + G M_i x'_i/|x'_i|^3
    (used for the operation count and by the GPU kernel) is the gradient of
    H_I: the two kicks agree to long-double rounding of V."""
    s = inputs.make_systems(16, 48, n_planets=None, n_range=(1, 8))
    s.m[:, :] *= 10.0          # heavier planets: larger interaction terms
    lm = live(s)
    Qa, Va = oracle.jacobi_kick(s, 0.05)
    Qb, Vb = oracle.jacobi_kick(s, 0.05, form="direct")
    dv = np.abs((Va - s.V.astype(LD))[lm]).max()
    assert dv > 1e-7                                          # the kick is not negligible
    assert np.abs((Va - Vb)[lm].astype(float)).max() < 2e-18
    assert np.abs((Qa - Qb)[lm].astype(float)).max() < 2e-18


def test_operation_count_of_the_jacobi_step():
    """One Jacobi step = the drifts (as in the DHC step) plus a kick whose
    extra work over the DHC interaction is linear in N (the coordinate sums
    and the star terms); no jump."""
    d = [oracle.count_ops(n)["flops"] for n in range(1, 9)]
    j = [oracle.count_ops_jacobi(n)["flops"] for n in range(1, 9)]
    extra = [jj - dd for jj, dd in zip(j, d)]
    steps = np.diff(extra)
    assert all(e > 0 for e in extra)
    assert np.all(steps == steps[0])          # exactly linear in N
    assert oracle.count_ops_jacobi(2)["div"] > 0 and oracle.count_ops_jacobi(2)["sqrt"] > 0


def test_gr_term_energy_identity_and_closed_form_kick():
    """With the GR potential of Sec. 3.3 (as read for the DHC map) added to
    H_I: H_K + H_I equals the DHC energy with GR, and the closed-form Jacobi
    acceleration (GR part: gr_i + sum_{k>=i} m_k gr_k / M_{i-1}) equals the
    dual-number gradient."""
    s = inputs.make_systems(12, 49, n_planets=None, n_range=(1, 8))
    c = 40.0
    lm = live(s)
    _, HK, HI = oracle.jacobi_parts(s, gr_c=c)
    E = oracle.energy(s, gr_c=c)
    assert np.abs((HK + HI - E) / E).max() < 1e-17
    Qa, Va = oracle.jacobi_kick(s, 0.05, gr_c=c)
    Qb, Vb = oracle.jacobi_kick(s, 0.05, form="direct", gr_c=c)
    Qc, Vc = oracle.jacobi_kick(s, 0.05)
    assert np.abs((Va - Vc)[lm].astype(float)).max() > 1e-4           # the GR part is not negligible
    assert np.abs((Va - Vb)[lm].astype(float)).max() < 2e-18


def test_gr_pericentre_precession_in_jacobi_coordinates():
    """One light planet: the Jacobi map with GR precesses the pericentre by the
    closed form of the -k/r^2 problem, 2 pi (1/sqrt(1 - 2k/h^2) - 1) per
    radial period (k = 3 mu^2/c^2, h^2 = mu a (1 - e^2))."""
    a, e, c = 1.0, 0.3, 20.0
    pos, vel = inputs.elements_to_cartesian(1.0, np.array([a]), np.array([e]), np.zeros(1), np.zeros(1),
                                            np.zeros(1), np.array([np.pi]))
    s = inputs.Systems(np.array([1], np.int32), np.array([1.0]), np.zeros((1, 8)), np.zeros((1, 8, 3)),
                       np.zeros((1, 8, 3)), np.array([0.0]))
    s.m[0, 0] = 1e-14
    s.Q[0, 0] = pos[0]
    s.V[0, 0] = vel[0]
    P = 2 * np.pi * a ** 1.5
    dt = P / 2000
    Q, V = s.Q.astype(LD), s.V.astype(LD)
    angles = []
    for _ in range(2 * 2000 + 200):
        Qn, Vn = oracle.jacobi_integrate(s, 1, Q=Q, V=V, dt=np.array([dt]), gr_c=c)
        eta0 = float((Q[0, 0] * V[0, 0]).sum()); eta1 = float((Qn[0, 0] * Vn[0, 0]).sum())
        if eta0 < 0 <= eta1:
            f = -eta0 / (eta1 - eta0)
            th0 = np.arctan2(float(Q[0, 0, 1]), float(Q[0, 0, 0]))
            th1 = np.arctan2(float(Qn[0, 0, 1]), float(Qn[0, 0, 0]))
            angles.append(th0 + f * np.angle(np.exp(1j * (th1 - th0))))
        Q, V = Qn, Vn
    prec = np.diff(np.unwrap(np.array(angles)))
    assert len(prec) >= 1
    k = 3.0 / c ** 2
    exact = 2 * np.pi * (1 / np.sqrt(1 - 2 * k / (a * (1 - e * e))) - 1)
    assert np.all(np.abs(prec - exact) < 2e-3 * exact), (prec, exact)


@pytest.mark.parametrize("scheme", ["dkd", "saba2"])
def test_gr_energy_error_bounded_second_order(scheme):
    s = heavy_system(n=2, seed=50)
    c = 100.0
    p_in = 2 * np.pi * np.sqrt(np.linalg.norm(s.Q[0, 0]) ** 3)
    def err(dt, n):
        E0 = oracle.energy(s, gr_c=c)[0]
        Q, V = s.Q.astype(LD), s.V.astype(LD)
        worst = 0.0
        for _ in range(n // 10):
            Q, V = oracle.jacobi_integrate(s, 10, scheme=scheme, Q=Q, V=V, dt=np.array([dt]), gr_c=c)
            worst = max(worst, abs(float((oracle.energy(s, Q, V, gr_c=c)[0] - E0) / E0)))
        return worst
    e1, e2 = err(p_in / 20, 400), err(p_in / 40, 800)
    lo, hi = (3.0, 5.0) if scheme == "dkd" else (3.0, 20.0)
    assert e1 < 1e-5 and lo < e1 / e2 < hi, (e1, e2)


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 0.0), ("dkd", 40.0), ("saba2", 0.0), ("saba3", 40.0)])
def test_tangent_matches_central_differences(scheme, gr_c):
    """The dual-number tangent of the Jacobi-coordinate map (DHC in and out,
    masses included) against central differences of the same long-double map."""
    s = inputs.make_systems(3, 61, n_planets=None, n_range=(2, 5))
    rng = np.random.default_rng(3)
    lm = np.arange(8)[None, :] < s.n_planets[:, None]
    dQ = rng.normal(size=(s.S, 8, 3)) * lm[:, :, None] * 0.1
    dV = rng.normal(size=(s.S, 8, 3)) * lm[:, :, None] * 0.01
    dm = rng.normal(size=(s.S, 8)) * lm * s.m
    dm0 = rng.normal(size=s.S) * 0.01
    n_steps = 60
    _, _, tQ, tV = oracle.tangent(s, n_steps, dQ, dV, dm, dm0, scheme=scheme, gr_c=gr_c, coords="jacobi")
    h = LD(1e-7)

    def run(sign):
        t = s.copy()
        t.m = (s.m.astype(LD) + sign * h * dm.astype(LD)).astype(float)
        Q = s.Q.astype(LD) + sign * h * dQ.astype(LD)
        V = s.V.astype(LD) + sign * h * dV.astype(LD)
        m = s.m.astype(LD) + sign * h * dm.astype(LD)
        m0 = s.m0.astype(LD) + sign * h * dm0.astype(LD)
        Qa, Va = Q.copy(), V.copy()
        oracle.lib().or_jacobi_integrate_ld(s.S, 8, s.n_planets.astype(np.int32), m0, m, Qa, Va, s.dt.astype(LD),
                                            n_steps, oracle.SCHEMES[scheme], LD(gr_c), 1)
        return Qa, Va

    Qp, Vp = run(1)
    Qm, Vm = run(-1)
    fQ = ((Qp - Qm) / (2 * h)).astype(float)
    fV = ((Vp - Vm) / (2 * h)).astype(float)
    assert np.abs(fQ - tQ.astype(float)).max() < 1e-7 * np.abs(fQ).max()
    assert np.abs(fV - tV.astype(float)).max() < 1e-7 * np.abs(fV).max()
