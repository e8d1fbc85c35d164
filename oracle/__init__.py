"""ORACLE -- test infrastructure, not part of the product.

ctypes front end of the plain CPU reference in wh_oracle.cpp (and the
brute-force Gragg-Bulirsch-Stoer pin in gbs.cpp).  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import this package.

Arrays follow the input generator's layout: n_planets int32 [S], m0 [S],
m [S, 8], Q [S, 8, 3], V [S, 8, 3], dt [S].  Long double is the parity
precision; double is the timing precision.  Besides the map itself:
osculating elements (numpy, plain definitions), the Jacobi-coordinate map
(jacobi_*), the SABA_n schemes ("saba2".."saba4"), the fixed-iteration
Kepler solver of App. A (kepler_fixed) and the operation counts.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
LD = np.longdouble
_PLD = np.ctypeslib.ndpointer(dtype=LD, flags="C_CONTIGUOUS")
_PD = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_PI = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_PL = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    """Load the oracle library, building it first if it is not there."""
    global _lib
    if _lib is None:
        path = os.environ.get("WH_ORACLE_LIB", _build.LIB)    # e.g. a sanitizer build of the same sources
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        i, l, ld, d = C.c_int, C.c_long, C.c_longdouble, C.c_double
        sig = {
            "or_max_threads": ([], i),
            "or_set_series_recur": ([i], None),
            "or_set_guess": ([i], None),
            "or_set_gd_form": ([i], None),
            "or_kepler_ld": ([i, _PLD, _PLD, _PLD, _PLD, _PLD], None),
            "or_kepler_fixed_ld": ([i, _PLD, _PLD, _PLD, _PLD, i, i, i, i], None),
            "or_kepler_fixed_d": ([i, _PD, _PD, _PD, _PD, i, i, i, i], None),
            "or_substep_ld": ([i, i, i, _PI, _PLD, _PLD, _PLD, _PLD, _PLD, ld], None),
            "or_integrate_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, _PLD, l, i, ld, i], None),
            "or_integrate_d": ([i, i, _PI, _PD, _PD, _PD, _PD, _PD, l, i, d, i], None),
            "or_energy_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, ld, _PLD], None),
            "or_angmom_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD], None),
            "or_tangent_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, _PLD, l, i, ld, _PLD, _PLD, _PLD, _PLD, i], None),
            "or_jacobi_tangent_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, _PLD, l, i, ld, _PLD, _PLD, _PLD, _PLD, i],
                                     None),
            "or_count_ops": ([i, i, i, i, i, i, _PL], None),
            "or_gbs_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, ld, l], ld),
            "or_jacobi_integrate_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, _PLD, l, i, ld, i], None),
            "or_jacobi_integrate_d": ([i, i, _PI, _PD, _PD, _PD, _PD, _PD, l, i, d, i], None),
            "or_jacobi_from_dhc_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, _PLD, _PLD], None),
            "or_jacobi_to_dhc_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, _PLD, _PLD], None),
            "or_jacobi_parts_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, ld, _PLD], None),
            "or_jacobi_kick_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, ld, ld], None),
            "or_jacobi_kick_direct_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, ld, ld], None),
            "or_count_ops_jacobi": ([i, i, i, i, i, i, _PL], None),
            "or_saba_coeffs": ([i, _PLD, _PLD], None),
            "or_corrector_coeffs": ([i, i, i, _PLD, _PLD], None),
            "or_corrector_F_series": ([i, i, _PLD], None),
            "or_jacobi_corrector_ld": ([i, i, _PI, _PLD, _PLD, _PLD, _PLD, _PLD, i, i, i, i, ld, i], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ld(a):
    return np.ascontiguousarray(a, dtype=LD)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


SCHEMES = {"dkd": 0, "kdk": 1, "saba2": 2, "saba3": 3, "saba4": 4}


def kepler(Q, V, mu, tau, return_X=False):
    """Exact Kepler drift of n particles: Q, V [n, 3]; mu, tau [n]."""
    Q = _ld(Q).copy(); V = _ld(V).copy()
    n = Q.shape[0]
    X = np.zeros(n, dtype=LD)
    lib().or_kepler_ld(n, Q, V, _ld(np.broadcast_to(mu, (n,))), _ld(np.broadcast_to(tau, (n,))), X)
    return (Q, V, X) if return_X else (Q, V)


def kepler_fixed(Q, V, mu, tau, n_halley=2, n_newton=2, terms_halley=4, terms_newton=8, precision="ld", recur=0, guess=0,
                 gd_form="direct"):
    """Fixed-iteration Kepler solve (App. A sweep mode).

    recur selects the series arrangement: `terms` terms are summed for
    c_{2+2r}, c_{3+2r} and r downward recurrences give c2, c3.
    gd_form: "direct" g' = 1 - mu G2 / r, or "wronskian" g' = (1 + f' g) / f.
    """
    n = np.asarray(Q).shape[0]
    lib().or_set_series_recur(int(recur))
    lib().or_set_guess(int(guess))
    lib().or_set_gd_form({"direct": 0, "wronskian": 1}[gd_form])
    if precision == "ld":
        Q = _ld(Q).copy(); V = _ld(V).copy()
        lib().or_kepler_fixed_ld(n, Q, V, _ld(np.broadcast_to(mu, (n,))), _ld(np.broadcast_to(tau, (n,))),
                                 n_halley, n_newton, terms_halley, terms_newton)
    else:
        Q = _d(Q).copy(); V = _d(V).copy()
        lib().or_kepler_fixed_d(n, Q, V, _d(np.broadcast_to(mu, (n,))), _d(np.broadcast_to(tau, (n,))),
                                n_halley, n_newton, terms_halley, terms_newton)
    return Q, V


def _unpack(sysm):
    S = sysm.S
    return S, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), _ld(sysm.Q).copy(), _ld(sysm.V).copy()


SUBSTEPS = {"kepler": 0, "jump": 1, "interaction": 2, "gr": 3}


def substep(which, sysm, tau, gr_c=0.0, Q=None, V=None):
    """Apply one sub-flow to every system; returns (Q, V) in long double."""
    S, np_, m0, m, Q0, V0 = _unpack(sysm)
    if Q is not None:
        Q0 = _ld(Q).copy()
    if V is not None:
        V0 = _ld(V).copy()
    lib().or_substep_ld(SUBSTEPS[which], S, 8, np_, m0, m, Q0, V0, _ld(np.broadcast_to(tau, (S,))), LD(gr_c))
    return Q0, V0


def integrate(sysm, n_steps, scheme="dkd", gr_c=0.0, precision="ld", nthreads=0, Q=None, V=None, dt=None):
    """n_steps plain-composition steps; returns final (Q, V)."""
    S = sysm.S
    dtv = sysm.dt if dt is None else dt
    if precision == "ld":
        Qa = _ld(sysm.Q if Q is None else Q).copy(); Va = _ld(sysm.V if V is None else V).copy()
        lib().or_integrate_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), Qa, Va, _ld(dtv),
                              int(n_steps), SCHEMES[scheme], LD(gr_c), nthreads)
    else:
        Qa = _d(sysm.Q if Q is None else Q).copy(); Va = _d(sysm.V if V is None else V).copy()
        lib().or_integrate_d(S, 8, _i(sysm.n_planets), _d(sysm.m0), _d(sysm.m), Qa, Va, _d(dtv),
                             int(n_steps), SCHEMES[scheme], float(gr_c), nthreads)
    return Qa, Va


def energy(sysm, Q=None, V=None, gr_c=0.0, m=None, m0=None):
    S = sysm.S
    E = np.zeros(S, dtype=LD)
    lib().or_energy_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m0 if m0 is None else m0), _ld(sysm.m if m is None else m),
                       _ld(sysm.Q if Q is None else Q), _ld(sysm.V if V is None else V), LD(gr_c), E)
    return E


def angmom(sysm, Q=None, V=None):
    S = sysm.S
    L = np.zeros((S, 3), dtype=LD)
    lib().or_angmom_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m), _ld(sysm.Q if Q is None else Q),
                       _ld(sysm.V if V is None else V), L)
    return L


def tangent(sysm, n_steps, dQ, dV, dm, dm0, scheme="dkd", gr_c=0.0, nthreads=0, coords="dhc"):
    """Forward tangent map along one direction per system (coords "jacobi":
    the Jacobi-coordinate map, DHC in and out).

    Returns (Q_T, V_T, dQ_T, dV_T) with dX_T = (d x_T / d x_0) . direction.
    """
    S = sysm.S
    Q = _ld(sysm.Q).copy(); V = _ld(sysm.V).copy()
    dQ = _ld(dQ).copy(); dV = _ld(dV).copy()
    f = lib().or_jacobi_tangent_ld if coords == "jacobi" else lib().or_tangent_ld
    f(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), Q, V, _ld(sysm.dt), int(n_steps), SCHEMES[scheme],
      LD(gr_c), _ld(dm0), _ld(dm), dQ, dV, nthreads)
    return Q, V, dQ, dV


def count_ops(n_planets=8, gr=False, n_halley=2, n_newton=2, terms_halley=4, terms_newton=8):
    """Operation count of one step of the method: dict add/mul/div/sqrt/flops."""
    c = np.zeros(4, dtype=np.int64)
    lib().or_set_series_recur(0)
    lib().or_set_guess(0)
    lib().or_set_gd_form(0)
    lib().or_count_ops(n_planets, int(gr), n_halley, n_newton, terms_halley, terms_newton, c)
    d = dict(add=int(c[0]), mul=int(c[1]), div=int(c[2]), sqrt=int(c[3]))
    d["flops"] = d["add"] + d["mul"] + d["div"] + d["sqrt"]
    return d


def gbs(sysm, t_total, n_macro, Q=None, V=None):
    """Brute-force N-body solution (Gragg-Bulirsch-Stoer); returns (Q, V, err)."""
    S = sysm.S
    Qa = _ld(sysm.Q if Q is None else Q).copy(); Va = _ld(sysm.V if V is None else V).copy()
    err = lib().or_gbs_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), Qa, Va, LD(t_total), int(n_macro))
    return Qa, Va, err


def max_threads() -> int:
    return int(lib().or_max_threads())


def elements(sysm, Q=None, V=None):
    """Osculating heliocentric semi-major axis and eccentricity, [S, 8] each.

    Two-body problem of the star and planet i: mu = G (m0 + m_i), position
    Q_i, velocity u_i = V_i + sum_j m_j V_j / m0 (heliocentric velocity from
    the barycentric one, Sec. 3.1: the star moves with -sum_j m_j V_j / m0);
    a = 1 / (2/r - u^2/mu), e = |u x (Q x u) / mu - Q / r|.  Slots beyond
    n_planets are NaN.
    """
    Q = _ld(sysm.Q if Q is None else Q); V = _ld(sysm.V if V is None else V)
    m = _ld(sysm.m); m0 = _ld(sysm.m0)
    live = np.arange(8)[None, :] < np.asarray(sysm.n_planets)[:, None]
    P = (np.where(live, m, 0)[..., None] * V).sum(axis=1)             # [S, 3]
    u = V + (P / m0[:, None])[:, None, :]
    mu = m0[:, None] + m
    with np.errstate(divide="ignore", invalid="ignore"):      # empty slots have r = 0
        r = np.sqrt((Q * Q).sum(-1))
        a = 1 / (2 / r - (u * u).sum(-1) / mu)
        h = np.cross(Q, u)
        evec = np.cross(u, h) / mu[..., None] - Q / r[..., None]
        e = np.sqrt((evec * evec).sum(-1))
    return np.where(live, a, np.nan), np.where(live, e, np.nan)


# ---- Wisdom-Holman map in Jacobi coordinates (Wisdom & Holman 1991) --------

def jacobi_integrate(sysm, n_steps, scheme="dkd", precision="ld", nthreads=0, Q=None, V=None, dt=None, gr_c=0.0):
    """n_steps of the Jacobi-coordinate map; DHC (Q, V) in and out."""
    S = sysm.S
    dtv = sysm.dt if dt is None else dt
    if precision == "ld":
        Qa = _ld(sysm.Q if Q is None else Q).copy(); Va = _ld(sysm.V if V is None else V).copy()
        lib().or_jacobi_integrate_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), Qa, Va, _ld(dtv),
                                     int(n_steps), SCHEMES[scheme], LD(gr_c), nthreads)
    else:
        Qa = _d(sysm.Q if Q is None else Q).copy(); Va = _d(sysm.V if V is None else V).copy()
        lib().or_jacobi_integrate_d(S, 8, _i(sysm.n_planets), _d(sysm.m0), _d(sysm.m), Qa, Va, _d(dtv),
                                    int(n_steps), SCHEMES[scheme], float(gr_c), nthreads)
    return Qa, Va


def jacobi_from_dhc(sysm, Q=None, V=None):
    S = sysm.S
    xp = np.zeros((S, 8, 3), dtype=LD); vp = np.zeros((S, 8, 3), dtype=LD)
    lib().or_jacobi_from_dhc_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), _ld(sysm.Q if Q is None else Q),
                                _ld(sysm.V if V is None else V), xp, vp)
    return xp, vp


def jacobi_to_dhc(sysm, xp, vp):
    S = sysm.S
    Q = np.zeros((S, 8, 3), dtype=LD); V = np.zeros((S, 8, 3), dtype=LD)
    lib().or_jacobi_to_dhc_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), _ld(xp), _ld(vp), Q, V)
    return Q, V


def jacobi_parts(sysm, Q=None, V=None, gr_c=0.0):
    """Per system (kinetic energy in Jacobi form, H_K, H_I)."""
    S = sysm.S
    out = np.zeros((S, 3), dtype=LD)
    lib().or_jacobi_parts_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), _ld(sysm.Q if Q is None else Q),
                             _ld(sysm.V if V is None else V), LD(gr_c), out)
    return out[:, 0], out[:, 1], out[:, 2]


def jacobi_kick(sysm, tau, Q=None, V=None, form="gradient", gr_c=0.0):
    """One kick of H_I: "gradient" = dual-number gradient of H_I, "direct" =
    the closed-form Jacobi acceleration."""
    S = sysm.S
    Qa = _ld(sysm.Q if Q is None else Q).copy(); Va = _ld(sysm.V if V is None else V).copy()
    f = lib().or_jacobi_kick_ld if form == "gradient" else lib().or_jacobi_kick_direct_ld
    f(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), Qa, Va, LD(tau), LD(gr_c))
    return Qa, Va


def count_ops_jacobi(n_planets=8, gr=False, n_halley=2, n_newton=2, terms_halley=4, terms_newton=8):
    """Operation count of one step of the Jacobi map."""
    c = np.zeros(4, dtype=np.int64)
    lib().or_set_series_recur(0)
    lib().or_set_guess(0)
    lib().or_set_gd_form(0)
    lib().or_count_ops_jacobi(n_planets, int(gr), n_halley, n_newton, terms_halley, terms_newton, c)
    d = dict(add=int(c[0]), mul=int(c[1]), div=int(c[2]), sqrt=int(c[3]))
    d["flops"] = d["add"] + d["mul"] + d["div"] + d["sqrt"]
    return d


def saba_coeffs(n):
    """SABA_n coefficients (c_1..c_{n+1}, d_1..d_n) from Gauss-Legendre quadrature."""
    c = np.zeros(n + 1, dtype=LD); d = np.zeros(n, dtype=LD)
    lib().or_saba_coeffs(int(n), c, d)
    return c, d


CORRECTOR_SIGN = 1     # the direction of the change of variables (pinned by the corrected energy error)


def corrector_coeffs(stages, scheme="dkd", sign=None):
    """(a, b) of the n-stage symplectic corrector (order 2n + 1) of the Jacobi
    map, scheme "dkd" or "kdk"."""
    a = np.zeros(stages, dtype=LD)
    b = np.zeros(stages, dtype=LD)
    lib().or_corrector_coeffs(int(stages), SCHEMES[scheme], CORRECTOR_SIGN if sign is None else int(sign), a, b)
    return a, b


def corrector_F_series(scheme, kmax):
    f = np.zeros(kmax + 1, dtype=LD)
    lib().or_corrector_F_series(SCHEMES[scheme], int(kmax), f)
    return f


def jacobi_corrector(sysm, stages, scheme="dkd", inverse=False, Q=None, V=None, gr_c=0.0, sign=None, nthreads=0):
    """The corrector C (or C^-1) of the Jacobi map on DHC states: mapping
    coordinates -> real coordinates (inverse: real -> mapping)."""
    S = sysm.S
    Qa = _ld(sysm.Q if Q is None else Q).copy(); Va = _ld(sysm.V if V is None else V).copy()
    lib().or_jacobi_corrector_ld(S, 8, _i(sysm.n_planets), _ld(sysm.m0), _ld(sysm.m), Qa, Va, _ld(sysm.dt),
                                 int(stages), SCHEMES[scheme], CORRECTOR_SIGN if sign is None else int(sign),
                                 int(bool(inverse)), LD(gr_c), nthreads)
    return Qa, Va


def jacobi_integrate_corrected(sysm, n_steps, stages, scheme="dkd", gr_c=0.0, sign=None):
    """The corrected Jacobi map: C^-1 at the start, n_steps of the map, C at
    the output; DHC in and out."""
    Q, V = jacobi_corrector(sysm, stages, scheme, inverse=True, gr_c=gr_c, sign=sign)
    Q, V = jacobi_integrate(sysm, n_steps, scheme=scheme, Q=Q, V=V, gr_c=gr_c)
    return jacobi_corrector(sysm, stages, scheme, inverse=False, Q=Q, V=V, gr_c=gr_c, sign=sign)
