"""GPU path vs the CPU oracle on the same seeded inputs (parity tests).

Tolerance: 1e-12 relative, per planet and norm-wise,
  |Q_gpu - Q_oracle| / |Q_oracle| and |V_gpu - V_oracle| / |V_oracle|,
after 1e3 steps.  The oracle runs the plain composition in long double with
converged Kepler solves; the GPU runs the fixed-iteration solver in double
with combined drifts (and combined jumps without GR), so the two agree up to
the accumulated double rounding of the GPU path.
"""
import numpy as np
import pytest
from scipy.stats import ks_2samp
import torch

import oracle
from paper_2307_05683_amd import inputs
from paper_2307_05683_amd.ensemble import Ensemble
from paper_2307_05683_amd import _lib

pytestmark = pytest.mark.gpu
TOL = 1e-12


def live(s):
    return np.arange(8)[None, :] < s.n_planets[:, None]


def rel_err(s, Qg, Vg, Qo, Vo):
    lm = live(s)
    Qo = Qo.astype(np.float64); Vo = Vo.astype(np.float64)
    with np.errstate(invalid="ignore"):     # padding entries are 0/0 and masked below
        eq = np.linalg.norm(Qg - Qo, axis=2) / np.linalg.norm(Qo, axis=2)
        ev = np.linalg.norm(Vg - Vo, axis=2) / np.linalg.norm(Vo, axis=2)
    per_sys = np.where(lm, np.maximum(eq, ev), 0).max(axis=1)
    print("relative error per system: median %.2e  p90 %.2e  max %.2e" % (np.median(per_sys), np.percentile(per_sys, 90),
                                                                          per_sys.max()), flush=True)
    return eq[lm].max(), ev[lm].max()


def gpu_run(s, n_steps, **kw):
    e = Ensemble.from_systems(s, **kw)
    e.step(n_steps)
    Q, V = e.state()
    torch.cuda.synchronize()
    out = Q.cpu().numpy(), V.cpu().numpy()
    e.close()
    return out


def check(s, n_steps, scheme="dkd", gr_c=0.0, tol=TOL, **kw):
    print("case: S=%d n_steps=%d scheme=%s gr_c=%g %s" % (s.S, n_steps, scheme, gr_c, kw), flush=True)
    Qg, Vg = gpu_run(s, n_steps, scheme=scheme, gr_c=gr_c, **kw)
    Qo, Vo = oracle.integrate(s, n_steps, scheme=scheme, gr_c=gr_c)
    eq, ev = rel_err(s, Qg, Vg, Qo, Vo)
    assert eq < tol and ev < tol, (eq, ev)
    return eq, ev


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
def test_single_system_1000_steps(scheme):
    check(inputs.workload("single8"), 1000, scheme)


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
def test_uniform_ensemble_1000_steps(scheme):
    check(inputs.workload("uniform8", S=72), 1000, scheme)


@pytest.mark.parametrize("exchange", ["dpp", "lds"])
@pytest.mark.parametrize("packing", ["pow2", "g8"])
@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
def test_uneven_batch_1000_steps(packing, scheme, exchange):
    s = inputs.make_systems(150, 2, n_planets=None, n_range=(1, 8), dt_mode="u15_30")
    check(s, 1000, scheme, packing=packing, exchange=exchange)


@pytest.mark.parametrize("scheme", ["dkd", "kdk"])
@pytest.mark.parametrize("gr_c", [10065.0, 40.0])
def test_gr_1000_steps(scheme, gr_c):
    s = inputs.make_systems(40, 4, n_planets=None, n_range=(2, 8))
    check(s, 1000, scheme, gr_c=gr_c)


@pytest.mark.parametrize("exchange", ["dpp", "lds"])
@pytest.mark.parametrize("n_steps", [1, 2, 3, 17])
@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 0.0), ("dkd", 40.0), ("kdk", 40.0)])
def test_few_steps(n_steps, scheme, gr_c, exchange):
    s = inputs.make_systems(20, 7, n_planets=None, n_range=(1, 8))
    check(s, n_steps, scheme, gr_c=gr_c, tol=1e-14, exchange=exchange)


def test_zero_steps_returns_input():
    s = inputs.make_systems(9, 8, n_planets=None, n_range=(1, 8))
    Qg, Vg = gpu_run(s, 0)
    lm = live(s)
    assert np.array_equal(Qg[lm], s.Q[lm]) and np.array_equal(Vg[lm], s.V[lm])


def test_keep_unsynchronized_is_bitwise_reproducible():
    """Sec. 3.5: outputs synchronize a copy; the run itself does not depend on
    how many outputs were taken."""
    s = inputs.make_systems(40, 9, n_planets=None, n_range=(2, 8))
    a = Ensemble.from_systems(s, chunk_steps=32)
    a.step(200)
    Qa, Va = a.state()
    b = Ensemble.from_systems(s, chunk_steps=32)
    for _ in range(20):
        b.step(10)
        b.state()
        b.energy()
    Qb, Vb = b.state()
    assert torch.equal(Qa, Qb) and torch.equal(Va, Vb)
    a.close(); b.close()


@pytest.mark.parametrize("packing", ["auto", "pair", "split", "serial"])
def test_graph_replay_matches_direct_launches_bitwise(packing):
    """Replays of the captured chunk graph (with the program's own launches
    and synchronizations between them) equal direct launches bit for bit."""
    s = inputs.make_systems(40, 10, n_planets=None, n_range=(2, 8))
    a = Ensemble.from_systems(s, chunk_steps=16, graph_launches=4, packing=packing)
    b = Ensemble.from_systems(s, chunk_steps=16, graph_launches=-1, packing=packing)
    for e in (a, b):
        e.step(3 * 64 + 21)
        e.energy()
        torch.cuda.synchronize()
        e.step(64)
    Qa, Va = a.state()
    Qb, Vb = b.state()
    assert torch.equal(Qa, Qb) and torch.equal(Va, Vb)
    a.close(); b.close()


@pytest.mark.parametrize("packing", ["auto", "pair", "split", "serial"])
def test_chunk_length_does_not_change_results(packing):
    """The state goes to memory and back between launches without loss, so
    the steps per launch do not change a single bit."""
    s = inputs.make_systems(40, 12, n_planets=None, n_range=(1, 8))
    out = []
    for chunk in (1, 7, 4096):
        e = Ensemble.from_systems(s, chunk_steps=chunk, packing=packing)
        e.step(150)
        out.append(e.state())
        e.close()
    for Q, V in out[1:]:
        assert torch.equal(Q, out[0][0]) and torch.equal(V, out[0][1])


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 40.0)])
def test_plain_per_size_path_matches_fused_bitwise(scheme, gr_c):
    s = inputs.make_systems(70, 11, n_planets=None, n_range=(1, 8), dt_mode="u15_30")
    a = Ensemble.from_systems(s, packing="g8", scheme=scheme, gr_c=gr_c, chunk_steps=50)
    b = Ensemble.from_systems(s, packing="g8", scheme=scheme, gr_c=gr_c)
    a.step(120)
    b.step_plain(120)
    Qa, Va = a.state()
    Qb, Vb = b.state()
    assert torch.equal(Qa, Qb) and torch.equal(Va, Vb)
    a.close(); b.close()


def test_exchanges_agree():
    """The DPP and LDS-crossbar schedules pair the planets in a different order
    and so differ only by rounding."""
    s = inputs.make_systems(60, 17, n_planets=None, n_range=(1, 8))
    Qa, Va = gpu_run(s, 300, exchange="dpp")
    Qb, Vb = gpu_run(s, 300, exchange="lds")
    lm = live(s)
    assert np.abs(Qa - Qb)[lm].max() < 1e-13 * np.abs(Qb)[lm].max()
    one = s.n_planets == 1          # no partner: identical arithmetic
    assert np.array_equal(Qa[one], Qb[one])


def test_packings_agree_and_eight_planet_systems_bitwise():
    s = inputs.make_systems(60, 12, n_planets=None, n_range=(1, 8))
    Qa, Va = gpu_run(s, 300, packing="pow2")
    Qb, Vb = gpu_run(s, 300, packing="g8")
    lm = live(s)
    assert np.abs(Qa - Qb)[lm].max() < 1e-13 * np.abs(Qb)[lm].max()
    eight = s.n_planets == 8
    assert np.array_equal(Qa[eight], Qb[eight]) and np.array_equal(Va[eight], Vb[eight])


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 0.0), ("dkd", 10065.0)])
def test_energy_matches_oracle(scheme, gr_c):
    s = inputs.make_systems(33, 13, n_planets=None, n_range=(1, 8))
    e = Ensemble.from_systems(s, scheme=scheme, gr_c=gr_c)
    E0 = e.energy().cpu().numpy()
    Eo0 = oracle.energy(s, gr_c=gr_c).astype(float)
    assert np.abs((E0 - Eo0) / Eo0).max() < 1e-14
    e.step(500)
    Q, V = e.state()
    E1 = e.energy().cpu().numpy()
    Eo1 = oracle.energy(s, Q.cpu().numpy(), V.cpu().numpy(), gr_c=gr_c).astype(float)
    assert np.abs((E1 - Eo1) / Eo1).max() < 1e-14
    e.close()


@pytest.mark.parametrize("packing", ["auto", "pair", "split", "serial"])
def test_flags_isolated_and_healthy_systems_unaffected(packing):
    s = inputs.make_systems(24, 14, n_planets=None, n_range=(2, 8))
    bad = s.copy()
    # system 3: one planet on an unbound orbit; system 7: a NaN velocity;
    # system 11: two planets starting at the same place (the first half drift
    # separates them; whatever follows stays inside that system)
    bad.V[3, 0] *= 3.0
    bad.V[7, 1, 0] = np.nan
    bad.Q[11, 1] = bad.Q[11, 0]
    e = Ensemble.from_systems(bad, packing=packing)
    e.step(50)
    f = e.flags().cpu().numpy()
    Qb, Vb = e.state()
    e.close()
    assert f[3] & _lib.WH_F_HYPERBOLIC
    assert f[7] & _lib.WH_F_NONFINITE
    others = [k for k in range(s.S) if k not in (3, 7, 11)]
    assert np.all(f[others] == 0)
    good = s.subset(others)
    g = Ensemble.from_systems(good, packing=packing)
    g.step(50)
    Qg, Vg = g.state()
    g.close()
    assert torch.equal(Qb[others], Qg) and torch.equal(Vb[others], Vg)


def test_zmax_flag_on_large_step():
    s = inputs.make_systems(8, 15, n_planets=3)
    s.dt[2] *= 8.0            # z ~ (2 pi 8 / 20)^2 ~ 6 for the inner planet
    e = Ensemble.from_systems(s)
    e.step(5)
    f = e.flags().cpu().numpy()
    e.close()
    assert f[2] & _lib.WH_F_ZMAX
    assert np.all(f[[0, 1, 3, 4, 5, 6, 7]] == 0)


@pytest.mark.parametrize("field,value", [("dt", 0.0), ("dt", -1.0), ("dt", float("nan")), ("m0", 0.0),
                                         ("m0", float("inf")), ("m", -1e-5), ("m", float("nan"))])
def test_invalid_inputs_rejected(field, value):
    s = inputs.make_systems(4, 16, n_planets=3)
    good = inputs.make_systems(4, 16, n_planets=3)
    getattr(s, field)[1] = value
    with pytest.raises(_lib.WHError) as ei:
        Ensemble.from_systems(s)
    assert ei.value.code == _lib.WH_EINVAL
    # a rejected call leaves nothing behind: the same systems, valid, still integrate
    e = Ensemble.from_systems(good)
    e.step(10)
    Q, V = e.state()
    assert e.steps_done == 10
    e.close()
    Qo, Vo = oracle.integrate(good, 10)
    eq, ev = rel_err(good, Q.cpu().numpy(), V.cpu().numpy(), Qo, Vo)
    assert eq < TOL and ev < TOL, (eq, ev)


def test_uniform_full_size_sampled():
    """The benchmark's workload (4096 eight-planet systems) in the default
    one-planet-per-lane layout (the benchmark's own split layout is covered
    in test_gpu_split): sampled systems checked one by one against the
    oracle."""
    s = inputs.workload("uniform8")
    e = Ensemble.from_systems(s)
    e.step(1000)
    Q, V = e.state()
    Q = Q.cpu().numpy(); V = V.cpu().numpy()
    e.close()
    idx = np.random.default_rng(0).choice(s.S, 48, replace=False)
    sub = s.subset(idx)
    Qo, Vo = oracle.integrate(sub, 1000)
    eq, ev = rel_err(sub, Q[idx], V[idx], Qo, Vo)
    assert eq < TOL and ev < TOL, (eq, ev)


_ORACLE_WORST = {}


def oracle_energy_worst(gr_c):
    """Per-system maximum relative energy error of the oracle over 20 samples
    of 1000 steps on 64 systems of the uniform workload (cached per gr_c)."""
    if gr_c not in _ORACLE_WORST:
        s = inputs.workload("uniform8", S=64)
        Q, V = s.Q.astype(np.longdouble), s.V.astype(np.longdouble)
        Eo0 = oracle.energy(s, gr_c=gr_c).astype(float)
        worst_o = np.zeros(s.S)
        for _ in range(20):
            Q, V = oracle.integrate(s, 1000, gr_c=gr_c, Q=Q, V=V)
            Eo = oracle.energy(s, Q, V, gr_c=gr_c).astype(float)
            worst_o = np.maximum(worst_o, np.abs((Eo - Eo0) / Eo0))
        _ORACLE_WORST[gr_c] = (s, worst_o)
    return _ORACLE_WORST[gr_c]


@pytest.mark.parametrize("packing,gr_c", [("auto", 0.0), ("pair", 0.0), ("split", 0.0), ("serial", 0.0),
                                         ("pair", 10065.0), ("serial", 10065.0)])
def test_energy_error_statistics_match_oracle(packing, gr_c):
    """Over a longer run the per-system maximum relative energy error of the
    GPU path matches the oracle's (ratio within [0.5, 2] for >= 95% of the
    systems, medians within 10%), in every lane layout and with GR."""
    s, worst_o = oracle_energy_worst(gr_c)
    e = Ensemble.from_systems(s, packing=packing, gr_c=gr_c)
    E0 = e.energy().cpu().numpy()
    worst_g = np.zeros(s.S)
    for _ in range(20):
        e.step(1000)
        Eg = e.energy().cpu().numpy()
        worst_g = np.maximum(worst_g, np.abs((Eg - E0) / E0))
    e.close()
    ratio = worst_g / worst_o
    assert np.mean((ratio > 0.5) & (ratio < 2.0)) >= 0.95
    assert abs(np.median(worst_g) / np.median(worst_o) - 1) < 0.1
    # the two distributions of log10 max |dE/E| are not distinguishable
    assert ks_2samp(np.log10(worst_g), np.log10(worst_o)).pvalue > 0.01


@pytest.mark.parametrize("opts", [{}, {"block_waves": 4, "chunk_steps": 1024}])
def test_uneven_full_size_sampled(opts):
    """The uneven batch at full size (16384 systems of 2..8 planets, per-system
    dt), in the default and the autotuned launch configurations; sampled
    systems checked one by one against the oracle."""
    s = inputs.workload("uneven2to8")
    e = Ensemble.from_systems(s, **opts)
    e.step(1000)
    Q, V = e.state()
    Q = Q.cpu().numpy(); V = V.cpu().numpy()
    e.close()
    idx = np.random.default_rng(1).choice(s.S, 32, replace=False)
    sub = s.subset(idx)
    Qo, Vo = oracle.integrate(sub, 1000)
    eq, ev = rel_err(sub, Q[idx], V[idx], Qo, Vo)
    assert eq < TOL and ev < TOL, (eq, ev)


def test_large_gr_full_size_sampled():
    """65536 eight-planet systems with GR (c = 10065) at full size."""
    s = inputs.workload("large8gr")
    e = Ensemble.from_systems(s, gr_c=inputs.GR_C)
    e.step(1000)
    Q, V = e.state()
    Q = Q.cpu().numpy(); V = V.cpu().numpy()
    flags = e.flags().cpu().numpy()
    e.close()
    assert not flags.any()
    idx = np.random.default_rng(2).choice(s.S, 24, replace=False)
    sub = s.subset(idx)
    Qo, Vo = oracle.integrate(sub, 1000, gr_c=inputs.GR_C)
    eq, ev = rel_err(sub, Q[idx], V[idx], Qo, Vo)
    assert eq < TOL and ev < TOL, (eq, ev)


@pytest.mark.parametrize("packing", ["auto", "pair", "split", "serial"])
def test_million_systems_tiled(packing):
    """2^20 eight-planet systems (one planet per lane: 8.4 million lanes,
    131072 wavefronts; pair: 65536; split: 262144; one lane per system: 16384):
    the 4096 distinct systems
    of the uniform workload tiled 256 times.  Systems are independent, so
    every copy must end bitwise equal to the first, and sampled ones match
    the oracle."""
    base = inputs.workload("uniform8")
    reps = 256
    t = inputs.Systems(np.tile(base.n_planets, reps), np.tile(base.m0, reps), np.tile(base.m, (reps, 1)),
                       np.tile(base.Q, (reps, 1, 1)), np.tile(base.V, (reps, 1, 1)), np.tile(base.dt, reps))
    assert t.S == 1 << 20
    e = Ensemble.from_systems(t, packing=packing)
    e.step(300)
    Q, V = e.state()
    e.close()
    Q = Q.view(reps, base.S, 8, 3)
    V = V.view(reps, base.S, 8, 3)
    assert torch.equal(Q, Q[:1].expand_as(Q)) and torch.equal(V, V[:1].expand_as(V))
    idx = np.random.default_rng(4).choice(base.S, 16, replace=False)
    sub = base.subset(idx)
    Qo, Vo = oracle.integrate(sub, 300)
    eq, ev = rel_err(sub, Q[-1].cpu().numpy()[idx], V[-1].cpu().numpy()[idx], Qo, Vo)
    assert eq < TOL and ev < TOL, (eq, ev)


@pytest.mark.parametrize("packing,scheme,gr_c", [("auto", "dkd", 0.0), ("auto", "kdk", 10065.0), ("pair", "dkd", 40.0),
                                                 ("split", "saba3", 0.0), ("serial", "dkd", 10065.0)])
def test_massless_planets(packing, scheme, gr_c):
    """Test particles (m = 0, which the method allows) inside real systems:
    they feel the planets and the star but act on nothing.  Parity with the
    oracle after 1e3 steps, and the energy of a synchronized copy equals the
    oracle's on the same state (a test particle's terms vanish; a system of
    test particles only has E = 0)."""
    s = inputs.make_systems(40, 71, n_planets=None, n_range=(2, 8))
    rng = np.random.default_rng(4)
    lm = live(s)
    zero = lm & (rng.random(lm.shape) < 0.3)
    s.m[zero] = 0.0
    check(s, 1000, scheme=scheme, gr_c=gr_c, packing=packing)
    # the energy is that of the massive bodies alone: a test particle's terms vanish
    e = Ensemble.from_systems(s, scheme=scheme, gr_c=gr_c, packing=packing)
    e.step(100)
    Q, V = e.state()
    E = e.energy().cpu().numpy()
    e.close()
    Eo = oracle.energy(s, Q.cpu().numpy(), V.cpu().numpy(), gr_c=gr_c).astype(float)
    # (a system whose planets are all test particles has E = 0 exactly)
    assert np.all(np.abs(E - Eo) <= 1e-14 * np.abs(Eo))


@pytest.mark.parametrize("packing", ["auto", "pair"])
def test_massless_planets_reverse_mode(packing):
    """The gradient with respect to a test particle's (zero) mass is the
    derivative of the map there, which the oracle's tangent gives."""
    s = inputs.make_systems(16, 72, n_planets=None, n_range=(2, 8))
    rng = np.random.default_rng(5)
    lm = live(s)
    zero = lm & (rng.random(lm.shape) < 0.3)
    s.m[zero] = 0.0
    gQ_T = rng.normal(size=(s.S, 8, 3)) * lm[:, :, None]
    gV_T = rng.normal(size=(s.S, 8, 3)) * lm[:, :, None]
    e = Ensemble.from_systems(s, packing=packing)
    e.forward_ckpt(200, 64)
    gQ0, gV0, gm, gm0 = [x.cpu().numpy() for x in e.adjoint(gQ_T, gV_T)]
    e.close()
    dm = np.where(zero, 1e-6, 0.0)
    z3 = np.zeros((s.S, 8, 3))
    _, _, tQ, tV = oracle.tangent(s, 200, z3, z3, dm, np.zeros(s.S))
    lhs = (gm * dm).sum(1)
    rhs = (gQ_T * tQ.astype(float)).sum((1, 2)) + (gV_T * tV.astype(float)).sum((1, 2))
    scale = np.abs(gQ_T * tQ.astype(float)).sum((1, 2)) + np.abs(gV_T * tV.astype(float)).sum((1, 2))
    has = zero.any(axis=1)
    rel = np.abs(lhs - rhs)[has] / scale[has]
    print("test-particle mass direction: max mismatch %.2e" % rel.max(), flush=True)
    assert rel.max() < 1e-9


@pytest.mark.parametrize("packing,scheme,gr_c", [("auto", "dkd", 0.0), ("pair", "kdk", 10065.0),
                                                 ("split", "dkd", 40.0), ("serial", "saba3", 0.0),
                                                 ("g8", "dkd", 0.0)])
def test_time_reversal(packing, scheme, gr_c):
    """Backward integration is the same map with the velocities flipped
    (Sec. 3.5; the splittings are symmetric): n steps forward, flip V, n steps,
    flip V returns to the initial state to rounding."""
    s = inputs.make_systems(48, 73, n_planets=None, n_range=(1, 8))
    n = 1000
    Q1, V1 = gpu_run(s, n, scheme=scheme, gr_c=gr_c, packing=packing)
    b = s.copy()
    b.Q = Q1.copy()
    b.V = -V1
    Q2, V2 = gpu_run(b, n, scheme=scheme, gr_c=gr_c, packing=packing)
    eq, ev = rel_err(s, Q2, -V2, s.Q.astype(np.longdouble), s.V.astype(np.longdouble))
    assert eq < 1e-12 and ev < 1e-12, (eq, ev)
