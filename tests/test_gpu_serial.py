"""One-lane-per-system packing (WH_PACK_SERIAL) against the oracle and
against the one-planet-per-lane packing."""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_05683_amd import _lib, inputs
from paper_2307_05683_amd.ensemble import Ensemble, _stream

pytestmark = pytest.mark.gpu
TOL = 1e-12


def live(s):
    return np.arange(8)[None, :] < s.n_planets[:, None]


def run(s, n_steps, **kw):
    e = Ensemble.from_systems(s, **kw)
    e.step(n_steps)
    Q, V = e.state()
    out = Q.cpu().numpy(), V.cpu().numpy(), e.energy().cpu().numpy(), e.flags().cpu().numpy()
    e.close()
    return out


def rel(s, Qg, Vg, Qo, Vo):
    lm = live(s)
    Qo = Qo.astype(float); Vo = Vo.astype(float)
    with np.errstate(invalid="ignore"):
        eq = np.linalg.norm(Qg - Qo, axis=2) / np.linalg.norm(Qo, axis=2)
        ev = np.linalg.norm(Vg - Vo, axis=2) / np.linalg.norm(Vo, axis=2)
    err = np.where(lm, np.maximum(eq, ev), 0).max(axis=1)
    print("relative error per system: median %.2e  max %.2e" % (np.median(err), err.max()), flush=True)
    return err.max()


@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 0.0), ("dkd", 10065.0), ("kdk", 40.0),
                                         ("saba3", 0.0)])
def test_uneven_batch_1000_steps(scheme, gr_c):
    # 71 systems of 1..8 planets: every wavefront mixes planet counts (it
    # runs the body of its largest count) and the last holds empty groups
    s = inputs.make_systems(71, 301, n_planets=None, n_range=(1, 8), dt_mode="u15_30")
    print("case: scheme=%s gr_c=%g" % (scheme, gr_c), flush=True)
    Qg, Vg, _, flags = run(s, 1000, packing="serial", scheme=scheme, gr_c=gr_c)
    Qo, Vo = oracle.integrate(s, 1000, scheme=scheme, gr_c=gr_c)
    assert rel(s, Qg, Vg, Qo, Vo) < TOL
    assert not flags.any()


@pytest.mark.parametrize("n_planets", [1, 2, 3, 5, 8])
def test_each_planet_count(n_planets):
    # a wavefront of one planet count runs that count's body alone
    s = inputs.make_systems(9, 302 + n_planets, n_planets=n_planets)
    Qg, Vg, _, flags = run(s, 1000, packing="serial")
    Qo, Vo = oracle.integrate(s, 1000)
    assert rel(s, Qg, Vg, Qo, Vo) < TOL
    assert not flags.any()


@pytest.mark.parametrize("n_steps", [0, 1, 2, 17])
def test_few_steps(n_steps):
    s = inputs.make_systems(30, 311, n_planets=None, n_range=(1, 8))
    for scheme in ("dkd", "kdk", "saba2"):
        Qg, Vg, _, _ = run(s, n_steps, packing="serial", scheme=scheme)
        Qo, Vo = oracle.integrate(s, n_steps, scheme=scheme)
        assert rel(s, Qg, Vg, Qo, Vo) < 1e-14


def test_agrees_with_one_planet_per_lane():
    s = inputs.make_systems(64, 312, n_planets=None, n_range=(1, 8))
    Qa, Va, Ea, _ = run(s, 300, packing="serial")
    Qb, Vb, Eb, _ = run(s, 300, packing="pow2")
    lm = live(s)
    assert np.abs(Qa - Qb)[lm].max() < 1e-13 * np.abs(Qb)[lm].max()
    assert np.abs((Ea - Eb) / Eb).max() < 1e-14


def test_energy_and_elements_match_oracle_on_same_state():
    s = inputs.make_systems(33, 313, n_planets=None, n_range=(1, 8))
    for gr_c in (0.0, 10065.0):
        e = Ensemble.from_systems(s, packing="serial", gr_c=gr_c)
        e.step(200)
        Q, V = e.state()
        E = e.energy().cpu().numpy()
        a, ecc = e.elements()
        L = e.angular_momentum().cpu().numpy()
        e.close()
        Qn, Vn = Q.cpu().numpy(), V.cpu().numpy()
        Eo = oracle.energy(s, Qn, Vn, gr_c=gr_c).astype(float)
        assert np.abs((E - Eo) / Eo).max() < 1e-14
        ao, eo = oracle.elements(s, Qn, Vn)
        lm = live(s)
        assert np.abs(ecc.cpu().numpy()[lm] - eo[lm].astype(float)).max() < 1e-13
        assert np.abs(a.cpu().numpy()[lm] / ao[lm].astype(float) - 1).max() < 1e-13
        Lo = np.einsum("sp,spk->sk", s.m * lm, np.cross(Qn, Vn))
        assert np.abs(L - Lo).max() < 1e-14 * np.abs(Lo).max()


def test_outputs_leave_padding_entries_untouched():
    s = inputs.make_systems(6, 314, n_planets=None, n_range=(1, 7))
    e = Ensemble.from_systems(s, packing="serial")
    e.step(10)
    dev = e.device
    Q = torch.full((s.S, 8, 3), 7.0, dtype=torch.float64, device=dev)
    V = torch.full((s.S, 8, 3), 7.0, dtype=torch.float64, device=dev)
    _lib.check(_lib.load().wh_get_state(e._ctx, Q.data_ptr(), V.data_ptr(), _stream(dev)))
    torch.cuda.synchronize(dev)
    e.close()
    pad = ~live(s)
    assert (Q.cpu().numpy()[pad] == 7.0).all() and (V.cpu().numpy()[pad] == 7.0).all()


def test_keep_unsynchronized_is_bitwise_reproducible():
    s = inputs.make_systems(40, 315, n_planets=None, n_range=(2, 8))
    a = Ensemble.from_systems(s, packing="serial", chunk_steps=32)
    a.step(200)
    Qa, Va = a.state()
    b = Ensemble.from_systems(s, packing="serial", chunk_steps=32)
    for _ in range(20):
        b.step(10)
        b.state()
        b.energy()
    Qb, Vb = b.state()
    assert torch.equal(Qa, Qb) and torch.equal(Va, Vb)
    a.close(); b.close()


def test_launch_shape_and_graph_leave_results_bitwise_unchanged():
    # every thread integrates its own system: workgroup size, launch length
    # and graph replay cannot change a bit
    s = inputs.make_systems(200, 316, n_planets=None, n_range=(1, 8))
    ref = None
    for bw, chunk, graphs in ((1, 4096, 8), (2, 100, -1), (4, 37, 3)):
        e = Ensemble.from_systems(s, packing="serial", block_waves=bw, chunk_steps=chunk, graph_launches=graphs)
        e.step(1500)
        Q, V = e.state()
        e.close()
        if ref is None:
            ref = (Q, V)
        else:
            assert torch.equal(Q, ref[0]) and torch.equal(V, ref[1])


def test_unsupported_combinations_rejected():
    s = inputs.make_systems(4, 317, n_planets=3)
    for kw in (dict(coords="jacobi"), dict(scheme="saba2", gr_c=10065.0)):
        with pytest.raises(_lib.WHError):
            Ensemble.from_systems(s, packing="serial", **kw)
    e = Ensemble.from_systems(s, packing="serial")
    with pytest.raises(_lib.WHError):        # the per-size path is the G8 packing's
        e.step_plain(1)
    e.close()


def test_flags_isolated():
    s = inputs.make_systems(24, 318, n_planets=None, n_range=(2, 8))
    bad = s.copy()
    bad.V[3, 0] *= 3.0          # unbound innermost planet of system 3
    _, _, _, flags = run(bad, 50, packing="serial")
    assert flags[3] & _lib.WH_F_HYPERBOLIC
    others = np.delete(np.arange(s.S), 3)
    assert not flags[others].any()


def test_full_size_sampled():
    """The GR workload (65536 eight-planet systems, c = 10065) in the
    packing's launch configuration (4096-step launches); sampled systems
    checked one by one against the oracle."""
    s = inputs.workload("large8gr")
    Qg, Vg, _, flags = run(s, 1000, packing="serial", gr_c=inputs.GR_C, chunk_steps=4096)
    assert not flags.any()
    idx = np.random.default_rng(7).choice(s.S, 48, replace=False)
    sub = s.subset(idx)
    Qo, Vo = oracle.integrate(sub, 1000, gr_c=inputs.GR_C)
    assert rel(sub, Qg[idx], Vg[idx], Qo, Vo) < TOL


def test_reverse_mode_matches_one_planet_per_lane():
    """The serial packing records its segments with its own step and sweeps
    them with the G8 layout's adjoint: its gradients agree with those of the
    one-planet-per-lane packing to rounding (the two forward runs differ only
    in summation order)."""
    s = inputs.make_systems(40, 319, n_planets=None, n_range=(1, 8))
    rng = np.random.default_rng(3)
    gQ_T = rng.normal(size=(s.S, 8, 3)) * live(s)[:, :, None]
    gV_T = rng.normal(size=(s.S, 8, 3)) * live(s)[:, :, None]
    out = {}
    for packing in ("serial", "g8"):
        e = Ensemble.from_systems(s, packing=packing, gr_c=inputs.GR_C)
        e.forward_ckpt(300, 64)
        out[packing] = [x.cpu().numpy() for x in e.adjoint(gQ_T, gV_T)]
        e.close()
    for a, b in zip(out["serial"], out["g8"]):
        scale = np.abs(b).max()
        assert np.abs(a - b).max() <= 1e-10 * scale


def test_forward_ckpt_equals_step():
    # the checkpointed forward run is the step kernel's run, bit for bit
    s = inputs.make_systems(30, 320, n_planets=None, n_range=(1, 8))
    a = Ensemble.from_systems(s, packing="serial")
    a.forward_ckpt(250, 60)
    b = Ensemble.from_systems(s, packing="serial")
    b.step(250)
    Qa, Va = a.state()
    Qb, Vb = b.state()
    assert torch.equal(Qa, Qb) and torch.equal(Va, Vb)
    a.close(); b.close()
