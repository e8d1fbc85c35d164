"""SABA_n splittings on the GPU vs the oracle's (parity), both coordinates."""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_05683_amd import _lib, inputs
from paper_2307_05683_amd.diagnostics import scan
from paper_2307_05683_amd.ensemble import Ensemble

pytestmark = pytest.mark.gpu
TOL = 1e-12


def live(s):
    return np.arange(8)[None, :] < s.n_planets[:, None]


def check(s, n_steps, scheme, coords, tol=TOL, **kw):
    print("case: S=%d n_steps=%d scheme=%s coords=%s %s" % (s.S, n_steps, scheme, coords, kw), flush=True)
    e = Ensemble.from_systems(s, scheme=scheme, coords=coords, **kw)
    e.step(n_steps)
    Q, V = e.state()
    Qg, Vg = Q.cpu().numpy(), V.cpu().numpy()
    e.close()
    f = oracle.jacobi_integrate if coords == "jacobi" else oracle.integrate
    Qo, Vo = f(s, n_steps, scheme=scheme)
    lm = live(s)
    Qo = Qo.astype(float); Vo = Vo.astype(float)
    with np.errstate(invalid="ignore"):
        eq = np.linalg.norm(Qg - Qo, axis=2) / np.linalg.norm(Qo, axis=2)
        ev = np.linalg.norm(Vg - Vo, axis=2) / np.linalg.norm(Vo, axis=2)
    err = np.where(lm, np.maximum(eq, ev), 0).max(axis=1)
    print("relative error per system: median %.2e  max %.2e" % (np.median(err), err.max()), flush=True)
    assert err.max() < tol


@pytest.mark.parametrize("coords", ["dhc", "jacobi"])
@pytest.mark.parametrize("scheme", ["saba2", "saba3", "saba4"])
def test_uneven_batch_1000_steps(scheme, coords):
    s = inputs.make_systems(48, 91, n_planets=None, n_range=(1, 8), dt_mode="u15_30")
    check(s, 1000, scheme, coords)


@pytest.mark.parametrize("exchange", ["dpp", "lds"])
@pytest.mark.parametrize("packing", ["pow2", "g8"])
def test_packings_and_exchanges(packing, exchange):
    s = inputs.make_systems(40, 92, n_planets=None, n_range=(1, 8))
    check(s, 500, "saba2", "dhc", packing=packing, exchange=exchange)


@pytest.mark.parametrize("scheme", ["saba2", "saba3", "saba4"])
@pytest.mark.parametrize("packing", ["pair", "split", "serial"])
def test_pair_split_and_serial_layouts(packing, scheme):
    s = inputs.make_systems(45, 97, n_planets=None, n_range=(1, 8), dt_mode="u15_30")
    check(s, 1000, scheme, "dhc", packing=packing)


@pytest.mark.parametrize("packing", ["pair", "split", "serial"])
def test_pair_split_and_serial_few_steps_and_outputs(packing):
    s = inputs.make_systems(20, 98, n_planets=None, n_range=(1, 8))
    for n in (1, 2, 5):
        check(s, n, "saba3", "dhc", tol=1e-14, packing=packing)
    # keep unsynchronized: outputs between chunks leave the run bitwise unchanged
    a = Ensemble.from_systems(s, scheme="saba2", chunk_steps=32, packing=packing)
    a.step(200)
    Qa, Va = a.state()
    b = Ensemble.from_systems(s, scheme="saba2", chunk_steps=32, packing=packing)
    for _ in range(20):
        b.step(10)
        b.state()
        b.energy()
    Qb, Vb = b.state()
    assert torch.equal(Qa, Qb) and torch.equal(Va, Vb)
    a.close(); b.close()


@pytest.mark.parametrize("n_steps", [1, 2, 5])
@pytest.mark.parametrize("coords", ["dhc", "jacobi"])
def test_few_steps(n_steps, coords):
    s = inputs.make_systems(20, 93, n_planets=None, n_range=(1, 8))
    check(s, n_steps, "saba3", coords, tol=1e-14)


def test_keep_unsynchronized_is_bitwise_reproducible():
    s = inputs.make_systems(40, 94, n_planets=None, n_range=(2, 8))
    a = Ensemble.from_systems(s, scheme="saba2", chunk_steps=32)
    a.step(200)
    Qa, Va = a.state()
    b = Ensemble.from_systems(s, scheme="saba2", chunk_steps=32)
    for _ in range(20):
        b.step(10)
        b.state()
    Qb, Vb = b.state()
    assert torch.equal(Qa, Qb) and torch.equal(Va, Vb)
    a.close(); b.close()


def test_gr_in_dhc_rejected():
    s = inputs.make_systems(4, 95, n_planets=3)
    with pytest.raises(_lib.WHError):
        Ensemble.from_systems(s, scheme="saba2", gr_c=10065.0)


@pytest.mark.parametrize("coords", ["dhc", "jacobi"])
def test_fourth_order_energy_error(coords):
    """SABA_2: the energy error falls ~16x per halving of dt for small
    perturbations (eps = 1e-5), as the oracle's does."""
    s = inputs.make_systems(64, 96, n_planets=2)
    s.m[:, :2] = 1e-5
    worst = []
    for k in (1, 2):
        t = s.copy()
        t.dt = s.dt / k
        e = Ensemble.from_systems(t, scheme="saba2", coords=coords)
        r = scan(e, 10, 100 * k, e_crit=1.0)
        worst.append(np.abs(r["dE"]).max(axis=0))
        e.close()
    ratio = worst[0] / worst[1]
    print("%s: median ratio per halving %.1f" % (coords, np.median(ratio)), flush=True)
    assert 12 < np.median(ratio) < 20
