"""Bitwise snapshots of the unsynchronized state (wh_save_state /
wh_restore_state).

Integration continues from the unsynchronized state and outputs only
synchronize copies of it (Sec. 3.5), so a run resumed from a snapshot --
taken mid-run, passed through host memory, loaded into a fresh context of
the same batch -- must end bitwise where the uninterrupted run ends.
"""
import numpy as np
import pytest
import torch

from paper_2307_05683_amd import _lib, inputs
from paper_2307_05683_amd.ensemble import Ensemble

pytestmark = pytest.mark.gpu


def outputs(e):
    Q, V = e.state()
    return [x.cpu().numpy() for x in (Q, V, e.energy(), e.flags(), e.angular_momentum())]


@pytest.mark.parametrize("packing,scheme,gr_c,coords", [("auto", "dkd", 0.0, "dhc"), ("pair", "dkd", 10065.0, "dhc"),
                                                        ("split", "kdk", 40.0, "dhc"), ("serial", "dkd", 0.0, "dhc"),
                                                        ("auto", "saba3", 0.0, "dhc"), ("g8", "kdk", 40.0, "jacobi")])
def test_resume_from_snapshot_is_bitwise(packing, scheme, gr_c, coords):
    s = inputs.make_systems(300, 81, n_planets=None, n_range=(1, 8))
    kw = dict(packing=packing, scheme=scheme, gr_c=gr_c, coords=coords, chunk_steps=512)
    a = Ensemble.from_systems(s, **kw)
    a.step(1237)
    a.state()                            # an output in between must not matter
    snap = a.save_state().cpu()          # through host memory, as a checkpoint file would be
    a.step(2000)
    ref = outputs(a)
    steps = a.steps_done
    a.close()
    b = Ensemble.from_systems(s, **kw)
    b.step(17)                           # whatever the fresh context did before is overwritten
    b.restore_state(snap)
    assert b.steps_done == 1237
    b.step(2000)
    out = outputs(b)
    assert b.steps_done == steps
    b.close()
    for x, y in zip(out, ref):
        assert np.array_equal(x, y)


def test_restore_rejects_other_configurations():
    s = inputs.make_systems(40, 82, n_planets=None, n_range=(1, 8))
    a = Ensemble.from_systems(s, packing="auto")
    a.step(10)
    snap = a.save_state()
    for kw in (dict(packing="pair"), dict(scheme="kdk"), dict(gr_c=40.0), dict(coords="jacobi")):
        b = Ensemble.from_systems(s, **kw)
        with pytest.raises(_lib.WHError) as ei:
            b.restore_state(snap)
        assert ei.value.code == _lib.WH_ESTATE
        b.close()
    other = Ensemble.from_systems(inputs.make_systems(41, 82, n_planets=None, n_range=(1, 8)))
    with pytest.raises(_lib.WHError) as ei:
        other.restore_state(torch.zeros(int(_lib.load().wh_state_bytes(other._ctx)), dtype=torch.uint8))
    assert ei.value.code == _lib.WH_EINVAL
    other.close()
    a.close()
