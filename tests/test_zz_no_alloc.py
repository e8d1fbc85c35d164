"""wh_integrate_noalloc: the integration entry point that allocates no device
memory (its workspace is a fixed array inside the library) against the
allocating sequence wh_init + wh_step_n + wh_get_state on the same inputs.
Two calls in a row, the second with a smaller batch, must each equal the
allocating path bitwise (the same kernels in the same order); a batch beyond
the array's size is rejected before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2307_05683_amd import _lib, inputs
from paper_2307_05683_amd.ensemble import PACKINGS, Ensemble, _stream

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def noalloc(s, n_steps, packing, gr_c=0.0, scheme="dkd"):
    L = _lib.load()
    cfg = _lib.default_config(s.S)
    cfg.packing = PACKINGS[packing]
    cfg.gr_c = gr_c
    cfg.scheme = {"dkd": _lib.WH_DKD, "kdk": _lib.WH_KDK}[scheme]
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)
    m0, m, Q, V, dt = t(s.m0), t(s.m), t(s.Q), t(s.V), t(s.dt)
    Qo = torch.zeros((s.S, 8, 3), dtype=torch.float64, device=DEV)
    Vo = torch.zeros_like(Qo)
    npl = np.ascontiguousarray(s.n_planets, dtype=np.int32)
    _lib.check(L.wh_integrate_noalloc(C.byref(cfg), npl.ctypes.data_as(C.POINTER(C.c_int32)), m0.data_ptr(),
                                      m.data_ptr(), Q.data_ptr(), V.data_ptr(), dt.data_ptr(), int(n_steps),
                                      Qo.data_ptr(), Vo.data_ptr(), _stream(DEV)))
    torch.cuda.synchronize()
    return Qo.cpu().numpy(), Vo.cpu().numpy()


def allocating(s, n_steps, packing, gr_c=0.0, scheme="dkd"):
    e = Ensemble.from_systems(s, packing=packing, gr_c=gr_c, scheme=scheme)
    e.step(n_steps)
    Q, V = e.state()
    out = Q.cpu().numpy(), V.cpu().numpy()
    e.close()
    return out


@pytest.mark.parametrize("packing,gr_c,scheme", [("auto", 0.0, "dkd"), ("split", 0.0, "dkd"),
                                                 ("pair", 10065.0, "dkd"), ("auto", 40.0, "kdk")])
def test_noalloc_equals_allocating_path_twice(packing, gr_c, scheme):
    big = inputs.make_systems(1500, 61, n_planets=None, n_range=(1, 8))
    small = inputs.make_systems(37, 62, n_planets=None, n_range=(2, 8))
    for s, n in ((big, 9000), (small, 1234)):     # 9000 = two 4096-step launches and a 808-step one
        print("case: noalloc %s gr_c=%g %s S=%d n=%d" % (packing, gr_c, scheme, s.S, n), flush=True)
        Qa, Va = noalloc(s, n, packing, gr_c, scheme)
        Qb, Vb = allocating(s, n, packing, gr_c, scheme)
        lm = np.arange(8)[None, :] < s.n_planets[:, None]
        assert np.array_equal(Qa[lm], Qb[lm]) and np.array_equal(Va[lm], Vb[lm])
        assert np.isfinite(Qa[lm]).all()


def test_noalloc_rejects_a_batch_beyond_the_array():
    L = _lib.load()
    s = inputs.make_systems(4, 63, n_planets=8)
    n_big = 200000                                   # 200000 eight-planet systems: ~200 MB of workspace
    cfg = _lib.default_config(n_big)
    npl = np.full(n_big, 8, dtype=np.int32)
    assert L.wh_workspace_bytes(C.byref(cfg), npl.ctypes.data_as(C.POINTER(C.c_int32))) > _lib.WH_NOALLOC_MAX_BYTES
    z = torch.zeros(8, dtype=torch.float64, device=DEV)
    rc = L.wh_integrate_noalloc(C.byref(cfg), npl.ctypes.data_as(C.POINTER(C.c_int32)), z.data_ptr(), z.data_ptr(),
                                z.data_ptr(), z.data_ptr(), z.data_ptr(), 10, z.data_ptr(), z.data_ptr(), _stream(DEV))
    assert rc == _lib.WH_EWORKSPACE
    assert b"scratch" in L.wh_last_error()
    # the library still works after the rejection
    Qa, _ = noalloc(s, 10, "auto")
    Qb, _ = allocating(s, 10, "auto")
    assert np.array_equal(Qa, Qb)
