"""Host-side checks of the C-ABI library (no GPU call is made here)."""
import ctypes as C

import numpy as np
import pytest

from paper_2307_05683_amd import _lib


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = _lib.header_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    # the binding declares exactly the header's functions
    assert sorted(_lib._SIGS) == names


def _ws(cfg, n):
    n = np.ascontiguousarray(n, dtype=np.int32)
    return _lib.load().wh_workspace_bytes(C.byref(cfg), n.ctypes.data_as(C.POINTER(C.c_int32)))


def test_workspace_size_follows_packing():
    n = np.array([2, 3, 5, 8, 1, 4, 7], dtype=np.int32)
    cfg = _lib.default_config(len(n))
    cfg.packing = _lib.WH_PACK_POW2
    a = _ws(cfg, n)
    cfg.packing = _lib.WH_PACK_G8
    b = _ws(cfg, n)
    assert a > 0 and b > 0
    # G8 keeps every planet count on its own waves: 7 counts -> 7 waves of 64 lanes
    per_slot = 7 * 8 + 2 * 8 + 2 * 4
    assert b >= 7 * 64 * per_slot
    # pow2 packs groups of 1/2/4/8 lanes: one wave per group size here
    assert a < b


def _layout_bytes(S, ns):
    a = lambda x: (x + 255) // 256 * 256
    return a(13 * 8 * ns) + 2 * a(8 * ns) + 2 * a(4 * ns) + 2 * a(4 * S)


@pytest.mark.parametrize("S", [1, 4, 7, 64, 1001])
def test_split_packing_takes_16_lanes_per_system(S):
    cfg = _lib.default_config(S)
    cfg.packing = _lib.WH_PACK_SPLIT
    n = np.random.default_rng(S).integers(1, 9, S)
    assert _ws(cfg, n) == _layout_bytes(S, 64 * ((S + 3) // 4))


@pytest.mark.parametrize("packing,max_systems", [(_lib.WH_PACK_POW2, 1 << 24), (_lib.WH_PACK_SPLIT, 1 << 23),
                                                 (_lib.WH_PACK_PAIR, 1 << 25), (_lib.WH_PACK_SERIAL, 1 << 24)])
def test_lane_slot_cap(packing, max_systems):
    # 32-bit device indexing: at most 2^27 lane slots; eight-planet systems
    # take 8 (one planet per lane), 16 (split) or 4 (pair) slots each
    cfg = _lib.default_config(max_systems + 1)
    cfg.packing = packing
    assert _ws(cfg, np.full(max_systems + 1, 8, dtype=np.int32)) == 0
    cfg.n_systems = 1000
    assert _ws(cfg, np.full(1000, 8, dtype=np.int32)) > 0


@pytest.mark.parametrize("packing", [_lib.WH_PACK_POW2, _lib.WH_PACK_G8, _lib.WH_PACK_PAIR, _lib.WH_PACK_SPLIT,
                                     _lib.WH_PACK_SERIAL])
def test_slot_count_matches_the_layout_rules(packing):
    # the library builds the slot tables and checks them against its own
    # closed-form count; here the count is rebuilt from the layout rules
    rng = np.random.default_rng(7)
    for S in (1, 5, 64, 333):
        n = rng.integers(1, 9, S)
        cnt = np.bincount(n, minlength=9)
        w = lambda k, per: -(-int(k) // per)
        if packing == _lib.WH_PACK_POW2:
            ns = 64 * (w(cnt[1], 64) + w(cnt[2], 32) + w(cnt[3] + cnt[4], 16) + w(cnt[5:].sum(), 8))
        elif packing in (_lib.WH_PACK_G8, _lib.WH_PACK_SERIAL):
            # the one-lane-per-system packing keeps the G8 storage
            ns = 64 * sum(w(cnt[k], 8) for k in range(1, 9))
        elif packing == _lib.WH_PACK_PAIR:
            ns = 128 * (w(cnt[1] + cnt[2], 64) + w(cnt[3] + cnt[4], 32) + w(cnt[5:].sum(), 16))
        else:
            ns = 64 * w(S, 4)
        cfg = _lib.default_config(S)
        cfg.packing = packing
        assert _ws(cfg, n) == _layout_bytes(S, ns), (S, packing)


@pytest.mark.parametrize("packing", [_lib.WH_PACK_PAIR, _lib.WH_PACK_SPLIT, _lib.WH_PACK_SERIAL])
def test_pair_split_and_serial_packings_need_dhc(packing):
    cfg = _lib.default_config(3)
    cfg.packing = packing
    for scheme in (_lib.WH_DKD, _lib.WH_KDK, _lib.WH_SABA2, _lib.WH_SABA4):
        cfg.scheme = scheme
        assert _ws(cfg, [2, 5, 8]) > 0
    cfg.gr_c = 10065.0            # SABA_n with GR needs Jacobi coordinates
    assert _ws(cfg, [2, 5, 8]) == 0
    cfg.gr_c = 0.0
    cfg.scheme = _lib.WH_DKD
    cfg.coords = _lib.WH_COORDS_JACOBI
    assert _ws(cfg, [2, 5, 8]) == 0


@pytest.mark.parametrize("bad", [
    dict(G=2.0), dict(scheme=5), dict(packing=6), dict(packing=7), dict(block_waves=3), dict(chunk_steps=-1), dict(n_systems=0),
    dict(exchange=9),
])
def test_invalid_configs_rejected(bad):
    cfg = _lib.default_config(3)
    for k, v in bad.items():
        setattr(cfg, k, v)
    assert _ws(cfg, [2, 2, 2]) == 0


def test_mixed_packing_configurations():
    # shared 8-lane groups: DHC drift-kick-drift or kick-drift-kick, the DPP
    # exchange, the paper's Kepler counts; a 5- and a 3-planet system share
    # a group (one wave), the 8-planet system has its own
    cfg = _lib.default_config(3)
    cfg.packing = _lib.WH_PACK_MIXED
    assert _ws(cfg, [5, 3, 8]) > 0
    cfg.scheme = _lib.WH_KDK
    assert _ws(cfg, [5, 3, 8]) > 0
    for k, v in (("scheme", _lib.WH_SABA2), ("coords", _lib.WH_COORDS_JACOBI), ("exchange", _lib.WH_EXCH_LDS),
                 ("kepler_counts", 1)):
        c = _lib.default_config(3)
        c.packing = _lib.WH_PACK_MIXED
        setattr(c, k, v)
        assert _ws(c, [5, 3, 8]) == 0, k


@pytest.mark.parametrize("counts", [[0, 2], [9], [3, -1]])
def test_invalid_planet_counts_rejected(counts):
    cfg = _lib.default_config(len(counts))
    assert _ws(cfg, counts) == 0


def test_defaults():
    cfg = _lib.default_config(4)
    assert cfg.G == 1.0 and cfg.scheme == _lib.WH_DKD and cfg.gr_c == 0.0
    assert cfg.chunk_steps > 0 and cfg.z_max > 0


def test_noalloc_entry_point_rejects_oversized_batches_before_any_device_call():
    """wh_integrate_noalloc checks the batch against its fixed scratch array
    before touching the device (so this runs without a GPU): 200000
    eight-planet systems need ~200 MB of workspace against 16 MiB."""
    import ctypes as C
    import numpy as np
    L = _lib.load()
    n = 200000
    cfg = _lib.default_config(n)
    npl = np.full(n, 8, dtype=np.int32)
    p = npl.ctypes.data_as(C.POINTER(C.c_int32))
    assert L.wh_workspace_bytes(C.byref(cfg), p) > _lib.WH_NOALLOC_MAX_BYTES
    rc = L.wh_integrate_noalloc(C.byref(cfg), p, None, None, None, None, None, 10, 8, 8, None)
    assert rc == _lib.WH_EWORKSPACE
    assert b"scratch" in L.wh_last_error()
    rc = L.wh_integrate_noalloc(C.byref(cfg), p, None, None, None, None, None, -1, 8, 8, None)
    assert rc == _lib.WH_EINVAL


@pytest.mark.parametrize("bad", [dict(packing=_lib.WH_PACK_SERIAL), dict(coords=_lib.WH_COORDS_JACOBI),
                                 dict(scheme=_lib.WH_SABA2), dict(exchange=_lib.WH_EXCH_LDS), dict(kepler_counts=2)])
def test_cheaper_kepler_counts_only_where_compiled(bad):
    L = _lib.load()
    cfg = _lib.default_config(4)
    cfg.kepler_counts = 1
    for k, v in bad.items():
        setattr(cfg, k, v)
    npl = np.full(4, 3, dtype=np.int32)
    assert L.wh_workspace_bytes(C.byref(cfg), npl.ctypes.data_as(C.POINTER(C.c_int32))) == 0
    cfg = _lib.default_config(4)
    cfg.kepler_counts = 1
    assert L.wh_workspace_bytes(C.byref(cfg), npl.ctypes.data_as(C.POINTER(C.c_int32))) > 0


@pytest.mark.parametrize("bad", [dict(coords=_lib.WH_COORDS_DHC), dict(scheme=_lib.WH_SABA2), dict(corrector=4),
                                 dict(corrector=-1)])
def test_correctors_need_jacobi_and_a_second_order_scheme(bad):
    L = _lib.load()
    npl = np.full(4, 3, dtype=np.int32)
    cfg = _lib.default_config(4)
    cfg.coords = _lib.WH_COORDS_JACOBI
    cfg.corrector = 2
    assert L.wh_workspace_bytes(C.byref(cfg), npl.ctypes.data_as(C.POINTER(C.c_int32))) > 0
    for k, v in bad.items():
        setattr(cfg, k, v)
    assert L.wh_workspace_bytes(C.byref(cfg), npl.ctypes.data_as(C.POINTER(C.c_int32))) == 0
