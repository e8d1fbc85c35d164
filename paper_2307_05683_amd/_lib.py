"""ctypes binding of libwh.so (the C interface in include/wh.h).

Argument marshalling only: every step of the integration runs in the HIP
kernels of libwh.so.  There is no CPU path; if the library is missing the
import of the binding fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libwh.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "wh.h")

WH_OK, WH_EINVAL, WH_EWORKSPACE, WH_EHIP, WH_ESTATE = 0, -1, -2, -3, -4
WH_DKD, WH_KDK = 0, 1
WH_SABA2, WH_SABA3, WH_SABA4 = 2, 3, 4
WH_PACK_AUTO, WH_PACK_POW2, WH_PACK_G8, WH_PACK_PAIR, WH_PACK_SPLIT, WH_PACK_SERIAL, WH_PACK_MIXED = -1, 0, 1, 2, 3, 4, 5
WH_F_NONFINITE, WH_F_HYPERBOLIC, WH_F_ZMAX = 1, 2, 4
WH_EXCH_AUTO, WH_EXCH_LDS, WH_EXCH_DPP = 0, 1, 2
WH_COORDS_DHC, WH_COORDS_JACOBI = 0, 1
WH_NOALLOC_MAX_BYTES = 16 << 20
ERRORS = {WH_EINVAL: "WH_EINVAL", WH_EWORKSPACE: "WH_EWORKSPACE", WH_EHIP: "WH_EHIP", WH_ESTATE: "WH_ESTATE"}


class WHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("n_systems", C.c_int32),
        ("G", C.c_double),
        ("gr_c", C.c_double),
        ("scheme", C.c_int32),
        ("packing", C.c_int32),
        ("block_waves", C.c_int32),
        ("chunk_steps", C.c_int32),
        ("graph_launches", C.c_int32),
        ("z_max", C.c_double),
        ("exchange", C.c_int32),
        ("coords", C.c_int32),
        ("balance", C.c_int32),
        ("kepler_counts", C.c_int32),
        ("corrector", C.c_int32),
    ]


_lib = None
vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_SIGS = {
    "wh_config_default": ([C.POINTER(Config), i32], None),
    "wh_workspace_bytes": ([C.POINTER(Config), C.POINTER(i32)], sz),
    "wh_init": ([C.POINTER(vp), C.POINTER(Config), C.POINTER(i32), vp, vp, vp, vp, vp, vp, sz, vp], i32),
    "wh_step_n": ([vp, i64, vp], i32),
    "wh_step_n_plain": ([vp, i64, vp], i32),
    "wh_get_state": ([vp, vp, vp, vp], i32),
    "wh_energy": ([vp, vp, vp], i32),
    "wh_status_flags": ([vp, vp, vp], i32),
    "wh_elements": ([vp, vp, vp, vp], i32),
    "wh_angular_momentum": ([vp, vp, vp], i32),
    "wh_steps_done": ([vp], i64),
    "wh_launch_windows": ([vp, C.POINTER(i32)], i32),
    "wh_state_bytes": ([vp], sz),
    "wh_save_state": ([vp, vp, sz, vp], i32),
    "wh_restore_state": ([vp, vp, sz, vp], i32),
    "wh_tape_bytes": ([vp, i64, i64], sz),
    "wh_forward_ckpt": ([vp, i64, i64, vp, sz, vp], i32),
    "wh_adjoint_n": ([vp, vp, sz, vp, vp, vp, vp, vp, vp, vp], i32),
    "wh_kepler_envelope": ([i64, vp, vp, vp, vp, i64, i32, i32, i32, i32, vp, vp, vp, vp, vp], i32),
    "wh_integrate_noalloc": ([C.POINTER(Config), C.POINTER(i32), vp, vp, vp, vp, vp, i64, vp, vp, vp], i32),
    "wh_last_error": ([], C.c_char_p),
    "wh_destroy": ([vp], None),
}


def header_symbols() -> list[str]:
    """Function names declared in include/wh.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(wh_[a-z_0-9]+)\s*\(", text)))


def load():
    """Load libwh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libwh.so is not built: run __graft_entry__.build() (or python -m "
                               "paper_2307_05683_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(code: int):
    if code != WH_OK:
        raise WHError(code, load().wh_last_error().decode())


def default_config(n_systems: int) -> Config:
    cfg = Config()
    load().wh_config_default(C.byref(cfg), int(n_systems))
    return cfg
