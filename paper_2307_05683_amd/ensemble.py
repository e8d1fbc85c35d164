"""Python front end: an ensemble of planetary systems integrated on the GPU.

PyTorch provides device memory and the stream; every computation runs in
libwh.so through the C interface (include/wh.h).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check

SCHEMES = {"dkd": _lib.WH_DKD, "kdk": _lib.WH_KDK, "saba2": _lib.WH_SABA2, "saba3": _lib.WH_SABA3,
           "saba4": _lib.WH_SABA4}
PACKINGS = {"auto": _lib.WH_PACK_AUTO, "pow2": _lib.WH_PACK_POW2, "g8": _lib.WH_PACK_G8, "pair": _lib.WH_PACK_PAIR,
            "split": _lib.WH_PACK_SPLIT, "serial": _lib.WH_PACK_SERIAL, "mixed": _lib.WH_PACK_MIXED}
EXCHANGES = {"auto": _lib.WH_EXCH_AUTO, "lds": _lib.WH_EXCH_LDS, "dpp": _lib.WH_EXCH_DPP}
COORDS = {"dhc": _lib.WH_COORDS_DHC, "jacobi": _lib.WH_COORDS_JACOBI}


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_f64(x, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=device)


class Ensemble:
    """S independent systems (star + 1..8 planets) in democratic heliocentric
    coordinates; see include/wh.h for the conventions.

    Arrays: n_planets [S] (host ints), m0 [S], m [S, 8], Q [S, 8, 3],
    V [S, 8, 3], dt [S] (float64; numpy or torch).
    """

    def __init__(self, n_planets, m0, m, Q, V, dt, *, gr_c=0.0, scheme="dkd", packing="auto", block_waves=1,
                 chunk_steps=4096, graph_launches=8, z_max=1.0, exchange="auto", coords="dhc", balance=0,
                 kepler_counts=0, corrector=0, device="cuda"):
        L = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("Ensemble needs a GPU (no CPU path exists)")
        self.device = torch.device(device)
        np_ = np.ascontiguousarray(np.asarray(n_planets), dtype=np.int32)
        S = int(np_.shape[0])
        self.S = S
        self.n_planets = np_
        cfg = _lib.default_config(S)
        cfg.gr_c = float(gr_c)
        cfg.scheme = SCHEMES[scheme]
        cfg.packing = PACKINGS[packing] if isinstance(packing, str) else int(packing)
        cfg.block_waves = int(block_waves)
        cfg.chunk_steps = int(chunk_steps)
        cfg.graph_launches = int(graph_launches)
        cfg.z_max = float(z_max)
        cfg.exchange = EXCHANGES[exchange] if isinstance(exchange, str) else int(exchange)
        cfg.coords = COORDS[coords] if isinstance(coords, str) else int(coords)
        cfg.balance = int(balance)
        cfg.kepler_counts = int(kepler_counts)
        cfg.corrector = int(corrector)
        self.cfg = cfg
        self.gr_c = float(gr_c)
        self.scheme = scheme
        nptr = np_.ctypes.data_as(C.POINTER(C.c_int32))
        nbytes = L.wh_workspace_bytes(C.byref(cfg), nptr)
        if nbytes == 0:
            raise _lib.WHError(_lib.WH_EINVAL, "invalid configuration or planet counts")
        self.workspace = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.m0 = _dev_f64(m0, self.device)
        self.m = _dev_f64(m, self.device)
        Qd, Vd = _dev_f64(Q, self.device), _dev_f64(V, self.device)
        self.dt = _dev_f64(dt, self.device)
        for name, t, shape in (("m0", self.m0, (S,)), ("m", self.m, (S, 8)), ("Q", Qd, (S, 8, 3)),
                               ("V", Vd, (S, 8, 3)), ("dt", self.dt, (S,))):
            if tuple(t.shape) != shape:
                raise ValueError("%s must have shape %s, got %s" % (name, shape, tuple(t.shape)))
        ctx = C.c_void_p()
        check(L.wh_init(C.byref(ctx), C.byref(cfg), nptr, self.m0.data_ptr(), self.m.data_ptr(), Qd.data_ptr(),
                        Vd.data_ptr(), self.dt.data_ptr(), self._ws_ptr, int(nbytes), _stream(self.device)))
        self._ctx = ctx

    @classmethod
    def from_systems(cls, systems, **kw):
        return cls(systems.n_planets, systems.m0, systems.m, systems.Q, systems.V, systems.dt, **kw)

    # ---- integration -----------------------------------------------------
    def step(self, n_steps: int):
        check(_lib.load().wh_step_n(self._ctx, int(n_steps), _stream(self.device)))
        return self

    def step_plain(self, n_steps: int):
        check(_lib.load().wh_step_n_plain(self._ctx, int(n_steps), _stream(self.device)))
        return self

    @property
    def steps_done(self) -> int:
        return int(_lib.load().wh_steps_done(self._ctx))

    @property
    def launch_windows(self):
        """(launches per chunk, wavefronts per window) of wh_step_n."""
        slots = C.c_int32(0)
        n = int(_lib.load().wh_launch_windows(self._ctx, C.byref(slots)))
        return n, int(slots.value)

    # ---- outputs (synchronized copies) -------------------------------------
    def state(self):
        Q = torch.zeros((self.S, 8, 3), dtype=torch.float64, device=self.device)
        V = torch.zeros((self.S, 8, 3), dtype=torch.float64, device=self.device)
        check(_lib.load().wh_get_state(self._ctx, Q.data_ptr(), V.data_ptr(), _stream(self.device)))
        return Q, V

    def energy(self):
        E = torch.zeros(self.S, dtype=torch.float64, device=self.device)
        check(_lib.load().wh_energy(self._ctx, E.data_ptr(), _stream(self.device)))
        return E

    def elements(self):
        """Osculating heliocentric (a, e) of every planet: [S, 8] each."""
        a = torch.zeros((self.S, 8), dtype=torch.float64, device=self.device)
        e = torch.zeros((self.S, 8), dtype=torch.float64, device=self.device)
        check(_lib.load().wh_elements(self._ctx, a.data_ptr(), e.data_ptr(), _stream(self.device)))
        return a, e

    def angular_momentum(self):
        """Total angular momentum sum_i Q_i x m_i V_i of every system: [S, 3]."""
        L = torch.zeros((self.S, 3), dtype=torch.float64, device=self.device)
        check(_lib.load().wh_angular_momentum(self._ctx, L.data_ptr(), _stream(self.device)))
        return L

    def flags(self):
        f = torch.zeros(self.S, dtype=torch.int32, device=self.device)
        check(_lib.load().wh_status_flags(self._ctx, f.data_ptr(), _stream(self.device)))
        return f

    # ---- snapshots -----------------------------------------------------------
    def save_state(self):
        """Bitwise snapshot of the unsynchronized state (a device byte tensor;
        .cpu() it to keep it in a file)."""
        L = _lib.load()
        nbytes = int(L.wh_state_bytes(self._ctx))
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + nbytes]
        check(L.wh_save_state(self._ctx, view.data_ptr(), nbytes, _stream(self.device)))
        return view

    def restore_state(self, snap):
        """Load a snapshot taken by save_state of a context of the same batch
        and configuration (a host copy is moved to the device first)."""
        L = _lib.load()
        nbytes = int(L.wh_state_bytes(self._ctx))
        buf = torch.empty(int(snap.numel()) + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + int(snap.numel())]
        view.copy_(snap)
        check(L.wh_restore_state(self._ctx, view.data_ptr(), int(snap.numel()), _stream(self.device)))
        return self

    # ---- reverse mode ------------------------------------------------------
    def forward_ckpt(self, n_steps: int, ckpt_every: int):
        """Advance n_steps from the initial state, storing a checkpoint every
        ckpt_every steps; returns the tape (a device byte tensor)."""
        L = _lib.load()
        nbytes = int(L.wh_tape_bytes(self._ctx, int(n_steps), int(ckpt_every)))
        if nbytes == 0:
            raise _lib.WHError(_lib.WH_EINVAL, "bad n_steps or ckpt_every")
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (buf.data_ptr() + 255) & ~255
        check(L.wh_forward_ckpt(self._ctx, int(n_steps), int(ckpt_every), ptr, nbytes, _stream(self.device)))
        self._tape = (buf, ptr, nbytes)
        return buf

    def adjoint(self, gQ_T, gV_T):
        """dL/d(Q0, V0, m, m0) from dL/d(Q_T, V_T) of the synchronized final
        state, for the run recorded by forward_ckpt."""
        if getattr(self, "_tape", None) is None:
            raise _lib.WHError(_lib.WH_ESTATE, "call forward_ckpt first")
        _, ptr, nbytes = self._tape
        gQ_T = _dev_f64(gQ_T, self.device)
        gV_T = _dev_f64(gV_T, self.device)
        gQ0 = torch.zeros((self.S, 8, 3), dtype=torch.float64, device=self.device)
        gV0 = torch.zeros_like(gQ0)
        gm = torch.zeros((self.S, 8), dtype=torch.float64, device=self.device)
        gm0 = torch.zeros(self.S, dtype=torch.float64, device=self.device)
        check(_lib.load().wh_adjoint_n(self._ctx, ptr, nbytes, gQ_T.data_ptr(), gV_T.data_ptr(), gQ0.data_ptr(),
                                       gV0.data_ptr(), gm.data_ptr(), gm0.data_ptr(), _stream(self.device)))
        return gQ0, gV0, gm, gm0

    def close(self):
        if getattr(self, "_ctx", None):
            torch.cuda.synchronize(self.device)      # nothing of this context may still be in flight
            _lib.load().wh_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Integrate(torch.autograd.Function):
    """(Q0, V0, m, m0) -> (Q_T, V_T) after n_steps; backward by the
    hand-written adjoint with checkpoint recomputation.

    The context's workspace and its tape (checkpoints plus two segment
    buffers: ~1.4 GB for 1024 eight-planet systems at 1e5 steps with
    checkpoints every 1000) are tensors saved for backward: torch frees them
    once a backward pass has run without retain_graph (a second backward
    through the graph then raises, as for any saved tensor) and keeps them
    while the graph is retained."""

    @staticmethod
    def forward(ctx, Q0, V0, m, m0, dt, n_planets, n_steps, ckpt_every, gr_c, opts):
        ens = Ensemble(n_planets, m0.detach(), m.detach(), Q0.detach(), V0.detach(), dt.detach(), gr_c=gr_c,
                       device=Q0.device, **opts)
        tape = ens.forward_ckpt(n_steps, ckpt_every)
        QT, VT = ens.state()
        ctx.save_for_backward(ens.workspace, tape)
        # from here on the saved tensors own the device memory the context uses
        ens.workspace = None
        ens._tape = (None,) + tuple(ens._tape[1:])
        ctx.ens = ens
        return QT, VT

    @staticmethod
    def backward(ctx, gQ, gV):
        workspace, tape = ctx.saved_tensors        # raises once torch has freed them
        ens = ctx.ens
        if gQ is None:
            gQ = torch.zeros((ens.S, 8, 3), dtype=torch.float64, device=ens.device)
        if gV is None:
            gV = torch.zeros((ens.S, 8, 3), dtype=torch.float64, device=ens.device)
        gQ0, gV0, gm, gm0 = ens.adjoint(gQ.contiguous(), gV.contiguous())
        del workspace, tape
        return gQ0, gV0, gm, gm0, None, None, None, None, None, None


def integrate(Q0, V0, m, m0, dt, n_planets, n_steps, ckpt_every=1000, gr_c=0.0, **opts):
    """Differentiable ensemble integration.  The options go to Ensemble
    (scheme "dkd", "kdk", "saba2".."saba4"; any packing; coords "dhc" or
    "jacobi").

    Q0, V0: [S, 8, 3], m: [S, 8], m0, dt: [S] float64 CUDA tensors;
    n_planets: host ints [S].  Returns the synchronized (Q_T, V_T).
    Gradients flow to Q0, V0, m and m0.
    """
    return _Integrate.apply(Q0, V0, m, m0, dt, np.asarray(n_planets), int(n_steps), int(ckpt_every), float(gr_c),
                            opts)
