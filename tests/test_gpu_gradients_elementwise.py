"""Reverse mode, component by component.

Every component of the GPU gradient (dL/dQ0, dL/dV0, dL/dm, dL/dm0) is
compared with the same component built from the oracle's forward tangent
map (dual numbers in long double, Kepler solved to convergence): the
tangent along basis direction e_k gives column k of the Jacobian M of the
map, and dL/dx0_k = <dL/dx_T, M e_k>.  The 57 basis directions of a system
(8 planets x (3 position + 3 velocity + 1 mass) + the star mass) run as 57
copies of it in one oracle call.  Planet slots beyond a system's planet
count have no direction and must come out zero on the GPU.

The full-length check of the adjoint configuration (1e5 steps, checkpoints
every 1000) adds central finite differences of the GPU forward map on every
input of sampled systems, with h = 1e-7 relative and Richardson's
extrapolation [4 D(h/2) - D(h)] / 3.
"""
import functools

import numpy as np
import pytest
import torch

import oracle
from paper_2307_05683_amd import inputs
from paper_2307_05683_amd.ensemble import Ensemble

pytestmark = pytest.mark.gpu

NDIR = 57   # 24 position + 24 velocity components, 8 planet masses, the star mass


def live(s):
    return np.arange(8)[None, :] < s.n_planets[:, None]


def basis_directions(s):
    """Replicate every system NDIR times (system-major) and give copy k the
    k-th basis direction; directions on padding slots stay zero."""
    rep = s.subset(np.repeat(np.arange(s.S), NDIR))
    R = rep.S
    dQ = np.zeros((R, 8, 3)); dV = np.zeros((R, 8, 3)); dm = np.zeros((R, 8)); dm0 = np.zeros(R)
    lm = live(s)
    for i in range(s.S):
        for k in range(NDIR):
            r = i * NDIR + k
            if k < 24:
                p, c = divmod(k, 3)
                dQ[r, p, c] = lm[i, p]
            elif k < 48:
                p, c = divmod(k - 24, 3)
                dV[r, p, c] = lm[i, p]
            elif k < 56:
                dm[r, k - 48] = lm[i, k - 48]
            else:
                dm0[r] = 1.0
    return rep, dQ, dV, dm, dm0


def unpack(col):
    """[S, NDIR] -> gQ [S, 8, 3], gV [S, 8, 3], gm [S, 8], gm0 [S]."""
    S = col.shape[0]
    return (col[:, :24].reshape(S, 8, 3), col[:, 24:48].reshape(S, 8, 3), col[:, 48:56].copy(), col[:, 56].copy())


def oracle_gradient(s, n_steps, gQ_T, gV_T, scheme="dkd", gr_c=0.0, coords="dhc"):
    rep, dQ, dV, dm, dm0 = basis_directions(s)
    _, _, tQ, tV = oracle.tangent(rep, n_steps, dQ, dV, dm, dm0, scheme=scheme, gr_c=gr_c, coords=coords)
    tQ = tQ.astype(float).reshape(s.S, NDIR, 8, 3)
    tV = tV.astype(float).reshape(s.S, NDIR, 8, 3)
    col = (np.einsum("spc,skpc->sk", gQ_T, tQ) + np.einsum("spc,skpc->sk", gV_T, tV))
    return unpack(col)


def seeds(s, seed):
    rng = np.random.default_rng(seed)
    lm = live(s)
    return rng.normal(size=(s.S, 8, 3)) * lm[:, :, None], rng.normal(size=(s.S, 8, 3)) * lm[:, :, None]


SMALL_STEPS, SMALL_EVERY = 300, 64


@functools.lru_cache(maxsize=None)
def small_case_reference(scheme, gr_c, coords):
    s = inputs.make_systems(16, 51, n_planets=None, n_range=(1, 8))
    gQ_T, gV_T = seeds(s, 52)
    return s, gQ_T, gV_T, oracle_gradient(s, SMALL_STEPS, gQ_T, gV_T, scheme, gr_c, coords)


def compare_blocks(gpu, ref, lm, label, tol_block, tol_elem, floor):
    """Each component against the oracle: |g - g_ref| <= tol_block |block of
    the system| and <= tol_elem max(|g_ref|, floor |block|); padding slots
    exactly zero."""
    names = ("dQ0", "dV0", "dm", "dm0")
    worst = {}
    for name, g, r in zip(names, gpu, ref):
        S = r.shape[0]
        if name == "dm0":
            mask = np.ones(S, bool)
            norm = np.abs(r)
        else:
            mask = lm if g.ndim == 2 else np.repeat(lm[:, :, None], 3, axis=2)
            norm = np.sqrt((r.reshape(S, -1) ** 2).sum(1))
        bshape = (S,) + (1,) * (r.ndim - 1)
        nb = norm.reshape(bshape)
        d = np.abs(g - r)
        assert not g[~mask].any(), "%s: non-zero gradient on a padding slot" % name
        eb = np.where(mask, d / np.maximum(nb, 1e-300), 0.0)
        ee = np.where(mask, d / np.maximum(np.maximum(np.abs(r), floor * nb), 1e-300), 0.0)
        worst[name] = (eb.max(), ee.max())
    print("%s: " % label + ", ".join("%s block %.1e elem %.1e" % (k, v[0], v[1]) for k, v in worst.items()),
          flush=True)
    for name, (eb, ee) in worst.items():
        assert eb < tol_block, (name, eb)
        assert ee < tol_elem, (name, ee)


DHC_CASES = [("dkd", 0.0), ("dkd", 40.0), ("kdk", 0.0), ("kdk", 40.0), ("saba2", 0.0), ("saba3", 0.0)]


@pytest.mark.parametrize("packing", ["auto", "split", "pair", "serial"])
@pytest.mark.parametrize("scheme,gr_c", DHC_CASES)
def test_every_gradient_component_matches_the_oracle(scheme, gr_c, packing):
    """16 systems of 1..8 planets, 300 steps, checkpoints every 64."""
    s, gQ_T, gV_T, ref = small_case_reference(scheme, gr_c, "dhc")
    print("case: %s gr_c=%g packing=%s" % (scheme, gr_c, packing), flush=True)
    e = Ensemble.from_systems(s, gr_c=gr_c, scheme=scheme, packing=packing)
    e.forward_ckpt(SMALL_STEPS, SMALL_EVERY)
    g = [x.cpu().numpy() for x in e.adjoint(gQ_T, gV_T)]
    e.close()
    compare_blocks(g, ref, live(s), "%s/%s/%g" % (packing, scheme, gr_c), 1e-9, 1e-7, 1e-3)


@pytest.mark.parametrize("packing", ["auto", "g8"])
@pytest.mark.parametrize("scheme,gr_c", [("dkd", 0.0), ("kdk", 40.0), ("saba2", 0.0), ("dkd", 10065.0)])
def test_every_jacobi_gradient_component_matches_the_oracle(scheme, gr_c, packing):
    s, gQ_T, gV_T, ref = small_case_reference(scheme, gr_c, "jacobi")
    print("case: jacobi %s gr_c=%g packing=%s" % (scheme, gr_c, packing), flush=True)
    e = Ensemble.from_systems(s, gr_c=gr_c, scheme=scheme, packing=packing, coords="jacobi")
    e.forward_ckpt(SMALL_STEPS, SMALL_EVERY)
    g = [x.cpu().numpy() for x in e.adjoint(gQ_T, gV_T)]
    e.close()
    compare_blocks(g, ref, live(s), "jacobi %s/%s/%g" % (packing, scheme, gr_c), 1e-9, 1e-7, 1e-3)


# ---------------------------------------------------------------------------
# The adjoint configuration at full length: 1024 eight-planet systems, 1e5
# steps, checkpoints every 1000, loss L = sum_i |Q_i(T)|^2.  Sampled systems.

FULL_STEPS, FULL_EVERY = 100_000, 1000
SAMPLED = np.array([0, 311, 650, 1023])


@functools.lru_cache(maxsize=None)
def full_length_adjoint(packing):
    s = inputs.workload("adjoint8")
    e = Ensemble.from_systems(s, packing=packing)
    e.forward_ckpt(FULL_STEPS, FULL_EVERY)
    QT, VT = e.state()
    g = [x.cpu().numpy() for x in e.adjoint(2 * QT, torch.zeros_like(VT))]
    QT = QT.cpu().numpy()
    e.close()
    return s, QT, g


@functools.lru_cache(maxsize=None)
def full_length_oracle():
    sub = inputs.workload("adjoint8").subset(SAMPLED)
    Qo, _ = oracle.integrate(sub, FULL_STEPS)
    gQ_T = 2 * Qo.astype(float) * live(sub)[:, :, None]
    return sub, oracle_gradient(sub, FULL_STEPS, gQ_T, np.zeros_like(gQ_T))


@pytest.mark.parametrize("packing", ["auto", "split"])
def test_full_length_gradient_components_match_the_oracle(packing):
    """Every component of the gradient of 4 sampled systems of the adjoint
    configuration at its full 1e5 steps against the oracle tangent (the
    oracle's loss seed 2 Q_T is its own final state)."""
    s, QT, g = full_length_adjoint(packing)
    sub, ref = full_length_oracle()
    gs = [x[SAMPLED] for x in g]
    compare_blocks(gs, ref, live(sub), "1e5 steps, %s" % packing, 1e-6, 1e-5, 1e-3)


def central_difference_check(sub, n_steps, col, label, min_decided, block_tol=None, **ens_kw):
    """Central differences of the GPU forward map on all 57 inputs of every
    system of `sub`: h = 1e-7 |Q_i| (|V_i|) for a position (velocity)
    component, 1e-7 m_i for a planet mass, 1e-7 m0 for the star mass, each
    at h and h/2; the perturbed copies integrate as one batch of independent
    systems.  col: the adjoint's gradient [S, 57] of L = sum_i |Q_i(T)|^2.
    The comparison value is Richardson's R = [4 D(h/2) - D(h)] / 3.  A
    central difference is itself uncertain: by its truncation, estimated as
    the spread of D(h/2), D(h), D(2h), and by the rounding noise of the loss
    divided by h: each perturbed run rounds differently at every step (in
    plain double the oracle's own central differences scatter by 1e-4 on a
    planet mass), so the spread of three independently rounded differences
    is the measure, plus sigma: three more copies of each system start one
    ulp away (every coordinate times 1 + 2^-52 or 1 - 2^-52) and sigma =
    max |L(copy) - L(x)| after the run.  Where u = spread + 2 sigma / h is
    below 5e-7 |R| the difference decides to 1e-6 and the
    adjoint must match R to 1e-6 relative (floor: 1e-3 of the system's
    gradient block); elsewhere the adjoint must lie within 1e-6 |R| + 4 u of
    R.  At least min_decided of the components must decide.  block_tol: the
    norm-wise reading of the 1e-6 (per system and group -- positions,
    velocities, the star mass -- max |adjoint - R| over the group's norm of R);
    None to report it only."""
    lm = live(sub)
    nS = sub.S
    copies = []          # (system, input k, sign, scale)
    fracs = (1.0, 0.5, 2.0)
    for i in range(nS):
        for k in range(NDIR):
            for frac in fracs:
                for sign in (1.0, -1.0):
                    copies.append((i, k, sign, frac))
    n_ulp = 3
    rows = [c[0] for c in copies] + [i for i in range(nS) for _ in range(n_ulp)] + list(range(nS))
    rep = sub.subset(rows)
    hs = np.zeros(len(copies))
    valid = np.zeros(len(copies), bool)
    for r, (i, k, sign, frac) in enumerate(copies):
        if k < 24:
            p, c = divmod(k, 3)
            h = 1e-7 * np.linalg.norm(sub.Q[i, p]) * frac
            rep.Q[r, p, c] += sign * h
            valid[r] = lm[i, p]
        elif k < 48:
            p, c = divmod(k - 24, 3)
            h = 1e-7 * np.linalg.norm(sub.V[i, p]) * frac
            rep.V[r, p, c] += sign * h
            valid[r] = lm[i, p]
        elif k < 56:
            p = k - 48
            h = 1e-7 * sub.m[i, p] * frac
            rep.m[r, p] += sign * h
            valid[r] = lm[i, p]
        else:
            h = 1e-7 * sub.m0[i] * frac
            rep.m0[r] += sign * h
            valid[r] = True
        hs[r] = h
    rng = np.random.default_rng(71)
    base_ulp = len(copies)
    for j in range(nS * n_ulp):
        r = base_ulp + j
        for arr in (rep.Q, rep.V):
            arr[r] *= 1.0 + rng.choice([-1.0, 1.0], size=arr[r].shape) * 2.0 ** -52
    e = Ensemble.from_systems(rep, **ens_kw)
    e.step(n_steps)
    Q, _ = e.state()
    e.close()
    Q = Q.cpu().numpy()
    L = (Q ** 2 * live(rep)[:, :, None]).sum((1, 2))
    L0 = L[-nS:]
    sigma = np.abs(L[base_ulp:base_ulp + nS * n_ulp].reshape(nS, n_ulp) - L0[:, None]).max(1)
    nf = len(fracs)
    Lc = L[:len(copies)].reshape(nS, NDIR, nf, 2)         # [system, input, (h, h/2, 2h), (+, -)]
    H = hs.reshape(nS, NDIR, nf, 2)[:, :, :, 0]
    with np.errstate(invalid="ignore", divide="ignore"):   # padding inputs have h = 0
        D = (Lc[..., 0] - Lc[..., 1]) / (2 * H)             # [system, input, (h, h/2, 2h)]
        rich = (4 * D[..., 1] - D[..., 0]) / 3
        # three differences with independent rounding: their spread bounds
        # truncation and rounding noise together (two may agree by chance)
        unc = D.max(axis=2) - D.min(axis=2) + 2 * sigma[:, None] / H[..., 0]
    ok_in = valid.reshape(nS, NDIR, nf, 2)[:, :, 0, 0]
    blocks = [slice(0, 24), slice(24, 48), slice(48, 56), slice(56, 57)]
    n_res = n_unres = 0
    worst_res = worst_unres = 0.0
    worst_block = {"dQ0": 0.0, "dV0": 0.0, "dm": 0.0, "dm0": 0.0}
    for i in range(nS):
        for bname, b in zip(worst_block, blocks):
            norm = np.linalg.norm(col[i, b])
            rnorm = np.linalg.norm(np.where(ok_in[i, b], rich[i, b], 0.0))
            dev = np.where(ok_in[i, b], np.abs(col[i, b] - rich[i, b]), 0.0).max()
            worst_block[bname] = max(worst_block[bname], dev / rnorm)
            for k in range(b.start, b.stop):
                if not ok_in[i, k]:
                    assert col[i, k] == 0.0
                    continue
                d = abs(col[i, k] - rich[i, k])
                if unc[i, k] <= 5e-7 * abs(rich[i, k]):
                    n_res += 1
                    err = d / max(abs(rich[i, k]), 1e-3 * norm)
                    worst_res = max(worst_res, err)
                    assert err < 1e-6, (label, i, k, col[i, k], rich[i, k], D[i, k], unc[i, k])
                else:
                    n_unres += 1
                    worst_unres = max(worst_unres, (d - 1e-6 * abs(rich[i, k])) / unc[i, k])
                    assert d <= 1e-6 * abs(rich[i, k]) + 4 * unc[i, k], (label, i, k, col[i, k], D[i, k], unc[i, k])
    print("%s: loss rounding noise (relative) up to %.1e; %d components decide to 1e-6 (worst relative error "
          "%.2e), %d do not (worst (|adjoint - R| - 1e-6 |R|) / u = %.2f); norm-wise per group: %s"
          % (label, (sigma / np.abs(L0)).max(), n_res, worst_res, n_unres, worst_unres,
             ", ".join("%s %.1e" % kv for kv in worst_block.items())), flush=True)
    assert n_res >= min_decided * (n_res + n_unres)
    if block_tol is not None:
        for bname in ("dQ0", "dV0", "dm0"):
            assert worst_block[bname] < block_tol, (bname, worst_block[bname])


def adjoint_columns(g, idx):
    n = len(idx)
    return np.concatenate([g[0][idx].reshape(n, 24), g[1][idx].reshape(n, 24), g[2][idx], g[3][idx][:, None]],
                          axis=1)


@pytest.mark.parametrize("packing,scheme,every", [("auto", "dkd", 100), ("auto", "dkd", 1000), ("split", "dkd", 64),
                                                  ("pair", "kdk", 100), ("serial", "dkd", 1000),
                                                  ("auto", "saba2", 50)])
def test_gradients_match_central_differences_on_every_input(packing, scheme, every):
    """8 eight-planet systems, 400 steps: every one of the 57 inputs of every
    system by central differences with h = 1e-7 relative (the adjoint
    configuration's step and, in two cases, its checkpoint interval of 1000
    steps).  Even at 400 steps the loss's rounding noise (~1e-15 of itself)
    over h keeps central differences from deciding the components of the
    inner planets to 1e-6 (a third decide); every component agrees within
    the difference's own uncertainty, and each group norm-wise to 1e-6."""
    s = inputs.make_systems(8, 53, n_planets=8)
    n_steps = 400
    e = Ensemble.from_systems(s, packing=packing, scheme=scheme)
    e.forward_ckpt(n_steps, every)
    QT, VT = e.state()
    g = [x.cpu().numpy() for x in e.adjoint(2 * QT, torch.zeros_like(VT))]
    e.close()
    col = adjoint_columns(g, np.arange(s.S))
    central_difference_check(s, n_steps, col, "400 steps %s/%s/K=%d" % (packing, scheme, every), 0.2, 1e-6,
                             packing=packing, scheme=scheme)


def test_full_length_gradients_match_central_differences():
    """The adjoint configuration's sampled systems at 1e5 steps (checkpoints
    every 1000).  After 1e5 steps the loss carries rounding noise of ~1e-15
    to 1e-14 of itself, while a 1e-7 relative step moves it by ~1e-7 of
    itself (positions, velocities) down to ~1e-11 (the mass of a light
    planet): only a part of the components can be decided to 1e-6 by central
    differences at this length (at 400 steps above, nearly all), and the
    element-wise comparison with the oracle tangent is the exact check."""
    s, _, g = full_length_adjoint("auto")
    sub = s.subset(SAMPLED)
    central_difference_check(sub, FULL_STEPS, adjoint_columns(g, SAMPLED), "1e5 steps", 0.2)
