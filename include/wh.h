/*
 * wh.h -- C interface of the MI355X Wisdom-Holman ensemble integrator.
 *
 * The library integrates many independent planetary systems (a star of mass
 * m0 and 1..8 planets each) with the Wisdom-Holman map in democratic
 * heliocentric coordinates of the WHFast512 paper (Javaheri, Rein & Tamayo
 * 2023, Sec. 3): per step a Kepler drift of every planet about the star
 * (Sec. 3.2), the planet-planet interaction kick (Sec. 3.3, acceleration
 * equation), the jump step (Sec. 3.4, jump equation) and an optional 1/r^2
 * GR kick (Sec. 3.3, final paragraphs), composed drift-kick-drift as in
 * Sec. 3.1 with combined drifts and "keep unsynchronized" output (Sec. 3.5).
 * Options (wh_config): kick-drift-kick and SABA_n compositions, Jacobi
 * coordinates, lane packings; besides the integration the library evaluates
 * energies and osculating elements, runs reverse mode (wh_forward_ckpt,
 * wh_adjoint_n) and the Kepler-solver envelope explorer.
 *
 * Conventions (Sec. 3.5 assumptions):
 *   - G = 1; masses constant; dt fixed per system and > 0 (integrate
 *     backwards by flipping the velocities).  Changing dt or masses needs a
 *     new wh_init.
 *   - Q = planet position relative to the star (heliocentric), V = P/m =
 *     barycentric velocity.  All floating point is IEEE binary64.
 *
 * Memory: every device buffer (inputs, outputs, workspace, tape) is owned by
 * the caller; the library never allocates device memory.  Host pointers are
 * marked "host"; every other pointer is a device pointer.  Array layouts:
 *   m0[S], dt[S], E[S], flags[S]               one value per system
 *   m[S*8]            planet p of system s at  m[s*8 + p]
 *   Q[S*8*3], V[...]  component c at          Q[(s*8 + p)*3 + c]
 * Entries of planets p >= n_planets[s] are ignored on input and left
 * untouched on output.
 *
 * Streams: every call is enqueued on `stream` and returns once enqueued;
 * buffers must stay valid until the stream has passed the call.  One context
 * is driven by one stream at a time; calls that overlap on one context race.
 *
 * Errors: calls return WH_OK (0) or a negative code; they validate their
 * arguments before enqueueing anything and never abort.  wh_last_error()
 * gives a message for the calling thread's last failure.  Numerical trouble
 * inside a system (non-finite state, an unbound orbit, a Kepler step outside
 * the validated range) is not an error: it sets sticky per-system flag bits
 * and the integration continues without branching.
 */
#ifndef WH_H
#define WH_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wh_ctx wh_ctx;
typedef int32_t wh_status;

enum {
  WH_OK = 0,
  WH_EINVAL = -1,     /* invalid argument (sizes, dt <= 0, G != 1, null pointer) */
  WH_EWORKSPACE = -2, /* workspace or tape smaller than required */
  WH_EHIP = -3,       /* HIP runtime error (text in wh_last_error) */
  WH_ESTATE = -4      /* call not valid in the context's current state */
};

/* Step composition (Sec. 3.1). */
enum {
  WH_DKD = 0,   /* K(dt/2) J(dt/2) I(dt) J(dt/2) K(dt/2): the paper's step */
  WH_KDK = 1,   /* I(dt/2) J(dt/2) K(dt) J(dt/2) I(dt/2)  (I includes GR) */
  /* Higher-order splittings (Sec. 3.1 mentions them; the paper uses none):
   * SABA_n of Laskar & Robutel (2001), K(c_1 dt) B(d_1 dt) K(c_2 dt) ...
   * B(d_n dt) K(c_{n+1} dt) with Gauss-Legendre coefficients and B the whole
   * perturbation (I and J together in DHC, the Jacobi kick in Jacobi
   * coordinates); error O(eps dt^(2n) + eps^2 dt^2), n drifts' and kicks'
   * cost per step.  GR only in Jacobi coordinates (in DHC its flow does not
   * commute with the jump's); not in reverse mode. */
  WH_SABA2 = 2,
  WH_SABA3 = 3,
  WH_SABA4 = 4
};

/* Lane packings of systems onto 64-lane wavefronts. */
enum {
  WH_PACK_AUTO = -1, /* WH_PACK_POW2 (an autotuner may pass an explicit id) */
  WH_PACK_POW2 = 0,  /* one group of 1/2/4/8 lanes per system (next power of 2 >= N) */
  WH_PACK_G8 = 1,    /* one 8-lane group per system whatever N */
  WH_PACK_PAIR = 2,  /* two planets per lane: a group of 1/2/4 lanes per system (2 lanes per 3-4 planets,
                        4 per 5-8); DHC only */
  WH_PACK_SPLIT = 3, /* two lanes per planet: a 16-lane group per system whatever N, the interaction kick
                        divided between the two copies of each planet (for ensembles with fewer
                        wavefronts than the GPU has SIMDs); DHC only */
  WH_PACK_SERIAL = 4, /* one lane per system: the storage of WH_PACK_G8, but one thread runs all planets of
                         a system (every pair visited once, no cross-lane traffic; 64 systems per wave, for
                         very large ensembles); DHC only */
  WH_PACK_MIXED = 5   /* WH_PACK_POW2, except that a 5-planet system shares an 8-lane group with a 3- or
                         2-planet one and a 6-planet system with a 2-planet one (the larger system in the
                         group's first lanes): the sums and the interaction kick of a group keep the two
                         systems apart, and a non-finite state in one never reaches the other.  DHC with
                         WH_DKD or WH_KDK, the DPP exchange and kepler_counts 0; forward only (reverse
                         mode: WH_ESTATE) */
};

/* Partner exchange of the interaction kick inside a lane group. */
enum {
  WH_EXCH_AUTO = 0, /* WH_EXCH_DPP */
  WH_EXCH_LDS = 1,  /* third-law rotation rounds through the LDS crossbar (ds_bpermute) */
  WH_EXCH_DPP = 2   /* DPP row moves only (one more pair round for 8-lane groups) */
};

/* Coordinates of the splitting. */
enum {
  WH_COORDS_DHC = 0,    /* democratic heliocentric (the paper's, Sec. 3) */
  WH_COORDS_JACOBI = 1  /* Jacobi coordinates (Wisdom & Holman 1991; the paper names them for systems of
                           two or four planets, Sec. 3.5 footnote and Sec. 6): planets in lane order, each
                           drifting about the centre of mass of the star and the planets inside it with
                           mu = G (m0 + m_1 + ... + m_i), and a kick of the remaining Hamiltonian; no jump.
                           Inputs and outputs stay in the DHC layout; GR (the same potential) enters
                           the kick; one planet per lane (WH_PACK_POW2 or WH_PACK_G8). */
};

/* Sticky per-system status bits. */
enum {
  WH_F_NONFINITE = 1u,  /* a position or velocity became NaN or infinite */
  WH_F_HYPERBOLIC = 2u, /* a Kepler drift saw an unbound orbit (beta <= 0) */
  WH_F_ZMAX = 4u        /* a Kepler drift's Stumpff argument exceeded z_max */
};

typedef struct {
  int32_t n_systems;   /* S >= 1; the packing may use at most 2^27 lane slots (16.7 million
                          eight-planet systems with one planet per lane or WH_PACK_SERIAL,
                          8.4 million with WH_PACK_SPLIT, 33.5 million with WH_PACK_PAIR) */
  double G;            /* must be 1.0 (Sec. 3.5) */
  double gr_c;         /* speed of light for the GR kick; <= 0 turns GR off */
  int32_t scheme;      /* WH_DKD, WH_KDK or WH_SABA2..4 */
  int32_t packing;     /* WH_PACK_* */
  int32_t block_waves; /* wavefronts per workgroup: 1, 2 or 4 (0 = 1) */
  int32_t chunk_steps; /* steps per kernel launch (0 = 4096) */
  int32_t graph_launches; /* launches per replayed HIP graph (0 = 8, < 0 = no graph) */
  double z_max;        /* WH_F_ZMAX threshold on the Stumpff argument (0 = 1.0) */
  int32_t exchange;    /* WH_EXCH_* */
  int32_t coords;      /* WH_COORDS_* */
  int32_t balance;     /* 1: balanced launch windows.  When the packing has more wavefronts than the GPU
                          can hold at its occupancy, one launch per chunk leaves some SIMDs a wave more
                          than others; instead each chunk of chunk_steps steps runs as a sequence of
                          launches ("windows") of at most (resident waves per SIMD) x (SIMDs)
                          wavefronts, each wave given a share of the chunk's steps in inverse proportion
                          to its per-step cost (group size), so that every SIMD carries about the same
                          work in every window.  Results are bitwise those of balance = 0 (a launch
                          boundary only stores and reloads the state).  WH_PACK_SERIAL ignores it.
                          0: one launch per chunk. */
  int32_t kepler_counts; /* iteration counts of the step's Kepler solve (Sec. 3.2, App. A): 0 the paper's
                            (2 Halley steps with 4 series terms, then 2 Newton steps with 8); 1 one Halley
                            step with 3 terms, then the same 2 Newton steps -- the cheapest set the envelope
                            explorer finds within App. A's accuracy bound for eccentricities up to 0.6 at
                            App. A's step (validate it on a batch first: autotune does).  Set 1: DHC
                            drift-kick-drift or kick-drift-kick with the DPP exchange in the POW2, G8, PAIR
                            and SPLIT packings, forward stepping only (no reverse mode: WH_ESTATE); the
                            synchronized outputs' closing half drift keeps the paper's counts. */
  int32_t corrector;   /* symplectic corrector stages (Wisdom, Holman & Touma 1996) of the Jacobi map: 0 none,
                          n = 1..3 a corrector of order 2n + 1.  The integration runs in mapping coordinates:
                          wh_init applies the inverse change of variables to the input state and every output
                          (state, energy, elements, angular momentum) applies the change to its synchronized
                          copy, removing the map's first-order-in-mass error terms through dt^(2n).  Each stage
                          is a kick carried by the Kepler flow: drift a dt, kick b dt, drift -2a dt, kick -b dt,
                          drift a dt, with a_i = i/(2n) and b_i from the conditions on the series of
                          (x/2)/sinh(x/2) (drift-kick-drift) or (x/2)coth(x/2) (kick-drift-kick).  Needs
                          WH_COORDS_JACOBI with WH_DKD or WH_KDK.  Reverse mode differentiates through both
                          changes of variables (the input's inverse and the output's). */
} wh_config;

/* Fills *cfg with the defaults above (DKD, no GR, auto packing, DHC). */
void wh_config_default(wh_config* cfg, int32_t n_systems);

/* Device workspace the context needs for this configuration and these planet
 * counts (n_planets: host array [S], each in 1..8).  0 on invalid input. */
size_t wh_workspace_bytes(const wh_config* cfg, const int32_t* n_planets);

/* Create a context and load the initial state.  n_planets is host memory;
 * m0, m, Q, V, dt are device arrays in the layout above; workspace is
 * caller-owned device memory of at least wh_workspace_bytes(), 256-byte
 * aligned, kept alive until wh_destroy.  The state starts synchronized. */
wh_status wh_init(wh_ctx** out, const wh_config* cfg, const int32_t* n_planets, const double* m0,
                  const double* m, const double* Q, const double* V, const double* dt, void* workspace,
                  size_t workspace_bytes, hipStream_t stream);

/* Advance every system by n_steps >= 0 steps of the fused persistent kernel.
 * Drifts are combined across steps (Sec. 3.1, 3.5): the stored state stays
 * unsynchronized until a reader synchronizes a copy of it. */
wh_status wh_step_n(wh_ctx* ctx, int64_t n_steps, hipStream_t stream);

/* Reference path with the same device math: one 8-lane group per system,
 * one launch per planet count per step, state read from and written to
 * device memory every step, no graph.  Results equal wh_step_n's up to
 * rounding order. */
wh_status wh_step_n_plain(wh_ctx* ctx, int64_t n_steps, hipStream_t stream);

/* Synchronized copy of the state (Q_out, V_out: device [S*8*3]); the
 * context keeps integrating the unsynchronized state (Sec. 3.5). */
wh_status wh_get_state(wh_ctx* ctx, double* Q_out, double* V_out, hipStream_t stream);

/* Energy of the synchronized copy, E_out device [S]:
 *   sum_i [m_i V_i^2/2 - m0 m_i/|Q_i|] - sum_{i<j} m_i m_j/|Q_i - Q_j|
 *   + |sum_i m_i V_i|^2/(2 m0)  [- sum_i 3 m0^2 m_i/(c^2 |Q_i|^2) with GR]
 * (the Hamiltonian of Sec. 3.1 without the constant barycentre term). */
wh_status wh_energy(wh_ctx* ctx, double* E_out, hipStream_t stream);

/* Osculating heliocentric semi-major axis and eccentricity of every planet
 * of the synchronized copy (a_out, e_out: device [S*8]), for the two-body
 * problem of star and planet (mu = G (m0 + m_i)) with the heliocentric
 * velocity u_i = V_i + sum_j m_j V_j / m0.  The paper's Sec. 5 declares a
 * Solar-System run unstable once Mercury's eccentricity exceeds 0.65.
 * a < 0 marks an unbound orbit. */
wh_status wh_elements(wh_ctx* ctx, double* a_out, double* e_out, hipStream_t stream);

/* Total angular momentum L = sum_i Q_i x m_i V_i of every system's
 * synchronized copy (L_out: device [S*3]).  In democratic heliocentric
 * coordinates with barycentric momenta this is the angular momentum of the
 * whole system about its barycentre; the drift, the jump, the interaction
 * kick and the GR kick of Sec. 3 each conserve it exactly, so its change
 * measures rounding alone. */
wh_status wh_angular_momentum(wh_ctx* ctx, double* L_out, hipStream_t stream);

/* Copy the sticky WH_F_* bits (flags_out: device uint32 [S]). */
wh_status wh_status_flags(wh_ctx* ctx, uint32_t* flags_out, hipStream_t stream);

/* Steps taken so far by every system (identical for all systems). */
int64_t wh_steps_done(const wh_ctx* ctx);

/* ---- bitwise snapshots of the unsynchronized state ----------------------
 * wh_save_state copies the context's internal state -- the unsynchronized,
 * compensated state of every lane slot (Sec. 3.5: integration continues from
 * it, outputs only synchronize copies), the sticky flags, the per-system
 * synchronized markers and the step count -- into a caller-owned, 256-byte
 * aligned device buffer of wh_state_bytes() bytes.  wh_restore_state loads
 * such a snapshot into a context created for the same batch (same planet
 * counts and order), packing, scheme, coordinates and GR setting (WH_ESTATE
 * otherwise, WH_EINVAL for a buffer that is not a snapshot): stepping on
 * from it gives bitwise the results the saved context would have given.  The
 * buffer may be copied to the host and back in between (checkpoint files).
 * Restore reads the snapshot's header back to the host (a stream
 * synchronization) and drops any recorded reverse-mode tape. */
size_t wh_state_bytes(const wh_ctx* ctx);
wh_status wh_save_state(wh_ctx* ctx, void* dst, size_t bytes, hipStream_t stream);
wh_status wh_restore_state(wh_ctx* ctx, const void* src, size_t bytes, hipStream_t stream);

/* Launches per chunk of wh_step_n: 1 without balanced windows (or when the
 * packing fits the GPU's resident wavefronts), else the number of windows;
 * *slots (may be null) receives the wavefronts per window the plan assumed
 * resident (0 without a plan).  -1 for a null context.  Host-only query. */
int32_t wh_launch_windows(const wh_ctx* ctx, int32_t* slots);

/* ---- reverse mode ------------------------------------------------------
 * Gradients of a loss of the synchronized final state with respect to the
 * initial synchronized state (Q0, V0), the planet masses and the star mass.
 * Usage: wh_init; wh_forward_ckpt(n, K, tape) (advances the context like
 * wh_step_n and stores a checkpoint every K steps in the tape);
 * wh_adjoint_n(tape, dL/dQ_T, dL/dV_T) -> dL/dQ_0, dL/dV_0, dL/dm, dL/dm0.
 * The adjoint re-runs each K-step segment from its checkpoint, records the
 * segment's per-step states and converged Kepler anomalies in the tape, and
 * sweeps it backwards with the hand-written transposed Jacobian of every
 * sub-step (the Kepler drift through the implicit function theorem); the
 * tape holds two segment buffers, so that segment k - 1 is recorded while
 * segment k is swept.  wh_tape_bytes gives the size: 96 B per lane slot per
 * checkpoint plus 2 x 80 B per lane slot and step of a segment (2 x n x 80 B
 * for SABA_n, which records its n drift-kick units; ckpt_every x n must not
 * exceed 2^30).  Every scheme, packing and coordinate system: with WH_KDK a
 * step of the tape is the kick block followed by the drift, and the
 * synchronized output's pending half kick is differentiated too; with SABA_n
 * the pending drift K(c_1 dt); in Jacobi coordinates the gradients are those
 * of the DHC inputs and outputs, through both coordinate transforms. */
size_t wh_tape_bytes(const wh_ctx* ctx, int64_t n_steps, int64_t ckpt_every);
wh_status wh_forward_ckpt(wh_ctx* ctx, int64_t n_steps, int64_t ckpt_every, void* tape, size_t tape_bytes,
                          hipStream_t stream);
wh_status wh_adjoint_n(wh_ctx* ctx, void* tape, size_t tape_bytes, const double* gQ_T, const double* gV_T,
                       double* gQ_0, double* gV_0, double* gm, double* gm0, hipStream_t stream);

/* ---- Kepler-solver envelope (Sec. 3.2, Fig. 1; App. A) ------------------
 * Advances n massless test particles, each about its own star (mu[i] = G m0)
 * with its own step tau[i] > 0, through n_steps Kepler drifts of the fixed
 * solver with n_halley Halley steps (terms_halley series terms) then
 * n_newton Newton steps (terms_newton terms), and writes the relative change
 * of the osculating semi-major axis, a_err[i] = (a_end - a_0) / a_0 with
 * a = 1 / (2/|Q| - |V|^2/mu) (zero for the exact flow; NaN where the solve
 * broke down).  The integrator's own solver is n_halley = 2, n_newton = 2,
 * terms 4 and 8.  With n_newton = 0 the series are evaluated once more at
 * the last Halley iterate.
 *   Q, V: device [n*3] initial positions / velocities, Q[i*3 + c];
 *   mu, tau: device [n];  a_err: device [n] (required);
 *   Q_out, V_out: device [n*3] final state, both or neither (may alias Q, V);
 *   zmax_out: device [n] or null, largest Stumpff argument beta X^2 of a
 *   final evaluation (the series assume it small).
 * Limits: 0 <= n_halley, n_newton <= 8, n_halley + n_newton >= 1, series
 * lengths 1..14; otherwise WH_EINVAL.  n = 0 enqueues nothing. */
wh_status wh_kepler_envelope(int64_t n, const double* Q, const double* V, const double* mu, const double* tau,
                             int64_t n_steps, int32_t n_halley, int32_t n_newton, int32_t terms_halley,
                             int32_t terms_newton, double* Q_out, double* V_out, double* a_err, double* zmax_out,
                             hipStream_t stream);

/* ---- integration without device allocation -----------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one call
 * that does what wh_init + wh_step_n(n_steps) + wh_get_state + wh_destroy do,
 * with the context's workspace in a fixed device array inside the library
 * instead of a caller buffer, and direct launches instead of a replayed HIP
 * graph (cfg->graph_launches is ignored); results are bitwise those of that
 * sequence with the same configuration.  It calls no hipMalloc, hipFree or
 * other allocating routine.
 *   cfg, n_planets (host [S]): as for wh_init; m0, m, Q, V, dt: device
 *   inputs in the layout above (read during the call's kernels, so they must
 *   stay valid until the stream has passed it); Q_out, V_out: device
 *   [S*8*3], the synchronized state after n_steps >= 0 steps.
 * The array holds WH_NOALLOC_MAX_BYTES per GPU (allocated when the library's
 * code object is loaded on that GPU, kept until the process ends); a batch
 * whose wh_workspace_bytes() exceeds it is rejected with WH_EWORKSPACE before
 * anything is enqueued (16 MiB: about 16000 eight-planet systems with one
 * planet per lane, 8000 with WH_PACK_SPLIT).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (different streams or
 * threads without ordering between them) race; calls on one stream are
 * ordered and safe.  Like wh_init it reads the masses and steps back to the
 * host to validate them (a stream synchronization). */
#define WH_NOALLOC_MAX_BYTES (16u << 20)
wh_status wh_integrate_noalloc(const wh_config* cfg, const int32_t* n_planets, const double* m0, const double* m,
                               const double* Q, const double* V, const double* dt, int64_t n_steps, double* Q_out,
                               double* V_out, hipStream_t stream);

/* Message of the calling thread's last failed call ("" if none). */
const char* wh_last_error(void);

/* Free the host context (the caller frees the workspace). */
void wh_destroy(wh_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* WH_H */
