// MI355X (gfx950) Wisdom-Holman ensemble integrator: kernels and the C ABI
// declared in include/wh.h.
//
// Hot path: one persistent kernel advances every system by a chunk of steps
// with the state held in VGPRs.  In the default layout each lane carries one
// planet, each aligned group of G lanes one system, each 64-lane wavefront
// 64/G systems; further layouts put two planets on a lane (wh_pair.h), one
// planet on two lanes (wh_split.h) or a whole system on one lane (the serial
// step below).  The
// step is the drift-kick-drift composition of the WHFast512 paper (Sec. 3.1)
// with the drifts of consecutive steps merged and, without GR, the two half
// jumps merged (they commute with the interaction kick then).  Output reads
// synchronize a register copy (Sec. 3.5, "keep unsynchronized").
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "wh.h"
#include "wh_device.h"
#include "wh_adjoint.h"
#include "wh_pair.h"
#include "wh_split.h"
#include "wh_step.h"
#include "wh_host.h"

using namespace wh;
using namespace wh_host;

// ===========================================================================
// Device side
// ===========================================================================
namespace {

// The kernel parameters, lane state, drift and the pair layout's kick and
// step are in wh_step.h; the pair step kernel itself in wh_pair_step.hip.

// Partner exchange of the interaction kick: EXCH 0 = rotation rounds over the
// LDS crossbar (ds_bpermute), EXCH 1 = DPP rounds.
template <int G, int EXCH> struct Exch;
template <int G> struct Exch<G, 0> {
  GroupTopo<G> t;
  __device__ __forceinline__ void init(int lane, double m) { make_topo<G>(t, lane, m); }
  __device__ __forceinline__ void momentum(double m, double vx, double vy, double vz, double& sx, double& sy,
                                           double& sz) const {
    group_momentum<G>(m, vx, vy, vz, sx, sy, sz);
  }
  __device__ __forceinline__ void accel(double qx, double qy, double qz, double m, double& ax, double& ay,
                                        double& az) const {
    interaction_accel<G>(t, qx, qy, qz, m, ax, ay, az);
  }
};
template <int G> struct Exch<G, 1> {
  DppMass t;
  __device__ __forceinline__ void init(int, double m) { make_dpp_mass<G>(t, m); }
  __device__ __forceinline__ void momentum(double m, double vx, double vy, double vz, double& sx, double& sy,
                                           double& sz) const {
    group_momentum<G>(m, vx, vy, vz, sx, sy, sz);
  }
  __device__ __forceinline__ void accel(double qx, double qy, double qz, double m, double& ax, double& ay,
                                        double& az) const {
    interaction_accel_dpp<G>(t, qx, qy, qz, m, ax, ay, az);
  }
};
// The split layout (two lanes per planet, wh_split.h) has one schedule, all
// DPP, whatever the exchange option.
struct ExchSplit {
  SplitMass t;
  __device__ __forceinline__ void init(int lane, double m) { t = make_split_mass(lane, m); }
  __device__ __forceinline__ void momentum(double m, double vx, double vy, double vz, double& sx, double& sy,
                                           double& sz) const {
    group_momentum<G_SPLIT>(m, vx, vy, vz, sx, sy, sz);
  }
  __device__ __forceinline__ void accel(double qx, double qy, double qz, double m, double& ax, double& ay,
                                        double& az) const {
    accel_split(t, qx, qy, qz, m, ax, ay, az);
  }
};
template <> struct Exch<G_SPLIT, 0> : ExchSplit {};
template <> struct Exch<G_SPLIT, 1> : ExchSplit {};

// Two systems in one 8-lane group (the mixed packing): system a in the
// group's first lanes, system b after it (padding lanes belong to b).  The
// DPP rounds of the one-system kick run over all eight lanes; a pair across
// the two systems gets zero partner mass and zero reaction weight, its
// squared distance is kept above 1e-200 (planets of two systems may
// coincide) and every position is taken finite, so that neither system's
// planets feel the other's and a non-finite state stays in its own system.
// Sums over the group run twice, once per system, each with the other
// system's lanes replaced by zeros (a select, which does not carry a NaN
// across).  System a meets the partners of its own 8-lane group in the same
// order; with the selects the compiler's contractions differ, so its results
// agree with that group's to rounding, not bit for bit.
struct ExchMixed {
  DppMass t;          // partner masses of the rounds, zero across the systems
  double r1, r3;      // own mass for the reactions of rounds 1 and 3, zero across
  bool a;             // the lane belongs to the group's first system
  // pl: the lane's planet index (-1: padding); p: its lane in the group
  __device__ __forceinline__ void init_mixed(double m, int pl, int p) {
    a = pl == p;
    make_dpp_mass<8>(t, m);
    const int s = a ? 1 : 0;
    const int s0 = dpp_i<QP_NEXT>(s), s1 = dpp_i<DPP_XOR2>(s), sm = dpp_i<DPP_HALF_MIRROR>(s);
    const int s2 = dpp_i<QP_R3>(sm), s3 = dpp_i<QP_R4>(sm), s4 = dpp_i<QP_R5>(sm);
    t.m[0] = s0 == s ? t.m[0] : 0.0;
    t.m[1] = s1 == s ? t.m[1] : 0.0;
    t.m[2] = s2 == s ? t.m[2] : 0.0;
    t.m[3] = s3 == s ? t.m[3] : 0.0;
    t.m[4] = s4 == s ? t.m[4] : 0.0;
    r1 = s0 == s ? m : 0.0;
    r3 = s2 == s ? m : 0.0;
  }
  __device__ __forceinline__ double sum(double v) const {
    const double sa = group_sum<8>(a ? v : 0.0);
    const double sb = group_sum<8>(a ? 0.0 : v);
    return a ? sa : sb;
  }
  __device__ __forceinline__ int any(int f) const {
    const int fa = group_or<8>(a ? f : 0);
    const int fb = group_or<8>(a ? 0 : f);
    return a ? fa : fb;
  }
  __device__ __forceinline__ void momentum(double m, double vx, double vy, double vz, double& sx, double& sy,
                                           double& sz) const {
    sx = sum(m * vx);
    sy = sum(m * vy);
    sz = sum(m * vz);
  }
  static __device__ __forceinline__ double pair(double qx, double qy, double qz, double px, double py, double pz,
                                                double mj, double& ax, double& ay, double& az, double& dx, double& dy,
                                                double& dz) {
    dx = qx - px; dy = qy - py; dz = qz - pz;
    const double r2 = fmax(fma(dx, dx, fma(dy, dy, dz * dz)), 1.0e-200);
    const double ir3 = rsqrt3_full(r2);
    const double w = mj * ir3;
    ax = fma(-w, dx, ax);
    ay = fma(-w, dy, ay);
    az = fma(-w, dz, az);
    return ir3;
  }
  // the rounds of interaction_accel_dpp<8>
  __device__ __forceinline__ void accel(double qx, double qy, double qz, double, double& ax, double& ay,
                                        double& az) const {
    qx = __builtin_isfinite(qx) ? qx : 0.0;
    qy = __builtin_isfinite(qy) ? qy : 0.0;
    qz = __builtin_isfinite(qz) ? qz : 0.0;
    ax = 0.0; ay = 0.0; az = 0.0;
    double dx, dy, dz;
    double ir3 = pair(qx, qy, qz, dpp<QP_NEXT>(qx), dpp<QP_NEXT>(qy), dpp<QP_NEXT>(qz), t.m[0], ax, ay, az, dx, dy,
                      dz);
    double wi = r1 * ir3;
    ax += dpp<QP_PREV>(wi * dx);
    ay += dpp<QP_PREV>(wi * dy);
    az += dpp<QP_PREV>(wi * dz);
    pair(qx, qy, qz, dpp<DPP_XOR2>(qx), dpp<DPP_XOR2>(qy), dpp<DPP_XOR2>(qz), t.m[1], ax, ay, az, dx, dy, dz);
    const double mx = dpp<DPP_HALF_MIRROR>(qx), my = dpp<DPP_HALF_MIRROR>(qy), mz = dpp<DPP_HALF_MIRROR>(qz);
    ir3 = pair(qx, qy, qz, dpp<QP_R3>(mx), dpp<QP_R3>(my), dpp<QP_R3>(mz), t.m[2], ax, ay, az, dx, dy, dz);
    wi = r3 * ir3;
    ax += dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(wi * dx));
    ay += dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(wi * dy));
    az += dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(wi * dz));
    pair(qx, qy, qz, dpp<QP_R4>(mx), dpp<QP_R4>(my), dpp<QP_R4>(mz), t.m[3], ax, ay, az, dx, dy, dz);
    pair(qx, qy, qz, dpp<QP_R5>(mx), dpp<QP_R5>(my), dpp<QP_R5>(mz), t.m[4], ax, ay, az, dx, dy, dz);
  }
};
template <> struct Exch<8, 2> : ExchMixed {};

// Kick block of the loop on the compensated state.  With GR:
// J(ta) [I + GR](ti) J(tc); without GR the jumps commute with I and merge:
// I(ti) J(ta + tc).  Increments go to the low parts; the state is
// renormalized at the end.  (vkx, vky, vkz) receive the velocity after the
// kick (kept by the adjoint).  kj = tau/m0 for the jumps (Sec. 3.4).
template <int G, bool GR, int EXCH>
__device__ __forceinline__ void kick_block(Lane& L, const Exch<G, EXCH>& ex, double inv_m0, double kg, double ta,
                                           double ti, double tc, double& vkx, double& vky, double& vkz) {
  double ax, ay, az, sx, sy, sz;
  if (GR) {
    ex.momentum(L.m, L.vx, L.vy, L.vz, sx, sy, sz);
    double k1 = ta * inv_m0;
    double dqx = k1 * sx, dqy = k1 * sy, dqz = k1 * sz;
    L.cqx += dqx; L.cqy += dqy; L.cqz += dqz;
    double qx = L.qx + dqx, qy = L.qy + dqy, qz = L.qz + dqz;
    ex.accel(qx, qy, qz, L.m, ax, ay, az);
    double gx, gy, gz;
    gr_accel(qx, qy, qz, kg, gx, gy, gz);
    ax += gx; ay += gy; az += gz;
  } else {
    ex.accel(L.qx, L.qy, L.qz, L.m, ax, ay, az);
  }
  double dvx = ti * ax, dvy = ti * ay, dvz = ti * az;
  L.cvx += dvx; L.cvy += dvy; L.cvz += dvz;
  vkx = L.vx + dvx; vky = L.vy + dvy; vkz = L.vz + dvz;
  ex.momentum(L.m, vkx, vky, vkz, sx, sy, sz);
  double k2 = (GR ? tc : ta + tc) * inv_m0;
  L.cqx += k2 * sx; L.cqy += k2 * sy; L.cqz += k2 * sz;
  renorm_all(L);
}

// ---------------------------------------------------------------------------
// Jacobi coordinates (Wisdom & Holman 1991; the paper names them for systems
// of two or four planets).  In a Jacobi context the state rows hold each
// planet's Jacobi position and velocity, measured from the centre of mass of
// the star and the planets inside it (planet order = lane order of the group).
// Per lane: M_i = m0 + m_1 + ... + m_i (the Kepler mass of its drift),
// 1/M_{i-1}, and w_i = m_i / M_i, with which heliocentric vectors follow as
//   h_i = x'_i + sum_{j<i} w_j x'_j.
struct JacConst {
  double Mi, inv_Mim1, w, ratio;   // ratio = m0 / M_{i-1} (exactly 1 for the innermost planet)
};
template <int G> __device__ __forceinline__ JacConst jac_const(double m0, double m, int p) {
  JacConst c;
  const double Mim1 = m0 + group_scan_excl<G>(m, p);
  c.Mi = Mim1 + m;
  c.inv_Mim1 = 1.0 / Mim1;
  c.w = m / c.Mi;
  c.ratio = m0 / Mim1;
  return c;
}
template <int G> __device__ __forceinline__ double jac_to_helio(double x, double w, int p) {
  return x + group_scan_excl<G>(w * x, p);
}

// Interaction kick over tau in Jacobi coordinates.  With H_I = U + sum_i G
// M_i m'_i / |x'_i| (m'_i = m_i M_{i-1} / M_i) the Jacobi acceleration is
//   a'_i = a_i - A_{i-1} + G M_i x'_i / |x'_i|^3,
// a_i the Newtonian acceleration of planet i, A_{i-1} that of the centre of
// mass of the bodies inside it; the mutual forces of those bodies cancel, so
//   M_{i-1} A_{i-1} = G m0 sum_{k>=i} m_k Q_k / |Q_k|^3 + sum_{j<i} m_j a^pl_j
// (Q heliocentric, a^pl the planet-planet part of a).  The star terms of
// planet i itself are grouped as
//   G M_i (x'_i / |x'_i|^3 - (m0 / M_{i-1}) Q_i / |Q_i|^3),
// which is exactly zero for the innermost planet (x'_1 = Q_1, M_0 = m0) and
// small for the others, leaving
//   a'_i = a^pl_i - (m0 / M_{i-1}) sum_{k>i} m_k Q_k / |Q_k|^3
//          - (1 / M_{i-1}) sum_{j<i} m_j a^pl_j + [the grouped star terms].
// Prefix and suffix sums run as group scans.  Increments go to the low
// parts, as in kick_block.
// a x - b y with both products rounded (no contraction), so that equal
// products cancel exactly.
__device__ __forceinline__ double diff_of_products(double a, double x, double b, double y) {
#pragma clang fp contract(off)
  return a * x - b * y;
}

//
// With GR (the potential of the DHC map, a function of the heliocentric
// positions) the force m_k gr_k on each planet and its reaction on the star
// add  gr_i + (sum_{k>=i} m_k gr_k) / M_{i-1}  to a'_i.
template <int G, int EXCH, bool GR = false>
__device__ __forceinline__ void kick_jacobi(Lane& L, const Exch<G, EXCH>& ex, const JacConst& jc, int p, double tau,
                                            double& vkx, double& vky, double& vkz, double kg = 0.0) {
  const double qx = jac_to_helio<G>(L.qx, jc.w, p);
  const double qy = jac_to_helio<G>(L.qy, jc.w, p);
  const double qz = jac_to_helio<G>(L.qz, jc.w, p);
  double ax, ay, az;
  ex.accel(qx, qy, qz, L.m, ax, ay, az);
  const double irq3 = rsqrt3_full(fma(qx, qx, fma(qy, qy, qz * qz)));
  const double kp = jc.Mi * rsqrt3_full(fma(L.qx, L.qx, fma(L.qy, L.qy, L.qz * L.qz)));
  const double kq = (jc.Mi * jc.ratio) * irq3;
  const double wq = L.m * irq3;
  const double cx = fma(jc.ratio, group_suffix_excl<G>(wq * qx, p), group_scan_excl<G>(L.m * ax, p) * jc.inv_Mim1);
  const double cy = fma(jc.ratio, group_suffix_excl<G>(wq * qy, p), group_scan_excl<G>(L.m * ay, p) * jc.inv_Mim1);
  const double cz = fma(jc.ratio, group_suffix_excl<G>(wq * qz, p), group_scan_excl<G>(L.m * az, p) * jc.inv_Mim1);
  double dvx = tau * ((ax - cx) + diff_of_products(kp, L.qx, kq, qx));
  double dvy = tau * ((ay - cy) + diff_of_products(kp, L.qy, kq, qy));
  double dvz = tau * ((az - cz) + diff_of_products(kp, L.qz, kq, qz));
  if (GR) {
    double gx, gy, gz;
    gr_accel(qx, qy, qz, kg, gx, gy, gz);
    dvx = fma(tau, fma(group_suffix_incl<G>(L.m * gx, p), jc.inv_Mim1, gx), dvx);
    dvy = fma(tau, fma(group_suffix_incl<G>(L.m * gy, p), jc.inv_Mim1, gy), dvy);
    dvz = fma(tau, fma(group_suffix_incl<G>(L.m * gz, p), jc.inv_Mim1, gz), dvz);
  }
  L.cvx += dvx; L.cvy += dvy; L.cvz += dvz;
  vkx = L.vx + dvx; vky = L.vy + dvy; vkz = L.vz + dvz;
  renorm_all(L);
}

// Jacobi state of the lane -> democratic heliocentric (Q heliocentric, V
// barycentric): heliocentric u from v', then V = u - sum_j m_j u_j / M_n.
template <int G> __device__ __forceinline__ void jacobi_to_dhc(Lane& L, int p) {
  const JacConst jc = jac_const<G>(L.m0, L.m, p);
  const double Mn = L.m0 + group_sum<G>(L.m);
  const double ux = jac_to_helio<G>(L.vx, jc.w, p);
  const double uy = jac_to_helio<G>(L.vy, jc.w, p);
  const double uz = jac_to_helio<G>(L.vz, jc.w, p);
  L.qx = jac_to_helio<G>(L.qx, jc.w, p);
  L.qy = jac_to_helio<G>(L.qy, jc.w, p);
  L.qz = jac_to_helio<G>(L.qz, jc.w, p);
  double px, py, pz;
  group_momentum<G>(L.m, ux, uy, uz, px, py, pz);
  L.vx = ux - px / Mn;
  L.vy = uy - py / Mn;
  L.vz = uz - pz / Mn;
}

// Democratic heliocentric -> Jacobi: u = V + sum_j m_j V_j / m0 (heliocentric
// velocity), x'_i = h_i - sum_{j<i} m_j h_j / M_{i-1} for h = Q and u.
template <int G> __device__ __forceinline__ void dhc_to_jacobi(Lane& L, int p) {
  const JacConst jc = jac_const<G>(L.m0, L.m, p);
  double px, py, pz;
  group_momentum<G>(L.m, L.vx, L.vy, L.vz, px, py, pz);
  const double ux = L.vx + px / L.m0, uy = L.vy + py / L.m0, uz = L.vz + pz / L.m0;
  L.vx = ux - group_scan_excl<G>(L.m * ux, p) * jc.inv_Mim1;
  L.vy = uy - group_scan_excl<G>(L.m * uy, p) * jc.inv_Mim1;
  L.vz = uz - group_scan_excl<G>(L.m * uz, p) * jc.inv_Mim1;
  const double qx = L.qx, qy = L.qy, qz = L.qz;
  L.qx = qx - group_scan_excl<G>(L.m * qx, p) * jc.inv_Mim1;
  L.qy = qy - group_scan_excl<G>(L.m * qy, p) * jc.inv_Mim1;
  L.qz = qz - group_scan_excl<G>(L.m * qz, p) * jc.inv_Mim1;
}

// n_steps steps for one lane.  The stored state X_u is "after a kick block,
// before its closing drift" (DKD) or "after a drift" (KDK):
//   DKD loop body: K(tk) . J(h) I(dt) J(h)        tk = h on the first step out
//                                                 of a synchronized state
//   KDK loop body: J(ta) I(ti) J(h) . K(dt)       (ta, ti) = (0, h) first,
//                                                 (h, dt) afterwards
// (operators in the order they act).  The state is kept as a double-double
// (rounded value + compensation); see drift and kick_block.
//
// In Jacobi coordinates (JAC) the loop bodies are K(tk) . I(dt) (DKD) and
// I(ti) . K(dt) (KDK), each planet drifting about mu = G M_i, with no jump.
template <int G, bool GR, int SCHEME, int EXCH, bool JAC = false, int KC = 0>
__device__ __forceinline__ void step_lane(const StepParams& p, Lane& L, int lane) {
  Exch<G, EXCH> ex;
  ex.init(lane, L.m);
  const double dt = L.dt;
  const double h = 0.5 * dt;
  const double inv_m0 = 1.0 / L.m0;
  const double kg = GR ? p.kgr * L.m0 * L.m0 : 0.0;
  KepDiag dg{0.0, 1.0e300};
  double vkx, vky, vkz;
  if constexpr (SCHEME == SCHEME_SABA) {
    // SABA_n: K(c_1 dt) B(d_1 dt) K(c_2 dt) ... B(d_n dt) K(c_{n+1} dt), the
    // closing drift merged with the next step's opening one (c_{n+1} = c_1).
    // B is the whole perturbation: I and J together in DHC (their flows
    // commute without GR), the Jacobi kick in Jacobi coordinates.
    const int pg = lane & (G - 1);
    JacConst jc{0.0, 0.0, 0.0, 0.0};
    if constexpr (JAC) jc = jac_const<G>(L.m0, L.m, pg);
    const double mu = JAC ? jc.Mi : L.m0;
    const double c1dt = p.sc[0] * dt;
    double tk = L.first ? c1dt : 2.0 * c1dt;
    for (int s = 0; s < p.n_steps; ++s) {
      drift(L, mu, tk, dg);
      tk = 2.0 * c1dt;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < p.saba_n) {
          const double tb = p.sd[k] * dt;
          if constexpr (JAC) kick_jacobi<G, EXCH, GR>(L, ex, jc, pg, tb, vkx, vky, vkz, kg);
          else kick_block<G, false, EXCH>(L, ex, inv_m0, 0.0, 0.5 * tb, tb, 0.5 * tb, vkx, vky, vkz);
          if (k + 1 < p.saba_n) drift(L, mu, p.sc[k + 1] * dt, dg);
        }
      }
    }
  } else if constexpr (JAC) {
    const int pg = lane & (G - 1);
    const JacConst jc = jac_const<G>(L.m0, L.m, pg);
    if (SCHEME == WH_DKD) {
      double tk = L.first ? h : dt;
      for (int s = 0; s < p.n_steps; ++s) {
        drift(L, jc.Mi, tk, dg);
        tk = dt;
        kick_jacobi<G, EXCH, GR>(L, ex, jc, pg, dt, vkx, vky, vkz, kg);
      }
    } else {
      double ti = L.first ? h : dt;
      for (int s = 0; s < p.n_steps; ++s) {
        kick_jacobi<G, EXCH, GR>(L, ex, jc, pg, ti, vkx, vky, vkz, kg);
        ti = dt;
        drift(L, jc.Mi, dt, dg);
      }
    }
  } else if (SCHEME == WH_DKD) {
    double tk = L.first ? h : dt;
    for (int s = 0; s < p.n_steps; ++s) {
      drift<KC>(L, L.m0, tk, dg);
      tk = dt;
      kick_block<G, GR, EXCH>(L, ex, inv_m0, kg, h, dt, h, vkx, vky, vkz);
    }
  } else {
    double ta = L.first ? 0.0 : h;
    double ti = L.first ? h : dt;
    for (int s = 0; s < p.n_steps; ++s) {
      kick_block<G, GR, EXCH>(L, ex, inv_m0, kg, ta, ti, h, vkx, vky, vkz);
      ta = h;
      ti = dt;
      drift<KC>(L, L.m0, dt, dg);
    }
  }
  int f = 0;
  if (L.pl >= 0) {
    bool fin = __builtin_isfinite(L.qx) && __builtin_isfinite(L.qy) && __builtin_isfinite(L.qz) &&
               __builtin_isfinite(L.vx) && __builtin_isfinite(L.vy) && __builtin_isfinite(L.vz);
    if (!fin) f |= WH_F_NONFINITE;
    if (!(dg.bmin > 0.0)) f |= WH_F_HYPERBOLIC;
    if (!(dg.zmax <= p.zlim)) f |= WH_F_ZMAX;
  }
  f = group_or<G>(f);
  if ((lane & (G - 1)) == 0 && L.sys >= 0) {
    p.flags[L.sys] |= (uint32_t)f;
    p.synced[L.sys] = 0;
  }
}

template <int G, bool GR, int SCHEME, int EXCH, bool JAC, int KC = 0>
__device__ void step_group(const StepParams& p, int slot, int lane) {
  Lane L = load_lane(p, slot);
  step_lane<G, GR, SCHEME, EXCH, JAC, KC>(p, L, lane);
  store_lane(p, slot, L);
}

// The compiler fits every variant in 128 VGPRs without spills, so four
// wavefronts stay resident per SIMD; a launch holds one wave per 64 lanes of
// the packed ensemble and each wave runs its whole chunk of steps.
template <bool GR, int SCHEME, int EXCH, bool JAC = false, int KC = 0>
__global__ __launch_bounds__(256) void k_step(StepParams p) {
  const int lane = threadIdx.x & 63;
  int wave;
  if (!launch_wave(p, (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), wave,
                   p.n_steps))
    return;
  const int slot = wave * 64 + lane;
  if (wave < p.w1) step_group<1, GR, SCHEME, EXCH, JAC, KC>(p, slot, lane);
  else if (wave < p.w2) step_group<2, GR, SCHEME, EXCH, JAC, KC>(p, slot, lane);
  else if (wave < p.w4) step_group<4, GR, SCHEME, EXCH, JAC, KC>(p, slot, lane);
  else step_group<8, GR, SCHEME, EXCH, JAC, KC>(p, slot, lane);
}


// ---------------------------------------------------------------------------
// The mixed packing (WH_PACK_MIXED): waves [wm, w8) hold two systems per
// 8-lane group (ExchMixed); the other waves are those of the one-planet
// layout.  DHC, drift-kick-drift or kick-drift-kick, the paper's Kepler
// counts.  Each system's flags are written from its planet 0.
template <bool GR, int SCHEME>
__device__ __forceinline__ void step_lane_mixed(const StepParams& p, Lane& L, int lane) {
  Exch<8, 2> ex;
  ex.init_mixed(L.m, L.pl, lane & 7);
  const double dt = L.dt;
  const double h = 0.5 * dt;
  const double inv_m0 = 1.0 / L.m0;
  const double kg = GR ? p.kgr * L.m0 * L.m0 : 0.0;
  KepDiag dg{0.0, 1.0e300};
  double vkx, vky, vkz;
  if (SCHEME == WH_DKD) {
    double tk = L.first ? h : dt;
    for (int s = 0; s < p.n_steps; ++s) {
      drift(L, L.m0, tk, dg);
      tk = dt;
      kick_block<8, GR, 2>(L, ex, inv_m0, kg, h, dt, h, vkx, vky, vkz);
    }
  } else {
    double ta = L.first ? 0.0 : h;
    double ti = L.first ? h : dt;
    for (int s = 0; s < p.n_steps; ++s) {
      kick_block<8, GR, 2>(L, ex, inv_m0, kg, ta, ti, h, vkx, vky, vkz);
      ta = h;
      ti = dt;
      drift(L, L.m0, dt, dg);
    }
  }
  const int f = ex.any(lane_flags(L, dg, p.zlim));
  if (L.pl == 0 && L.sys >= 0) {
    p.flags[L.sys] |= (uint32_t)f;
    p.synced[L.sys] = 0;
  }
}

template <bool GR, int SCHEME>
__global__ __launch_bounds__(256) void k_step_mixed(StepParams p) {
  const int lane = threadIdx.x & 63;
  int wave;
  if (!launch_wave(p, (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), wave, p.n_steps)) return;
  const int slot = wave * 64 + lane;
  if (wave < p.w1) step_group<1, GR, SCHEME, 1, false>(p, slot, lane);
  else if (wave < p.w2) step_group<2, GR, SCHEME, 1, false>(p, slot, lane);
  else if (wave < p.w4) step_group<4, GR, SCHEME, 1, false>(p, slot, lane);
  else if (wave < p.wm) step_group<8, GR, SCHEME, 1, false>(p, slot, lane);
  else {
    Lane L = load_lane(p, slot);
    step_lane_mixed<GR, SCHEME>(p, L, lane);
    store_lane(p, slot, L);
  }
}

// ---------------------------------------------------------------------------
// Two lanes per planet (WH_PACK_SPLIT, see wh_split.h): every wave holds four
// 16-lane groups, one system each, planet p in lanes 2p and 2p + 1.  The step
// is the one-planet step with the split interaction and the planet sums of
// that layout.
template <bool GR, int SCHEME, int KC = 0>
__global__ __launch_bounds__(256) void k_step_split(StepParams p) {
  const int lane = threadIdx.x & 63;
  int wave;
  if (!launch_wave(p, (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), wave,
                   p.n_steps))
    return;
  step_group<G_SPLIT, GR, SCHEME, 1, false, KC>(p, wave * 64 + lane, lane);
}

// ---------------------------------------------------------------------------
// One lane per system (WH_PACK_SERIAL): the storage is that of the G8 packing
// (planet p of a system in slot p of its 8-slot group, each planet count on
// waves of its own), but thread t runs the whole system of group t, as the
// paper runs one system per core.  The interaction kick visits each of the
// N(N-1)/2 pairs once and gives both planets their share (Sec. 3.3,
// acceleration equation), and the jump sums the momenta in the thread
// (Sec. 3.4): no cross-lane traffic, 64 systems per wave.  The body is
// compiled for each planet count NP and a wave runs the one for the largest
// count among its systems; slots beyond a system's own count are padding
// planets (zero mass, far orbits), integrated like the G8 layout's padding
// lanes.
//
// Registers hold the rounded state (Q, V, m) of every planet; the
// compensation terms live in LDS (a thread-private [6][8] block of doubles,
// lane-interleaved), since eight planets' full state would overflow the
// thread's registers.  Each planet's terms are read once per step: its kick
// increments, renormalization and next drift run back to back.
constexpr int SERIAL_LDS_PER_WAVE = 6 * 8 * 64;   // doubles

template <int NP> struct SerialState {
  double qx[NP], qy[NP], qz[NP], vx[NP], vy[NP], vz[NP], m[NP];
};

// element (k, i) of the thread's compensation block: k = 0..5 (Q then V), planet i
__device__ __forceinline__ double& comp_at(double* cl, int k, int i) { return cl[(k * 8 + i) * 64]; }

template <int NP> __device__ __forceinline__ Lane serial_get(const SerialState<NP>& S, double* cl, int i) {
  Lane L{};
  L.qx = S.qx[i]; L.qy = S.qy[i]; L.qz = S.qz[i];
  L.vx = S.vx[i]; L.vy = S.vy[i]; L.vz = S.vz[i];
  L.m = S.m[i];
  L.cqx = comp_at(cl, 0, i); L.cqy = comp_at(cl, 1, i); L.cqz = comp_at(cl, 2, i);
  L.cvx = comp_at(cl, 3, i); L.cvy = comp_at(cl, 4, i); L.cvz = comp_at(cl, 5, i);
  return L;
}

template <int NP> __device__ __forceinline__ void serial_put(SerialState<NP>& S, double* cl, int i, const Lane& L) {
  S.qx[i] = L.qx; S.qy[i] = L.qy; S.qz[i] = L.qz;
  S.vx[i] = L.vx; S.vy[i] = L.vy; S.vz[i] = L.vz;
  comp_at(cl, 0, i) = L.cqx; comp_at(cl, 1, i) = L.cqy; comp_at(cl, 2, i) = L.cqz;
  comp_at(cl, 3, i) = L.cvx; comp_at(cl, 4, i) = L.cvy; comp_at(cl, 5, i) = L.cvz;
}

// Kepler drift K(tau) of one planet; the diagnostics count the system's own
// planets only.  Returns the anomaly X.
__device__ __forceinline__ double serial_drift(Lane& L, double mu, double tau, bool own, KepDiag& dg) {
  KepDiag d{0.0, 1.0e300};
  const double X = drift(L, mu, tau, d);
  if (own) {
    dg.zmax = fmax(dg.zmax, d.zmax);
    dg.bmin = fmin(dg.bmin, d.bmin);
  }
  return X;
}

// J(ta) [I + GR](ti) J(tc) of one system (the operations of kick_block on
// every planet), then, if do_drift, the next drift K(tau) of each planet
// right after its renormalization.  REC: the velocities after the kick go to
// vk[r * ns + i] (r = 0..2), as the adjoint's tape keeps them, and, if xrec
// is given, the drift's anomaly to xrec[i].  Contraction
// is off here so that the recording instantiation (whose extra stores would
// otherwise let the compiler fuse different products) rounds exactly as the
// step kernel does.
template <int NP, bool GR, bool REC = false>
__device__ __forceinline__ void serial_kick_drift(SerialState<NP>& S, double* cl, int n, double m0, double inv_m0,
                                                  double kg, double ta, double ti, double tc, double tau,
                                                  bool do_drift, KepDiag& dg, double* vk = nullptr, int ns = 0,
                                                  double* xrec = nullptr) {
#pragma clang fp contract(off)
  double qx[NP], qy[NP], qz[NP], ax[NP], ay[NP], az[NP];
  double dqx = 0.0, dqy = 0.0, dqz = 0.0;
  if (GR) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      sx = fma(S.m[i], S.vx[i], sx);
      sy = fma(S.m[i], S.vy[i], sy);
      sz = fma(S.m[i], S.vz[i], sz);
    }
    const double k1 = ta * inv_m0;
    dqx = k1 * sx; dqy = k1 * sy; dqz = k1 * sz;
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    qx[i] = GR ? S.qx[i] + dqx : S.qx[i];
    qy[i] = GR ? S.qy[i] + dqy : S.qy[i];
    qz[i] = GR ? S.qz[i] + dqz : S.qz[i];
    ax[i] = 0.0; ay[i] = 0.0; az[i] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = i + 1; j < NP; ++j) {
      double dx, dy, dz;
      const double ir3 = pair_accel(qx[i], qy[i], qz[i], qx[j], qy[j], qz[j], S.m[j], ax[i], ay[i], az[i], dx, dy,
                                    dz);
      const double w = S.m[i] * ir3;   // planet j's acceleration is +w d
      ax[j] = fma(w, dx, ax[j]);
      ay[j] = fma(w, dy, ay[j]);
      az[j] = fma(w, dz, az[j]);
    }
  double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    if (GR) {
      double gx, gy, gz;
      gr_accel(qx[i], qy[i], qz[i], kg, gx, gy, gz);
      ax[i] += gx; ay[i] += gy; az[i] += gz;
    }
    ax[i] *= ti; ay[i] *= ti; az[i] *= ti;   // now the velocity increments
    if (REC) {
      vk[i] = S.vx[i] + ax[i];
      vk[ns + i] = S.vy[i] + ay[i];
      vk[2 * ns + i] = S.vz[i] + az[i];
    }
    sx = fma(S.m[i], S.vx[i] + ax[i], sx);
    sy = fma(S.m[i], S.vy[i] + ay[i], sy);
    sz = fma(S.m[i], S.vz[i] + az[i], sz);
  }
  const double k2 = (GR ? tc : ta + tc) * inv_m0;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    Lane L = serial_get(S, cl, i);
    if (GR) { L.cqx += dqx; L.cqy += dqy; L.cqz += dqz; }
    L.cvx += ax[i]; L.cvy += ay[i]; L.cvz += az[i];
    L.cqx += k2 * sx; L.cqy += k2 * sy; L.cqz += k2 * sz;
    renorm_all(L);
    if (do_drift) {
      const double X = serial_drift(L, m0, tau, i < n, dg);
      if (REC && xrec) xrec[i] = X;
    }
    serial_put(S, cl, i, L);
    // one planet at a time: hoisting the next planets' loads and solves
    // would overflow the registers
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int NP, bool GR, int SCHEME>
__device__ void step_serial(const StepParams& p, int base, int n, double* cl) {
  const double* st = p.st;
  const int ns = p.ns;
  SerialState<NP> S;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    S.qx[i] = st[base + i];
    S.qy[i] = st[ns + base + i];
    S.qz[i] = st[2 * ns + base + i];
    S.vx[i] = st[3 * ns + base + i];
    S.vy[i] = st[4 * ns + base + i];
    S.vz[i] = st[5 * ns + base + i];
    S.m[i] = st[6 * ns + base + i];
#pragma unroll
    for (int k = 0; k < 6; ++k) comp_at(cl, k, i) = st[(7 + k) * ns + base + i];
  }
  const int sys = p.slot_sys[base];
  const double dt = p.dts[base];
  const double h = 0.5 * dt;
  const double m0 = p.m0s[base];
  const double inv_m0 = 1.0 / m0;
  const double kg = GR ? p.kgr * m0 * m0 : 0.0;
  const bool first = p.synced[sys] != 0;
  KepDiag dg{0.0, 1.0e300};
  auto drift_all = [&](double tau) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      Lane L = serial_get(S, cl, i);
      serial_drift(L, m0, tau, i < n, dg);
      serial_put(S, cl, i, L);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  const int ns_steps = p.n_steps;
  if constexpr (SCHEME == SCHEME_SABA) {
    // K(c_1 dt) B(d_1 dt) K(c_2 dt) ... B(d_n dt), the closing drift merged
    // with the next step's opening one; each kick is followed by the drift
    // after it, except the last kick of the last step
    const double c1dt = p.sc[0] * dt;
    if (ns_steps > 0) drift_all(first ? c1dt : 2.0 * c1dt);
    for (int s = 0; s < ns_steps; ++s) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < p.saba_n) {
          const double tb = p.sd[k] * dt;
          const bool inner = k + 1 < p.saba_n;
          const double tau = inner ? p.sc[k + 1] * dt : 2.0 * c1dt;
          serial_kick_drift<NP, false>(S, cl, n, m0, inv_m0, 0.0, 0.5 * tb, tb, 0.5 * tb, tau,
                                       inner || s + 1 < ns_steps, dg);
        }
      }
    }
  } else if (SCHEME == WH_DKD) {
    if (ns_steps > 0) drift_all(first ? h : dt);
    for (int s = 0; s < ns_steps; ++s)
      serial_kick_drift<NP, GR>(S, cl, n, m0, inv_m0, kg, h, dt, h, dt, s + 1 < ns_steps, dg);
  } else {
    double ta = first ? 0.0 : h;
    double ti = first ? h : dt;
    for (int s = 0; s < ns_steps; ++s) {
      serial_kick_drift<NP, GR>(S, cl, n, m0, inv_m0, kg, ta, ti, h, dt, true, dg);
      ta = h;
      ti = dt;
    }
  }
  int f = 0;
  double* so = p.st;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const bool fin = __builtin_isfinite(S.qx[i]) && __builtin_isfinite(S.qy[i]) && __builtin_isfinite(S.qz[i]) &&
                     __builtin_isfinite(S.vx[i]) && __builtin_isfinite(S.vy[i]) && __builtin_isfinite(S.vz[i]);
    if (i < n && !fin) f |= WH_F_NONFINITE;
    so[base + i] = S.qx[i];
    so[ns + base + i] = S.qy[i];
    so[2 * ns + base + i] = S.qz[i];
    so[3 * ns + base + i] = S.vx[i];
    so[4 * ns + base + i] = S.vy[i];
    so[5 * ns + base + i] = S.vz[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) so[(7 + k) * ns + base + i] = comp_at(cl, k, i);
  }
  if (!(dg.bmin > 0.0)) f |= WH_F_HYPERBOLIC;
  if (!(dg.zmax <= p.zlim)) f |= WH_F_ZMAX;
  p.flags[sys] |= (uint32_t)f;
  p.synced[sys] = 0;
}

// Dynamic LDS: SERIAL_LDS_PER_WAVE doubles per wave of the block.
template <bool GR, int SCHEME>
__global__ __launch_bounds__(256) void k_step_serial(StepParams p) {
  extern __shared__ double serial_lds[];
  const int g = p.wave0 * 8 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (g >= p.w8 * 8) return;
  const int base = g * 8;
  if (p.slot_sys[base] < 0) return;   // an empty group
  double* cl = serial_lds + (threadIdx.x >> 6) * SERIAL_LDS_PER_WAVE + (threadIdx.x & 63);
  int n = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) n += p.slot_pl[base + i] >= 0;
  // the largest planet count among the wave's systems (wave-uniform)
  int nw = 1;
#pragma unroll
  for (int k = 2; k <= 8; ++k)
    if (__ballot(n >= k) != 0) nw = k;
  switch (nw) {
    case 1: step_serial<1, GR, SCHEME>(p, base, n, cl); break;
    case 2: step_serial<2, GR, SCHEME>(p, base, n, cl); break;
    case 3: step_serial<3, GR, SCHEME>(p, base, n, cl); break;
    case 4: step_serial<4, GR, SCHEME>(p, base, n, cl); break;
    case 5: step_serial<5, GR, SCHEME>(p, base, n, cl); break;
    case 6: step_serial<6, GR, SCHEME>(p, base, n, cl); break;
    case 7: step_serial<7, GR, SCHEME>(p, base, n, cl); break;
    default: step_serial<8, GR, SCHEME>(p, base, n, cl); break;
  }
}

// ---------------------------------------------------------------------------
// Synchronized copy: DKD applies the pending half drift K(h), SABA_n the
// pending drift K(c_1 dt); KDK applies the pending half kick J(h) [I + GR](h).
// A synchronized state is left as is.
// The result is the compensated state plus the half step's increments.
struct SyncParams {
  StepParams sp;
  double* Q_out;    // [S*8*3] or null
  double* V_out;
  double* E_out;    // [S] or null
  double* a_out;    // [S*8] or null
  double* e_out;
  double* L_out;    // [S*3] or null
};

// Angular momentum m (Q x V) of one planet.
__device__ __forceinline__ void planet_angmom(const Lane& L, double& lx, double& ly, double& lz) {
  lx = L.m * (L.qy * L.vz - L.qz * L.vy);
  ly = L.m * (L.qz * L.vx - L.qx * L.vz);
  lz = L.m * (L.qx * L.vy - L.qy * L.vx);
}

// Symplectic corrector of the Jacobi map on a lane's (compensated) state:
// the change from mapping to real coordinates C, or its inverse.  A stage
// Z(a, b) drifts a dt, kicks b dt, drifts -2a dt, kicks -b dt and drifts a dt
// (a kick carried by the Kepler flow and back); C applies the stages from
// the last to the first, C^-1 the first to the last with a negated, which is
// the exact inverse.  Coefficients from the host (corrector_coefficients).
template <int G, bool GR>
__device__ void apply_corrector(const StepParams& p, Lane& L, int lane, bool inverse) {
  const int pg = lane & (G - 1);
  const JacConst jc = jac_const<G>(L.m0, L.m, pg);
  Exch<G, 0> ex;
  ex.init(lane, L.m);
  const double kg = GR ? p.kgr * L.m0 * L.m0 : 0.0;
  KepDiag dg{0.0, 1.0e300};
  double vkx, vky, vkz;
  const double h = L.dt;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < p.corr_n) {
      const int i = inverse ? k : p.corr_n - 1 - k;
      const double a = (inverse ? -p.corr_a[i] : p.corr_a[i]) * h;
      const double b = p.corr_b[i] * h;
      drift(L, jc.Mi, a, dg);
      kick_jacobi<G, 0, GR>(L, ex, jc, pg, b, vkx, vky, vkz, kg);
      drift(L, jc.Mi, -2.0 * a, dg);
      kick_jacobi<G, 0, GR>(L, ex, jc, pg, -b, vkx, vky, vkz, kg);
      drift(L, jc.Mi, a, dg);
    }
  }
}

// Substep j of the corrector's sequence in the order C (or C^-1) applies
// them (as apply_corrector: stage by stage, D(a) K(b) D(-2a) K(-b) D(a) in
// units of dt).  Returns true for a drift; tau is the substep's time.
__device__ __forceinline__ bool corrector_substep(const StepParams& p, int j, bool inverse, double h, double& tau) {
  const int k = j / 5, sub = j - 5 * k;
  const int i = inverse ? k : p.corr_n - 1 - k;
  const double a = (inverse ? -p.corr_a[i] : p.corr_a[i]) * h;
  const double b = p.corr_b[i] * h;
  if (sub == 0 || sub == 4) { tau = a; return true; }
  if (sub == 2) { tau = -2.0 * a; return true; }
  tau = sub == 1 ? b : -b;
  return false;
}

// The first n_sub substeps of C (or C^-1) on a lane's compensated state.
template <int G, bool GR>
__device__ void corrector_run(const StepParams& p, Lane& L, int lane, bool inverse, int n_sub) {
  const int pg = lane & (G - 1);
  const JacConst jc = jac_const<G>(L.m0, L.m, pg);
  Exch<G, 0> ex;
  ex.init(lane, L.m);
  const double kg = GR ? p.kgr * L.m0 * L.m0 : 0.0;
  KepDiag dg{0.0, 1.0e300};
  double vkx, vky, vkz;
  for (int j = 0; j < n_sub; ++j) {
    double tau;
    if (corrector_substep(p, j, inverse, L.dt, tau)) drift(L, jc.Mi, tau, dg);
    else kick_jacobi<G, 0, GR>(L, ex, jc, pg, tau, vkx, vky, vkz, kg);
  }
}

template <int G, bool GR, int SCHEME, bool JAC = false>
__device__ void sync_lane(const StepParams& p, Lane& L, int lane) {
  const int pg = lane & (G - 1);
  if (!L.first) {   // uniform over the group: one system, one flag
    const double h = 0.5 * L.dt;
    if (SCHEME == WH_DKD || SCHEME == SCHEME_SABA) {
      KepDiag dg{0.0, 1.0e300};
      const double tau = SCHEME == SCHEME_SABA ? p.sc[0] * L.dt : h;
      double mu = L.m0;
      if constexpr (JAC) mu = jac_const<G>(L.m0, L.m, pg).Mi;
      drift(L, mu, tau, dg);
    } else {
      Exch<G, 0> ex;
      ex.init(lane, L.m);
      double vkx, vky, vkz;
      if constexpr (JAC)
        kick_jacobi<G, 0, GR>(L, ex, jac_const<G>(L.m0, L.m, pg), pg, h, vkx, vky, vkz,
                              GR ? p.kgr * L.m0 * L.m0 : 0.0);
      else kick_block<G, GR, 0>(L, ex, 1.0 / L.m0, GR ? p.kgr * L.m0 * L.m0 : 0.0, h, h, 0.0, vkx, vky, vkz);
    }
  }
  // the output is in real coordinates: the corrector takes the synchronized
  // mapping coordinates there (uniform over the group: one system)
  if constexpr (JAC)
    if (p.corr_n > 0) apply_corrector<G, GR>(p, L, lane, false);
  L.qx += L.cqx; L.qy += L.cqy; L.qz += L.cqz;
  L.vx += L.cvx; L.vy += L.cvy; L.vz += L.cvz;
  if constexpr (JAC) jacobi_to_dhc<G>(L, pg);
}

// Energy of the lane's system (every lane of the group gets it).
template <int G, bool GR> __device__ double group_energy(const StepParams& p, const Lane& L, int lane) {
  const double r2 = L.qx * L.qx + L.qy * L.qy + L.qz * L.qz;
  const double r = sqrt(r2);
  double e = 0.5 * L.m * (L.vx * L.vx + L.vy * L.vy + L.vz * L.vz) - L.m0 * L.m / r;
  if (GR) e -= 0.5 * p.kgr * L.m0 * L.m0 * L.m / r2;   // 3 m0^2 m / (c^2 r^2)
  // planets of the group and lanes per planet (2 in the split layout, where
  // lane ^ 2k holds planet p ^ k)
  constexpr int NP = G == G_SPLIT ? 8 : G;
  constexpr int LS = G == G_SPLIT ? 2 : 1;
  double pair = 0.0;
#pragma unroll
  for (int k = 1; k < NP; ++k) {
    int src = (lane ^ (k * LS)) << 2;
    double px = bperm(src, L.qx), py = bperm(src, L.qy), pz = bperm(src, L.qz), pm = bperm(src, L.m);
    double dx = L.qx - px, dy = L.qy - py, dz = L.qz - pz;
    pair += pm / sqrt(dx * dx + dy * dy + dz * dz);
  }
  e -= 0.5 * L.m * pair;
  e = group_sum<G>(e);
  double sx = group_sum<G>(L.m * L.vx), sy = group_sum<G>(L.m * L.vy), sz = group_sum<G>(L.m * L.vz);
  return e + (sx * sx + sy * sy + sz * sz) / (2.0 * L.m0);
}

template <int G, bool GR, int SCHEME, bool JAC> __device__ void sync_group(const SyncParams& q, int slot, int lane) {
  const StepParams& p = q.sp;
  Lane L = load_lane(p, slot);
  sync_lane<G, GR, SCHEME, JAC>(p, L, lane);
  // one writer per planet (the split layout holds two copies)
  const bool writer = L.sys >= 0 && L.pl >= 0 && (G != G_SPLIT || (lane & 1) == 0);
  if (q.Q_out && writer) {
    size_t o = ((size_t)L.sys * 8 + L.pl) * 3;
    q.Q_out[o] = L.qx; q.Q_out[o + 1] = L.qy; q.Q_out[o + 2] = L.qz;
    q.V_out[o] = L.vx; q.V_out[o + 1] = L.vy; q.V_out[o + 2] = L.vz;
  }
  if (q.E_out) {
    double E = group_energy<G, GR>(p, L, lane);
    if ((lane & (G - 1)) == 0 && L.sys >= 0) q.E_out[L.sys] = E;
  }
  if (q.L_out) {
    double lx, ly, lz;
    planet_angmom(L, lx, ly, lz);
    lx = group_sum<G>(lx); ly = group_sum<G>(ly); lz = group_sum<G>(lz);
    if ((lane & (G - 1)) == 0 && L.sys >= 0) {
      q.L_out[(size_t)L.sys * 3] = lx; q.L_out[(size_t)L.sys * 3 + 1] = ly; q.L_out[(size_t)L.sys * 3 + 2] = lz;
    }
  }
  if (q.a_out) {
    // heliocentric velocity u = V + sum_j m_j V_j / m0, two-body elements
    double sx, sy, sz;
    group_momentum<G>(L.m, L.vx, L.vy, L.vz, sx, sy, sz);
    double ux = L.vx + sx / L.m0, uy = L.vy + sy / L.m0, uz = L.vz + sz / L.m0;
    double mu = L.m0 + L.m;
    double r = sqrt(L.qx * L.qx + L.qy * L.qy + L.qz * L.qz);
    double u2 = ux * ux + uy * uy + uz * uz;
    double a = 1.0 / (2.0 / r - u2 / mu);
    double hx = L.qy * uz - L.qz * uy, hy = L.qz * ux - L.qx * uz, hz = L.qx * uy - L.qy * ux;
    double ex = (uy * hz - uz * hy) / mu - L.qx / r;
    double ey = (uz * hx - ux * hz) / mu - L.qy / r;
    double ez = (ux * hy - uy * hx) / mu - L.qz / r;
    if (writer) {
      size_t o = (size_t)L.sys * 8 + L.pl;
      q.a_out[o] = a;
      q.e_out[o] = sqrt(ex * ex + ey * ey + ez * ez);
    }
  }
}

template <bool GR, int SCHEME, bool JAC = false>
__global__ __launch_bounds__(256) void k_sync(SyncParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (wave < p.w1) sync_group<1, GR, SCHEME, JAC>(q, slot, lane);
  else if (wave < p.w2) sync_group<2, GR, SCHEME, JAC>(q, slot, lane);
  else if (wave < p.w4) sync_group<4, GR, SCHEME, JAC>(q, slot, lane);
  else sync_group<8, GR, SCHEME, JAC>(q, slot, lane);
}

template <bool GR, int SCHEME>
__global__ __launch_bounds__(256) void k_sync_split(SyncParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  sync_group<G_SPLIT, GR, SCHEME, false>(q, wave * 64 + lane, lane);
}

// Synchronized copy of the pair layout: as sync_group for both slots.
__device__ __forceinline__ void osculating(const Lane& L, double sx, double sy, double sz, double& a, double& e) {
  const double ux = L.vx + sx / L.m0, uy = L.vy + sy / L.m0, uz = L.vz + sz / L.m0;
  const double mu = L.m0 + L.m;
  const double r = sqrt(L.qx * L.qx + L.qy * L.qy + L.qz * L.qz);
  const double u2 = ux * ux + uy * uy + uz * uz;
  a = 1.0 / (2.0 / r - u2 / mu);
  const double hx = L.qy * uz - L.qz * uy, hy = L.qz * ux - L.qx * uz, hz = L.qx * uy - L.qy * ux;
  const double ex = (uy * hz - uz * hy) / mu - L.qx / r;
  const double ey = (uz * hx - ux * hz) / mu - L.qy / r;
  const double ez = (ux * hy - uy * hx) / mu - L.qz / r;
  e = sqrt(ex * ex + ey * ey + ez * ez);
}

__device__ __forceinline__ double planet_energy(const Lane& L, double kgr) {
  const double r2 = L.qx * L.qx + L.qy * L.qy + L.qz * L.qz;
  double e = 0.5 * L.m * (L.vx * L.vx + L.vy * L.vy + L.vz * L.vz) - L.m0 * L.m / sqrt(r2);
  if (kgr > 0) e -= 0.5 * kgr * L.m0 * L.m0 * L.m / r2;
  return e;
}

// Synchronized copy of a shared 8-lane group (the mixed packing): as
// sync_group, with the pending half kick, the energy's pair terms and every
// sum kept within each system; results written from each system's planet 0.
template <bool GR, int SCHEME> __device__ void sync_group_mixed(const SyncParams& q, int slot, int lane) {
  const StepParams& p = q.sp;
  Lane L = load_lane(p, slot);
  Exch<8, 2> ex;
  ex.init_mixed(L.m, L.pl, lane & 7);
  if (!L.first) {
    const double h = 0.5 * L.dt;
    if (SCHEME == WH_DKD) {
      KepDiag dg{0.0, 1.0e300};
      drift(L, L.m0, h, dg);
    } else {
      double vkx, vky, vkz;
      kick_block<8, GR, 2>(L, ex, 1.0 / L.m0, GR ? p.kgr * L.m0 * L.m0 : 0.0, h, h, 0.0, vkx, vky, vkz);
    }
  }
  L.qx += L.cqx; L.qy += L.cqy; L.qz += L.cqz;
  L.vx += L.cvx; L.vy += L.cvy; L.vz += L.cvz;
  const bool writer = L.sys >= 0 && L.pl >= 0;
  if (q.Q_out && writer) {
    size_t o = ((size_t)L.sys * 8 + L.pl) * 3;
    q.Q_out[o] = L.qx; q.Q_out[o + 1] = L.qy; q.Q_out[o + 2] = L.qz;
    q.V_out[o] = L.vx; q.V_out[o + 1] = L.vy; q.V_out[o + 2] = L.vz;
  }
  if (q.E_out) {
    const double r2 = L.qx * L.qx + L.qy * L.qy + L.qz * L.qz;
    double e = 0.5 * L.m * (L.vx * L.vx + L.vy * L.vy + L.vz * L.vz) - L.m0 * L.m / sqrt(r2);
    if (GR) e -= 0.5 * p.kgr * L.m0 * L.m0 * L.m / r2;
    const int own = ex.a ? 1 : 0;
    double pair = 0.0;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      const int src = (lane ^ k) << 2;
      const double px = bperm(src, L.qx), py = bperm(src, L.qy), pz = bperm(src, L.qz), pm = bperm(src, L.m);
      const bool same = __builtin_amdgcn_ds_bpermute(src, own) == own;
      const double dx = L.qx - px, dy = L.qy - py, dz = L.qz - pz;
      const double d2 = same ? dx * dx + dy * dy + dz * dz : 1.0;
      pair += (same ? pm : 0.0) / sqrt(d2);
    }
    e -= 0.5 * L.m * pair;
    e = ex.sum(e);
    double sx, sy, sz;
    ex.momentum(L.m, L.vx, L.vy, L.vz, sx, sy, sz);
    const double E = e + (sx * sx + sy * sy + sz * sz) / (2.0 * L.m0);
    if (L.pl == 0 && L.sys >= 0) q.E_out[L.sys] = E;
  }
  if (q.L_out) {
    double lx, ly, lz;
    planet_angmom(L, lx, ly, lz);
    lx = ex.sum(lx); ly = ex.sum(ly); lz = ex.sum(lz);
    if (L.pl == 0 && L.sys >= 0) {
      q.L_out[(size_t)L.sys * 3] = lx; q.L_out[(size_t)L.sys * 3 + 1] = ly; q.L_out[(size_t)L.sys * 3 + 2] = lz;
    }
  }
  if (q.a_out) {
    double sx, sy, sz;
    ex.momentum(L.m, L.vx, L.vy, L.vz, sx, sy, sz);
    double a, e;
    osculating(L, sx, sy, sz, a, e);
    if (writer) {
      size_t o = (size_t)L.sys * 8 + L.pl;
      q.a_out[o] = a;
      q.e_out[o] = e;
    }
  }
}

template <bool GR, int SCHEME>
__global__ __launch_bounds__(256) void k_sync_mixed(SyncParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (wave < p.w1) sync_group<1, GR, SCHEME, false>(q, slot, lane);
  else if (wave < p.w2) sync_group<2, GR, SCHEME, false>(q, slot, lane);
  else if (wave < p.w4) sync_group<4, GR, SCHEME, false>(q, slot, lane);
  else if (wave < p.wm) sync_group<8, GR, SCHEME, false>(q, slot, lane);
  else sync_group_mixed<GR, SCHEME>(q, slot, lane);
}

template <int G, bool GR> __device__ double group_energy_pair(const StepParams& p, const Lane& A, const Lane& B,
                                                              int lane) {
  double e = planet_energy(A, GR ? p.kgr : 0.0) + planet_energy(B, GR ? p.kgr : 0.0);
  {
    const double dx = A.qx - B.qx, dy = A.qy - B.qy, dz = A.qz - B.qz;
    e -= A.m * B.m / sqrt(dx * dx + dy * dy + dz * dz);
  }
  double pair = 0.0;
#pragma unroll
  for (int k = 1; k < G; ++k) {
    const int src = (lane ^ k) << 2;
    const double pax = bperm(src, A.qx), pay = bperm(src, A.qy), paz = bperm(src, A.qz), pma = bperm(src, A.m);
    const double pbx = bperm(src, B.qx), pby = bperm(src, B.qy), pbz = bperm(src, B.qz), pmb = bperm(src, B.m);
    double dx, dy, dz;
    dx = A.qx - pax; dy = A.qy - pay; dz = A.qz - paz; pair += A.m * pma / sqrt(dx * dx + dy * dy + dz * dz);
    dx = A.qx - pbx; dy = A.qy - pby; dz = A.qz - pbz; pair += A.m * pmb / sqrt(dx * dx + dy * dy + dz * dz);
    dx = B.qx - pax; dy = B.qy - pay; dz = B.qz - paz; pair += B.m * pma / sqrt(dx * dx + dy * dy + dz * dz);
    dx = B.qx - pbx; dy = B.qy - pby; dz = B.qz - pbz; pair += B.m * pmb / sqrt(dx * dx + dy * dy + dz * dz);
  }
  e -= 0.5 * pair;
  e = group_sum<G>(e);
  double sx, sy, sz;
  pair_momentum<G>(A.m, A.vx, A.vy, A.vz, B.m, B.vx, B.vy, B.vz, sx, sy, sz);
  return e + (sx * sx + sy * sy + sz * sz) / (2.0 * A.m0);
}

__device__ __forceinline__ void write_state(const SyncParams& q, const Lane& L) {
  if (q.Q_out && L.sys >= 0 && L.pl >= 0) {
    size_t o = ((size_t)L.sys * 8 + L.pl) * 3;
    q.Q_out[o] = L.qx; q.Q_out[o + 1] = L.qy; q.Q_out[o + 2] = L.qz;
    q.V_out[o] = L.vx; q.V_out[o + 1] = L.vy; q.V_out[o + 2] = L.vz;
  }
}

template <int G, bool GR, int SCHEME> __device__ void sync_group_pair(const SyncParams& q, int sa, int lane) {
  const StepParams& p = q.sp;
  Lane A = load_lane(p, sa);
  Lane B = load_lane(p, sa + 64);
  if (!A.first) {
    const double h = 0.5 * A.dt;
    if (SCHEME == WH_DKD || SCHEME == SCHEME_SABA) {
      KepDiag dg{0.0, 1.0e300};
      const double tau = SCHEME == SCHEME_SABA ? p.sc[0] * A.dt : h;
      drift(A, A.m0, tau, dg);
      drift(B, B.m0, tau, dg);
    } else {
      const PairMass pm = make_pair_mass<G>(A.m, B.m);
      double vka[3], vkb[3];
      kick_block_pair<G, GR>(A, B, pm, 1.0 / A.m0, GR ? p.kgr * A.m0 * A.m0 : 0.0, h, h, 0.0, vka, vkb);
    }
  }
  A.qx += A.cqx; A.qy += A.cqy; A.qz += A.cqz; A.vx += A.cvx; A.vy += A.cvy; A.vz += A.cvz;
  B.qx += B.cqx; B.qy += B.cqy; B.qz += B.cqz; B.vx += B.cvx; B.vy += B.cvy; B.vz += B.cvz;
  write_state(q, A);
  write_state(q, B);
  if (q.E_out) {
    const double E = group_energy_pair<G, GR>(p, A, B, lane);
    if ((lane & (G - 1)) == 0 && A.sys >= 0) q.E_out[A.sys] = E;
  }
  if (q.L_out) {
    double ax, ay, az, bx, by, bz;
    planet_angmom(A, ax, ay, az);
    planet_angmom(B, bx, by, bz);
    const double lx = group_sum<G>(ax + bx), ly = group_sum<G>(ay + by), lz = group_sum<G>(az + bz);
    if ((lane & (G - 1)) == 0 && A.sys >= 0) {
      q.L_out[(size_t)A.sys * 3] = lx; q.L_out[(size_t)A.sys * 3 + 1] = ly; q.L_out[(size_t)A.sys * 3 + 2] = lz;
    }
  }
  if (q.a_out) {
    double sx, sy, sz, a, e;
    pair_momentum<G>(A.m, A.vx, A.vy, A.vz, B.m, B.vx, B.vy, B.vz, sx, sy, sz);
    osculating(A, sx, sy, sz, a, e);
    if (A.sys >= 0 && A.pl >= 0) { q.a_out[(size_t)A.sys * 8 + A.pl] = a; q.e_out[(size_t)A.sys * 8 + A.pl] = e; }
    osculating(B, sx, sy, sz, a, e);
    if (B.sys >= 0 && B.pl >= 0) { q.a_out[(size_t)B.sys * 8 + B.pl] = a; q.e_out[(size_t)B.sys * 8 + B.pl] = e; }
  }
}

template <bool GR, int SCHEME>
__global__ __launch_bounds__(256) void k_sync_pair(SyncParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int sa = wave * 128 + lane;
  if (wave < p.w1) sync_group_pair<1, GR, SCHEME>(q, sa, lane);
  else if (wave < p.w2) sync_group_pair<2, GR, SCHEME>(q, sa, lane);
  else sync_group_pair<4, GR, SCHEME>(q, sa, lane);
}

// Initial state of a Jacobi context: the gathered DHC state (compensation
// zero) converted in place.
template <int G> __device__ void to_jacobi_group(const StepParams& p, int slot, int lane) {
  Lane L = load_lane(p, slot);
  dhc_to_jacobi<G>(L, lane & (G - 1));
  store_lane(p, slot, L);
}
// Inverse corrector at set-up: real -> mapping coordinates (Jacobi state).
template <int G, bool GR> __device__ void corrector_in_group(const StepParams& p, int slot, int lane) {
  Lane L = load_lane(p, slot);
  apply_corrector<G, GR>(p, L, lane, true);
  renorm_all(L);
  store_lane(p, slot, L);
}
template <bool GR> __global__ __launch_bounds__(256) void k_corrector_in(StepParams p) {
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (wave < p.w1) corrector_in_group<1, GR>(p, slot, lane);
  else if (wave < p.w2) corrector_in_group<2, GR>(p, slot, lane);
  else if (wave < p.w4) corrector_in_group<4, GR>(p, slot, lane);
  else corrector_in_group<8, GR>(p, slot, lane);
}

__global__ __launch_bounds__(256) void k_to_jacobi(StepParams p) {
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (wave < p.w1) to_jacobi_group<1>(p, slot, lane);
  else if (wave < p.w2) to_jacobi_group<2>(p, slot, lane);
  else if (wave < p.w4) to_jacobi_group<4>(p, slot, lane);
  else to_jacobi_group<8>(p, slot, lane);
}

// ---------------------------------------------------------------------------
// Reverse mode (drift-kick-drift).  Checkpoints hold the double-double state
// [12][ns] (Q, V, then their compensation); a segment tape holds, per step,
// the rounded state entering the step, the step's Kepler anomaly and the
// velocity after the step's kick, [step][TAPE_ROWS][ns]; the adjoint state is
// [8][ns]: gQ, gV, gm, and the lane's share of gm0.  Segments are swept from
// the last to the first; while segment k is swept, the next launch's input,
// segment k - 1, is recorded by other wavefronts of the same launch into the
// second of two segment tapes.
constexpr int TAPE_ROWS = WH_TAPE_ROWS;
struct AdjParams {
  StepParams sp;
  const double* ck;    // k_adj_init: the final checkpoint
  double* tape;        // tape of the segment being swept
  double* grad;        // adjoint state
  const double* gQ_T;  // caller layout [S*8*3]
  const double* gV_T;
  double* gQ_0;
  double* gV_0;
  double* gm;          // [S*8]
  double* gm0;         // [S]
  int n_seg;           // steps of the segment being swept
  int first_synced;    // it starts from the synchronized initial state
  int sweep_waves;     // wavefronts of the sweeping role (0: the launch only records)
  const double* ck_rec;  // recording role: checkpoint of the segment to record,
  double* tape_rec;      // the tape to fill,
  int n_rec;             // its steps,
  int rec_first_synced;  // and whether it starts from the synchronized initial state
};

__device__ __forceinline__ void load_ck(const double* ck, int ns, int slot, Lane& L) {
  L.qx = ck[slot]; L.qy = ck[ns + slot]; L.qz = ck[2 * ns + slot];
  L.vx = ck[3 * ns + slot]; L.vy = ck[4 * ns + slot]; L.vz = ck[5 * ns + slot];
  L.cqx = ck[6 * ns + slot]; L.cqy = ck[7 * ns + slot]; L.cqz = ck[8 * ns + slot];
  L.cvx = ck[9 * ns + slot]; L.cvy = ck[10 * ns + slot]; L.cvz = ck[11 * ns + slot];
}

__global__ void k_save_ck(const double* st, double* ck, int ns) {
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= ns) return;
  for (int r = 0; r < 6; ++r) ck[r * ns + slot] = st[r * ns + slot];
  for (int r = 0; r < 6; ++r) ck[(6 + r) * ns + slot] = st[(7 + r) * ns + slot];
}

struct Grad {
  double qx, qy, qz, vx, vy, vz, m, m0;
};

__device__ __forceinline__ void load_grad(const double* g, int ns, int slot, Grad& a) {
  a.qx = g[slot]; a.qy = g[ns + slot]; a.qz = g[2 * ns + slot];
  a.vx = g[3 * ns + slot]; a.vy = g[4 * ns + slot]; a.vz = g[5 * ns + slot];
  a.m = g[6 * ns + slot]; a.m0 = g[7 * ns + slot];
}
__device__ __forceinline__ void store_grad(double* g, int ns, int slot, const Grad& a) {
  g[slot] = a.qx; g[ns + slot] = a.qy; g[2 * ns + slot] = a.qz;
  g[3 * ns + slot] = a.vx; g[4 * ns + slot] = a.vy; g[5 * ns + slot] = a.vz;
  g[6 * ns + slot] = a.m; g[7 * ns + slot] = a.m0;
}

// Adjoint of the jump Q += kj sum_j m_j V_j (kj = tau/m0) given the group's
// momentum S = sum_j m_j V_j: gV_i += kj m_i sum_k gQ_k, gm_i += kj V_i .
// sum_k gQ_k, and gm0 gets -(kj/m0) S . sum_k gQ_k once per group.
template <int G>
__device__ __forceinline__ void jump_vjp(Grad& a, double m, double vx, double vy, double vz, double kj, double m0,
                                         double sx, double sy, double sz, bool leader) {
  double Gx = group_sum<G>(a.qx), Gy = group_sum<G>(a.qy), Gz = group_sum<G>(a.qz);
  double km = kj * m;
  a.vx = fma(km, Gx, a.vx);
  a.vy = fma(km, Gy, a.vy);
  a.vz = fma(km, Gz, a.vz);
  a.m += kj * (vx * Gx + vy * Gy + vz * Gz);
  if (leader) a.m0 -= kj / m0 * (sx * Gx + sy * Gy + sz * Gz);
}

// The jump adjoint in the pair layout: the sums run over both slots of the
// group's lanes.
template <int G>
__device__ __forceinline__ void jump_vjp_pair(Grad& a, Grad& b, double ma, double mb, const double va[3],
                                              const double vb[3], double kj, double m0, const double sm[3],
                                              bool leader) {
  const double Gx = group_sum<G>(a.qx + b.qx), Gy = group_sum<G>(a.qy + b.qy), Gz = group_sum<G>(a.qz + b.qz);
  a.vx = fma(kj * ma, Gx, a.vx); a.vy = fma(kj * ma, Gy, a.vy); a.vz = fma(kj * ma, Gz, a.vz);
  b.vx = fma(kj * mb, Gx, b.vx); b.vy = fma(kj * mb, Gy, b.vy); b.vz = fma(kj * mb, Gz, b.vz);
  a.m += kj * (va[0] * Gx + va[1] * Gy + va[2] * Gz);
  b.m += kj * (vb[0] * Gx + vb[1] * Gy + vb[2] * Gz);
  if (leader) a.m0 -= kj / m0 * (sm[0] * Gx + sm[1] * Gy + sm[2] * Gz);
}

// Adjoint of the interaction kick with the exchange the forward kick used.
template <int G>
__device__ __forceinline__ void interaction_vjp(const Exch<G, 1>& ex, double qx, double qy, double qz, double m,
                                                double tau, double gvx, double gvy, double gvz, double& gqx,
                                                double& gqy, double& gqz, double& gm) {
  if constexpr (G == G_SPLIT) interaction_vjp_split(ex.t, qx, qy, qz, m, tau, gvx, gvy, gvz, gqx, gqy, gqz, gm);
  else interaction_vjp_dpp<G>(ex.t, qx, qy, qz, m, tau, gvx, gvy, gvz, gqx, gqy, gqz, gm);
}

// Adjoint of the kick block J(ta) [I + GR](ti) J(tc) (J(ta + tc) I(ti)
// without GR) at the forward point (Q0, V0), with vk the velocity after the
// kick: a holds dL/d(output) and receives dL/d(input).
template <int G, bool GR>
__device__ __forceinline__ void kick_block_vjp(Grad& a, const Exch<G, 1>& ex, double m, double m0, double inv_m0,
                                               double kg, double q0x, double q0y, double q0z, double v0x, double v0y,
                                               double v0z, double vkx, double vky, double vkz, double ta, double ti,
                                               double tc, bool leader) {
  if (GR) {
    double s1x, s1y, s1z, s3x, s3y, s3z;
    group_momentum<G>(m, v0x, v0y, v0z, s1x, s1y, s1z);
    const double k1 = ta * inv_m0;
    const double q2x = q0x + k1 * s1x, q2y = q0y + k1 * s1y, q2z = q0z + k1 * s1z;
    group_momentum<G>(m, vkx, vky, vkz, s3x, s3y, s3z);
    jump_vjp<G>(a, m, vkx, vky, vkz, tc * inv_m0, m0, s3x, s3y, s3z, leader);
    double gmu = 0.0;
    interaction_vjp<G>(ex, q2x, q2y, q2z, m, ti, a.vx, a.vy, a.vz, a.qx, a.qy, a.qz, a.m);
    gr_vjp(q2x, q2y, q2z, kg, m0, ti, a.vx, a.vy, a.vz, a.qx, a.qy, a.qz, gmu);
    a.m0 += gmu;
    jump_vjp<G>(a, m, v0x, v0y, v0z, k1, m0, s1x, s1y, s1z, leader);
  } else {
    double s2x, s2y, s2z;
    group_momentum<G>(m, vkx, vky, vkz, s2x, s2y, s2z);
    jump_vjp<G>(a, m, vkx, vky, vkz, (ta + tc) * inv_m0, m0, s2x, s2y, s2z, leader);
    interaction_vjp<G>(ex, q0x, q0y, q0z, m, ti, a.vx, a.vy, a.vz, a.qx, a.qy, a.qz, a.m);
  }
}

// Forward recompute of a segment from its checkpoint, writing its tape.  Same
// arithmetic as the step kernel (DPP exchange).  Per step the tape holds the
// state at the start of the step, the anomaly X of its drift and the
// velocity after its kick; with KDK the step is the kick block followed by
// the drift.
template <int G, bool GR, int SCH = WH_DKD>
__device__ void adj_record_lane(const AdjParams& q, int slot, int lane) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  Lane L;
  load_ck(q.ck_rec, ns, slot, L);
  L.m = p.st[6 * ns + slot];
  L.m0 = p.m0s[slot];
  L.dt = p.dts[slot];
  Exch<G, 1> ex;
  ex.init(lane, L.m);
  const double dt = L.dt, h = 0.5 * dt;
  const double inv_m0 = 1.0 / L.m0;
  const double kg = GR ? p.kgr * L.m0 * L.m0 : 0.0;
  KepDiag dg{0.0, 1.0e300};
  if constexpr (SCH == SCHEME_SABA) {
    // SABA_n: n units per step, unit k = K(tau_k) then the perturbation kick
    // B(d_k dt); tau_0 = c_1 dt (2 c_1 dt after the first step), tau_k = c_{k+1} dt
    const int nu = p.saba_n;
    const double c1dt = p.sc[0] * dt;
    for (int s = 0; s < q.n_rec; ++s)
      for (int k = 0; k < nu; ++k) {
        double* row = q.tape_rec + ((size_t)s * nu + k) * TAPE_ROWS * ns + slot;
        const double tau = k > 0 ? p.sc[k] * dt : (q.rec_first_synced && s == 0 ? c1dt : 2.0 * c1dt);
        const double tb = p.sd[k] * dt;
        row[0] = L.qx; row[ns] = L.qy; row[2 * ns] = L.qz;
        row[3 * ns] = L.vx; row[4 * ns] = L.vy; row[5 * ns] = L.vz;
        row[6 * ns] = drift(L, L.m0, tau, dg);
        double vkx, vky, vkz;
        kick_block<G, false, 1>(L, ex, inv_m0, 0.0, 0.5 * tb, tb, 0.5 * tb, vkx, vky, vkz);
        row[7 * ns] = vkx; row[8 * ns] = vky; row[9 * ns] = vkz;
      }
    return;
  }
  if constexpr (SCH == WH_KDK) {
    double ta = q.rec_first_synced ? 0.0 : h;
    double ti = q.rec_first_synced ? h : dt;
    for (int s = 0; s < q.n_rec; ++s) {
      double* row = q.tape_rec + (size_t)s * TAPE_ROWS * ns + slot;
      row[0] = L.qx; row[ns] = L.qy; row[2 * ns] = L.qz;
      row[3 * ns] = L.vx; row[4 * ns] = L.vy; row[5 * ns] = L.vz;
      double vkx, vky, vkz;
      kick_block<G, GR, 1>(L, ex, inv_m0, kg, ta, ti, h, vkx, vky, vkz);
      row[7 * ns] = vkx; row[8 * ns] = vky; row[9 * ns] = vkz;
      ta = h;
      ti = dt;
      row[6 * ns] = drift(L, L.m0, dt, dg);
    }
    return;
  }
  double tk = q.rec_first_synced ? h : dt;
  for (int s = 0; s < q.n_rec; ++s) {
    double* row = q.tape_rec + (size_t)s * TAPE_ROWS * ns + slot;
    row[0] = L.qx; row[ns] = L.qy; row[2 * ns] = L.qz;
    row[3 * ns] = L.vx; row[4 * ns] = L.vy; row[5 * ns] = L.vz;
    row[6 * ns] = drift(L, L.m0, tk, dg);
    tk = dt;
    double vkx, vky, vkz;
    kick_block<G, GR, 1>(L, ex, inv_m0, kg, h, dt, h, vkx, vky, vkz);
    row[7 * ns] = vkx; row[8 * ns] = vky; row[9 * ns] = vkz;   // V after the kick
  }
}

// One step's row of a segment tape (TAPE_ROWS values of one slot).
struct TapeRow {
  double v[TAPE_ROWS];
};
__device__ __forceinline__ void load_tape_row(const double* row, int ns, TapeRow& r) {
#pragma unroll
  for (int i = 0; i < TAPE_ROWS; ++i) r.v[i] = row[(size_t)i * ns];
}
// The two slots of a pair-layout lane: slot 128 w + l and slot 128 w + 64 + l.
__device__ __forceinline__ void load_tape_rows_pair(const double* ra, int ns, TapeRow& a, TapeRow& b) {
  load_tape_row(ra, ns, a);
  load_tape_row(ra + 64, ns, b);
}

// Reverse sweep of a recorded segment: the adjoint state is carried back
// through the transposed Jacobian of every sub-step.
template <int G, bool GR, int SCH = WH_DKD>
__device__ void adj_sweep_lane(const AdjParams& q, int slot, int lane) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  const double m = p.st[6 * ns + slot], m0 = p.m0s[slot];
  Exch<G, 1> ex;
  ex.init(lane, m);
  const double dt = p.dts[slot], h = 0.5 * dt;
  const double inv_m0 = 1.0 / m0;
  const double kg = GR ? p.kgr * m0 * m0 : 0.0;
  Grad a;
  load_grad(q.grad, ns, slot, a);
  // the lane(s) of planet 0 add the star-mass terms of the jump (in the
  // split layout both copies, so that the copies keep equal bits)
  const bool leader = G == G_SPLIT ? (lane & 14) == 0 : (lane & (G - 1)) == 0;
  if constexpr (SCH == SCHEME_SABA) {
    const int nu = p.saba_n;
    const double c1dt = p.sc[0] * dt;
    const int nunits = q.n_seg * nu;
    TapeRow nxt;
    if (nunits > 0) load_tape_row(q.tape + (size_t)(nunits - 1) * TAPE_ROWS * ns + slot, ns, nxt);
    for (int u = nunits - 1; u >= 0; --u) {
      const int s = u / nu, k = u - s * nu;
      const TapeRow cur = nxt;
      if (u > 0) load_tape_row(q.tape + (size_t)(u - 1) * TAPE_ROWS * ns + slot, ns, nxt);
      const double q0x = cur.v[0], q0y = cur.v[1], q0z = cur.v[2];
      const double v0x = cur.v[3], v0y = cur.v[4], v0z = cur.v[5];
      const double vkx = cur.v[7], vky = cur.v[8], vkz = cur.v[9];
      const double tau = k > 0 ? p.sc[k] * dt : (q.first_synced && s == 0 ? c1dt : 2.0 * c1dt);
      const double tb = p.sd[k] * dt;
      KepFwd kf;
      kepler_at_X(q0x, q0y, q0z, v0x, v0y, v0z, m0, tau, cur.v[6], kf);
      const double q1x = kf.f * q0x + kf.g * v0x, q1y = kf.f * q0y + kf.g * v0y, q1z = kf.f * q0z + kf.g * v0z;
      const double v1x = kf.fd * q0x + kf.gd * v0x, v1y = kf.fd * q0y + kf.gd * v0y, v1z = kf.fd * q0z + kf.gd * v0z;
      kick_block_vjp<G, false>(a, ex, m, m0, inv_m0, 0.0, q1x, q1y, q1z, v1x, v1y, v1z, vkx, vky, vkz, 0.5 * tb, tb,
                               0.5 * tb, leader);
      double gmu = 0.0;
      kepler_vjp(kf, q0x, q0y, q0z, v0x, v0y, v0z, m0, a.qx, a.qy, a.qz, a.vx, a.vy, a.vz, gmu);
      a.m0 += gmu;
    }
    store_grad(q.grad, ns, slot, a);
    return;
  }
  if constexpr (SCH == WH_KDK) {
    // step = kick block (ta, ti, h) then K(dt): the drift's adjoint first
    TapeRow nxt;
    if (q.n_seg > 0) load_tape_row(q.tape + (size_t)(q.n_seg - 1) * TAPE_ROWS * ns + slot, ns, nxt);
    for (int s = q.n_seg - 1; s >= 0; --s) {
      const TapeRow cur = nxt;
      if (s > 0) load_tape_row(q.tape + (size_t)(s - 1) * TAPE_ROWS * ns + slot, ns, nxt);
      const double q0x = cur.v[0], q0y = cur.v[1], q0z = cur.v[2];
      const double v0x = cur.v[3], v0y = cur.v[4], v0z = cur.v[5];
      const double X = cur.v[6];
      const double vkx = cur.v[7], vky = cur.v[8], vkz = cur.v[9];
      const bool first = q.first_synced && s == 0;
      const double ta = first ? 0.0 : h, ti = first ? h : dt;
      // the drift's starting point: positions after both jumps
      double s2x, s2y, s2z, q3x, q3y, q3z;
      group_momentum<G>(m, vkx, vky, vkz, s2x, s2y, s2z);
      if (GR) {
        double s1x, s1y, s1z;
        group_momentum<G>(m, v0x, v0y, v0z, s1x, s1y, s1z);
        const double k1 = ta * inv_m0, k2 = h * inv_m0;
        q3x = (q0x + k1 * s1x) + k2 * s2x;
        q3y = (q0y + k1 * s1y) + k2 * s2y;
        q3z = (q0z + k1 * s1z) + k2 * s2z;
      } else {
        const double k2 = (ta + h) * inv_m0;
        q3x = q0x + k2 * s2x; q3y = q0y + k2 * s2y; q3z = q0z + k2 * s2z;
      }
      KepFwd k;
      kepler_at_X(q3x, q3y, q3z, vkx, vky, vkz, m0, dt, X, k);
      double gmu = 0.0;
      kepler_vjp(k, q3x, q3y, q3z, vkx, vky, vkz, m0, a.qx, a.qy, a.qz, a.vx, a.vy, a.vz, gmu);
      a.m0 += gmu;
      kick_block_vjp<G, GR>(a, ex, m, m0, inv_m0, kg, q0x, q0y, q0z, v0x, v0y, v0z, vkx, vky, vkz, ta, ti, h,
                            leader);
    }
    store_grad(q.grad, ns, slot, a);
    return;
  }
  // The tape row of step s - 1 is loaded while step s is swept, so the
  // loads' latency hides behind a step's arithmetic (one wavefront per SIMD
  // has nothing else to switch to).
  TapeRow nxt;
  if (q.n_seg > 0) load_tape_row(q.tape + (size_t)(q.n_seg - 1) * TAPE_ROWS * ns + slot, ns, nxt);
  for (int s = q.n_seg - 1; s >= 0; --s) {
    const TapeRow cur = nxt;
    if (s > 0) load_tape_row(q.tape + (size_t)(s - 1) * TAPE_ROWS * ns + slot, ns, nxt);
    double q0x = cur.v[0], q0y = cur.v[1], q0z = cur.v[2];
    double v0x = cur.v[3], v0y = cur.v[4], v0z = cur.v[5];
    double X = cur.v[6];
    double vkx = cur.v[7], vky = cur.v[8], vkz = cur.v[9];
    double tau = (q.first_synced && s == 0) ? h : dt;
    KepFwd k;
    kepler_at_X(q0x, q0y, q0z, v0x, v0y, v0z, m0, tau, X, k);
    double q1x = k.f * q0x + k.g * v0x, q1y = k.f * q0y + k.g * v0y, q1z = k.f * q0z + k.g * v0z;
    double v1x = k.fd * q0x + k.gd * v0x, v1y = k.fd * q0y + k.gd * v0y, v1z = k.fd * q0z + k.gd * v0z;
    if (GR) {
      double s1x, s1y, s1z;
      group_momentum<G>(m, v1x, v1y, v1z, s1x, s1y, s1z);
      double kj = h * inv_m0;
      double q2x = q1x + kj * s1x, q2y = q1y + kj * s1y, q2z = q1z + kj * s1z;
      double v3x = vkx, v3y = vky, v3z = vkz;   // V after the kick, from the tape
      double s3x, s3y, s3z;
      group_momentum<G>(m, v3x, v3y, v3z, s3x, s3y, s3z);
      jump_vjp<G>(a, m, v3x, v3y, v3z, kj, m0, s3x, s3y, s3z, leader);
      double gmu = 0.0;
      interaction_vjp<G>(ex, q2x, q2y, q2z, m, dt, a.vx, a.vy, a.vz, a.qx, a.qy, a.qz, a.m);
      gr_vjp(q2x, q2y, q2z, kg, m0, dt, a.vx, a.vy, a.vz, a.qx, a.qy, a.qz, gmu);
      a.m0 += gmu;
      jump_vjp<G>(a, m, v1x, v1y, v1z, kj, m0, s1x, s1y, s1z, leader);
    } else {
      double v2x = vkx, v2y = vky, v2z = vkz;   // V after the kick, from the tape
      double s2x, s2y, s2z;
      group_momentum<G>(m, v2x, v2y, v2z, s2x, s2y, s2z);
      jump_vjp<G>(a, m, v2x, v2y, v2z, dt * inv_m0, m0, s2x, s2y, s2z, leader);
      interaction_vjp<G>(ex, q1x, q1y, q1z, m, dt, a.vx, a.vy, a.vz, a.qx, a.qy, a.qz, a.m);
    }
    double gmu = 0.0;
    kepler_vjp(k, q0x, q0y, q0z, v0x, v0y, v0z, m0, a.qx, a.qy, a.qz, a.vx, a.vy, a.vz, gmu);
    a.m0 += gmu;
  }
  store_grad(q.grad, ns, slot, a);
}

// Adjoint of the kick block in the pair layout (as kick_block_vjp, for both
// slots of the lane).
template <int G, bool GR>
__device__ __forceinline__ void kick_block_vjp_pair(Grad& a, Grad& b, const PairMass& pm, double ma, double mb,
                                                    double m0, double inv_m0, double kg, const double q0a[3],
                                                    const double v0a[3], const double q0b[3], const double v0b[3],
                                                    const double vka[3], const double vkb[3], double ta, double ti,
                                                    double tc, bool leader) {
  double gqa[3], gqb[3];
  if (GR) {
    double s1[3], s3[3], q2a[3], q2b[3];
    pair_momentum<G>(ma, v0a[0], v0a[1], v0a[2], mb, v0b[0], v0b[1], v0b[2], s1[0], s1[1], s1[2]);
    const double k1 = ta * inv_m0;
    for (int k = 0; k < 3; ++k) { q2a[k] = q0a[k] + k1 * s1[k]; q2b[k] = q0b[k] + k1 * s1[k]; }
    pair_momentum<G>(ma, vka[0], vka[1], vka[2], mb, vkb[0], vkb[1], vkb[2], s3[0], s3[1], s3[2]);
    jump_vjp_pair<G>(a, b, ma, mb, vka, vkb, tc * inv_m0, m0, s3, leader);
    const double gva[3] = {a.vx, a.vy, a.vz}, gvb[3] = {b.vx, b.vy, b.vz};
    gqa[0] = a.qx; gqa[1] = a.qy; gqa[2] = a.qz; gqb[0] = b.qx; gqb[1] = b.qy; gqb[2] = b.qz;
    interaction_vjp_pair<G>(pm, ma, mb, q2a, q2b, gva, gvb, ti, gqa, gqb, a.m, b.m);
    double gmu_a = 0.0, gmu_b = 0.0;
    gr_vjp(q2a[0], q2a[1], q2a[2], kg, m0, ti, gva[0], gva[1], gva[2], gqa[0], gqa[1], gqa[2], gmu_a);
    gr_vjp(q2b[0], q2b[1], q2b[2], kg, m0, ti, gvb[0], gvb[1], gvb[2], gqb[0], gqb[1], gqb[2], gmu_b);
    a.qx = gqa[0]; a.qy = gqa[1]; a.qz = gqa[2]; b.qx = gqb[0]; b.qy = gqb[1]; b.qz = gqb[2];
    a.m0 += gmu_a;
    b.m0 += gmu_b;
    jump_vjp_pair<G>(a, b, ma, mb, v0a, v0b, k1, m0, s1, leader);
  } else {
    double s2[3];
    pair_momentum<G>(ma, vka[0], vka[1], vka[2], mb, vkb[0], vkb[1], vkb[2], s2[0], s2[1], s2[2]);
    jump_vjp_pair<G>(a, b, ma, mb, vka, vkb, (ta + tc) * inv_m0, m0, s2, leader);
    const double gva[3] = {a.vx, a.vy, a.vz}, gvb[3] = {b.vx, b.vy, b.vz};
    gqa[0] = a.qx; gqa[1] = a.qy; gqa[2] = a.qz; gqb[0] = b.qx; gqb[1] = b.qy; gqb[2] = b.qz;
    interaction_vjp_pair<G>(pm, ma, mb, q0a, q0b, gva, gvb, ti, gqa, gqb, a.m, b.m);
    a.qx = gqa[0]; a.qy = gqa[1]; a.qz = gqa[2]; b.qx = gqb[0]; b.qy = gqb[1]; b.qz = gqb[2];
  }
}

// The same two roles in the pair layout: lane l of wave w holds slots
// 128 w + l (a) and 128 w + 64 + l (b).
template <int G, bool GR, int SCH = WH_DKD>
__device__ void adj_record_pair(const AdjParams& q, int sa) {
  const StepParams& p = q.sp;
  const int ns = p.ns, sb = sa + 64;
  Lane A, B;
  load_ck(q.ck_rec, ns, sa, A);
  load_ck(q.ck_rec, ns, sb, B);
  A.m = p.st[6 * ns + sa]; B.m = p.st[6 * ns + sb];
  A.m0 = p.m0s[sa]; B.m0 = p.m0s[sb];
  const PairMass pm = make_pair_mass<G>(A.m, B.m);
  const double dt = p.dts[sa], h = 0.5 * dt;
  const double inv_m0 = 1.0 / A.m0;
  const double kg = GR ? p.kgr * A.m0 * A.m0 : 0.0;
  KepDiag dga{0.0, 1.0e300}, dgb{0.0, 1.0e300};
  if constexpr (SCH == SCHEME_SABA) {
    const int nu = p.saba_n;
    const double c1dt = p.sc[0] * dt;
    for (int s = 0; s < q.n_rec; ++s)
      for (int k = 0; k < nu; ++k) {
        double* ra = q.tape_rec + ((size_t)s * nu + k) * TAPE_ROWS * ns + sa;
        double* rb = ra + 64;
        const double tau = k > 0 ? p.sc[k] * dt : (q.rec_first_synced && s == 0 ? c1dt : 2.0 * c1dt);
        const double tb = p.sd[k] * dt;
        ra[0] = A.qx; ra[ns] = A.qy; ra[2 * ns] = A.qz; ra[3 * ns] = A.vx; ra[4 * ns] = A.vy; ra[5 * ns] = A.vz;
        rb[0] = B.qx; rb[ns] = B.qy; rb[2 * ns] = B.qz; rb[3 * ns] = B.vx; rb[4 * ns] = B.vy; rb[5 * ns] = B.vz;
        ra[6 * ns] = drift(A, A.m0, tau, dga);
        rb[6 * ns] = drift(B, B.m0, tau, dgb);
        double vka[3], vkb[3];
        kick_block_pair<G, false>(A, B, pm, inv_m0, 0.0, 0.5 * tb, tb, 0.5 * tb, vka, vkb);
        ra[7 * ns] = vka[0]; ra[8 * ns] = vka[1]; ra[9 * ns] = vka[2];
        rb[7 * ns] = vkb[0]; rb[8 * ns] = vkb[1]; rb[9 * ns] = vkb[2];
      }
    return;
  }
  if constexpr (SCH == WH_KDK) {
    double ta = q.rec_first_synced ? 0.0 : h;
    double ti = q.rec_first_synced ? h : dt;
    for (int s = 0; s < q.n_rec; ++s) {
      double* ra = q.tape_rec + (size_t)s * TAPE_ROWS * ns + sa;
      double* rb = ra + 64;
      ra[0] = A.qx; ra[ns] = A.qy; ra[2 * ns] = A.qz; ra[3 * ns] = A.vx; ra[4 * ns] = A.vy; ra[5 * ns] = A.vz;
      rb[0] = B.qx; rb[ns] = B.qy; rb[2 * ns] = B.qz; rb[3 * ns] = B.vx; rb[4 * ns] = B.vy; rb[5 * ns] = B.vz;
      double vka[3], vkb[3];
      kick_block_pair<G, GR>(A, B, pm, inv_m0, kg, ta, ti, h, vka, vkb);
      ra[7 * ns] = vka[0]; ra[8 * ns] = vka[1]; ra[9 * ns] = vka[2];
      rb[7 * ns] = vkb[0]; rb[8 * ns] = vkb[1]; rb[9 * ns] = vkb[2];
      ta = h;
      ti = dt;
      ra[6 * ns] = drift(A, A.m0, dt, dga);
      rb[6 * ns] = drift(B, B.m0, dt, dgb);
    }
    return;
  }
  double tk = q.rec_first_synced ? h : dt;
  for (int s = 0; s < q.n_rec; ++s) {
    double* ra = q.tape_rec + (size_t)s * TAPE_ROWS * ns + sa;
    double* rb = ra + 64;
    ra[0] = A.qx; ra[ns] = A.qy; ra[2 * ns] = A.qz; ra[3 * ns] = A.vx; ra[4 * ns] = A.vy; ra[5 * ns] = A.vz;
    rb[0] = B.qx; rb[ns] = B.qy; rb[2 * ns] = B.qz; rb[3 * ns] = B.vx; rb[4 * ns] = B.vy; rb[5 * ns] = B.vz;
    ra[6 * ns] = drift(A, A.m0, tk, dga);
    rb[6 * ns] = drift(B, B.m0, tk, dgb);
    tk = dt;
    double vka[3], vkb[3];
    kick_block_pair<G, GR>(A, B, pm, inv_m0, kg, h, dt, h, vka, vkb);
    ra[7 * ns] = vka[0]; ra[8 * ns] = vka[1]; ra[9 * ns] = vka[2];
    rb[7 * ns] = vkb[0]; rb[8 * ns] = vkb[1]; rb[9 * ns] = vkb[2];
  }
}

template <int G, bool GR, int SCH = WH_DKD>
__device__ void adj_sweep_pair(const AdjParams& q, int sa, int lane) {
  const StepParams& p = q.sp;
  const int ns = p.ns, sb = sa + 64;
  const double ma = p.st[6 * ns + sa], mb = p.st[6 * ns + sb], m0 = p.m0s[sa];
  const PairMass pm = make_pair_mass<G>(ma, mb);
  const double dt = p.dts[sa], h = 0.5 * dt;
  const double inv_m0 = 1.0 / m0;
  const double kg = GR ? p.kgr * m0 * m0 : 0.0;
  Grad a, b;
  load_grad(q.grad, ns, sa, a);
  load_grad(q.grad, ns, sb, b);
  const bool leader = (lane & (G - 1)) == 0;
  if constexpr (SCH == SCHEME_SABA) {
    const int nu = p.saba_n;
    const double c1dt = p.sc[0] * dt;
    const int nunits = q.n_seg * nu;
    TapeRow na, nb;
    if (nunits > 0) load_tape_rows_pair(q.tape + (size_t)(nunits - 1) * TAPE_ROWS * ns + sa, ns, na, nb);
    for (int u = nunits - 1; u >= 0; --u) {
      const int s = u / nu, k = u - s * nu;
      const TapeRow ca = na, cb = nb;
      if (u > 0) load_tape_rows_pair(q.tape + (size_t)(u - 1) * TAPE_ROWS * ns + sa, ns, na, nb);
      const double q0a[3] = {ca.v[0], ca.v[1], ca.v[2]}, v0a[3] = {ca.v[3], ca.v[4], ca.v[5]};
      const double q0b[3] = {cb.v[0], cb.v[1], cb.v[2]}, v0b[3] = {cb.v[3], cb.v[4], cb.v[5]};
      const double vka[3] = {ca.v[7], ca.v[8], ca.v[9]}, vkb[3] = {cb.v[7], cb.v[8], cb.v[9]};
      const double tau = k > 0 ? p.sc[k] * dt : (q.first_synced && s == 0 ? c1dt : 2.0 * c1dt);
      const double tb = p.sd[k] * dt;
      KepFwd ka, kb;
      kepler_at_X(q0a[0], q0a[1], q0a[2], v0a[0], v0a[1], v0a[2], m0, tau, ca.v[6], ka);
      kepler_at_X(q0b[0], q0b[1], q0b[2], v0b[0], v0b[1], v0b[2], m0, tau, cb.v[6], kb);
      double q1a[3], v1a[3], q1b[3], v1b[3];
      for (int c = 0; c < 3; ++c) {
        q1a[c] = ka.f * q0a[c] + ka.g * v0a[c]; v1a[c] = ka.fd * q0a[c] + ka.gd * v0a[c];
        q1b[c] = kb.f * q0b[c] + kb.g * v0b[c]; v1b[c] = kb.fd * q0b[c] + kb.gd * v0b[c];
      }
      kick_block_vjp_pair<G, false>(a, b, pm, ma, mb, m0, inv_m0, 0.0, q1a, v1a, q1b, v1b, vka, vkb, 0.5 * tb, tb,
                                    0.5 * tb, leader);
      double gmu = 0.0;
      kepler_vjp(ka, q0a[0], q0a[1], q0a[2], v0a[0], v0a[1], v0a[2], m0, a.qx, a.qy, a.qz, a.vx, a.vy, a.vz, gmu);
      a.m0 += gmu;
      gmu = 0.0;
      kepler_vjp(kb, q0b[0], q0b[1], q0b[2], v0b[0], v0b[1], v0b[2], m0, b.qx, b.qy, b.qz, b.vx, b.vy, b.vz, gmu);
      b.m0 += gmu;
    }
    store_grad(q.grad, ns, sa, a);
    store_grad(q.grad, ns, sb, b);
    return;
  }
  if constexpr (SCH == WH_KDK) {
    TapeRow na, nb;
    if (q.n_seg > 0) load_tape_rows_pair(q.tape + (size_t)(q.n_seg - 1) * TAPE_ROWS * ns + sa, ns, na, nb);
    for (int s = q.n_seg - 1; s >= 0; --s) {
      const TapeRow ca = na, cb = nb;
      if (s > 0) load_tape_rows_pair(q.tape + (size_t)(s - 1) * TAPE_ROWS * ns + sa, ns, na, nb);
      const double q0a[3] = {ca.v[0], ca.v[1], ca.v[2]}, v0a[3] = {ca.v[3], ca.v[4], ca.v[5]};
      const double q0b[3] = {cb.v[0], cb.v[1], cb.v[2]}, v0b[3] = {cb.v[3], cb.v[4], cb.v[5]};
      const double vka[3] = {ca.v[7], ca.v[8], ca.v[9]}, vkb[3] = {cb.v[7], cb.v[8], cb.v[9]};
      const bool first = q.first_synced && s == 0;
      const double ta = first ? 0.0 : h, ti = first ? h : dt;
      double s2[3], q3a[3], q3b[3];
      pair_momentum<G>(ma, vka[0], vka[1], vka[2], mb, vkb[0], vkb[1], vkb[2], s2[0], s2[1], s2[2]);
      if (GR) {
        double s1[3];
        pair_momentum<G>(ma, v0a[0], v0a[1], v0a[2], mb, v0b[0], v0b[1], v0b[2], s1[0], s1[1], s1[2]);
        const double k1 = ta * inv_m0, k2 = h * inv_m0;
        for (int k = 0; k < 3; ++k) {
          q3a[k] = (q0a[k] + k1 * s1[k]) + k2 * s2[k];
          q3b[k] = (q0b[k] + k1 * s1[k]) + k2 * s2[k];
        }
      } else {
        const double k2 = (ta + h) * inv_m0;
        for (int k = 0; k < 3; ++k) { q3a[k] = q0a[k] + k2 * s2[k]; q3b[k] = q0b[k] + k2 * s2[k]; }
      }
      KepFwd ka, kb;
      kepler_at_X(q3a[0], q3a[1], q3a[2], vka[0], vka[1], vka[2], m0, dt, ca.v[6], ka);
      kepler_at_X(q3b[0], q3b[1], q3b[2], vkb[0], vkb[1], vkb[2], m0, dt, cb.v[6], kb);
      double gmu = 0.0;
      kepler_vjp(ka, q3a[0], q3a[1], q3a[2], vka[0], vka[1], vka[2], m0, a.qx, a.qy, a.qz, a.vx, a.vy, a.vz, gmu);
      a.m0 += gmu;
      gmu = 0.0;
      kepler_vjp(kb, q3b[0], q3b[1], q3b[2], vkb[0], vkb[1], vkb[2], m0, b.qx, b.qy, b.qz, b.vx, b.vy, b.vz, gmu);
      b.m0 += gmu;
      kick_block_vjp_pair<G, GR>(a, b, pm, ma, mb, m0, inv_m0, kg, q0a, v0a, q0b, v0b, vka, vkb, ta, ti, h,
                                 leader);
    }
    store_grad(q.grad, ns, sa, a);
    store_grad(q.grad, ns, sb, b);
    return;
  }
  TapeRow na, nb;
  if (q.n_seg > 0) load_tape_rows_pair(q.tape + (size_t)(q.n_seg - 1) * TAPE_ROWS * ns + sa, ns, na, nb);
  for (int s = q.n_seg - 1; s >= 0; --s) {
    const TapeRow ca = na, cb = nb;
    if (s > 0) load_tape_rows_pair(q.tape + (size_t)(s - 1) * TAPE_ROWS * ns + sa, ns, na, nb);
    const double q0a[3] = {ca.v[0], ca.v[1], ca.v[2]}, v0a[3] = {ca.v[3], ca.v[4], ca.v[5]};
    const double q0b[3] = {cb.v[0], cb.v[1], cb.v[2]}, v0b[3] = {cb.v[3], cb.v[4], cb.v[5]};
    const double vka[3] = {ca.v[7], ca.v[8], ca.v[9]}, vkb[3] = {cb.v[7], cb.v[8], cb.v[9]};
    const double tau = (q.first_synced && s == 0) ? h : dt;
    KepFwd ka, kb;
    kepler_at_X(q0a[0], q0a[1], q0a[2], v0a[0], v0a[1], v0a[2], m0, tau, ca.v[6], ka);
    kepler_at_X(q0b[0], q0b[1], q0b[2], v0b[0], v0b[1], v0b[2], m0, tau, cb.v[6], kb);
    double q1a[3], v1a[3], q1b[3], v1b[3];
    for (int k = 0; k < 3; ++k) {
      q1a[k] = ka.f * q0a[k] + ka.g * v0a[k]; v1a[k] = ka.fd * q0a[k] + ka.gd * v0a[k];
      q1b[k] = kb.f * q0b[k] + kb.g * v0b[k]; v1b[k] = kb.fd * q0b[k] + kb.gd * v0b[k];
    }
    double gqa[3] = {a.qx, a.qy, a.qz}, gqb[3] = {b.qx, b.qy, b.qz};
    if (GR) {
      double s1[3], s3[3];
      pair_momentum<G>(ma, v1a[0], v1a[1], v1a[2], mb, v1b[0], v1b[1], v1b[2], s1[0], s1[1], s1[2]);
      const double kj = h * inv_m0;
      double q2a[3], q2b[3];
      for (int k = 0; k < 3; ++k) { q2a[k] = q1a[k] + kj * s1[k]; q2b[k] = q1b[k] + kj * s1[k]; }
      pair_momentum<G>(ma, vka[0], vka[1], vka[2], mb, vkb[0], vkb[1], vkb[2], s3[0], s3[1], s3[2]);
      jump_vjp_pair<G>(a, b, ma, mb, vka, vkb, kj, m0, s3, leader);
      const double gva[3] = {a.vx, a.vy, a.vz}, gvb[3] = {b.vx, b.vy, b.vz};
      gqa[0] = a.qx; gqa[1] = a.qy; gqa[2] = a.qz; gqb[0] = b.qx; gqb[1] = b.qy; gqb[2] = b.qz;
      interaction_vjp_pair<G>(pm, ma, mb, q2a, q2b, gva, gvb, dt, gqa, gqb, a.m, b.m);
      double gmu_a = 0.0, gmu_b = 0.0;
      gr_vjp(q2a[0], q2a[1], q2a[2], kg, m0, dt, gva[0], gva[1], gva[2], gqa[0], gqa[1], gqa[2], gmu_a);
      gr_vjp(q2b[0], q2b[1], q2b[2], kg, m0, dt, gvb[0], gvb[1], gvb[2], gqb[0], gqb[1], gqb[2], gmu_b);
      a.qx = gqa[0]; a.qy = gqa[1]; a.qz = gqa[2]; b.qx = gqb[0]; b.qy = gqb[1]; b.qz = gqb[2];
      a.m0 += gmu_a;
      b.m0 += gmu_b;
      jump_vjp_pair<G>(a, b, ma, mb, v1a, v1b, kj, m0, s1, leader);
    } else {
      double s2[3];
      pair_momentum<G>(ma, vka[0], vka[1], vka[2], mb, vkb[0], vkb[1], vkb[2], s2[0], s2[1], s2[2]);
      jump_vjp_pair<G>(a, b, ma, mb, vka, vkb, dt * inv_m0, m0, s2, leader);
      const double gva[3] = {a.vx, a.vy, a.vz}, gvb[3] = {b.vx, b.vy, b.vz};
      gqa[0] = a.qx; gqa[1] = a.qy; gqa[2] = a.qz; gqb[0] = b.qx; gqb[1] = b.qy; gqb[2] = b.qz;
      interaction_vjp_pair<G>(pm, ma, mb, q1a, q1b, gva, gvb, dt, gqa, gqb, a.m, b.m);
      a.qx = gqa[0]; a.qy = gqa[1]; a.qz = gqa[2]; b.qx = gqb[0]; b.qy = gqb[1]; b.qz = gqb[2];
    }
    double gmu = 0.0;
    kepler_vjp(ka, q0a[0], q0a[1], q0a[2], v0a[0], v0a[1], v0a[2], m0, a.qx, a.qy, a.qz, a.vx, a.vy, a.vz, gmu);
    a.m0 += gmu;
    gmu = 0.0;
    kepler_vjp(kb, q0b[0], q0b[1], q0b[2], v0b[0], v0b[1], v0b[2], m0, b.qx, b.qy, b.qz, b.vx, b.vy, b.vz, gmu);
    b.m0 += gmu;
  }
  store_grad(q.grad, ns, sa, a);
  store_grad(q.grad, ns, sb, b);
}

template <bool GR, int SCH> __global__ __launch_bounds__(256) void k_adj_segment_pair(AdjParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const bool sweep = wave < q.sweep_waves;
  if (!sweep) wave -= q.sweep_waves;
  if (wave >= p.w8) return;
  const int sa = wave * 128 + lane;
  if (sweep) {
    if (wave < p.w1) adj_sweep_pair<1, GR, SCH>(q, sa, lane);
    else if (wave < p.w2) adj_sweep_pair<2, GR, SCH>(q, sa, lane);
    else adj_sweep_pair<4, GR, SCH>(q, sa, lane);
  } else {
    if (wave < p.w1) adj_record_pair<1, GR, SCH>(q, sa);
    else if (wave < p.w2) adj_record_pair<2, GR, SCH>(q, sa);
    else adj_record_pair<4, GR, SCH>(q, sa);
  }
}

// Waves [0, sweep_waves) sweep one segment, the waves after them record the
// previous segment; each role covers the packing's waves once.
template <bool GR, bool SPLIT, int SCH> __global__ __launch_bounds__(256) void k_adj_segment(AdjParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const bool sweep = wave < q.sweep_waves;
  if (!sweep) wave -= q.sweep_waves;
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (SPLIT) {
    if (sweep) adj_sweep_lane<G_SPLIT, GR, SCH>(q, slot, lane);
    else adj_record_lane<G_SPLIT, GR, SCH>(q, slot, lane);
  } else if (sweep) {
    if (wave < p.w1) adj_sweep_lane<1, GR, SCH>(q, slot, lane);
    else if (wave < p.w2) adj_sweep_lane<2, GR, SCH>(q, slot, lane);
    else if (wave < p.w4) adj_sweep_lane<4, GR, SCH>(q, slot, lane);
    else adj_sweep_lane<8, GR, SCH>(q, slot, lane);
  } else {
    if (wave < p.w1) adj_record_lane<1, GR, SCH>(q, slot, lane);
    else if (wave < p.w2) adj_record_lane<2, GR, SCH>(q, slot, lane);
    else if (wave < p.w4) adj_record_lane<4, GR, SCH>(q, slot, lane);
    else adj_record_lane<8, GR, SCH>(q, slot, lane);
  }
}

// The one-lane-per-system packing keeps the G8 storage, so its reverse sweep
// is the G8 layout's; the recording runs the serial forward step (the same
// arithmetic as k_step_serial, so the recomputed segment equals the forward
// run bit for bit) and writes the tape rows of every slot of the group.
// Slots the wave's body does not integrate (beyond its largest planet count,
// or an empty group) never change: their rows hold the stored state, X = 0
// and the velocity, finite values that the zero masses keep out of every sum.
__device__ __forceinline__ void record_static(const AdjParams& q, int base, int from) {
  const int ns = q.sp.ns;
  const int rows = q.n_rec * (q.sp.saba_n > 0 ? q.sp.saba_n : 1);   // SABA_n: n units per step
  for (int i = from; i < 8; ++i) {
    const int slot = base + i;
    double v[6];
    for (int r = 0; r < 6; ++r) v[r] = q.ck_rec[r * ns + slot];
    for (int s = 0; s < rows; ++s) {
      double* row = q.tape_rec + (size_t)s * TAPE_ROWS * ns + slot;
      for (int r = 0; r < 6; ++r) row[r * ns] = v[r];
      row[6 * ns] = 0.0;
      for (int r = 0; r < 3; ++r) row[(7 + r) * ns] = v[3 + r];
    }
  }
}

template <int NP, bool GR, int SCH>
__device__ void adj_record_serial(const AdjParams& q, int base, int n, double* cl) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  SerialState<NP> S;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int slot = base + i;
    S.qx[i] = q.ck_rec[slot]; S.qy[i] = q.ck_rec[ns + slot]; S.qz[i] = q.ck_rec[2 * ns + slot];
    S.vx[i] = q.ck_rec[3 * ns + slot]; S.vy[i] = q.ck_rec[4 * ns + slot]; S.vz[i] = q.ck_rec[5 * ns + slot];
    S.m[i] = p.st[6 * ns + slot];
#pragma unroll
    for (int k = 0; k < 6; ++k) comp_at(cl, k, i) = q.ck_rec[(6 + k) * ns + slot];
  }
  const double dt = p.dts[base], h = 0.5 * dt;
  const double m0 = p.m0s[base];
  const double inv_m0 = 1.0 / m0;
  const double kg = GR ? p.kgr * m0 * m0 : 0.0;
  KepDiag dg{0.0, 1.0e300};
  if constexpr (SCH == SCHEME_SABA) {
    const int nu = p.saba_n;
    const double c1dt = p.sc[0] * dt;
    for (int s = 0; s < q.n_rec; ++s)
      for (int k = 0; k < nu; ++k) {
        double* row = q.tape_rec + ((size_t)s * nu + k) * TAPE_ROWS * ns + base;
        const double tau = k > 0 ? p.sc[k] * dt : (q.rec_first_synced && s == 0 ? c1dt : 2.0 * c1dt);
        const double tb = p.sd[k] * dt;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          row[i] = S.qx[i]; row[ns + i] = S.qy[i]; row[2 * ns + i] = S.qz[i];
          row[3 * ns + i] = S.vx[i]; row[4 * ns + i] = S.vy[i]; row[5 * ns + i] = S.vz[i];
          Lane L = serial_get(S, cl, i);
          row[6 * ns + i] = serial_drift(L, m0, tau, i < n, dg);
          serial_put(S, cl, i, L);
          __builtin_amdgcn_sched_barrier(0);
        }
        serial_kick_drift<NP, false, true>(S, cl, n, m0, inv_m0, 0.0, 0.5 * tb, tb, 0.5 * tb, 0.0, false, dg,
                                           row + 7 * ns, ns);
      }
    record_static(q, base, NP);
    return;
  }
  if constexpr (SCH == WH_KDK) {
    double ta = q.rec_first_synced ? 0.0 : h;
    double ti = q.rec_first_synced ? h : dt;
    for (int s = 0; s < q.n_rec; ++s) {
      double* row = q.tape_rec + (size_t)s * TAPE_ROWS * ns + base;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        row[i] = S.qx[i]; row[ns + i] = S.qy[i]; row[2 * ns + i] = S.qz[i];
        row[3 * ns + i] = S.vx[i]; row[4 * ns + i] = S.vy[i]; row[5 * ns + i] = S.vz[i];
      }
      serial_kick_drift<NP, GR, true>(S, cl, n, m0, inv_m0, kg, ta, ti, h, dt, true, dg, row + 7 * ns, ns,
                                      row + 6 * ns);
      ta = h;
      ti = dt;
    }
    record_static(q, base, NP);
    return;
  }
  double tk = q.rec_first_synced ? h : dt;
  for (int s = 0; s < q.n_rec; ++s) {
    double* row = q.tape_rec + (size_t)s * TAPE_ROWS * ns + base;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      row[i] = S.qx[i]; row[ns + i] = S.qy[i]; row[2 * ns + i] = S.qz[i];
      row[3 * ns + i] = S.vx[i]; row[4 * ns + i] = S.vy[i]; row[5 * ns + i] = S.vz[i];
      Lane L = serial_get(S, cl, i);
      row[6 * ns + i] = serial_drift(L, m0, tk, i < n, dg);
      serial_put(S, cl, i, L);
      __builtin_amdgcn_sched_barrier(0);
    }
    tk = dt;
    serial_kick_drift<NP, GR, true>(S, cl, n, m0, inv_m0, kg, h, dt, h, 0.0, false, dg, row + 7 * ns, ns);
  }
  record_static(q, base, NP);
}

// Waves [0, sweep_waves) sweep (G8 waves, one planet per lane); the others
// record, one thread per 8-slot group, with SERIAL_LDS_PER_WAVE doubles of
// dynamic LDS per wave (one-wave workgroups).
template <bool GR, int SCH> __global__ __launch_bounds__(64) void k_adj_segment_serial(AdjParams q) {
  extern __shared__ double serial_lds[];
  const StepParams& p = q.sp;
  const int lane = threadIdx.x;
  const int wave = blockIdx.x;
  if (wave < q.sweep_waves) {
    if (wave < p.w8) adj_sweep_lane<8, GR, SCH>(q, wave * 64 + lane, lane);
    return;
  }
  const int g = (wave - q.sweep_waves) * 64 + lane;
  if (g >= p.w8 * 8) return;
  const int base = g * 8;
  if (p.slot_sys[base] < 0) {
    record_static(q, base, 0);
    return;
  }
  double* cl = serial_lds + lane;
  int n = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) n += p.slot_pl[base + i] >= 0;
  int nw = 1;
#pragma unroll
  for (int k = 2; k <= 8; ++k)
    if (__ballot(n >= k) != 0) nw = k;
  switch (nw) {
    case 1: adj_record_serial<1, GR, SCH>(q, base, n, cl); break;
    case 2: adj_record_serial<2, GR, SCH>(q, base, n, cl); break;
    case 3: adj_record_serial<3, GR, SCH>(q, base, n, cl); break;
    case 4: adj_record_serial<4, GR, SCH>(q, base, n, cl); break;
    case 5: adj_record_serial<5, GR, SCH>(q, base, n, cl); break;
    case 6: adj_record_serial<6, GR, SCH>(q, base, n, cl); break;
    case 7: adj_record_serial<7, GR, SCH>(q, base, n, cl); break;
    default: adj_record_serial<8, GR, SCH>(q, base, n, cl); break;
  }
}

// ---------------------------------------------------------------------------
// Reverse mode in Jacobi coordinates (one planet per lane).  The masses enter
// through the interior masses: M_{i-1} = m0 + sum_{j<i} m_j, M_i, 1/M_{i-1},
// w_i = m_i / M_i and ratio_i = m0 / M_{i-1}.  jac_mass_adj turns adjoints of
// M_i, 1/M_{i-1}, w and ratio into those of m_i, m0 and M_{i-1}; the adjoint
// of M_{i-1} is collected per lane and handed to m0 and the inner planets'
// masses by jac_fold_mim1 (a suffix sum over the group).
struct JacAdj {
  double Mi, inv, w, ratio;
};

__device__ __forceinline__ void jac_mass_adj(const JacConst& jc, double m0, const JacAdj& g, Grad& a,
                                             double& gMim1) {
  const double gMi = g.Mi - jc.w * g.w / jc.Mi;
  a.m += g.w / jc.Mi + gMi;
  a.m0 += jc.inv_Mim1 * g.ratio;
  const double ginv = g.inv + m0 * g.ratio;
  gMim1 += gMi - jc.inv_Mim1 * jc.inv_Mim1 * ginv;
}

template <int G> __device__ __forceinline__ void jac_fold_mim1(Grad& a, double& gMim1, int p) {
  a.m0 += gMim1;
  a.m += group_suffix_excl<G>(gMim1, p);
  gMim1 = 0.0;
}

// Adjoint of the Jacobi kick V' += tau a'(X', m) of kick_jacobi at Jacobi
// positions (xx, xy, xz): a.v (unchanged by the kick's adjoint) gives
// dL/dX' (added to a.q), dL/dm, dL/dm0 and the M_{i-1} adjoint.
template <int G, bool GR>
__device__ __forceinline__ void kick_jacobi_vjp(Grad& a, double& gMim1, const Exch<G, 1>& ex, const JacConst& jc,
                                                int p, double m, double m0, double kg, double xx, double xy,
                                                double xz, double tau) {
  // forward values
  const double qx = jac_to_helio<G>(xx, jc.w, p);
  const double qy = jac_to_helio<G>(xy, jc.w, p);
  const double qz = jac_to_helio<G>(xz, jc.w, p);
  double ax, ay, az;
  ex.accel(qx, qy, qz, m, ax, ay, az);
  const double irq = rsqrt_full(fma(qx, qx, fma(qy, qy, qz * qz)));
  const double irq2 = irq * irq, irq3 = irq2 * irq;
  const double irp = rsqrt_full(fma(xx, xx, fma(xy, xy, xz * xz)));
  const double irp2 = irp * irp, irp3 = irp2 * irp;
  const double kp = jc.Mi * irp3, kq = (jc.Mi * jc.ratio) * irq3, wq = m * irq3;
  const double sx = group_suffix_excl<G>(wq * qx, p), sy = group_suffix_excl<G>(wq * qy, p),
               sz = group_suffix_excl<G>(wq * qz, p);
  const double px = group_scan_excl<G>(m * ax, p), py = group_scan_excl<G>(m * ay, p),
               pz = group_scan_excl<G>(m * az, p);
  // adjoint of the acceleration a'
  const double Gx = tau * a.vx, Gy = tau * a.vy, Gz = tau * a.vz;
  JacAdj g{0.0, 0.0, 0.0, 0.0};
  double gqx = -kq * Gx, gqy = -kq * Gy, gqz = -kq * Gz;
  a.qx += kp * Gx; a.qy += kp * Gy; a.qz += kp * Gz;
  const double gkp = Gx * xx + Gy * xy + Gz * xz;
  const double gkq = -(Gx * qx + Gy * qy + Gz * qz);
  // c = ratio * sum_{k>i} wq_k q_k + (sum_{j<i} m_j a_j) / M_{i-1}, entering as -c
  g.ratio -= Gx * sx + Gy * sy + Gz * sz;
  g.inv -= Gx * px + Gy * py + Gz * pz;
  const double ux = group_scan_excl<G>(-jc.ratio * Gx, p), uy = group_scan_excl<G>(-jc.ratio * Gy, p),
               uz = group_scan_excl<G>(-jc.ratio * Gz, p);
  const double gwq = ux * qx + uy * qy + uz * qz;
  gqx += wq * ux; gqy += wq * uy; gqz += wq * uz;
  const double hx = group_suffix_excl<G>(-jc.inv_Mim1 * Gx, p), hy = group_suffix_excl<G>(-jc.inv_Mim1 * Gy, p),
               hz = group_suffix_excl<G>(-jc.inv_Mim1 * Gz, p);
  const double gax = Gx + m * hx, gay = Gy + m * hy, gaz = Gz + m * hz;
  a.m += hx * ax + hy * ay + hz * az;
  if (GR) {
    // + gr_i + (sum_{k>=i} m_k gr_k) / M_{i-1}
    double grx, gry, grz;
    gr_accel(qx, qy, qz, kg, grx, gry, grz);
    const double SGx = group_suffix_incl<G>(m * grx, p), SGy = group_suffix_incl<G>(m * gry, p),
                 SGz = group_suffix_incl<G>(m * grz, p);
    g.inv += Gx * SGx + Gy * SGy + Gz * SGz;
    const double vx = group_scan_incl<G>(jc.inv_Mim1 * Gx, p), vy = group_scan_incl<G>(jc.inv_Mim1 * Gy, p),
                 vz = group_scan_incl<G>(jc.inv_Mim1 * Gz, p);
    a.m += vx * grx + vy * gry + vz * grz;
    double gmu = 0.0;
    gr_vjp(qx, qy, qz, kg, m0, 1.0, Gx + m * vx, Gy + m * vy, Gz + m * vz, gqx, gqy, gqz, gmu);
    a.m0 += gmu;
  }
  // wq = m |q|^-3, kq = M_i ratio |q|^-3, kp = M_i |x'|^-3
  a.m += irq3 * gwq;
  const double girq3 = m * gwq + (jc.Mi * jc.ratio) * gkq;
  g.Mi += jc.ratio * irq3 * gkq + irp3 * gkp;
  g.ratio += jc.Mi * irq3 * gkq;
  const double cq = -3.0 * girq3 * irq3 * irq2;
  gqx += cq * qx; gqy += cq * qy; gqz += cq * qz;
  const double cp = -3.0 * (jc.Mi * gkp) * irp3 * irp2;
  a.qx += cp * xx; a.qy += cp * xy; a.qz += cp * xz;
  // the planet-planet accelerations at the heliocentric positions
  interaction_vjp<G>(ex, qx, qy, qz, m, 1.0, gax, gay, gaz, gqx, gqy, gqz, a.m);
  // q = x' + sum_{j<i} w_j x'_j
  const double tx = group_suffix_excl<G>(gqx, p), ty = group_suffix_excl<G>(gqy, p),
               tz = group_suffix_excl<G>(gqz, p);
  a.qx += gqx + jc.w * tx; a.qy += gqy + jc.w * ty; a.qz += gqz + jc.w * tz;
  g.w += tx * xx + ty * xy + tz * xz;
  jac_mass_adj(jc, m0, g, a, gMim1);
}

// Adjoint of the Jacobi drift K(tau) about mu = G M_i at (x0, v0) with the
// recorded anomaly X: a goes from the drift's output to its input.
__device__ __forceinline__ void jac_drift_vjp(Grad& a, double& gMim1, double mi, double x0x, double x0y, double x0z,
                                              double v0x, double v0y, double v0z, double tau, double X, KepFwd& k) {
  kepler_at_X(x0x, x0y, x0z, v0x, v0y, v0z, mi, tau, X, k);
  double gmu = 0.0;
  kepler_vjp(k, x0x, x0y, x0z, v0x, v0y, v0z, mi, a.qx, a.qy, a.qz, a.vx, a.vy, a.vz, gmu);
  a.m += gmu;      // M_i = M_{i-1} + m_i
  gMim1 += gmu;
}

// Adjoint of the output transform Jacobi -> DHC (jacobi_to_dhc) at the
// Jacobi state (x', v'): a.q, a.v hold dL/dQ, dL/dV and receive dL/dx',
// dL/dv'.
template <int G>
__device__ __forceinline__ void jac_to_dhc_vjp(Grad& a, double& gMim1, const JacConst& jc, int p, double m,
                                               double m0, double xx, double xy, double xz, double vx, double vy,
                                               double vz) {
  const double Mn = m0 + group_sum<G>(m);
  const double ux = jac_to_helio<G>(vx, jc.w, p), uy = jac_to_helio<G>(vy, jc.w, p),
               uz = jac_to_helio<G>(vz, jc.w, p);
  double Px, Py, Pz;
  group_momentum<G>(m, ux, uy, uz, Px, Py, Pz);
  const double Sx = group_sum<G>(a.vx), Sy = group_sum<G>(a.vy), Sz = group_sum<G>(a.vz);
  const double iMn = 1.0 / Mn;
  const double gux = a.vx - m * Sx * iMn, guy = a.vy - m * Sy * iMn, guz = a.vz - m * Sz * iMn;
  a.m -= (ux * Sx + uy * Sy + uz * Sz) * iMn;
  const double gMn = (Px * Sx + Py * Sy + Pz * Sz) * iMn * iMn;   // Mn = m0 + sum_j m_j
  a.m += gMn;
  if (p == 0) a.m0 += gMn;
  JacAdj g{0.0, 0.0, 0.0, 0.0};
  const double tux = group_suffix_excl<G>(gux, p), tuy = group_suffix_excl<G>(guy, p),
               tuz = group_suffix_excl<G>(guz, p);
  a.vx = gux + jc.w * tux; a.vy = guy + jc.w * tuy; a.vz = guz + jc.w * tuz;
  const double tqx = group_suffix_excl<G>(a.qx, p), tqy = group_suffix_excl<G>(a.qy, p),
               tqz = group_suffix_excl<G>(a.qz, p);
  g.w = tux * vx + tuy * vy + tuz * vz + tqx * xx + tqy * xy + tqz * xz;
  a.qx += jc.w * tqx; a.qy += jc.w * tqy; a.qz += jc.w * tqz;
  jac_mass_adj(jc, m0, g, a, gMim1);
}

// Adjoint of the input transform DHC -> Jacobi (dhc_to_jacobi) at the DHC
// state (Q, V): a.q, a.v hold dL/dx', dL/dv' and receive dL/dQ, dL/dV.
template <int G>
__device__ __forceinline__ void dhc_to_jac_vjp(Grad& a, double& gMim1, const JacConst& jc, int p, double m,
                                               double m0, double Qx, double Qy, double Qz, double Vx, double Vy,
                                               double Vz) {
  double Px, Py, Pz;
  group_momentum<G>(m, Vx, Vy, Vz, Px, Py, Pz);
  const double ux = Vx + Px / m0, uy = Vy + Py / m0, uz = Vz + Pz / m0;
  JacAdj g{0.0, 0.0, 0.0, 0.0};
  // x' = Q - (sum_{j<i} m_j Q_j) / M_{i-1}
  const double bx = group_suffix_excl<G>(jc.inv_Mim1 * a.qx, p), by = group_suffix_excl<G>(jc.inv_Mim1 * a.qy, p),
               bz = group_suffix_excl<G>(jc.inv_Mim1 * a.qz, p);
  g.inv -= a.qx * group_scan_excl<G>(m * Qx, p) + a.qy * group_scan_excl<G>(m * Qy, p) +
           a.qz * group_scan_excl<G>(m * Qz, p);
  a.m -= Qx * bx + Qy * by + Qz * bz;
  a.qx -= m * bx; a.qy -= m * by; a.qz -= m * bz;
  // v' = u - (sum_{j<i} m_j u_j) / M_{i-1}
  const double cx = group_suffix_excl<G>(jc.inv_Mim1 * a.vx, p), cy = group_suffix_excl<G>(jc.inv_Mim1 * a.vy, p),
               cz = group_suffix_excl<G>(jc.inv_Mim1 * a.vz, p);
  g.inv -= a.vx * group_scan_excl<G>(m * ux, p) + a.vy * group_scan_excl<G>(m * uy, p) +
           a.vz * group_scan_excl<G>(m * uz, p);
  a.m -= ux * cx + uy * cy + uz * cz;
  const double gux = a.vx - m * cx, guy = a.vy - m * cy, guz = a.vz - m * cz;
  // u = V + (sum_j m_j V_j) / m0
  const double Sx = group_sum<G>(gux), Sy = group_sum<G>(guy), Sz = group_sum<G>(guz);
  a.vx = gux + m * Sx / m0; a.vy = guy + m * Sy / m0; a.vz = guz + m * Sz / m0;
  a.m += (Vx * Sx + Vy * Sy + Vz * Sz) / m0;
  if (p == 0) a.m0 -= (Px * Sx + Py * Sy + Pz * Sz) / (m0 * m0);
  jac_mass_adj(jc, m0, g, a, gMim1);
}

// Recording and sweeping of a Jacobi context (per lane; tape rows as in DHC:
// the state at the start of the step or unit, the drift's X, V' after the
// kick).
template <int G, bool GR, int SCH>
__device__ void adj_record_jac(const AdjParams& q, int slot, int lane) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  const int pg = lane & (G - 1);
  Lane L;
  load_ck(q.ck_rec, ns, slot, L);
  L.m = p.st[6 * ns + slot];
  L.m0 = p.m0s[slot];
  Exch<G, 1> ex;
  ex.init(lane, L.m);
  const JacConst jc = jac_const<G>(L.m0, L.m, pg);
  const double dt = p.dts[slot], h = 0.5 * dt;
  const double kg = GR ? p.kgr * L.m0 * L.m0 : 0.0;
  KepDiag dg{0.0, 1.0e300};
  auto put_state = [&](double* row) {
    row[0] = L.qx; row[ns] = L.qy; row[2 * ns] = L.qz;
    row[3 * ns] = L.vx; row[4 * ns] = L.vy; row[5 * ns] = L.vz;
  };
  double vkx, vky, vkz;
  if constexpr (SCH == SCHEME_SABA) {
    const int nu = p.saba_n;
    const double c1dt = p.sc[0] * dt;
    for (int s = 0; s < q.n_rec; ++s)
      for (int k = 0; k < nu; ++k) {
        double* row = q.tape_rec + ((size_t)s * nu + k) * TAPE_ROWS * ns + slot;
        const double tau = k > 0 ? p.sc[k] * dt : (q.rec_first_synced && s == 0 ? c1dt : 2.0 * c1dt);
        put_state(row);
        row[6 * ns] = drift(L, jc.Mi, tau, dg);
        kick_jacobi<G, 1, GR>(L, ex, jc, pg, p.sd[k] * dt, vkx, vky, vkz, kg);
        row[7 * ns] = vkx; row[8 * ns] = vky; row[9 * ns] = vkz;
      }
  } else if constexpr (SCH == WH_KDK) {
    double ti = q.rec_first_synced ? h : dt;
    for (int s = 0; s < q.n_rec; ++s) {
      double* row = q.tape_rec + (size_t)s * TAPE_ROWS * ns + slot;
      put_state(row);
      kick_jacobi<G, 1, GR>(L, ex, jc, pg, ti, vkx, vky, vkz, kg);
      row[7 * ns] = vkx; row[8 * ns] = vky; row[9 * ns] = vkz;
      ti = dt;
      row[6 * ns] = drift(L, jc.Mi, dt, dg);
    }
  } else {
    double tk = q.rec_first_synced ? h : dt;
    for (int s = 0; s < q.n_rec; ++s) {
      double* row = q.tape_rec + (size_t)s * TAPE_ROWS * ns + slot;
      put_state(row);
      row[6 * ns] = drift(L, jc.Mi, tk, dg);
      tk = dt;
      kick_jacobi<G, 1, GR>(L, ex, jc, pg, dt, vkx, vky, vkz, kg);
      row[7 * ns] = vkx; row[8 * ns] = vky; row[9 * ns] = vkz;
    }
  }
}

template <int G, bool GR, int SCH>
__device__ void adj_sweep_jac(const AdjParams& q, int slot, int lane) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  const int pg = lane & (G - 1);
  const double m = p.st[6 * ns + slot], m0 = p.m0s[slot];
  Exch<G, 1> ex;
  ex.init(lane, m);
  const JacConst jc = jac_const<G>(m0, m, pg);
  const double dt = p.dts[slot], h = 0.5 * dt;
  const double kg = GR ? p.kgr * m0 * m0 : 0.0;
  Grad a;
  load_grad(q.grad, ns, slot, a);
  double gMim1 = 0.0;
  KepFwd k;
  if constexpr (SCH == SCHEME_SABA) {
    const int nu = p.saba_n;
    const double c1dt = p.sc[0] * dt;
    const int nunits = q.n_seg * nu;
    TapeRow nxt;
    if (nunits > 0) load_tape_row(q.tape + (size_t)(nunits - 1) * TAPE_ROWS * ns + slot, ns, nxt);
    for (int u = nunits - 1; u >= 0; --u) {
      const int s = u / nu, kk = u - s * nu;
      const TapeRow cur = nxt;
      if (u > 0) load_tape_row(q.tape + (size_t)(u - 1) * TAPE_ROWS * ns + slot, ns, nxt);
      const double tau = kk > 0 ? p.sc[kk] * dt : (q.first_synced && s == 0 ? c1dt : 2.0 * c1dt);
      const double x0x = cur.v[0], x0y = cur.v[1], x0z = cur.v[2];
      const double v0x = cur.v[3], v0y = cur.v[4], v0z = cur.v[5];
      kepler_at_X(x0x, x0y, x0z, v0x, v0y, v0z, jc.Mi, tau, cur.v[6], k);
      const double x1x = k.f * x0x + k.g * v0x, x1y = k.f * x0y + k.g * v0y, x1z = k.f * x0z + k.g * v0z;
      kick_jacobi_vjp<G, GR>(a, gMim1, ex, jc, pg, m, m0, kg, x1x, x1y, x1z, p.sd[kk] * dt);
      jac_drift_vjp(a, gMim1, jc.Mi, x0x, x0y, x0z, v0x, v0y, v0z, tau, cur.v[6], k);
      jac_fold_mim1<G>(a, gMim1, pg);
    }
  } else if constexpr (SCH == WH_KDK) {
    TapeRow nxt;
    if (q.n_seg > 0) load_tape_row(q.tape + (size_t)(q.n_seg - 1) * TAPE_ROWS * ns + slot, ns, nxt);
    for (int s = q.n_seg - 1; s >= 0; --s) {
      const TapeRow cur = nxt;
      if (s > 0) load_tape_row(q.tape + (size_t)(s - 1) * TAPE_ROWS * ns + slot, ns, nxt);
      const double x0x = cur.v[0], x0y = cur.v[1], x0z = cur.v[2];
      const double ti = (q.first_synced && s == 0) ? h : dt;
      // K(dt) from (x0, V' after the kick), then the kick at x0
      jac_drift_vjp(a, gMim1, jc.Mi, x0x, x0y, x0z, cur.v[7], cur.v[8], cur.v[9], dt, cur.v[6], k);
      kick_jacobi_vjp<G, GR>(a, gMim1, ex, jc, pg, m, m0, kg, x0x, x0y, x0z, ti);
      jac_fold_mim1<G>(a, gMim1, pg);
    }
  } else {
    TapeRow nxt;
    if (q.n_seg > 0) load_tape_row(q.tape + (size_t)(q.n_seg - 1) * TAPE_ROWS * ns + slot, ns, nxt);
    for (int s = q.n_seg - 1; s >= 0; --s) {
      const TapeRow cur = nxt;
      if (s > 0) load_tape_row(q.tape + (size_t)(s - 1) * TAPE_ROWS * ns + slot, ns, nxt);
      const double tau = (q.first_synced && s == 0) ? h : dt;
      const double x0x = cur.v[0], x0y = cur.v[1], x0z = cur.v[2];
      const double v0x = cur.v[3], v0y = cur.v[4], v0z = cur.v[5];
      kepler_at_X(x0x, x0y, x0z, v0x, v0y, v0z, jc.Mi, tau, cur.v[6], k);
      const double x1x = k.f * x0x + k.g * v0x, x1y = k.f * x0y + k.g * v0y, x1z = k.f * x0z + k.g * v0z;
      kick_jacobi_vjp<G, GR>(a, gMim1, ex, jc, pg, m, m0, kg, x1x, x1y, x1z, dt);
      jac_drift_vjp(a, gMim1, jc.Mi, x0x, x0y, x0z, v0x, v0y, v0z, tau, cur.v[6], k);
      jac_fold_mim1<G>(a, gMim1, pg);   // per step, so the sums do not depend on the segments
    }
  }
  store_grad(q.grad, ns, slot, a);
}

template <bool GR, int SCH> __global__ __launch_bounds__(256) void k_adj_segment_jac(AdjParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const bool sweep = wave < q.sweep_waves;
  if (!sweep) wave -= q.sweep_waves;
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (sweep) {
    if (wave < p.w1) adj_sweep_jac<1, GR, SCH>(q, slot, lane);
    else if (wave < p.w2) adj_sweep_jac<2, GR, SCH>(q, slot, lane);
    else if (wave < p.w4) adj_sweep_jac<4, GR, SCH>(q, slot, lane);
    else adj_sweep_jac<8, GR, SCH>(q, slot, lane);
  } else {
    if (wave < p.w1) adj_record_jac<1, GR, SCH>(q, slot, lane);
    else if (wave < p.w2) adj_record_jac<2, GR, SCH>(q, slot, lane);
    else if (wave < p.w4) adj_record_jac<4, GR, SCH>(q, slot, lane);
    else adj_record_jac<8, GR, SCH>(q, slot, lane);
  }
}

// Adjoint of the corrector C (or C^-1) entered at the lane state L0: a.q,
// a.v hold dL/d(its output) on entry and dL/d(its input) on return; mass
// terms go to a.m, a.m0 and gMim1.  The substeps' inputs are recomputed
// from L0 (the sequence is at most 15 substeps long, and this runs once per
// reverse pass).
template <int G, bool GR>
__device__ void corrector_vjp(const StepParams& p, const Lane& L0, int lane, bool inverse, Grad& a,
                              double& gMim1) {
  const int pg = lane & (G - 1);
  const JacConst jc = jac_const<G>(L0.m0, L0.m, pg);
  Exch<G, 1> ex;
  ex.init(lane, L0.m);
  const double kg = GR ? p.kgr * L0.m0 * L0.m0 : 0.0;
  for (int j = 5 * p.corr_n - 1; j >= 0; --j) {
    Lane L = L0;
    corrector_run<G, GR>(p, L, lane, inverse, j);   // the state entering substep j
    double tau;
    if (corrector_substep(p, j, inverse, L0.dt, tau)) {
      Lane Lx = L;
      KepDiag dg{0.0, 1.0e300};
      const double X = drift(Lx, jc.Mi, tau, dg);
      KepFwd k;
      jac_drift_vjp(a, gMim1, jc.Mi, L.qx, L.qy, L.qz, L.vx, L.vy, L.vz, tau, X, k);
    } else {
      kick_jacobi_vjp<G, GR>(a, gMim1, ex, jc, pg, L.m, L.m0, kg, L.qx, L.qy, L.qz, tau);
    }
  }
}

// The synchronized output of a Jacobi context: the pending operation (K(h),
// K(c_1 dt) or the half kick) on the stored state, then the transform to
// DHC.  The grad rows hold the caller's dL/dQ_T, dL/dV_T on entry and
// dL/d(stored state) on return.
template <int G, bool GR, int SCH> __device__ void adj_init_jac_lane(const AdjParams& q, int slot, int lane,
                                                                   int synced) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  const int pg = lane & (G - 1);
  Grad a;
  load_grad(q.grad, ns, slot, a);
  Lane L;
  load_ck(q.ck, ns, slot, L);
  L.m = p.st[6 * ns + slot];
  const double m0 = p.m0s[slot], dt = p.dts[slot];
  L.m0 = m0;
  L.dt = dt;
  const double kg = GR ? p.kgr * m0 * m0 : 0.0;
  const JacConst jc = jac_const<G>(m0, L.m, pg);
  Exch<G, 1> ex;
  ex.init(lane, L.m);
  double gMim1 = 0.0;
  const double x0x = L.qx, x0y = L.qy, x0z = L.qz, v0x = L.vx, v0y = L.vy, v0z = L.vz;
  double tau = 0.0, X = 0.0;
  if (!synced) {
    KepDiag dg{0.0, 1.0e300};
    if (SCH == WH_KDK) {
      double vkx, vky, vkz;
      kick_jacobi<G, 1, GR>(L, ex, jc, pg, 0.5 * dt, vkx, vky, vkz, kg);
    } else {
      tau = SCH == SCHEME_SABA ? p.sc[0] * dt : 0.5 * dt;
      X = drift(L, jc.Mi, tau, dg);
    }
  }
  // the output's corrector C (real coordinates) sits between the pending
  // operation and the transform
  const Lane Lp = L;
  if (p.corr_n > 0) apply_corrector<G, GR>(p, L, lane, false);
  jac_to_dhc_vjp<G>(a, gMim1, jc, pg, L.m, m0, L.qx + L.cqx, L.qy + L.cqy, L.qz + L.cqz, L.vx + L.cvx,
                    L.vy + L.cvy, L.vz + L.cvz);
  if (p.corr_n > 0) corrector_vjp<G, GR>(p, Lp, lane, false, a, gMim1);
  if (!synced) {
    if (SCH == WH_KDK) {
      kick_jacobi_vjp<G, GR>(a, gMim1, ex, jc, pg, L.m, m0, kg, x0x, x0y, x0z, 0.5 * dt);
    } else {
      KepFwd k;
      jac_drift_vjp(a, gMim1, jc.Mi, x0x, x0y, x0z, v0x, v0y, v0z, tau, X, k);
    }
  }
  jac_fold_mim1<G>(a, gMim1, pg);
  store_grad(q.grad, ns, slot, a);
}

template <bool GR, int SCH> __global__ __launch_bounds__(256) void k_adj_init_jac(AdjParams q, int synced) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (wave < p.w1) adj_init_jac_lane<1, GR, SCH>(q, slot, lane, synced);
  else if (wave < p.w2) adj_init_jac_lane<2, GR, SCH>(q, slot, lane, synced);
  else if (wave < p.w4) adj_init_jac_lane<4, GR, SCH>(q, slot, lane, synced);
  else adj_init_jac_lane<8, GR, SCH>(q, slot, lane, synced);
}

// Before the outputs: the grad rows hold dL/d(initial Jacobi state); the
// input transform's adjoint at the initial DHC state (rebuilt from the first
// checkpoint) turns them into dL/d(Q0, V0) and adds the mass terms.  With a
// corrector the stored initial state is C^-1 of the transformed input: C
// rebuilds that input (to rounding) and C^-1's adjoint runs first.
template <int G, bool GR> __device__ void adj_in_jac_lane(const AdjParams& q, int slot, int lane) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  const int pg = lane & (G - 1);
  Grad a;
  load_grad(q.grad, ns, slot, a);
  Lane L;
  load_ck(q.ck, ns, slot, L);
  L.m = p.st[6 * ns + slot];
  L.m0 = p.m0s[slot];
  L.dt = p.dts[slot];
  double gMim1 = 0.0;
  if (p.corr_n > 0) {
    apply_corrector<G, GR>(p, L, lane, false);
    corrector_vjp<G, GR>(p, L, lane, true, a, gMim1);
  }
  L.qx += L.cqx; L.qy += L.cqy; L.qz += L.cqz;
  L.vx += L.cvx; L.vy += L.cvy; L.vz += L.cvz;
  const JacConst jc = jac_const<G>(L.m0, L.m, pg);
  jacobi_to_dhc<G>(L, pg);
  dhc_to_jac_vjp<G>(a, gMim1, jc, pg, L.m, L.m0, L.qx, L.qy, L.qz, L.vx, L.vy, L.vz);
  jac_fold_mim1<G>(a, gMim1, pg);
  store_grad(q.grad, ns, slot, a);
}

template <bool GR> __global__ __launch_bounds__(256) void k_adj_in_jac(AdjParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (wave < p.w1) adj_in_jac_lane<1, GR>(q, slot, lane);
  else if (wave < p.w2) adj_in_jac_lane<2, GR>(q, slot, lane);
  else if (wave < p.w4) adj_in_jac_lane<4, GR>(q, slot, lane);
  else adj_in_jac_lane<8, GR>(q, slot, lane);
}

// Adjoint of the closing drift of the synchronized output (K(h), or K(c_1 dt)
// for SABA_n; the identity when no step was taken), from the caller's
// dL/dQ_T, dL/dV_T.
__global__ void k_adj_init(AdjParams q, int synced) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= ns) return;
  int sys = p.slot_sys[slot], pl = p.slot_pl[slot];
  Grad a{0, 0, 0, 0, 0, 0, 0, 0};
  if (sys >= 0 && pl >= 0) {
    size_t o = ((size_t)sys * 8 + pl) * 3;
    a.qx = q.gQ_T[o]; a.qy = q.gQ_T[o + 1]; a.qz = q.gQ_T[o + 2];
    a.vx = q.gV_T[o]; a.vy = q.gV_T[o + 1]; a.vz = q.gV_T[o + 2];
    if (!synced) {
      double qx = q.ck[slot], qy = q.ck[ns + slot], qz = q.ck[2 * ns + slot];
      double vx = q.ck[3 * ns + slot], vy = q.ck[4 * ns + slot], vz = q.ck[5 * ns + slot];
      // the pending drift: K(dt/2), or K(c_1 dt) for SABA_n
      double m0 = p.m0s[slot], h = p.saba_n > 0 ? p.sc[0] * p.dts[slot] : 0.5 * p.dts[slot];
      KepDiag dg{0.0, 1.0e300};
      KepCoef kc;
      double X = kepler_coeffs<KEP_NH, KEP_NN, KEP_KH, KEP_KN>(qx, qy, qz, vx, vy, vz, m0, h, dg, kc);
      KepFwd k;
      kepler_at_X(qx, qy, qz, vx, vy, vz, m0, h, X, k);
      double gmu = 0.0;
      kepler_vjp(k, qx, qy, qz, vx, vy, vz, m0, a.qx, a.qy, a.qz, a.vx, a.vy, a.vz, gmu);
      a.m0 = gmu;
    }
  }
  store_grad(q.grad, ns, slot, a);
}

// KDK: the synchronized output applies the pending half kick J(h) [I +
// GR](h) to the stored state; its adjoint needs the group's sums, so it runs
// per lane group.  The forward kick is re-evaluated at the stored state for
// the velocity after it.
__device__ __forceinline__ Grad gather_grad_T(const AdjParams& q, int slot) {
  const StepParams& p = q.sp;
  Grad a{0, 0, 0, 0, 0, 0, 0, 0};
  const int sys = p.slot_sys[slot], pl = p.slot_pl[slot];
  if (sys >= 0 && pl >= 0) {
    const size_t o = ((size_t)sys * 8 + pl) * 3;
    a.qx = q.gQ_T[o]; a.qy = q.gQ_T[o + 1]; a.qz = q.gQ_T[o + 2];
    a.vx = q.gV_T[o]; a.vy = q.gV_T[o + 1]; a.vz = q.gV_T[o + 2];
  }
  return a;
}

template <int G, bool GR> __device__ void adj_init_kdk_lane(const AdjParams& q, int slot, int lane, int synced) {
  const StepParams& p = q.sp;
  const int ns = p.ns;
  Grad a = gather_grad_T(q, slot);
  if (!synced) {
    Lane L;
    load_ck(q.ck, ns, slot, L);
    L.m = p.st[6 * ns + slot];
    const double m0 = p.m0s[slot], h = 0.5 * p.dts[slot], inv_m0 = 1.0 / m0;
    const double kg = GR ? p.kgr * m0 * m0 : 0.0;
    Exch<G, 1> ex;
    ex.init(lane, L.m);
    const double q0x = L.qx, q0y = L.qy, q0z = L.qz, v0x = L.vx, v0y = L.vy, v0z = L.vz;
    double vkx, vky, vkz;
    kick_block<G, GR, 1>(L, ex, inv_m0, kg, h, h, 0.0, vkx, vky, vkz);
    const bool leader = G == G_SPLIT ? (lane & 14) == 0 : (lane & (G - 1)) == 0;
    kick_block_vjp<G, GR>(a, ex, L.m, m0, inv_m0, kg, q0x, q0y, q0z, v0x, v0y, v0z, vkx, vky, vkz, h, h, 0.0,
                          leader);
  }
  store_grad(q.grad, ns, slot, a);
}

template <int G, bool GR> __device__ void adj_init_kdk_pair(const AdjParams& q, int sa, int lane, int synced) {
  const StepParams& p = q.sp;
  const int ns = p.ns, sb = sa + 64;
  Grad a = gather_grad_T(q, sa), b = gather_grad_T(q, sb);
  if (!synced) {
    Lane A, B;
    load_ck(q.ck, ns, sa, A);
    load_ck(q.ck, ns, sb, B);
    A.m = p.st[6 * ns + sa]; B.m = p.st[6 * ns + sb];
    const double m0 = p.m0s[sa], h = 0.5 * p.dts[sa], inv_m0 = 1.0 / m0;
    const double kg = GR ? p.kgr * m0 * m0 : 0.0;
    const PairMass pm = make_pair_mass<G>(A.m, B.m);
    const double q0a[3] = {A.qx, A.qy, A.qz}, v0a[3] = {A.vx, A.vy, A.vz};
    const double q0b[3] = {B.qx, B.qy, B.qz}, v0b[3] = {B.vx, B.vy, B.vz};
    double vka[3], vkb[3];
    kick_block_pair<G, GR>(A, B, pm, inv_m0, kg, h, h, 0.0, vka, vkb);
    kick_block_vjp_pair<G, GR>(a, b, pm, A.m, B.m, m0, inv_m0, kg, q0a, v0a, q0b, v0b, vka, vkb, h, h, 0.0,
                               (lane & (G - 1)) == 0);
  }
  store_grad(q.grad, ns, sa, a);
  store_grad(q.grad, ns, sb, b);
}

// LAYOUT: 0 one planet per lane (pow2, G8 and the serial packing's G8
// storage), 1 split, 2 pair.
template <bool GR, int LAYOUT> __global__ __launch_bounds__(256) void k_adj_init_kdk(AdjParams q, int synced) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  if (LAYOUT == 2) {
    const int sa = wave * 128 + lane;
    if (wave < p.w1) adj_init_kdk_pair<1, GR>(q, sa, lane, synced);
    else if (wave < p.w2) adj_init_kdk_pair<2, GR>(q, sa, lane, synced);
    else adj_init_kdk_pair<4, GR>(q, sa, lane, synced);
    return;
  }
  const int slot = wave * 64 + lane;
  if (LAYOUT == 1) adj_init_kdk_lane<G_SPLIT, GR>(q, slot, lane, synced);
  else if (wave < p.w1) adj_init_kdk_lane<1, GR>(q, slot, lane, synced);
  else if (wave < p.w2) adj_init_kdk_lane<2, GR>(q, slot, lane, synced);
  else if (wave < p.w4) adj_init_kdk_lane<4, GR>(q, slot, lane, synced);
  else adj_init_kdk_lane<8, GR>(q, slot, lane, synced);
}

template <int G> __device__ void adj_finish_lane(const AdjParams& q, int slot, int lane) {
  const StepParams& p = q.sp;
  Grad a;
  load_grad(q.grad, p.ns, slot, a);
  double g0 = group_sum<G>(a.m0);
  int sys = p.slot_sys[slot], pl = p.slot_pl[slot];
  if (sys >= 0 && pl >= 0 && (G != G_SPLIT || (lane & 1) == 0)) {
    size_t o = ((size_t)sys * 8 + pl) * 3;
    q.gQ_0[o] = a.qx; q.gQ_0[o + 1] = a.qy; q.gQ_0[o + 2] = a.qz;
    q.gV_0[o] = a.vx; q.gV_0[o + 1] = a.vy; q.gV_0[o + 2] = a.vz;
    q.gm[(size_t)sys * 8 + pl] = a.m;
  }
  if ((lane & (G - 1)) == 0 && sys >= 0) q.gm0[sys] = g0;
}

template <int G> __device__ void adj_finish_pair(const AdjParams& q, int sa, int lane) {
  const StepParams& p = q.sp;
  Grad g[2];
  load_grad(q.grad, p.ns, sa, g[0]);
  load_grad(q.grad, p.ns, sa + 64, g[1]);
  const double g0 = group_sum<G>(g[0].m0 + g[1].m0);
  for (int k = 0; k < 2; ++k) {
    const int slot = sa + 64 * k;
    const int sys = p.slot_sys[slot], pl = p.slot_pl[slot];
    if (sys >= 0 && pl >= 0) {
      size_t o = ((size_t)sys * 8 + pl) * 3;
      q.gQ_0[o] = g[k].qx; q.gQ_0[o + 1] = g[k].qy; q.gQ_0[o + 2] = g[k].qz;
      q.gV_0[o] = g[k].vx; q.gV_0[o + 1] = g[k].vy; q.gV_0[o + 2] = g[k].vz;
      q.gm[(size_t)sys * 8 + pl] = g[k].m;
    }
  }
  const int sys = p.slot_sys[sa];
  if ((lane & (G - 1)) == 0 && sys >= 0) q.gm0[sys] = g0;
}

__global__ __launch_bounds__(256) void k_adj_finish_pair(AdjParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int sa = wave * 128 + lane;
  if (wave < p.w1) adj_finish_pair<1>(q, sa, lane);
  else if (wave < p.w2) adj_finish_pair<2>(q, sa, lane);
  else adj_finish_pair<4>(q, sa, lane);
}

template <bool SPLIT> __global__ __launch_bounds__(256) void k_adj_finish(AdjParams q) {
  const StepParams& p = q.sp;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wave >= p.w8) return;
  const int slot = wave * 64 + lane;
  if (SPLIT) adj_finish_lane<G_SPLIT>(q, slot, lane);
  else if (wave < p.w1) adj_finish_lane<1>(q, slot, lane);
  else if (wave < p.w2) adj_finish_lane<2>(q, slot, lane);
  else if (wave < p.w4) adj_finish_lane<4>(q, slot, lane);
  else adj_finish_lane<8>(q, slot, lane);
}

// ---------------------------------------------------------------------------
// Load the caller's arrays into the slot layout.  Padding lanes get a zero
// mass and a distinct circular orbit far outside the system, so their
// Kepler solves stay finite and their positions never coincide with another
// lane's (their zero mass keeps them out of every other lane's sums).
__global__ void k_gather(double* st, int ns, double* m0s, double* dts, const int* slot_sys, const int* slot_pl,
                         const double* m0, const double* m, const double* Q, const double* V, const double* dt,
                         int split) {
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= ns) return;
  int s = slot_sys[slot], pl = slot_pl[slot];
  double M0 = s >= 0 ? m0[s] : 1.0;
  m0s[slot] = M0;
  dts[slot] = s >= 0 ? dt[s] : 1.0e-3;
  if (s >= 0 && pl >= 0) {
    size_t o = ((size_t)s * 8 + pl) * 3;
    for (int c = 0; c < 3; ++c) {
      st[c * ns + slot] = Q[o + c];
      st[(3 + c) * ns + slot] = V[o + c];
    }
    st[6 * ns + slot] = m[(size_t)s * 8 + pl];
  } else {
    // distinct for the two slots of a lane in the pair layout; in the split
    // layout the planet's index, the same for both of its copies
    int k = split ? (slot >> 1) & 7 : (slot & 7) | ((slot >> 3) & 8);
    double a = 1.0e4 * (1.0 + 0.25 * k);
    double ph = 0.3 + 0.7 * k;
    double vc = sqrt(M0 / a);
    st[slot] = a * cos(ph);
    st[ns + slot] = a * sin(ph);
    st[2 * ns + slot] = 0.0;
    st[3 * ns + slot] = -vc * sin(ph);
    st[4 * ns + slot] = vc * cos(ph);
    st[5 * ns + slot] = 0.0;
    st[6 * ns + slot] = 0.0;
  }
  for (int r = 7; r < ROWS; ++r) st[r * ns + slot] = 0.0;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Header of a state snapshot (wh_save_state): what a restoring context must
// match, and the step count of the saved state.
struct StateHeader {
  uint64_t magic;
  int32_t version, S, ns, packing, coords, scheme, gr, rows;
  int64_t steps_done;
};
constexpr uint64_t STATE_MAGIC = 0x5748535441544531ull;   // "WHSTATE1"

__global__ void k_write_header(StateHeader h, StateHeader* dst) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = h;
}

__global__ void k_copy_u32(uint32_t* dst, const uint32_t* src, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

// ===========================================================================
// Kepler-solver envelope (Sec. 3.2 test of Fig. 1, App. A search): massless
// test particles about a star, each advanced n_steps Kepler drifts of its own
// tau with run-time iteration counts, and the relative change of the
// osculating semi-major axis a = 1 / (2/r - v^2/mu), which the exact flow
// conserves.  One lane per particle; the state is plain binary64, the update
// Q' = Q + ((f - 1) Q + g V), V' = V + (f' Q + (g' - 1) V).
// ===========================================================================
struct EnvParams {
  const double* Q;   // [n*3]
  const double* V;
  const double* mu;  // [n]
  const double* tau; // [n]
  double* Q_out;     // [n*3] or null (may alias Q)
  double* V_out;
  double* a_err;     // [n]
  double* zmax_out;  // [n] or null
  int64_t n;
  int64_t n_steps;
  KepCountsRun counts;
};

__device__ __forceinline__ double semi_major(double qx, double qy, double qz, double vx, double vy, double vz,
                                             double mu) {
  double r = sqrt(qx * qx + qy * qy + qz * qz);
  double v2 = vx * vx + vy * vy + vz * vz;
  return 1.0 / (2.0 / r - v2 / mu);
}

__global__ __launch_bounds__(256) void k_envelope(EnvParams p) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < p.n; i += (int64_t)gridDim.x * 256) {
    double qx = p.Q[3 * i], qy = p.Q[3 * i + 1], qz = p.Q[3 * i + 2];
    double vx = p.V[3 * i], vy = p.V[3 * i + 1], vz = p.V[3 * i + 2];
    const double mu = p.mu[i], tau = p.tau[i];
    const double a0 = semi_major(qx, qy, qz, vx, vy, vz, mu);
    KepDiag dg{0.0, 1e300};
    for (int64_t s = 0; s < p.n_steps; ++s) {
      KepCoef k;
      kepler_coeffs_p(p.counts, qx, qy, qz, vx, vy, vz, mu, tau, dg, k);
      double nqx = qx + fma(k.fm1, qx, k.g * vx);
      double nqy = qy + fma(k.fm1, qy, k.g * vy);
      double nqz = qz + fma(k.fm1, qz, k.g * vz);
      vx = vx + fma(k.fd, qx, k.gdm1 * vx);
      vy = vy + fma(k.fd, qy, k.gdm1 * vy);
      vz = vz + fma(k.fd, qz, k.gdm1 * vz);
      qx = nqx; qy = nqy; qz = nqz;
    }
    p.a_err[i] = (semi_major(qx, qy, qz, vx, vy, vz, mu) - a0) / a0;
    if (p.zmax_out) p.zmax_out[i] = dg.zmax;
    if (p.Q_out) {
      p.Q_out[3 * i] = qx; p.Q_out[3 * i + 1] = qy; p.Q_out[3 * i + 2] = qz;
    }
    if (p.V_out) {
      p.V_out[3 * i] = vx; p.V_out[3 * i + 1] = vy; p.V_out[3 * i + 2] = vz;
    }
  }
}

// ===========================================================================
// Host side
// ===========================================================================
namespace {

thread_local std::string g_err;

wh_status fail(wh_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

wh_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(WH_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return WH_OK;
}

}  // namespace

struct wh_ctx {
  wh_config cfg;
  int S = 0;
  Packing P;
  Layout lay;
  char* ws = nullptr;
  double* st = nullptr;
  double* m0s = nullptr;
  double* dts = nullptr;
  int* slot_sys = nullptr;
  int* slot_pl = nullptr;
  uint32_t* flags = nullptr;
  int* synced = nullptr;
  int64_t steps_done = 0;
  int block_waves = 1;
  int exchange = WH_EXCH_DPP;
  int chunk = 4096;
  int graph_launches = 8;
  // reverse mode: the tape the last wh_forward_ckpt filled
  const void* tape = nullptr;
  size_t tape_bytes = 0;
  int64_t tape_steps = 0, tape_every = 0, tape_end = -1;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // balanced launch windows of one chunk (empty: one launch per chunk):
  // window k covers entries [plan_off[k], plan_off[k + 1]) of the device
  // tables plan_wave / plan_steps
  std::vector<int> plan_off;
  int* plan_wave = nullptr;
  int* plan_steps = nullptr;
  int plan_slots = 0;   // wavefronts the GPU holds at the kernel's occupancy
};

namespace {

StepParams step_params(const wh_ctx* c, int n_steps) {
  StepParams p;
  p.st = c->st;
  p.ns = c->P.ns;
  p.m0s = c->m0s;
  p.dts = c->dts;
  p.slot_sys = c->slot_sys;
  p.slot_pl = c->slot_pl;
  p.flags = c->flags;
  p.synced = c->synced;
  p.wave0 = 0;
  p.w1 = c->P.w1; p.w2 = c->P.w2; p.w4 = c->P.w4; p.w8 = c->P.w8;
  p.wm = c->P.wm;
  p.n_steps = n_steps;
  p.kgr = c->cfg.gr_c > 0 ? 6.0 / (c->cfg.gr_c * c->cfg.gr_c) : 0.0;
  p.zlim = c->cfg.z_max > 0 ? c->cfg.z_max : 1.0;
  p.saba_n = 0;
  p.plan_wave = nullptr;
  p.plan_steps = nullptr;
  p.plan_n = 0;
  p.corr_n = c->cfg.corrector;
  for (int k = 0; k < 3; ++k) p.corr_a[k] = p.corr_b[k] = 0.0;
  if (p.corr_n > 0) corrector_coefficients(p.corr_n, c->cfg.scheme, p.corr_a, p.corr_b);
  for (int k = 0; k < 5; ++k) p.sc[k] = 0.0;
  for (int k = 0; k < 4; ++k) p.sd[k] = 0.0;
  if (c->cfg.scheme >= WH_SABA2) {
    p.saba_n = c->cfg.scheme;      // WH_SABA2..4 = 2..4
    saba_coefficients(p.saba_n, p.sc, p.sd);
  }
  return p;
}

// The step kernel of a context's configuration (host stub address, for
// hipLaunchKernel and the occupancy query).
template <int EXCH> const void* step_kernel_exch(const wh_ctx* c) {
  const bool gr = c->cfg.gr_c > 0;
  const bool jac = c->cfg.coords == WH_COORDS_JACOBI;
  const bool saba = c->cfg.scheme >= WH_SABA2, dkd = c->cfg.scheme == WH_DKD;
  if (c->cfg.kepler_counts == 1) {
    // the cheaper count set: DHC drift-kick-drift / kick-drift-kick in the
    // DPP-exchange layouts (config_ok refuses the rest)
    if (c->P.pair) {
      if (dkd) return gr ? (const void*)k_step_pair<true, WH_DKD, 1> : (const void*)k_step_pair<false, WH_DKD, 1>;
      return gr ? (const void*)k_step_pair<true, WH_KDK, 1> : (const void*)k_step_pair<false, WH_KDK, 1>;
    }
    if (c->P.split) {
      if (dkd) return gr ? (const void*)k_step_split<true, WH_DKD, 1> : (const void*)k_step_split<false, WH_DKD, 1>;
      return gr ? (const void*)k_step_split<true, WH_KDK, 1> : (const void*)k_step_split<false, WH_KDK, 1>;
    }
    if (dkd) return gr ? (const void*)k_step<true, WH_DKD, 1, false, 1> : (const void*)k_step<false, WH_DKD, 1, false, 1>;
    return gr ? (const void*)k_step<true, WH_KDK, 1, false, 1> : (const void*)k_step<false, WH_KDK, 1, false, 1>;
  }
  if (c->P.pair) {
    if (saba) return (const void*)k_step_pair<false, SCHEME_SABA>;
    if (dkd) return gr ? (const void*)k_step_pair<true, WH_DKD> : (const void*)k_step_pair<false, WH_DKD>;
    return gr ? (const void*)k_step_pair<true, WH_KDK> : (const void*)k_step_pair<false, WH_KDK>;
  }
  if (c->P.split) {
    if (saba) return (const void*)k_step_split<false, SCHEME_SABA>;
    if (dkd) return gr ? (const void*)k_step_split<true, WH_DKD> : (const void*)k_step_split<false, WH_DKD>;
    return gr ? (const void*)k_step_split<true, WH_KDK> : (const void*)k_step_split<false, WH_KDK>;
  }
  if (c->P.serial) {
    if (saba) return (const void*)k_step_serial<false, SCHEME_SABA>;
    if (dkd) return gr ? (const void*)k_step_serial<true, WH_DKD> : (const void*)k_step_serial<false, WH_DKD>;
    return gr ? (const void*)k_step_serial<true, WH_KDK> : (const void*)k_step_serial<false, WH_KDK>;
  }
  if (saba) {
    // (GR is allowed with SABA_n in Jacobi coordinates only)
    if (jac) return gr ? (const void*)k_step<true, SCHEME_SABA, EXCH, true>
                       : (const void*)k_step<false, SCHEME_SABA, EXCH, true>;
    return (const void*)k_step<false, SCHEME_SABA, EXCH, false>;
  }
  if (jac) {
    if (dkd) return gr ? (const void*)k_step<true, WH_DKD, EXCH, true> : (const void*)k_step<false, WH_DKD, EXCH, true>;
    return gr ? (const void*)k_step<true, WH_KDK, EXCH, true> : (const void*)k_step<false, WH_KDK, EXCH, true>;
  }
  if (dkd) return gr ? (const void*)k_step<true, WH_DKD, EXCH> : (const void*)k_step<false, WH_DKD, EXCH>;
  return gr ? (const void*)k_step<true, WH_KDK, EXCH> : (const void*)k_step<false, WH_KDK, EXCH>;
}

const void* step_kernel(const wh_ctx* c) {
  if (c->P.mixed) {
    const bool gr = c->cfg.gr_c > 0;
    if (c->cfg.scheme == WH_DKD) return gr ? (const void*)k_step_mixed<true, WH_DKD> : (const void*)k_step_mixed<false, WH_DKD>;
    return gr ? (const void*)k_step_mixed<true, WH_KDK> : (const void*)k_step_mixed<false, WH_KDK>;
  }
  return c->exchange == WH_EXCH_LDS ? step_kernel_exch<0>(c) : step_kernel_exch<1>(c);
}

// Workgroup shape of the step kernel: bw wavefronts per workgroup and the
// dynamic LDS per workgroup (the serial layout keeps its compensation terms
// there: one thread per 8-slot group, at most two waves per workgroup so the
// LDS stays within 64 KiB).
void step_block_shape(const wh_ctx* c, int& bw, size_t& smem) {
  bw = c->block_waves;
  smem = 0;
  if (c->P.serial) {
    bw = bw > 2 ? 2 : bw;
    smem = (size_t)bw * SERIAL_LDS_PER_WAVE * sizeof(double);
  }
}

// Launch the step kernel over n_waves wavefronts of the packing (units of the
// launch: waves, or for the serial layout one thread per 8-slot group).
void launch_step_kernel(const wh_ctx* c, const StepParams& p, int n_waves, hipStream_t st) {
  int bw;
  size_t smem;
  step_block_shape(c, bw, smem);
  const int units = c->P.serial ? (n_waves * 8 + 63) / 64 : n_waves;
  dim3 block(64 * bw), grid((units + bw - 1) / bw);
  StepParams q = p;
  void* args[] = {(void*)&q};
  (void)hipLaunchKernel(step_kernel(c), grid, block, args, smem, st);
}

void launch_step(const wh_ctx* c, int n_steps, hipStream_t st) {
  StepParams p = step_params(c, n_steps);
  launch_step_kernel(c, p, c->P.nwaves, st);
}

// Balanced launch windows for one chunk (wh_config.balance): slots =
// (resident waves per SIMD at the step kernel's occupancy) x (SIMDs), using at
// most as many waves per SIMD as the packing has waves for; plan_windows
// (wh_host.h) cuts the chunk.  No plan (one launch per chunk) when the
// packing has no more waves than slots, or more than 16 per slot (the single
// launch's imbalance is then small), or for the serial layout.
wh_status build_plan(wh_ctx* c, std::vector<int>& hw, std::vector<int>& hs) {
  c->plan_off.clear();
  c->plan_slots = 0;
  hw.clear();
  hs.clear();
  if (c->cfg.balance != 1 || c->P.serial) return WH_OK;
  int dev = 0, ncu = 0, nb = 0;
  wh_status st;
  if ((st = hip_check(hipGetDevice(&dev), "hipGetDevice")) ||
      (st = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "CU count")))
    return st;
  int bw;
  size_t smem;
  step_block_shape(c, bw, smem);
  if ((st = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel(c), 64 * bw, smem),
                      "occupancy query")))
    return st;
  const int simds = 4 * ncu;                 // CDNA: four SIMDs per compute unit
  const int per_simd = nb * bw / 4;          // resident wavefronts per SIMD
  const int W = c->P.nwaves;
  const int k = std::min(per_simd, W / std::max(simds, 1));
  if (k < 1) return WH_OK;
  const int slots = k * simds;
  if (W <= slots || W > 16 * slots) return WH_OK;
  std::vector<double> cost(W);
  for (int w = 0; w < W; ++w) cost[w] = wave_step_cost(c->P, c->cfg.gr_c > 0, w);
  plan_windows(cost, c->chunk, slots, PLAN_Q, hw, hs, c->plan_off);
  if (hw.size() > plan_capacity(&c->cfg, c->P)) return fail(WH_EHIP, "internal error: launch plan too large");
  c->plan_slots = slots;
  return WH_OK;
}

// One chunk of c->chunk steps for every wave: the balanced windows, or one
// launch.
void launch_chunk(const wh_ctx* c, hipStream_t st) {
  if (c->plan_off.size() < 2) {
    launch_step(c, c->chunk, st);
    return;
  }
  for (size_t k = 0; k + 1 < c->plan_off.size(); ++k) {
    StepParams p = step_params(c, 0);
    p.plan_wave = c->plan_wave + c->plan_off[k];
    p.plan_steps = c->plan_steps + c->plan_off[k];
    p.plan_n = c->plan_off[k + 1] - c->plan_off[k];
    launch_step_kernel(c, p, p.plan_n, st);
  }
}

wh_status launch_sync(wh_ctx* c, double* Q, double* V, double* E, hipStream_t st, double* a = nullptr,
                      double* e = nullptr, double* L = nullptr) {
  SyncParams q;
  q.sp = step_params(c, 0);
  q.Q_out = Q;
  q.V_out = V;
  q.E_out = E;
  q.a_out = a;
  q.e_out = e;
  q.L_out = L;
  dim3 block(64), grid(c->P.nwaves);
  const bool gr = c->cfg.gr_c > 0;
  if (c->P.mixed) {
    if (c->cfg.scheme == WH_DKD) {
      if (gr) hipLaunchKernelGGL((k_sync_mixed<true, WH_DKD>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync_mixed<false, WH_DKD>), grid, block, 0, st, q);
    } else {
      if (gr) hipLaunchKernelGGL((k_sync_mixed<true, WH_KDK>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync_mixed<false, WH_KDK>), grid, block, 0, st, q);
    }
  } else if (c->P.pair) {
    if (c->cfg.scheme >= WH_SABA2) {
      hipLaunchKernelGGL((k_sync_pair<false, SCHEME_SABA>), grid, block, 0, st, q);
    } else if (c->cfg.scheme == WH_DKD) {
      if (gr) hipLaunchKernelGGL((k_sync_pair<true, WH_DKD>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync_pair<false, WH_DKD>), grid, block, 0, st, q);
    } else {
      if (gr) hipLaunchKernelGGL((k_sync_pair<true, WH_KDK>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync_pair<false, WH_KDK>), grid, block, 0, st, q);
    }
  } else if (c->P.split) {
    if (c->cfg.scheme >= WH_SABA2) {
      hipLaunchKernelGGL((k_sync_split<false, SCHEME_SABA>), grid, block, 0, st, q);
    } else if (c->cfg.scheme == WH_DKD) {
      if (gr) hipLaunchKernelGGL((k_sync_split<true, WH_DKD>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync_split<false, WH_DKD>), grid, block, 0, st, q);
    } else {
      if (gr) hipLaunchKernelGGL((k_sync_split<true, WH_KDK>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync_split<false, WH_KDK>), grid, block, 0, st, q);
    }
  } else if (c->cfg.scheme >= WH_SABA2) {
    // (GR, allowed in Jacobi coordinates only, enters the energy of the copy)
    if (c->cfg.coords == WH_COORDS_JACOBI) {
      if (gr) hipLaunchKernelGGL((k_sync<true, SCHEME_SABA, true>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync<false, SCHEME_SABA, true>), grid, block, 0, st, q);
    } else {
      hipLaunchKernelGGL((k_sync<false, SCHEME_SABA, false>), grid, block, 0, st, q);
    }
  } else if (c->cfg.coords == WH_COORDS_JACOBI) {
    if (c->cfg.scheme == WH_DKD) {
      if (gr) hipLaunchKernelGGL((k_sync<true, WH_DKD, true>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync<false, WH_DKD, true>), grid, block, 0, st, q);
    } else {
      if (gr) hipLaunchKernelGGL((k_sync<true, WH_KDK, true>), grid, block, 0, st, q);
      else hipLaunchKernelGGL((k_sync<false, WH_KDK, true>), grid, block, 0, st, q);
    }
  } else if (c->cfg.scheme == WH_DKD) {
    if (gr) hipLaunchKernelGGL((k_sync<true, WH_DKD>), grid, block, 0, st, q);
    else hipLaunchKernelGGL((k_sync<false, WH_DKD>), grid, block, 0, st, q);
  } else {
    if (gr) hipLaunchKernelGGL((k_sync<true, WH_KDK>), grid, block, 0, st, q);
    else hipLaunchKernelGGL((k_sync<false, WH_KDK>), grid, block, 0, st, q);
  }
  return hip_check(hipGetLastError(), "sync kernel launch");
}

wh_status ensure_graph(wh_ctx* c) {
  if (c->gexec) return WH_OK;
  // a failed attempt releases what it made, so a later call starts afresh
  auto release = [c](wh_status s) {
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->graph = nullptr;
    c->cap_stream = nullptr;
    c->gexec = nullptr;
    return s;
  };
  wh_status s;
  if ((s = hip_check(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate")))
    return release(s);
  if ((s = hip_check(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture")))
    return release(s);
  for (int i = 0; i < c->graph_launches; ++i) launch_chunk(c, c->cap_stream);
  hipError_t le = hipGetLastError();
  hipError_t ee = hipStreamEndCapture(c->cap_stream, &c->graph);
  if ((s = hip_check(le, "launch during capture"))) return release(s);
  if ((s = hip_check(ee, "end capture"))) return release(s);
  if ((s = hip_check(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0), "graph instantiate")))
    return release(s);
  return WH_OK;
}

int tape_units(const wh_ctx* c) { return c->cfg.scheme >= WH_SABA2 ? c->cfg.scheme : 1; }

// One launch of the reverse pass: sweep_waves wavefronts sweep a segment and
// the following ones record the previous segment (record_waves wavefronts of
// the packing; the serial packing records with one thread per 8-slot group).
template <bool GR, int SCH>
void launch_adj_segment(const wh_ctx* c, const AdjParams& q, int sweep_waves, int record_waves, hipStream_t st) {
  if (c->P.serial) {
    const int rec = record_waves > 0 ? (record_waves * 8 + 63) / 64 : 0;
    const dim3 grid(sweep_waves + rec), block(64);
    const size_t smem = SERIAL_LDS_PER_WAVE * sizeof(double);
    hipLaunchKernelGGL((k_adj_segment_serial<GR, SCH>), grid, block, smem, st, q);
    return;
  }
  const dim3 grid(sweep_waves + record_waves), block(64);
  if (c->P.pair) hipLaunchKernelGGL((k_adj_segment_pair<GR, SCH>), grid, block, 0, st, q);
  else if (c->P.split) hipLaunchKernelGGL((k_adj_segment<GR, true, SCH>), grid, block, 0, st, q);
  else hipLaunchKernelGGL((k_adj_segment<GR, false, SCH>), grid, block, 0, st, q);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// Scratch array of wh_integrate_noalloc: that entry point's workspace, for
// callers that cannot allocate device memory.  Every GPU the library runs on
// holds its own copy (WH_NOALLOC_MAX_BYTES) until the process ends.  In host
// code the name is a stand-in, not a device address: the device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[WH_NOALLOC_MAX_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // device address of scratch, per device id

// Address of the current device's scratch array (looked up on the first call
// on each device, with that device current).
wh_status scratch_address(void** out) {
  int dev = -1;
  wh_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st) return st;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if ((st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))) return st;
    if (!p || ((uintptr_t)p & 255) != 0) return fail(WH_EHIP, "scratch array address is null or misaligned");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return WH_OK;
}
}  // namespace

extern "C" {

void wh_config_default(wh_config* cfg, int32_t n_systems) { config_defaults(cfg, n_systems); }

size_t wh_workspace_bytes(const wh_config* cfg, const int32_t* n_planets) {
  std::string why;
  if (!config_ok(cfg, why) || !n_planets) return 0;
  Packing P;
  if (!make_packing(cfg->n_systems, n_planets, eff_packing(cfg), P)) return 0;
  return make_layout(cfg->n_systems, P.ns, plan_capacity(cfg, P)).total;
}

wh_status wh_init(wh_ctx** out, const wh_config* cfg, const int32_t* n_planets, const double* m0, const double* m,
                  const double* Q, const double* V, const double* dt, void* workspace, size_t workspace_bytes,
                  hipStream_t stream) {
  std::string why;
  if (!out) return fail(WH_EINVAL, "null output pointer");
  *out = nullptr;
  if (!config_ok(cfg, why)) return fail(WH_EINVAL, why);
  if (!n_planets || !m0 || !m || !Q || !V || !dt || !workspace)
    return fail(WH_EINVAL, "null array pointer");
  if (((uintptr_t)workspace & 255) != 0) return fail(WH_EINVAL, "workspace must be 256-byte aligned");
  const int S = cfg->n_systems;
  wh_ctx* c = new wh_ctx();
  c->cfg = *cfg;
  c->S = S;
  if (!make_packing(S, n_planets, eff_packing(cfg), c->P, &why)) {
    delete c;
    return fail(WH_EINVAL, why);
  }
  c->lay = make_layout(S, c->P.ns, plan_capacity(cfg, c->P));
  if (workspace_bytes < c->lay.total) {
    delete c;
    return fail(WH_EWORKSPACE, "workspace too small: need " + std::to_string(c->lay.total) + " bytes");
  }
  // Validate the physical inputs (Sec. 3.5: dt > 0, positive star mass,
  // non-negative constant planet masses) before anything is enqueued.
  std::vector<double> h_m0(S), h_dt(S), h_m((size_t)S * 8);
  wh_status st;
  if ((st = hip_check(hipMemcpyAsync(h_m0.data(), m0, sizeof(double) * S, hipMemcpyDeviceToHost, stream), "copy m0")) ||
      (st = hip_check(hipMemcpyAsync(h_dt.data(), dt, sizeof(double) * S, hipMemcpyDeviceToHost, stream), "copy dt")) ||
      (st = hip_check(hipMemcpyAsync(h_m.data(), m, sizeof(double) * 8 * S, hipMemcpyDeviceToHost, stream), "copy m")) ||
      (st = hip_check(hipStreamSynchronize(stream), "synchronize"))) {
    (void)hipStreamSynchronize(stream);   // copies already queued write into the host vectors
    delete c;
    return st;
  }
  for (int s = 0; s < S; ++s) {
    if (!(h_dt[s] > 0.0) || !std::isfinite(h_dt[s])) {
      delete c;
      return fail(WH_EINVAL, "dt must be finite and > 0 (system " + std::to_string(s) + ")");
    }
    if (!(h_m0[s] > 0.0) || !std::isfinite(h_m0[s])) {
      delete c;
      return fail(WH_EINVAL, "star mass must be finite and > 0 (system " + std::to_string(s) + ")");
    }
    for (int p = 0; p < n_planets[s]; ++p)
      if (!(h_m[(size_t)s * 8 + p] >= 0.0) || !std::isfinite(h_m[(size_t)s * 8 + p])) {
        delete c;
        return fail(WH_EINVAL, "planet masses must be finite and >= 0 (system " + std::to_string(s) + ")");
      }
  }
  c->ws = (char*)workspace;
  c->st = (double*)(c->ws + c->lay.st);
  c->m0s = (double*)(c->ws + c->lay.m0s);
  c->dts = (double*)(c->ws + c->lay.dts);
  c->slot_sys = (int*)(c->ws + c->lay.slot_sys);
  c->slot_pl = (int*)(c->ws + c->lay.slot_pl);
  c->flags = (uint32_t*)(c->ws + c->lay.flags);
  c->synced = (int*)(c->ws + c->lay.synced);
  c->plan_wave = (int*)(c->ws + c->lay.plan_wave);
  c->plan_steps = (int*)(c->ws + c->lay.plan_steps);
  c->block_waves = cfg->block_waves > 0 ? cfg->block_waves : 1;
  c->exchange = cfg->exchange == WH_EXCH_LDS ? WH_EXCH_LDS : WH_EXCH_DPP;
  c->chunk = cfg->chunk_steps > 0 ? cfg->chunk_steps : 4096;
  c->graph_launches = cfg->graph_launches == 0 ? 8 : cfg->graph_launches;
  const int ns = c->P.ns;
  // from here on the stream may hold copies that read the context's slot
  // tables: drain it before freeing the context on a failure
  auto abandon = [&](wh_status s) {
    (void)hipStreamSynchronize(stream);
    delete c;
    return s;
  };
  std::vector<int> plan_w, plan_s;   // outlive the copies: the stream is synchronized below
  if ((st = build_plan(c, plan_w, plan_s))) return abandon(st);
  if (!plan_w.empty() &&
      ((st = hip_check(hipMemcpyAsync(c->plan_wave, plan_w.data(), sizeof(int) * plan_w.size(),
                                      hipMemcpyHostToDevice, stream), "upload launch plan")) ||
       (st = hip_check(hipMemcpyAsync(c->plan_steps, plan_s.data(), sizeof(int) * plan_s.size(),
                                      hipMemcpyHostToDevice, stream), "upload launch plan"))))
    return abandon(st);
  if ((st = hip_check(hipMemcpyAsync(c->slot_sys, c->P.slot_sys.data(), sizeof(int) * ns, hipMemcpyHostToDevice,
                                     stream), "upload slot table")) ||
      (st = hip_check(hipMemcpyAsync(c->slot_pl, c->P.slot_pl.data(), sizeof(int) * ns, hipMemcpyHostToDevice,
                                     stream), "upload slot table")))
    return abandon(st);
  hipLaunchKernelGGL(k_gather, dim3((ns + 255) / 256), dim3(256), 0, stream, c->st, ns, c->m0s, c->dts, c->slot_sys,
                     c->slot_pl, m0, m, Q, V, dt, c->P.split ? 1 : 0);
  hipLaunchKernelGGL(k_fill_u32, dim3((S + 255) / 256), dim3(256), 0, stream, c->flags, 0u, S);
  hipLaunchKernelGGL(k_fill_u32, dim3((S + 255) / 256), dim3(256), 0, stream, (uint32_t*)c->synced, 1u, S);
  if (cfg->coords == WH_COORDS_JACOBI)
    hipLaunchKernelGGL(k_to_jacobi, dim3(c->P.nwaves), dim3(64), 0, stream, step_params(c, 0));
  if (cfg->coords == WH_COORDS_JACOBI && cfg->corrector > 0) {
    if (cfg->gr_c > 0) hipLaunchKernelGGL(k_corrector_in<true>, dim3(c->P.nwaves), dim3(64), 0, stream, step_params(c, 0));
    else hipLaunchKernelGGL(k_corrector_in<false>, dim3(c->P.nwaves), dim3(64), 0, stream, step_params(c, 0));
  }
  if ((st = hip_check(hipGetLastError(), "init kernels"))) return abandon(st);
  // the slot tables live in the context and must outlive the async copies;
  // synchronize so the caller may free the input arrays right away
  if ((st = hip_check(hipStreamSynchronize(stream), "synchronize"))) {
    delete c;
    return st;
  }
  *out = c;
  return WH_OK;
}

wh_status wh_step_n(wh_ctx* c, int64_t n_steps, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (n_steps < 0) return fail(WH_EINVAL, "n_steps must be >= 0");
  if (n_steps == 0) return WH_OK;
  int64_t full = n_steps / c->chunk;
  int rem = (int)(n_steps % c->chunk);
  wh_status st;
  if (c->graph_launches > 0 && full >= c->graph_launches) {
    if ((st = ensure_graph(c))) return st;
    int64_t reps = full / c->graph_launches;
    for (int64_t r = 0; r < reps; ++r)
      if ((st = hip_check(hipGraphLaunch(c->gexec, stream), "graph launch"))) return st;
    full -= reps * c->graph_launches;
  }
  for (int64_t i = 0; i < full; ++i) launch_chunk(c, stream);
  if (rem) launch_step(c, rem, stream);
  if ((st = hip_check(hipGetLastError(), "step kernel launch"))) return st;
  c->steps_done += n_steps;
  return WH_OK;
}

wh_status wh_step_n_plain(wh_ctx* c, int64_t n_steps, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (n_steps < 0) return fail(WH_EINVAL, "n_steps must be >= 0");
  if (eff_packing(&c->cfg) != WH_PACK_G8)
    return fail(WH_ESTATE, "the per-size reference path needs a context created with WH_PACK_G8");
  for (int64_t s = 0; s < n_steps; ++s)
    for (int n = 1; n <= 8; ++n) {
      int b = c->P.plain_begin[n], e = c->P.plain_end[n];
      if (e <= b) continue;
      StepParams p = step_params(c, 1);
      p.wave0 = b;
      p.w1 = p.w2 = p.w4 = 0;
      p.w8 = e;
      launch_step_kernel(c, p, e - b, stream);
    }
  wh_status st = hip_check(hipGetLastError(), "step kernel launch");
  if (st) return st;
  c->steps_done += n_steps;
  return WH_OK;
}

wh_status wh_get_state(wh_ctx* c, double* Q_out, double* V_out, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!Q_out || !V_out) return fail(WH_EINVAL, "null output pointer");
  return launch_sync(c, Q_out, V_out, nullptr, stream);
}

wh_status wh_energy(wh_ctx* c, double* E_out, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!E_out) return fail(WH_EINVAL, "null output pointer");
  return launch_sync(c, nullptr, nullptr, E_out, stream);
}

wh_status wh_elements(wh_ctx* c, double* a_out, double* e_out, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!a_out || !e_out) return fail(WH_EINVAL, "null output pointer");
  return launch_sync(c, nullptr, nullptr, nullptr, stream, a_out, e_out);
}

wh_status wh_angular_momentum(wh_ctx* c, double* L_out, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!L_out) return fail(WH_EINVAL, "null output pointer");
  return launch_sync(c, nullptr, nullptr, nullptr, stream, nullptr, nullptr, L_out);
}

wh_status wh_status_flags(wh_ctx* c, uint32_t* flags_out, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!flags_out) return fail(WH_EINVAL, "null output pointer");
  hipLaunchKernelGGL(k_copy_u32, dim3((c->S + 255) / 256), dim3(256), 0, stream, flags_out, c->flags, c->S);
  return hip_check(hipGetLastError(), "flags copy");
}

int64_t wh_steps_done(const wh_ctx* c) { return c ? c->steps_done : -1; }

}  // extern "C"

namespace {
struct SnapLayout {
  size_t st, flags, synced, total;
};
SnapLayout snap_layout(const wh_ctx* c) {
  SnapLayout L;
  size_t o = align256(sizeof(StateHeader));
  L.st = o; o = align256(o + sizeof(double) * ROWS * (size_t)c->P.ns);
  L.flags = o; o = align256(o + sizeof(uint32_t) * (size_t)c->S);
  L.synced = o; o = align256(o + sizeof(int) * (size_t)c->S);
  L.total = o;
  return L;
}
StateHeader snap_header(const wh_ctx* c) {
  StateHeader h;
  h.magic = STATE_MAGIC;
  h.version = 1;
  h.S = c->S;
  h.ns = c->P.ns;
  h.packing = eff_packing(&c->cfg);
  h.coords = c->cfg.coords;
  h.scheme = c->cfg.scheme;
  h.gr = c->cfg.gr_c > 0 ? 1 : 0;
  h.rows = ROWS;
  h.steps_done = c->steps_done;
  return h;
}
}  // namespace

extern "C" {

size_t wh_state_bytes(const wh_ctx* c) { return c ? snap_layout(c).total : 0; }

wh_status wh_save_state(wh_ctx* c, void* dst, size_t bytes, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!dst) return fail(WH_EINVAL, "null snapshot buffer");
  if (((uintptr_t)dst & 255) != 0) return fail(WH_EINVAL, "snapshot buffer must be 256-byte aligned");
  const SnapLayout L = snap_layout(c);
  if (bytes < L.total) return fail(WH_EWORKSPACE, "snapshot buffer too small: need " + std::to_string(L.total));
  char* d = (char*)dst;
  hipLaunchKernelGGL(k_write_header, dim3(1), dim3(64), 0, stream, snap_header(c), (StateHeader*)d);
  wh_status st;
  if ((st = hip_check(hipGetLastError(), "snapshot header")) ||
      (st = hip_check(hipMemcpyAsync(d + L.st, c->st, sizeof(double) * ROWS * (size_t)c->P.ns,
                                     hipMemcpyDeviceToDevice, stream), "snapshot state")) ||
      (st = hip_check(hipMemcpyAsync(d + L.flags, c->flags, sizeof(uint32_t) * (size_t)c->S,
                                     hipMemcpyDeviceToDevice, stream), "snapshot flags")) ||
      (st = hip_check(hipMemcpyAsync(d + L.synced, c->synced, sizeof(int) * (size_t)c->S, hipMemcpyDeviceToDevice,
                                     stream), "snapshot synced")))
    return st;
  return WH_OK;
}

wh_status wh_restore_state(wh_ctx* c, const void* src, size_t bytes, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!src) return fail(WH_EINVAL, "null snapshot buffer");
  if (((uintptr_t)src & 255) != 0) return fail(WH_EINVAL, "snapshot buffer must be 256-byte aligned");
  const SnapLayout L = snap_layout(c);
  if (bytes < sizeof(StateHeader)) return fail(WH_EINVAL, "not a wh_save_state snapshot (too short)");
  StateHeader h;
  wh_status st;
  if ((st = hip_check(hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDeviceToHost, stream), "read snapshot header")) ||
      (st = hip_check(hipStreamSynchronize(stream), "synchronize")))
    return st;
  const StateHeader mine = snap_header(c);
  if (h.magic != STATE_MAGIC || h.version != 1) return fail(WH_EINVAL, "not a wh_save_state snapshot");
  if (h.S != mine.S || h.ns != mine.ns || h.packing != mine.packing || h.coords != mine.coords ||
      h.scheme != mine.scheme || h.gr != mine.gr || h.rows != mine.rows)
    return fail(WH_ESTATE, "snapshot of a context with another batch, packing, scheme, coordinates or GR setting");
  if (h.steps_done < 0) return fail(WH_EINVAL, "corrupt snapshot header");
  if (bytes < L.total) return fail(WH_EWORKSPACE, "snapshot buffer smaller than this context's state");
  const char* s = (const char*)src;
  if ((st = hip_check(hipMemcpyAsync(c->st, s + L.st, sizeof(double) * ROWS * (size_t)c->P.ns,
                                     hipMemcpyDeviceToDevice, stream), "restore state")) ||
      (st = hip_check(hipMemcpyAsync(c->flags, s + L.flags, sizeof(uint32_t) * (size_t)c->S,
                                     hipMemcpyDeviceToDevice, stream), "restore flags")) ||
      (st = hip_check(hipMemcpyAsync(c->synced, s + L.synced, sizeof(int) * (size_t)c->S, hipMemcpyDeviceToDevice,
                                     stream), "restore synced")))
    return st;
  c->steps_done = h.steps_done;
  c->tape = nullptr;      // a recorded tape belongs to the state it was recorded from
  c->tape_end = -1;
  return WH_OK;
}

int32_t wh_launch_windows(const wh_ctx* c, int32_t* slots) {
  if (!c) return -1;
  if (slots) *slots = c->plan_slots;
  return c->plan_off.size() < 2 ? 1 : (int32_t)c->plan_off.size() - 1;
}

size_t wh_tape_bytes(const wh_ctx* c, int64_t n_steps, int64_t ckpt_every) {
  if (!c || n_steps < 0 || ckpt_every < 1 || ckpt_every > (1 << 30)) return 0;
  if (ckpt_every * tape_units(c) > (1 << 30)) return 0;
  return tape_layout(c->P.ns, n_steps, ckpt_every, tape_units(c)).total;
}

wh_status wh_forward_ckpt(wh_ctx* c, int64_t n_steps, int64_t ckpt_every, void* tape, size_t tape_bytes,
                          hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!tape) return fail(WH_EINVAL, "null tape");
  if (n_steps < 0 || ckpt_every < 1 || ckpt_every > (1 << 30)) return fail(WH_EINVAL, "bad n_steps or ckpt_every");
  if (((uintptr_t)tape & 255) != 0) return fail(WH_EINVAL, "tape must be 256-byte aligned");
  if (c->cfg.scheme != WH_DKD && c->cfg.scheme != WH_KDK && c->cfg.scheme < WH_SABA2)
    return fail(WH_ESTATE, "reverse mode is implemented for WH_DKD, WH_KDK and WH_SABA2..4");
  if (c->cfg.kepler_counts != 0)
    return fail(WH_ESTATE, "reverse mode runs the paper's Kepler counts (kepler_counts = 0)");
  if (c->P.mixed) return fail(WH_ESTATE, "reverse mode does not run the mixed packing");
  if (c->steps_done != 0) return fail(WH_ESTATE, "wh_forward_ckpt must start from the initial state (no steps taken)");
  if (ckpt_every * tape_units(c) > (1 << 30)) return fail(WH_EINVAL, "ckpt_every too large for this scheme");
  TapeLayout T = tape_layout(c->P.ns, n_steps, ckpt_every, tape_units(c));
  if (T.total == 0) return fail(WH_EINVAL, "tape size overflows size_t for these n_steps and ckpt_every");
  if (tape_bytes < T.total) return fail(WH_EWORKSPACE, "tape too small: need " + std::to_string(T.total) + " bytes");
  const int ns = c->P.ns;
  double* ck = (double*)((char*)tape + T.ck);
  dim3 blk(256), grd((ns + 255) / 256);
  int64_t done = 0;
  for (int64_t k = 0; k <= T.n_seg; ++k) {
    hipLaunchKernelGGL(k_save_ck, grd, blk, 0, stream, c->st, ck + (size_t)k * 12 * ns, ns);
    if (k == T.n_seg) break;
    int64_t n = std::min(ckpt_every, n_steps - done);
    while (n > 0) {
      int m = (int)std::min<int64_t>(n, c->chunk);
      launch_step(c, m, stream);
      n -= m;
      done += m;
    }
  }
  wh_status st = hip_check(hipGetLastError(), "forward checkpoint launch");
  if (st) return st;
  c->steps_done += n_steps;
  c->tape = tape;
  c->tape_bytes = tape_bytes;
  c->tape_steps = n_steps;
  c->tape_every = ckpt_every;
  c->tape_end = c->steps_done;
  return WH_OK;
}

wh_status wh_adjoint_n(wh_ctx* c, void* tape, size_t tape_bytes, const double* gQ_T, const double* gV_T,
                       double* gQ_0, double* gV_0, double* gm, double* gm0, hipStream_t stream) {
  if (!c) return fail(WH_EINVAL, "null context");
  if (!tape || !gQ_T || !gV_T || !gQ_0 || !gV_0 || !gm || !gm0) return fail(WH_EINVAL, "null pointer");
  if (tape != c->tape || tape_bytes != c->tape_bytes || c->steps_done != c->tape_end)
    return fail(WH_ESTATE, "no matching wh_forward_ckpt for this tape (or steps taken since)");
  const int ns = c->P.ns;
  TapeLayout T = tape_layout(ns, c->tape_steps, c->tape_every, tape_units(c));
  double* ck = (double*)((char*)tape + T.ck);
  double* seg[2] = {(double*)((char*)tape + T.seg[0]), (double*)((char*)tape + T.seg[1])};
  AdjParams q;
  q.sp = step_params(c, 0);
  q.tape = seg[0];
  q.grad = (double*)((char*)tape + T.grad);
  q.gQ_T = gQ_T; q.gV_T = gV_T;
  q.gQ_0 = gQ_0; q.gV_0 = gV_0; q.gm = gm; q.gm0 = gm0;
  q.ck = ck + (size_t)T.n_seg * 12 * ns;
  q.n_seg = 0;
  q.first_synced = 0;
  q.sweep_waves = 0;
  q.ck_rec = nullptr;
  q.tape_rec = seg[1];
  q.n_rec = 0;
  q.rec_first_synced = 0;
  const bool gr = c->cfg.gr_c > 0;
  const bool kdk = c->cfg.scheme == WH_KDK;
  const bool jac = c->cfg.coords == WH_COORDS_JACOBI;
  const int nw = c->P.nwaves;
  const int synced_end = (int)(c->tape_steps == 0);
  if (jac) {
    // gather dL/dQ_T, dL/dV_T, then the output transform and pending operation per lane group
    hipLaunchKernelGGL(k_adj_init, dim3((ns + 255) / 256), dim3(256), 0, stream, q, 1);
    const dim3 g(nw), b(64);
    if (c->cfg.scheme >= WH_SABA2) {
      if (gr) hipLaunchKernelGGL((k_adj_init_jac<true, SCHEME_SABA>), g, b, 0, stream, q, synced_end);
      else hipLaunchKernelGGL((k_adj_init_jac<false, SCHEME_SABA>), g, b, 0, stream, q, synced_end);
    } else if (kdk) {
      if (gr) hipLaunchKernelGGL((k_adj_init_jac<true, WH_KDK>), g, b, 0, stream, q, synced_end);
      else hipLaunchKernelGGL((k_adj_init_jac<false, WH_KDK>), g, b, 0, stream, q, synced_end);
    } else {
      if (gr) hipLaunchKernelGGL((k_adj_init_jac<true, WH_DKD>), g, b, 0, stream, q, synced_end);
      else hipLaunchKernelGGL((k_adj_init_jac<false, WH_DKD>), g, b, 0, stream, q, synced_end);
    }
  } else if (!kdk) {
    hipLaunchKernelGGL(k_adj_init, dim3((ns + 255) / 256), dim3(256), 0, stream, q, synced_end);
  } else {
    const dim3 g(nw), b(64);
    if (c->P.pair) {
      if (gr) hipLaunchKernelGGL((k_adj_init_kdk<true, 2>), g, b, 0, stream, q, synced_end);
      else hipLaunchKernelGGL((k_adj_init_kdk<false, 2>), g, b, 0, stream, q, synced_end);
    } else if (c->P.split) {
      if (gr) hipLaunchKernelGGL((k_adj_init_kdk<true, 1>), g, b, 0, stream, q, synced_end);
      else hipLaunchKernelGGL((k_adj_init_kdk<false, 1>), g, b, 0, stream, q, synced_end);
    } else {
      if (gr) hipLaunchKernelGGL((k_adj_init_kdk<true, 0>), g, b, 0, stream, q, synced_end);
      else hipLaunchKernelGGL((k_adj_init_kdk<false, 0>), g, b, 0, stream, q, synced_end);
    }
  }
  auto seg_steps = [&](int64_t k) {
    return (int)std::min<int64_t>(c->tape_every, c->tape_steps - k * c->tape_every);
  };
  auto set_record = [&](int64_t k) {   // segment k into tape k mod 2
    q.ck_rec = ck + (size_t)k * 12 * ns;
    q.tape_rec = seg[k & 1];
    q.n_rec = seg_steps(k);
    q.rec_first_synced = (k == 0);
  };
  const bool saba = c->cfg.scheme >= WH_SABA2;
  auto launch = [&](int sweep_waves, int record_waves) {
    q.sweep_waves = sweep_waves;
    if (jac) {
      const dim3 grid(sweep_waves + record_waves), block(64);
      if (saba && gr) hipLaunchKernelGGL((k_adj_segment_jac<true, SCHEME_SABA>), grid, block, 0, stream, q);
      else if (saba) hipLaunchKernelGGL((k_adj_segment_jac<false, SCHEME_SABA>), grid, block, 0, stream, q);
      else if (kdk && gr) hipLaunchKernelGGL((k_adj_segment_jac<true, WH_KDK>), grid, block, 0, stream, q);
      else if (kdk) hipLaunchKernelGGL((k_adj_segment_jac<false, WH_KDK>), grid, block, 0, stream, q);
      else if (gr) hipLaunchKernelGGL((k_adj_segment_jac<true, WH_DKD>), grid, block, 0, stream, q);
      else hipLaunchKernelGGL((k_adj_segment_jac<false, WH_DKD>), grid, block, 0, stream, q);
      return;
    }
    if (saba) launch_adj_segment<false, SCHEME_SABA>(c, q, sweep_waves, record_waves, stream);
    else if (kdk && gr) launch_adj_segment<true, WH_KDK>(c, q, sweep_waves, record_waves, stream);
    else if (kdk) launch_adj_segment<false, WH_KDK>(c, q, sweep_waves, record_waves, stream);
    else if (gr) launch_adj_segment<true, WH_DKD>(c, q, sweep_waves, record_waves, stream);
    else launch_adj_segment<false, WH_DKD>(c, q, sweep_waves, record_waves, stream);
  };
  // record the last segment, then sweep segment k while recording k - 1
  if (T.n_seg > 0) {
    set_record(T.n_seg - 1);
    launch(0, nw);
  }
  for (int64_t k = T.n_seg - 1; k >= 0; --k) {
    q.tape = seg[k & 1];
    q.n_seg = seg_steps(k);
    q.first_synced = (k == 0);
    if (k > 0) {
      set_record(k - 1);
      launch(nw, nw);
    } else {
      launch(nw, 0);
    }
  }
  if (jac) {
    q.ck = ck;   // the first checkpoint: the initial state the input transform is differentiated at
    if (c->cfg.gr_c > 0) hipLaunchKernelGGL(k_adj_in_jac<true>, dim3(nw), dim3(64), 0, stream, q);
    else hipLaunchKernelGGL(k_adj_in_jac<false>, dim3(nw), dim3(64), 0, stream, q);
  }
  if (c->P.pair) hipLaunchKernelGGL(k_adj_finish_pair, dim3(nw), dim3(64), 0, stream, q);
  else if (c->P.split) hipLaunchKernelGGL(k_adj_finish<true>, dim3(nw), dim3(64), 0, stream, q);
  else hipLaunchKernelGGL(k_adj_finish<false>, dim3(nw), dim3(64), 0, stream, q);
  return hip_check(hipGetLastError(), "adjoint launch");
}

wh_status wh_kepler_envelope(int64_t n, const double* Q, const double* V, const double* mu, const double* tau,
                             int64_t n_steps, int32_t n_halley, int32_t n_newton, int32_t terms_halley,
                             int32_t terms_newton, double* Q_out, double* V_out, double* a_err, double* zmax_out,
                             hipStream_t stream) {
  if (n < 0 || n_steps < 0) return fail(WH_EINVAL, "n and n_steps must be >= 0");
  if (n_halley < 0 || n_halley > KEP_RT_MAX_NH || n_newton < 0 || n_newton > KEP_RT_MAX_NN ||
      n_halley + n_newton < 1)
    return fail(WH_EINVAL, "iteration counts must satisfy 0 <= n_halley, n_newton <= 8 and n_halley + n_newton >= 1");
  if (terms_halley < 1 || terms_halley > KEP_RT_MAX_TERMS || terms_newton < 1 || terms_newton > KEP_RT_MAX_TERMS)
    return fail(WH_EINVAL, "series lengths must be in 1..14");
  if (n == 0) return WH_OK;
  if (!Q || !V || !mu || !tau || !a_err) return fail(WH_EINVAL, "null array pointer");
  if ((Q_out == nullptr) != (V_out == nullptr)) return fail(WH_EINVAL, "Q_out and V_out must both be given or both null");
  EnvParams p;
  p.Q = Q; p.V = V; p.mu = mu; p.tau = tau;
  p.Q_out = Q_out; p.V_out = V_out; p.a_err = a_err; p.zmax_out = zmax_out;
  p.n = n; p.n_steps = n_steps;
  p.counts = KepCountsRun{n_halley, n_newton, terms_halley, terms_newton};
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_envelope, dim3((unsigned)blocks), dim3(256), 0, stream, p);
  return hip_check(hipGetLastError(), "envelope launch");
}

wh_status wh_integrate_noalloc(const wh_config* cfg, const int32_t* n_planets, const double* m0, const double* m,
                               const double* Q, const double* V, const double* dt, int64_t n_steps, double* Q_out,
                               double* V_out, hipStream_t stream) {
  std::string why;
  if (!config_ok(cfg, why)) return fail(WH_EINVAL, why);
  if (!n_planets) return fail(WH_EINVAL, "null planet-count array");
  if (n_steps < 0) return fail(WH_EINVAL, "n_steps must be >= 0");
  if (!Q_out || !V_out) return fail(WH_EINVAL, "null output pointer");
  // no graph: its instantiation may allocate device memory
  wh_config c2 = *cfg;
  c2.graph_launches = -1;
  const size_t need = wh_workspace_bytes(&c2, n_planets);
  if (need == 0) return fail(WH_EINVAL, "invalid planet counts or packing");
  if (need > (size_t)WH_NOALLOC_MAX_BYTES)
    return fail(WH_EWORKSPACE, "wh_integrate_noalloc: this batch needs " + std::to_string(need) +
                                   " bytes of workspace, more than the fixed scratch array of " +
                                   std::to_string((size_t)WH_NOALLOC_MAX_BYTES) + " bytes");
  void* ws = nullptr;
  wh_status st = scratch_address(&ws);
  if (st) return st;
  wh_ctx* c = nullptr;
  if ((st = wh_init(&c, &c2, n_planets, m0, m, Q, V, dt, ws, (size_t)WH_NOALLOC_MAX_BYTES, stream))) return st;
  st = wh_step_n(c, n_steps, stream);
  if (!st) st = wh_get_state(c, Q_out, V_out, stream);
  // the kernels hold everything they need by value: the host context may go
  // while they are still in flight
  wh_destroy(c);
  return st;
}

const char* wh_last_error(void) { return g_err.c_str(); }

void wh_destroy(wh_ctx* c) {
  if (!c) return;
  // teardown: nothing useful can be done with a failure here
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

}  // extern "C"
