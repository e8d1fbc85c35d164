// Step-kernel pieces shared by the library's two translation units: the
// kernel parameters, the per-lane state and its compensated updates, the
// Kepler drift of that state, and the pair layout's kick and step (two
// planets per lane).  wh.hip holds every other kernel and the C ABI;
// wh_pair_step.hip holds the pair layout's step kernel, compiled with the
// instruction scheduler set for latency (two resident wavefronts per SIMD;
// the default occupancy-first schedule, three resident, measured slower).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wh.h"
#include "wh_device.h"
#include "wh_pair.h"
#include "wh_host.h"

namespace wh {

// State arrays, structure of arrays over lane slots: rows 0-2 Q, 3-5 V,
// 6 m, 7-9 and 10-12 the compensation terms of Q and V (the low-order parts
// that rounding dropped from earlier increments).
constexpr int ROWS = wh_host::WH_STATE_ROWS;

struct StepParams {
  double* st;            // [ROWS][ns]
  int ns;                // number of lane slots (multiple of 64)
  const double* m0s;     // [ns] star mass of the slot's system
  const double* dts;     // [ns] timestep of the slot's system
  const int* slot_sys;   // [ns] system index, -1 for an empty group
  const int* slot_pl;    // [ns] planet index, -1 for a padding lane
  uint32_t* flags;       // [S]
  int* synced;           // [S] 1 while the stored state is synchronized
  int wave0;             // first wave of this launch
  int w1, w2, w4, w8;    // wave ranges [0,w1) G=1, [w1,w2) G=2, [w2,w4) G=4, [w4,w8) G=8
  int wm;                // [wm, w8): 8-lane groups of two systems (mixed packing; wm = w8 otherwise)
  int n_steps;
  double kgr;            // 6 / c^2, or 0 without GR
  double zlim;           // WH_F_ZMAX threshold
  int saba_n;            // SABA_n: number of kicks per step (0 otherwise)
  double sc[5];          // SABA_n drift coefficients c_1 .. c_{n+1} (c_{n+1} = c_1)
  double sd[4];          // SABA_n kick coefficients d_1 .. d_n
  // Balanced launch window (null: the launch covers waves wave0.. with
  // n_steps each): wavefront k of the launch runs wave plan_wave[k] of the
  // packing for plan_steps[k] steps, k < plan_n.
  const int* plan_wave;
  const int* plan_steps;
  int plan_n;
  // symplectic corrector of the Jacobi map: stages and their coefficients
  int corr_n;
  double corr_a[3], corr_b[3];
};

// Wave of the packing and step count of launch wavefront k (k uniform over
// the wavefront); false if the launch has no such wavefront.  (Declaring the
// values wave-uniform with readfirstlane turned the group-size dispatch into
// scalar branches and cost the pair kernel ~60 VGPRs, so they stay vector
// values.)
__device__ __forceinline__ bool launch_wave(const StepParams& p, int k, int& wave, int& n_steps) {
  if (p.plan_wave) {
    if (k >= p.plan_n) return false;
    wave = p.plan_wave[k];
    n_steps = p.plan_steps[k];
    return true;
  }
  wave = p.wave0 + k;
  n_steps = p.n_steps;
  return wave < p.w8;
}

// Kernel scheme id of the SABA_n family (n read from StepParams).
constexpr int SCHEME_SABA = 2;

struct Lane {
  double qx, qy, qz, vx, vy, vz, m, m0, dt;
  double cqx, cqy, cqz, cvx, cvy, cvz;
  int sys, pl, first;
};

__device__ __forceinline__ Lane load_lane(const StepParams& p, int slot) {
  Lane L;
  const double* st = p.st;
  const int ns = p.ns;
  L.qx = st[slot];
  L.qy = st[ns + slot];
  L.qz = st[2 * ns + slot];
  L.vx = st[3 * ns + slot];
  L.vy = st[4 * ns + slot];
  L.vz = st[5 * ns + slot];
  L.m = st[6 * ns + slot];
  L.cqx = st[7 * ns + slot];
  L.cqy = st[8 * ns + slot];
  L.cqz = st[9 * ns + slot];
  L.cvx = st[10 * ns + slot];
  L.cvy = st[11 * ns + slot];
  L.cvz = st[12 * ns + slot];
  L.m0 = p.m0s[slot];
  L.dt = p.dts[slot];
  L.sys = p.slot_sys[slot];
  L.pl = p.slot_pl[slot];
  L.first = L.sys >= 0 ? p.synced[L.sys] : 1;
  return L;
}

__device__ __forceinline__ void store_lane(const StepParams& p, int slot, const Lane& L) {
  double* st = p.st;
  const int ns = p.ns;
  st[slot] = L.qx;
  st[ns + slot] = L.qy;
  st[2 * ns + slot] = L.qz;
  st[3 * ns + slot] = L.vx;
  st[4 * ns + slot] = L.vy;
  st[5 * ns + slot] = L.vz;
  st[7 * ns + slot] = L.cqx;
  st[8 * ns + slot] = L.cqy;
  st[9 * ns + slot] = L.cqz;
  st[10 * ns + slot] = L.cvx;
  st[11 * ns + slot] = L.cvy;
  st[12 * ns + slot] = L.cvz;
}

// The state of a coordinate is the unevaluated sum s + c (rounded value and
// compensation).  Operators read the rounded values.  A Kepler drift adds
// its increment to s by an exact two-sum and sends the two-sum's error, the
// increment's own low part and the image of c under the drift to c; kicks and
// jumps add their (small) increments to c; one renormalization per step
// moves c back to at most half an ulp of s.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}
__device__ __forceinline__ void renorm(double& s, double& c) {
#pragma clang fp contract(off)
  double t = s + c;
  c = c - (t - s);
  s = t;
}
__device__ __forceinline__ void add_hi(double& s, double& c, double h, double l) {
#pragma clang fp contract(off)
  double t, e;
  two_sum(s, h, t, e);
  s = t;
  c = (c + l) + e;
}

// Kepler drift K(tau) of the compensated state.  The coefficients come from
// the rounded values; the increment (f-1)Q + gV, f'Q + (g'-1)V is formed in
// double-double (lin2_dd) and c is carried through the same linear map.
// Returns the anomaly X.
// KC selects the iteration counts of the solve (KepSet, wh_device.h).
template <int KC = 0>
__device__ __forceinline__ double drift(Lane& L, double mu, double tau, KepDiag& dg) {
  KepCoef k;
  double X = kepler_coeffs<KepSet<KC>::NH, KepSet<KC>::NN, KepSet<KC>::KH, KepSet<KC>::KN>(L.qx, L.qy, L.qz, L.vx,
                                                                                          L.vy, L.vz, mu, tau, dg, k);
  double hqx, hqy, hqz, hvx, hvy, hvz, lqx, lqy, lqz, lvx, lvy, lvz;
  lin2_dd(k.fm1, L.qx, k.g, L.vx, hqx, lqx);
  lin2_dd(k.fm1, L.qy, k.g, L.vy, hqy, lqy);
  lin2_dd(k.fm1, L.qz, k.g, L.vz, hqz, lqz);
  lin2_dd(k.gdm1, L.vx, k.fd, L.qx, hvx, lvx);
  lin2_dd(k.gdm1, L.vy, k.fd, L.qy, hvy, lvy);
  lin2_dd(k.gdm1, L.vz, k.fd, L.qz, hvz, lvz);
  lqx = fma(k.fm1, L.cqx, fma(k.g, L.cvx, lqx));
  lqy = fma(k.fm1, L.cqy, fma(k.g, L.cvy, lqy));
  lqz = fma(k.fm1, L.cqz, fma(k.g, L.cvz, lqz));
  lvx = fma(k.fd, L.cqx, fma(k.gdm1, L.cvx, lvx));
  lvy = fma(k.fd, L.cqy, fma(k.gdm1, L.cvy, lvy));
  lvz = fma(k.fd, L.cqz, fma(k.gdm1, L.cvz, lvz));
  add_hi(L.qx, L.cqx, hqx, lqx);
  add_hi(L.qy, L.cqy, hqy, lqy);
  add_hi(L.qz, L.cqz, hqz, lqz);
  add_hi(L.vx, L.cvx, hvx, lvx);
  add_hi(L.vy, L.cvy, hvy, lvy);
  add_hi(L.vz, L.cvz, hvz, lvz);
  return X;
}

__device__ __forceinline__ void renorm_all(Lane& L) {
  renorm(L.qx, L.cqx); renorm(L.qy, L.cqy); renorm(L.qz, L.cqz);
  renorm(L.vx, L.cvx); renorm(L.vy, L.cvy); renorm(L.vz, L.cvz);
}

// ---------------------------------------------------------------------------
// Two planets per lane (WH_PACK_PAIR, see wh_pair.h): wave w covers slots
// [128 w, 128 w + 128); lane l holds slot 128 w + l ("a") and 128 w + 64 + l
// ("b").  The step is the one-planet step applied to both slots, with the
// interaction and momentum sums of the pair layout.

// (vka, vkb) receive the velocities after the kick (kept by the adjoint).
template <int G, bool GR>
__device__ __forceinline__ void kick_block_pair(Lane& A, Lane& B, const PairMass& pm, double inv_m0, double kg,
                                                double ta, double ti, double tc, double vka[3], double vkb[3]) {
  double sx, sy, sz;
  double qax = A.qx, qay = A.qy, qaz = A.qz, qbx = B.qx, qby = B.qy, qbz = B.qz;
  if (GR) {
    pair_momentum<G>(A.m, A.vx, A.vy, A.vz, B.m, B.vx, B.vy, B.vz, sx, sy, sz);
    const double k1 = ta * inv_m0;
    const double dqx = k1 * sx, dqy = k1 * sy, dqz = k1 * sz;
    A.cqx += dqx; A.cqy += dqy; A.cqz += dqz;
    B.cqx += dqx; B.cqy += dqy; B.cqz += dqz;
    qax += dqx; qay += dqy; qaz += dqz;
    qbx += dqx; qby += dqy; qbz += dqz;
  }
  double aax, aay, aaz, abx, aby, abz;
  accel_pair<G>(pm, A.m, B.m, qax, qay, qaz, qbx, qby, qbz, aax, aay, aaz, abx, aby, abz);
  if (GR) {
    double gx, gy, gz;
    gr_accel(qax, qay, qaz, kg, gx, gy, gz);
    aax += gx; aay += gy; aaz += gz;
    gr_accel(qbx, qby, qbz, kg, gx, gy, gz);
    abx += gx; aby += gy; abz += gz;
  }
  const double dvax = ti * aax, dvay = ti * aay, dvaz = ti * aaz;
  const double dvbx = ti * abx, dvby = ti * aby, dvbz = ti * abz;
  A.cvx += dvax; A.cvy += dvay; A.cvz += dvaz;
  B.cvx += dvbx; B.cvy += dvby; B.cvz += dvbz;
  vka[0] = A.vx + dvax; vka[1] = A.vy + dvay; vka[2] = A.vz + dvaz;
  vkb[0] = B.vx + dvbx; vkb[1] = B.vy + dvby; vkb[2] = B.vz + dvbz;
  pair_momentum<G>(A.m, vka[0], vka[1], vka[2], B.m, vkb[0], vkb[1], vkb[2], sx, sy, sz);
  const double k2 = (GR ? tc : ta + tc) * inv_m0;
  A.cqx += k2 * sx; A.cqy += k2 * sy; A.cqz += k2 * sz;
  B.cqx += k2 * sx; B.cqy += k2 * sy; B.cqz += k2 * sz;
  renorm_all(A);
  renorm_all(B);
}

__device__ __forceinline__ int lane_flags(const Lane& L, const KepDiag& dg, double zlim) {
  int f = 0;
  if (L.pl >= 0) {
    bool fin = __builtin_isfinite(L.qx) && __builtin_isfinite(L.qy) && __builtin_isfinite(L.qz) &&
               __builtin_isfinite(L.vx) && __builtin_isfinite(L.vy) && __builtin_isfinite(L.vz);
    if (!fin) f |= WH_F_NONFINITE;
    if (!(dg.bmin > 0.0)) f |= WH_F_HYPERBOLIC;
    if (!(dg.zmax <= zlim)) f |= WH_F_ZMAX;
  }
  return f;
}

template <int G, bool GR, int SCHEME, int KC = 0>
__device__ __forceinline__ void step_lane_pair(const StepParams& p, Lane& A, Lane& B, int lane) {
  const PairMass pm = make_pair_mass<G>(A.m, B.m);
  const double dt = A.dt;
  const double h = 0.5 * dt;
  const double inv_m0 = 1.0 / A.m0;
  const double kg = GR ? p.kgr * A.m0 * A.m0 : 0.0;
  KepDiag dga{0.0, 1.0e300}, dgb{0.0, 1.0e300};
  double vka[3], vkb[3];
  if constexpr (SCHEME == SCHEME_SABA) {
    // SABA_n as in step_lane, B = I and J together (DHC, no GR)
    const double c1dt = p.sc[0] * dt;
    double tk = A.first ? c1dt : 2.0 * c1dt;
    for (int s = 0; s < p.n_steps; ++s) {
      drift(A, A.m0, tk, dga);
      drift(B, B.m0, tk, dgb);
      tk = 2.0 * c1dt;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < p.saba_n) {
          const double tb = p.sd[k] * dt;
          kick_block_pair<G, false>(A, B, pm, inv_m0, 0.0, 0.5 * tb, tb, 0.5 * tb, vka, vkb);
          if (k + 1 < p.saba_n) {
            drift(A, A.m0, p.sc[k + 1] * dt, dga);
            drift(B, B.m0, p.sc[k + 1] * dt, dgb);
          }
        }
      }
    }
  } else if (SCHEME == WH_DKD) {
    double tk = A.first ? h : dt;
    for (int s = 0; s < p.n_steps; ++s) {
      drift<KC>(A, A.m0, tk, dga);
      drift<KC>(B, B.m0, tk, dgb);
      tk = dt;
      kick_block_pair<G, GR>(A, B, pm, inv_m0, kg, h, dt, h, vka, vkb);
    }
  } else {
    double ta = A.first ? 0.0 : h;
    double ti = A.first ? h : dt;
    for (int s = 0; s < p.n_steps; ++s) {
      kick_block_pair<G, GR>(A, B, pm, inv_m0, kg, ta, ti, h, vka, vkb);
      ta = h;
      ti = dt;
      drift<KC>(A, A.m0, dt, dga);
      drift<KC>(B, B.m0, dt, dgb);
    }
  }
  int f = group_or<G>(lane_flags(A, dga, p.zlim) | lane_flags(B, dgb, p.zlim));
  if ((lane & (G - 1)) == 0 && A.sys >= 0) {
    p.flags[A.sys] |= (uint32_t)f;
    p.synced[A.sys] = 0;
  }
}

template <int G, bool GR, int SCHEME, int KC = 0>
__device__ void step_group_pair(const StepParams& p, int sa, int lane) {
  Lane A = load_lane(p, sa);
  Lane B = load_lane(p, sa + 64);
  step_lane_pair<G, GR, SCHEME, KC>(p, A, B, lane);
  store_lane(p, sa, A);
  store_lane(p, sa + 64, B);
}

// The pair layout's persistent step kernel, defined and instantiated in
// wh_pair_step.hip for GR in {false, true} with drift-kick-drift and
// kick-drift-kick (Kepler count sets 0 and 1) and SABA_n (GR off, set 0).
template <bool GR, int SCHEME, int KC = 0>
__global__ __launch_bounds__(256) void k_step_pair(StepParams p);

}  // namespace wh
