// Two planets per lane (the WH_PACK_PAIR layout).
//
// A system of N planets takes an aligned group of G = 1, 2 or 4 lanes with
// 2G >= N; lane l of the group holds planet l in its "a" slot and planet
// G + l in its "b" slot.  Every lane runs two independent Kepler solves per
// drift, which the compiler interleaves, and the interaction pairs cost fewer
// evaluations and cross-lane moves per planet than one planet per lane:
//   the lane's own pair (a, b), no exchange;
//   G = 2: the partner lane (xor 1), each side computing its own four pairs;
//   G = 4: the next lane of the quad with reactions returned (four pairs,
//          each evaluated once), then the opposite lane (xor 2), each side
//          computing its own four pairs;
// so 9 evaluations per lane cover the 28 pairs of an 8-planet system (32
// lanes' worth, against 40 with one planet per lane), with 18 two-word DPP
// moves per lane instead of 27.  Everything else is the one-planet math of
// wh_device.h applied to both slots.
#pragma once
#include "wh_adjoint.h"
#include "wh_device.h"

namespace wh {

// 1/|d|^3 for the separation d: rsqrt3_full's refinement with its two
// constants in one FMA, (1 - e)^(-3/2) = 1 + e (3/2 + (15/8) e) + O(e^3).
// An instruction takes one scalar operand, so 15/8 is held in a register
// across the step loop: the empty asm statement hides its value from the
// compiler, which would otherwise re-create it at every use.  One
// instruction fewer per evaluation than rsqrt3_full, within the pair
// layout's register budget (two resident wavefronts per SIMD); the
// one-planet kernels keep rsqrt3_full, where the extra live register would
// cost occupancy.
__device__ __forceinline__ double inv_r3(double dx, double dy, double dz) {
  const double x = fma(dx, dx, fma(dy, dy, dz * dz));
  const double y = __builtin_amdgcn_rsq(x);
  const double y2 = y * y;
  const double e = fma(-x, y2, 1.0);
  const double y3 = y2 * y;
  double c = 1.875;
  __asm__("" : "+v"(c));
  return fma(y3 * e, fma(c, e, 1.5), y3);
}

// Partner masses of the rounds (constant, Sec. 3.5).
struct PairMass {
  double a1, b1, a2, b2;   // round 1 partner's a and b; round 2 partner's a and b
};
template <int G> __device__ __forceinline__ PairMass make_pair_mass(double ma, double mb) {
  PairMass t{0.0, 0.0, 0.0, 0.0};
  if (G == 2) { t.a1 = dpp<DPP_XOR1>(ma); t.b1 = dpp<DPP_XOR1>(mb); }
  if (G == 4) {
    t.a1 = dpp<QP_NEXT>(ma); t.b1 = dpp<QP_NEXT>(mb);
    t.a2 = dpp<DPP_XOR2>(ma); t.b2 = dpp<DPP_XOR2>(mb);
  }
  return t;
}

// Accelerations (aa, ab) of the lane's two planets from all other planets of
// the system (Sec. 3.3, acceleration equation).
template <int G>
__device__ __forceinline__ void accel_pair(const PairMass& pm, double ma, double mb, double ax, double ay, double az,
                                           double bx, double by, double bz, double& aax, double& aay, double& aaz,
                                           double& abx, double& aby, double& abz) {
  // the lane's own pair
  {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    const double w = inv_r3(dx, dy, dz);
    const double wa = mb * w, wb = ma * w;
    aax = -wa * dx; aay = -wa * dy; aaz = -wa * dz;
    abx = wb * dx; aby = wb * dy; abz = wb * dz;
  }
  if (G == 2) {
    const double pax = dpp<DPP_XOR1>(ax), pay = dpp<DPP_XOR1>(ay), paz = dpp<DPP_XOR1>(az);
    const double pbx = dpp<DPP_XOR1>(bx), pby = dpp<DPP_XOR1>(by), pbz = dpp<DPP_XOR1>(bz);
    double dx, dy, dz, w;
    dx = ax - pax; dy = ay - pay; dz = az - paz; w = pm.a1 * inv_r3(dx, dy, dz);
    aax = fma(-w, dx, aax); aay = fma(-w, dy, aay); aaz = fma(-w, dz, aaz);
    dx = ax - pbx; dy = ay - pby; dz = az - pbz; w = pm.b1 * inv_r3(dx, dy, dz);
    aax = fma(-w, dx, aax); aay = fma(-w, dy, aay); aaz = fma(-w, dz, aaz);
    dx = bx - pax; dy = by - pay; dz = bz - paz; w = pm.a1 * inv_r3(dx, dy, dz);
    abx = fma(-w, dx, abx); aby = fma(-w, dy, aby); abz = fma(-w, dz, abz);
    dx = bx - pbx; dy = by - pby; dz = bz - pbz; w = pm.b1 * inv_r3(dx, dy, dz);
    abx = fma(-w, dx, abx); aby = fma(-w, dy, aby); abz = fma(-w, dz, abz);
  }
  if (G == 4) {
    // round 1: the next lane of the quad; its planets' reactions go back
    {
      const double pax = dpp<QP_NEXT>(ax), pay = dpp<QP_NEXT>(ay), paz = dpp<QP_NEXT>(az);
      const double pbx = dpp<QP_NEXT>(bx), pby = dpp<QP_NEXT>(by), pbz = dpp<QP_NEXT>(bz);
      double rax = 0.0, ray = 0.0, raz = 0.0, rbx = 0.0, rby = 0.0, rbz = 0.0;
      double dx, dy, dz, w;
      // (a, partner a)
      dx = ax - pax; dy = ay - pay; dz = az - paz; w = inv_r3(dx, dy, dz);
      aax = fma(-pm.a1 * w, dx, aax); aay = fma(-pm.a1 * w, dy, aay); aaz = fma(-pm.a1 * w, dz, aaz);
      rax = fma(ma * w, dx, rax); ray = fma(ma * w, dy, ray); raz = fma(ma * w, dz, raz);
      // (a, partner b)
      dx = ax - pbx; dy = ay - pby; dz = az - pbz; w = inv_r3(dx, dy, dz);
      aax = fma(-pm.b1 * w, dx, aax); aay = fma(-pm.b1 * w, dy, aay); aaz = fma(-pm.b1 * w, dz, aaz);
      rbx = fma(ma * w, dx, rbx); rby = fma(ma * w, dy, rby); rbz = fma(ma * w, dz, rbz);
      // (b, partner a)
      dx = bx - pax; dy = by - pay; dz = bz - paz; w = inv_r3(dx, dy, dz);
      abx = fma(-pm.a1 * w, dx, abx); aby = fma(-pm.a1 * w, dy, aby); abz = fma(-pm.a1 * w, dz, abz);
      rax = fma(mb * w, dx, rax); ray = fma(mb * w, dy, ray); raz = fma(mb * w, dz, raz);
      // (b, partner b)
      dx = bx - pbx; dy = by - pby; dz = bz - pbz; w = inv_r3(dx, dy, dz);
      abx = fma(-pm.b1 * w, dx, abx); aby = fma(-pm.b1 * w, dy, aby); abz = fma(-pm.b1 * w, dz, abz);
      rbx = fma(mb * w, dx, rbx); rby = fma(mb * w, dy, rby); rbz = fma(mb * w, dz, rbz);
      // the previous lane computed the reactions on this lane's planets
      aax += dpp<QP_PREV>(rax); aay += dpp<QP_PREV>(ray); aaz += dpp<QP_PREV>(raz);
      abx += dpp<QP_PREV>(rbx); aby += dpp<QP_PREV>(rby); abz += dpp<QP_PREV>(rbz);
    }
    // round 2: the opposite lane, each side its own four pairs
    {
      const double pax = dpp<DPP_XOR2>(ax), pay = dpp<DPP_XOR2>(ay), paz = dpp<DPP_XOR2>(az);
      const double pbx = dpp<DPP_XOR2>(bx), pby = dpp<DPP_XOR2>(by), pbz = dpp<DPP_XOR2>(bz);
      double dx, dy, dz, w;
      dx = ax - pax; dy = ay - pay; dz = az - paz; w = pm.a2 * inv_r3(dx, dy, dz);
      aax = fma(-w, dx, aax); aay = fma(-w, dy, aay); aaz = fma(-w, dz, aaz);
      dx = ax - pbx; dy = ay - pby; dz = az - pbz; w = pm.b2 * inv_r3(dx, dy, dz);
      aax = fma(-w, dx, aax); aay = fma(-w, dy, aay); aaz = fma(-w, dz, aaz);
      dx = bx - pax; dy = by - pay; dz = bz - paz; w = pm.a2 * inv_r3(dx, dy, dz);
      abx = fma(-w, dx, abx); aby = fma(-w, dy, aby); abz = fma(-w, dz, abz);
      dx = bx - pbx; dy = by - pby; dz = bz - pbz; w = pm.b2 * inv_r3(dx, dy, dz);
      abx = fma(-w, dx, abx); aby = fma(-w, dy, aby); abz = fma(-w, dz, abz);
    }
  }
}

// Momentum of the system, sum over both slots of every lane of the group.
template <int G>
__device__ __forceinline__ void pair_momentum(double ma, double vax, double vay, double vaz, double mb, double vbx,
                                              double vby, double vbz, double& sx, double& sy, double& sz) {
  sx = group_sum<G>(fma(ma, vax, mb * vbx));
  sy = group_sum<G>(fma(ma, vay, mb * vby));
  sz = group_sum<G>(fma(ma, vaz, mb * vbz));
}

// ---------------------------------------------------------------------------
// Reverse mode of the pair layout.  Vectors of the two slots are passed as
// double[3] arrays (a: the lane's first planet, b: its second).

// Adjoint of the interaction kick V += tau a(Q) for both slots: pair_vjp for
// every pair accel_pair evaluates, over the same rounds.  A pair evaluated
// once (the lane's own pair, the reaction round of G = 4) gives the partner
// the negated share; in the symmetric rounds each side takes its own.
template <int G>
__device__ __forceinline__ void interaction_vjp_pair(const PairMass& pm, double ma, double mb, const double qa[3],
                                                     const double qb[3], const double gva[3], const double gvb[3],
                                                     double tau, double gqa[3], double gqb[3], double& gma,
                                                     double& gmb) {
  double c[3], co, cp;
  auto vjp = [&](const double* q, const double* gv, double m, const double* p, const double* pg, double mj) {
    pair_vjp(q[0], q[1], q[2], gv[0], gv[1], gv[2], m, p[0], p[1], p[2], pg[0], pg[1], pg[2], mj, tau, c[0], c[1],
             c[2], co, cp);
  };
  vjp(qa, gva, ma, qb, gvb, mb);       // the lane's own pair
  for (int k = 0; k < 3; ++k) { gqa[k] += c[k]; gqb[k] -= c[k]; }
  gma += co; gmb += cp;
  if (G == 2 || G == 4) {
    // G = 4 round 1: the next lane of the quad, reactions returned
    double pa[3], pb[3], pga[3], pgb[3], ra[3] = {0.0, 0.0, 0.0}, rb[3] = {0.0, 0.0, 0.0}, ram = 0.0, rbm = 0.0;
    if (G == 4) {
      for (int k = 0; k < 3; ++k) {
        pa[k] = dpp<QP_NEXT>(qa[k]); pb[k] = dpp<QP_NEXT>(qb[k]);
        pga[k] = dpp<QP_NEXT>(gva[k]); pgb[k] = dpp<QP_NEXT>(gvb[k]);
      }
      vjp(qa, gva, ma, pa, pga, pm.a1);
      for (int k = 0; k < 3; ++k) { gqa[k] += c[k]; ra[k] -= c[k]; }
      gma += co; ram += cp;
      vjp(qa, gva, ma, pb, pgb, pm.b1);
      for (int k = 0; k < 3; ++k) { gqa[k] += c[k]; rb[k] -= c[k]; }
      gma += co; rbm += cp;
      vjp(qb, gvb, mb, pa, pga, pm.a1);
      for (int k = 0; k < 3; ++k) { gqb[k] += c[k]; ra[k] -= c[k]; }
      gmb += co; ram += cp;
      vjp(qb, gvb, mb, pb, pgb, pm.b1);
      for (int k = 0; k < 3; ++k) { gqb[k] += c[k]; rb[k] -= c[k]; }
      gmb += co; rbm += cp;
      for (int k = 0; k < 3; ++k) { gqa[k] += dpp<QP_PREV>(ra[k]); gqb[k] += dpp<QP_PREV>(rb[k]); }
      gma += dpp<QP_PREV>(ram);
      gmb += dpp<QP_PREV>(rbm);
    }
    // symmetric round: G = 2 the partner lane (xor 1), G = 4 the opposite lane (xor 2)
    double ma2, mb2;
    for (int k = 0; k < 3; ++k) {
      if (G == 2) {
        pa[k] = dpp<DPP_XOR1>(qa[k]); pb[k] = dpp<DPP_XOR1>(qb[k]);
        pga[k] = dpp<DPP_XOR1>(gva[k]); pgb[k] = dpp<DPP_XOR1>(gvb[k]);
      } else {
        pa[k] = dpp<DPP_XOR2>(qa[k]); pb[k] = dpp<DPP_XOR2>(qb[k]);
        pga[k] = dpp<DPP_XOR2>(gva[k]); pgb[k] = dpp<DPP_XOR2>(gvb[k]);
      }
    }
    ma2 = G == 2 ? pm.a1 : pm.a2;
    mb2 = G == 2 ? pm.b1 : pm.b2;
    vjp(qa, gva, ma, pa, pga, ma2);
    for (int k = 0; k < 3; ++k) gqa[k] += c[k];
    gma += co;
    vjp(qa, gva, ma, pb, pgb, mb2);
    for (int k = 0; k < 3; ++k) gqa[k] += c[k];
    gma += co;
    vjp(qb, gvb, mb, pa, pga, ma2);
    for (int k = 0; k < 3; ++k) gqb[k] += c[k];
    gmb += co;
    vjp(qb, gvb, mb, pb, pgb, mb2);
    for (int k = 0; k < 3; ++k) gqb[k] += c[k];
    gmb += co;
  }
}

}  // namespace wh
