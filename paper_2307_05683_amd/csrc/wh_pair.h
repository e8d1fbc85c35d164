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
#include "wh_device.h"

namespace wh {

// 1/|d|^3 for the separation d
__device__ __forceinline__ double inv_r3(double dx, double dy, double dz) {
  const double ir = rsqrt_full(fma(dx, dx, fma(dy, dy, dz * dz)));
  return ir * ir * ir;
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

}  // namespace wh
