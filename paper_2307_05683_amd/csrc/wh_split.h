// Two lanes per planet (the WH_PACK_SPLIT layout).
//
// A system takes one aligned 16-lane group, i.e. one DPP row: planet p
// (padding planets beyond N included) lives in lanes 2p and 2p + 1, which
// hold bitwise-identical copies of its state.  Both copies run the same drift,
// jump and GR kick; only the interaction kick (Sec. 3.3, acceleration
// equation) is divided between them.  This halves the lanes' share of the
// O(N^2) work at the cost of a duplicated Kepler solve, which pays when an
// ensemble has fewer wavefronts than the chip has SIMDs.
//
// Interaction schedule.  With row_ror moves inside the row, lane L reads
// lane L + s (mod 16).  For L = 2p + c and odd s = 2k + 1 the source is copy
// 1 - c of planet p + k + c, so one move gives the two copies different
// partners:
//   round 1 (s = 3): copy 0 pairs with planet p + 1, copy 1 with p + 2;
//   round 2 (s = 7): copy 0 pairs with planet p + 3, copy 1 with p + 4.
// Each lane returns its partner's reaction by the inverse rotation (lane L
// reads lane L - s, which computed the pair with L's planet).  Offsets 1..3
// give 24 distinct pairs and offset 4 the remaining 4, each twice: copy 1 of
// planets 4..7 carries zero weights in round 2.  Two evaluations per lane
// cover the 28 pairs of an 8-planet system; the copies then add their shares
// (a0 + a1 and a1 + a0 are the same bits, so the copies stay identical).
#pragma once
#include "wh_adjoint.h"
#include "wh_device.h"

namespace wh {

struct SplitMass {
  double m1, m2;   // partner mass of rounds 1 and 2 (constant, Sec. 3.5)
  double w2;       // own mass for the round-2 reaction
  double on2;      // 1, or 0 where round 2 repeats a pair
};

__device__ __forceinline__ SplitMass make_split_mass(int lane, double m) {
  SplitMass t;
  // copy 1 of planets 4..7 repeats pairs (p, p + 4) that copy 1 of p - 4 has
  const bool dup = (lane & 1) && (lane & 8);
  t.m1 = dpp<DPP_ROR13>(m);
  const double m2 = dpp<DPP_ROR9>(m);
  t.m2 = dup ? 0.0 : m2;
  t.w2 = dup ? 0.0 : m;
  t.on2 = dup ? 0.0 : 1.0;
  return t;
}

// Acceleration of the lane's planet from the other planets of the system;
// both copies receive the same bits.
__device__ __forceinline__ void accel_split(const SplitMass& t, double qx, double qy, double qz, double m,
                                            double& ax, double& ay, double& az) {
  ax = 0.0; ay = 0.0; az = 0.0;
  double dx, dy, dz;
  double ir3 = pair_accel(qx, qy, qz, dpp<DPP_ROR13>(qx), dpp<DPP_ROR13>(qy), dpp<DPP_ROR13>(qz), t.m1, ax, ay, az,
                          dx, dy, dz);
  double wi = m * ir3;   // the partner's acceleration is +wi * d
  ax += dpp<DPP_ROR3>(wi * dx);
  ay += dpp<DPP_ROR3>(wi * dy);
  az += dpp<DPP_ROR3>(wi * dz);
  ir3 = pair_accel(qx, qy, qz, dpp<DPP_ROR9>(qx), dpp<DPP_ROR9>(qy), dpp<DPP_ROR9>(qz), t.m2, ax, ay, az, dx, dy,
                   dz);
  wi = t.w2 * ir3;
  ax += dpp<DPP_ROR7>(wi * dx);
  ay += dpp<DPP_ROR7>(wi * dy);
  az += dpp<DPP_ROR7>(wi * dz);
  ax += dpp<DPP_XOR1>(ax);
  ay += dpp<DPP_XOR1>(ay);
  az += dpp<DPP_XOR1>(az);
}

// Adjoint of the split interaction kick V += tau a(Q) (pair_vjp per
// evaluated pair, over the same two rounds): each lane accumulates its own
// share and the share the inverse rotation returns for its planet, then the
// copies add their shares as in the forward kick, so both keep the same bits.
__device__ __forceinline__ void interaction_vjp_split(const SplitMass& t, double qx, double qy, double qz, double m,
                                                      double tau, double gvx, double gvy, double gvz, double& gqx,
                                                      double& gqy, double& gqz, double& gm) {
  double cx, cy, cz, co, cp;
  double sx, sy, sz, sm;
  pair_vjp(qx, qy, qz, gvx, gvy, gvz, m, dpp<DPP_ROR13>(qx), dpp<DPP_ROR13>(qy), dpp<DPP_ROR13>(qz),
           dpp<DPP_ROR13>(gvx), dpp<DPP_ROR13>(gvy), dpp<DPP_ROR13>(gvz), t.m1, tau, cx, cy, cz, co, cp);
  sx = cx - dpp<DPP_ROR3>(cx);
  sy = cy - dpp<DPP_ROR3>(cy);
  sz = cz - dpp<DPP_ROR3>(cz);
  sm = co + dpp<DPP_ROR3>(cp);
  pair_vjp(qx, qy, qz, gvx, gvy, gvz, m, dpp<DPP_ROR9>(qx), dpp<DPP_ROR9>(qy), dpp<DPP_ROR9>(qz),
           dpp<DPP_ROR9>(gvx), dpp<DPP_ROR9>(gvy), dpp<DPP_ROR9>(gvz), t.m2, tau * t.on2, cx, cy, cz, co, cp);
  sx += cx - dpp<DPP_ROR7>(cx);
  sy += cy - dpp<DPP_ROR7>(cy);
  sz += cz - dpp<DPP_ROR7>(cz);
  sm += co + dpp<DPP_ROR7>(cp);
  gqx += sx + dpp<DPP_XOR1>(sx);
  gqy += sy + dpp<DPP_XOR1>(sy);
  gqz += sz + dpp<DPP_XOR1>(sz);
  gm += sm + dpp<DPP_XOR1>(sm);
}

}  // namespace wh
