// Reverse-mode (adjoint) building blocks of the Wisdom-Holman step, FP64.
//
// Each function takes the adjoint (gradient) of a sub-step's outputs and
// returns the adjoint of its inputs, accumulating the adjoints of the masses.
// Notation of the forward step: K(tau) maps (Q, V) to (f Q + g V, f' Q + g' V);
// I(tau) adds tau a(Q) to V; J(tau) adds (tau/m0) sum_j m_j V_j to Q; the GR
// kick adds -tau 6 m0^2/c^2 Q/|Q|^4 to V.
#pragma once
#include "wh_device.h"

namespace wh {

// Stumpff functions c2..c5 by series (K terms of c4 and c5, then the
// recurrence c_n = 1/n! - z c_{n+2}), for the G functions G0..G5 the Kepler
// derivatives need.
template <int K> __device__ __forceinline__ void stumpff_c0_c5(double z, double c[6]) {
  c[4] = stumpff_series<K, 4>(z);
  c[5] = stumpff_series<K, 5>(z);
  c[2] = fma(-z, c[4], 0.5);
  c[3] = fma(-z, c[5], 1.0 / 6.0);
  c[0] = fma(-z, c[2], 1.0);
  c[1] = fma(-z, c[3], 1.0);
}

// Forward quantities of one Kepler drift at a known anomaly X.
struct KepFwd {
  double r0, eta, beta, zeta, X;
  double G[6];
  double r, f, g, fd, gd;
};

__device__ __forceinline__ void kepler_at_X(double qx, double qy, double qz, double vx, double vy, double vz,
                                            double mu, double tau, double X, KepFwd& k) {
  double r2 = fma(qx, qx, fma(qy, qy, qz * qz));
  double v2 = fma(vx, vx, fma(vy, vy, vz * vz));
  k.eta = fma(qx, vx, fma(qy, vy, qz * vz));
  k.r0 = sqrt(r2);
  k.beta = 2.0 * mu / k.r0 - v2;
  k.zeta = fma(-k.beta, k.r0, mu);
  k.X = X;
  double X2 = X * X;
  double c[6];
  stumpff_c0_c5<8>(k.beta * X2, c);
  double Xn = 1.0;
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    k.G[n] = Xn * c[n];
    Xn *= X;
  }
  k.r = fma(k.eta, k.G[1], fma(k.zeta, k.G[2], k.r0));
  k.f = 1.0 - mu * k.G[2] / k.r0;
  k.g = fma(-mu, k.G[3], tau);
  k.fd = -mu * k.G[1] / (k.r0 * k.r);
  k.gd = 1.0 - mu * k.G[2] / k.r;
}

// Adjoint of the Kepler drift.  In: (gQ1, gV1), the adjoint of the output.
// Out: (gQ, gV) the adjoint of the input, gmu += the adjoint of mu = G m0.
// The anomaly X is defined implicitly by F(X; r0, eta, zeta, beta) = 0, so by
// the implicit function theorem dX = -(F_r0 dr0 + F_eta deta + F_zeta dzeta +
// F_beta dbeta) / F_X with F_X = r, F_r0 = X, F_eta = G2, F_zeta = G3 and
// F_beta = eta dG2/dbeta + zeta dG3/dbeta, where dG_n/dbeta =
// (n G_{n+2} - X G_{n+1}) / 2 and dG_n/dX = G_{n-1}.
__device__ __forceinline__ void kepler_vjp(const KepFwd& k, double qx, double qy, double qz, double vx, double vy,
                                           double vz, double mu, double& gqx, double& gqy, double& gqz,
                                           double& gvx, double& gvy, double& gvz, double& gmu) {
  const double* G = k.G;
  // outputs Q1 = f Q + g V, V1 = f' Q + g' V
  double gf = gqx * qx + gqy * qy + gqz * qz;
  double gg = gqx * vx + gqy * vy + gqz * vz;
  double gfd = gvx * qx + gvy * qy + gvz * qz;
  double ggd = gvx * vx + gvy * vy + gvz * vz;
  double nqx = k.f * gqx + k.fd * gvx, nqy = k.f * gqy + k.fd * gvy, nqz = k.f * gqz + k.fd * gvz;
  double nvx = k.g * gqx + k.gd * gvx, nvy = k.g * gqy + k.gd * gvy, nvz = k.g * gqz + k.gd * gvz;
  // f = 1 - mu G2/r0, g = tau - mu G3, f' = -mu G1/(r0 r), g' = 1 - mu G2/r
  double ir0 = 1.0 / k.r0, ir = 1.0 / k.r;
  double gm = -gf * G[2] * ir0 - gg * G[3] + gfd * k.fd / mu - ggd * G[2] * ir;
  double gG1 = -gfd * mu * ir0 * ir;
  double gG2 = -gf * mu * ir0 - ggd * mu * ir;
  double gG3 = -gg * mu;
  double gr0 = gf * mu * G[2] * ir0 * ir0 - gfd * k.fd * ir0;
  double gr = -gfd * k.fd * ir + ggd * mu * G[2] * ir * ir;
  // r = r0 + eta G1 + zeta G2
  gr0 += gr;
  double geta = gr * G[1];
  double gzeta = gr * G[2];
  gG1 += gr * k.eta;
  gG2 += gr * k.zeta;
  // G_n(beta, X)
  const double X = k.X;
  double dG1b = 0.5 * (G[3] - X * G[2]);
  double dG2b = 0.5 * (2.0 * G[4] - X * G[3]);
  double dG3b = 0.5 * (3.0 * G[5] - X * G[4]);
  double gX = gG1 * G[0] + gG2 * G[1] + gG3 * G[2];
  double gbeta = gG1 * dG1b + gG2 * dG2b + gG3 * dG3b;
  // implicit function theorem for X
  double Fb = k.eta * dG2b + k.zeta * dG3b;
  double s = -gX * ir;        // -gX / F_X
  gr0 += s * X;
  geta += s * G[2];
  gzeta += s * G[3];
  gbeta += s * Fb;
  // zeta = mu - beta r0
  gm += gzeta;
  gbeta -= gzeta * k.r0;
  gr0 -= gzeta * k.beta;
  // beta = 2 mu / r0 - |V|^2
  gm += 2.0 * gbeta * ir0;
  gr0 -= 2.0 * gbeta * mu * ir0 * ir0;
  double gv2 = -gbeta;
  // eta = Q.V, |V|^2, r0 = |Q|
  nqx += geta * vx + gr0 * qx * ir0;
  nqy += geta * vy + gr0 * qy * ir0;
  nqz += geta * vz + gr0 * qz * ir0;
  nvx += geta * qx + 2.0 * gv2 * vx;
  nvy += geta * qy + 2.0 * gv2 * vy;
  nvz += geta * qz + 2.0 * gv2 * vz;
  gqx = nqx; gqy = nqy; gqz = nqz;
  gvx = nvx; gvy = nvy; gvz = nvz;
  gmu += gm;
}

// Adjoint of the interaction kick V += tau a(Q) inside a group, with the DPP
// rounds of interaction_accel_dpp.  With a_i = -sum_j m_j d_ij/|d_ij|^3,
// d_ij = Q_i - Q_j and T_ij = I/r^3 - 3 d d^T/r^5 (symmetric):
//   gQ_k += tau sum_{j != k} T_kj (m_k gV_j - m_j gV_k)
//   gm_k += tau sum_{i != k} gV_i . (Q_k - Q_i) / r^3
// For a pair computed once, the partner's share is the negative of the
// lane's own share, which two-sided rounds send back.
__device__ __forceinline__ void pair_vjp(double qx, double qy, double qz, double gvx, double gvy, double gvz,
                                         double m, double px, double py, double pz, double pgx, double pgy,
                                         double pgz, double mj, double tau, double& cx, double& cy, double& cz,
                                         double& cm_own, double& cm_partner) {
  double dx = qx - px, dy = qy - py, dz = qz - pz;
  double r2 = dx * dx + dy * dy + dz * dz;
  double ir = rsqrt_full(r2);
  double ir2 = ir * ir;
  double ir3 = ir2 * ir;
  double ux = m * pgx - mj * gvx, uy = m * pgy - mj * gvy, uz = m * pgz - mj * gvz;
  double du = dx * ux + dy * uy + dz * uz;
  double w = 3.0 * du * ir2;
  double t = tau * ir3;
  cx = t * (ux - w * dx);
  cy = t * (uy - w * dy);
  cz = t * (uz - w * dz);
  cm_own = t * (pgx * dx + pgy * dy + pgz * dz);
  cm_partner = -t * (gvx * dx + gvy * dy + gvz * dz);
}

template <int G>
__device__ __forceinline__ void interaction_vjp_dpp(const DppMass& t, double qx, double qy, double qz, double m,
                                                    double tau, double gvx, double gvy, double gvz, double& gqx,
                                                    double& gqy, double& gqz, double& gm) {
  double cx, cy, cz, co, cp;
  if (G == 2) {
    pair_vjp(qx, qy, qz, gvx, gvy, gvz, m, dpp<DPP_XOR1>(qx), dpp<DPP_XOR1>(qy), dpp<DPP_XOR1>(qz),
             dpp<DPP_XOR1>(gvx), dpp<DPP_XOR1>(gvy), dpp<DPP_XOR1>(gvz), t.m[0], tau, cx, cy, cz, co, cp);
    gqx += cx; gqy += cy; gqz += cz; gm += co;
  }
  if (G >= 4) {
    pair_vjp(qx, qy, qz, gvx, gvy, gvz, m, dpp<QP_NEXT>(qx), dpp<QP_NEXT>(qy), dpp<QP_NEXT>(qz),
             dpp<QP_NEXT>(gvx), dpp<QP_NEXT>(gvy), dpp<QP_NEXT>(gvz), t.m[0], tau, cx, cy, cz, co, cp);
    gqx += cx - dpp<QP_PREV>(cx);
    gqy += cy - dpp<QP_PREV>(cy);
    gqz += cz - dpp<QP_PREV>(cz);
    gm += co + dpp<QP_PREV>(cp);
    pair_vjp(qx, qy, qz, gvx, gvy, gvz, m, dpp<DPP_XOR2>(qx), dpp<DPP_XOR2>(qy), dpp<DPP_XOR2>(qz),
             dpp<DPP_XOR2>(gvx), dpp<DPP_XOR2>(gvy), dpp<DPP_XOR2>(gvz), t.m[1], tau, cx, cy, cz, co, cp);
    gqx += cx; gqy += cy; gqz += cz; gm += co;
  }
  if (G == 8) {
    double mx = dpp<DPP_HALF_MIRROR>(qx), my = dpp<DPP_HALF_MIRROR>(qy), mz = dpp<DPP_HALF_MIRROR>(qz);
    double hx = dpp<DPP_HALF_MIRROR>(gvx), hy = dpp<DPP_HALF_MIRROR>(gvy), hz = dpp<DPP_HALF_MIRROR>(gvz);
    pair_vjp(qx, qy, qz, gvx, gvy, gvz, m, dpp<QP_R3>(mx), dpp<QP_R3>(my), dpp<QP_R3>(mz), dpp<QP_R3>(hx),
             dpp<QP_R3>(hy), dpp<QP_R3>(hz), t.m[2], tau, cx, cy, cz, co, cp);
    gqx += cx - dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(cx));
    gqy += cy - dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(cy));
    gqz += cz - dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(cz));
    gm += co + dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(cp));
    pair_vjp(qx, qy, qz, gvx, gvy, gvz, m, dpp<QP_R4>(mx), dpp<QP_R4>(my), dpp<QP_R4>(mz), dpp<QP_R4>(hx),
             dpp<QP_R4>(hy), dpp<QP_R4>(hz), t.m[3], tau, cx, cy, cz, co, cp);
    gqx += cx; gqy += cy; gqz += cz; gm += co;
    pair_vjp(qx, qy, qz, gvx, gvy, gvz, m, dpp<QP_R5>(mx), dpp<QP_R5>(my), dpp<QP_R5>(mz), dpp<QP_R5>(hx),
             dpp<QP_R5>(hy), dpp<QP_R5>(hz), t.m[4], tau, cx, cy, cz, co, cp);
    gqx += cx; gqy += cy; gqz += cz; gm += co;
  }
}

// Adjoint of the GR kick V += tau * (-kg Q/|Q|^4), kg = 6 mu^2 / c^2:
//   gQ += -tau kg (gV/|Q|^4 - 4 Q (Q.gV)/|Q|^6),  gmu += tau gV.a_GR * 2/mu.
__device__ __forceinline__ void gr_vjp(double qx, double qy, double qz, double kg, double mu, double tau,
                                       double gvx, double gvy, double gvz, double& gqx, double& gqy, double& gqz,
                                       double& gmu) {
  double r2 = qx * qx + qy * qy + qz * qz;
  double ir2 = 1.0 / r2;
  double ir4 = ir2 * ir2;
  double qg = qx * gvx + qy * gvy + qz * gvz;
  double s = -tau * kg * ir4;
  double w = -4.0 * qg * ir2;
  gqx += s * (gvx + w * qx);
  gqy += s * (gvy + w * qy);
  gqz += s * (gvz + w * qz);
  gmu += 2.0 * s * qg / mu;
}

}  // namespace wh
