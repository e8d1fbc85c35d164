// Device math of the Wisdom-Holman step for CDNA4 (gfx950), FP64 throughout.
//
// One lane holds one planet.  A system of N planets occupies an aligned group
// of G = 1, 2, 4 or 8 lanes of a 64-lane wavefront; lanes of the group beyond
// N are inert padding (zero mass).  Cross-lane traffic never leaves the
// group: sums use DPP row operations, partner exchange uses ds_bpermute (the
// LDS crossbar, no LDS storage and no barrier).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wh {

// ---------------------------------------------------------------------------
// Reciprocal and reciprocal square root.  The hardware seeds (v_rcp_f64,
// v_rsq_f64) are good to about 2^-24; one Newton step with the second-order
// term, y (1 + e + e^2) for 1/x and y (1 + e/2 + 3e^2/8) for 1/sqrt(x), leaves
// an O(e^3) error below the final rounding.
__device__ __forceinline__ double rcp_seed(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ double rcp_full(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  return fma(y, fma(e, e, e), y);
}
__device__ __forceinline__ double rsqrt_full(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = x * y;
  double e = fma(-h, y, 1.0);
  double c = fma(0.375, e, 0.5);
  return fma(y * e, c, y);
}
// x^(-3/2), the 1/r^3 of the kicks, from the same seed in one step:
// (1 - e)^(-3/2) = 1 + (3e/2)(1 + 5e/4) + O(e^3) with e = 1 - x y^2, applied
// to y^3.  As many instructions as cubing rsqrt_full, and closer (within 2.5
// units of 2^-53 against 5.6, over 2e7 arguments with seeds off by up to
// 2^-21, against long double).  Every instruction takes at most one
// constant that is not an inline one (1.25, 1.5): the single form
// fma(15/8, e, 3/2) needs both in one instruction, which the VALU's one
// scalar operand turns into two register moves per evaluation.
__device__ __forceinline__ double rsqrt3_full(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double y2 = y * y;
  double e = fma(-x, y2, 1.0);
  double y3 = y2 * y;
  double s = fma(1.25, e, 1.0);
  return fma(1.5 * (y3 * e), s, y3);
}

// ---------------------------------------------------------------------------
// Cross-lane moves of 64-bit values (two 32-bit moves each), with bound_ctrl
// set: a lane whose source lies outside its 16-lane row reads 0 (only the row
// shifts of the group scans below do that, and they mask such lanes out).
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
  int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL> __device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
// DPP controls: quad_perm [1,0,3,2] (xor 1), [2,3,0,1] (xor 2), row_half_mirror
// (lane i of each 8-lane half-row reads lane 7-i).
constexpr int DPP_XOR1 = 0xB1;
constexpr int DPP_XOR2 = 0x4E;
constexpr int DPP_HALF_MIRROR = 0x141;

__device__ __forceinline__ double bperm(int src_byte_addr, double v) {
  int lo = __builtin_amdgcn_ds_bpermute(src_byte_addr, __double2loint(v));
  int hi = __builtin_amdgcn_ds_bpermute(src_byte_addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// row_ror:n -- lane l of a 16-lane row reads lane (l - n) mod 16
constexpr int DPP_ROR3 = 0x123, DPP_ROR7 = 0x127, DPP_ROR8 = 0x128, DPP_ROR9 = 0x129, DPP_ROR13 = 0x12D;

// Group of 16 lanes = the split layout (wh_split.h): planet p in lanes 2p and
// 2p + 1, which hold identical copies.
constexpr int G_SPLIT = 16;

// Sum over an aligned group of G lanes; every lane receives the same bits.
// Butterfly: after stage s each lane holds the sum of its 2^s-lane block
// (the GPU form of the three shuffle-and-add stages of Sec. 3.4).  In the
// split layout the sum runs over planets, each counted once: lanes xor 2 are
// planets p and p ^ 1 of one copy, after which every lane of a quad holds the
// same bits, and the half-row mirror and the row rotation by 8 add the other
// quad and the other half-row.
template <int G> __device__ __forceinline__ double group_sum(double v) {
  if (G == G_SPLIT) {
    v += dpp<DPP_XOR2>(v);
    v += dpp<DPP_HALF_MIRROR>(v);
    return v + dpp<DPP_ROR8>(v);
  }
  if (G >= 2) v += dpp<DPP_XOR1>(v);
  if (G >= 4) v += dpp<DPP_XOR2>(v);
  if (G >= 8) v += dpp<DPP_HALF_MIRROR>(v);
  return v;
}
template <int G> __device__ __forceinline__ int group_or(int v) {
  if (G >= 2) v |= dpp_i<DPP_XOR1>(v);
  if (G >= 4) v |= dpp_i<DPP_XOR2>(v);
  if (G >= 8) v |= dpp_i<DPP_HALF_MIRROR>(v);
  if (G >= 16) v |= dpp_i<DPP_ROR8>(v);
  return v;
}

// Prefix and suffix sums inside an aligned G-lane group (p = lane index in
// the group), Hillis-Steele over DPP row shifts: row_shr:n hands lane l the
// value of lane l - n, row_shl:n that of lane l + n.  Groups never straddle a
// 16-lane row, so every needed source is in the row; sources from the
// neighbouring group are masked off.
constexpr int DPP_ROW_SHL1 = 0x101, DPP_ROW_SHL2 = 0x102, DPP_ROW_SHL4 = 0x104;
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114;

// sum over lanes p' <= p
template <int G> __device__ __forceinline__ double group_scan_incl(double v, int p) {
  if (G >= 2) { double t = dpp<DPP_ROW_SHR1>(v); v += (p >= 1) ? t : 0.0; }
  if (G >= 4) { double t = dpp<DPP_ROW_SHR2>(v); v += (p >= 2) ? t : 0.0; }
  if (G >= 8) { double t = dpp<DPP_ROW_SHR4>(v); v += (p >= 4) ? t : 0.0; }
  return v;
}
// sum over lanes p' < p
template <int G> __device__ __forceinline__ double group_scan_excl(double v, int p) {
  if (G == 1) return 0.0;
  double t = dpp<DPP_ROW_SHR1>(v);
  return group_scan_incl<G>((p >= 1) ? t : 0.0, p);
}
// sum over lanes p' >= p
template <int G> __device__ __forceinline__ double group_suffix_incl(double v, int p) {
  if (G >= 2) { double t = dpp<DPP_ROW_SHL1>(v); v += (p + 1 < G) ? t : 0.0; }
  if (G >= 4) { double t = dpp<DPP_ROW_SHL2>(v); v += (p + 2 < G) ? t : 0.0; }
  if (G >= 8) { double t = dpp<DPP_ROW_SHL4>(v); v += (p + 4 < G) ? t : 0.0; }
  return v;
}
// sum over lanes p' > p
template <int G> __device__ __forceinline__ double group_suffix_excl(double v, int p) {
  if (G == 1) return 0.0;
  double t = dpp<DPP_ROW_SHL1>(v);
  return group_suffix_incl<G>((p + 1 < G) ? t : 0.0, p);
}

// ---------------------------------------------------------------------------
// Stumpff functions by truncated series (Sec. 3.2): K terms of
//   c2(z) = sum_k (-z)^k / (2k+2)!,   c3(z) = sum_k (-z)^k / (2k+3)!
// evaluated by Horner's rule with exact inverse factorials.
__host__ __device__ constexpr double inv_factorial(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;   // exact up to 18!
  return 1.0 / f;
}
template <int K, int N0> __device__ __forceinline__ double stumpff_series(double z) {
  double s = inv_factorial(N0 + 2 * (K - 1));
#pragma unroll
  for (int k = K - 2; k >= 0; --k) s = fma(-z, s, inv_factorial(N0 + 2 * k));
  return s;
}

// Per-lane running diagnostics of the Kepler solves.
struct KepDiag {
  double zmax;   // largest Stumpff argument of a final evaluation
  double bmin;   // smallest beta = 2 mu / r0 - v^2 (<= 0: unbound)
};

// Lagrange coefficients of a Kepler drift: the drift maps (Q, V) to
// (f Q + g V, f' Q + g' V); kept as f - 1, g, f', g' - 1 so increments are
// formed without cancellation.
struct KepCoef {
  double fm1, g, fd, gdm1;
};

// Iteration counts of the fixed Kepler solve: NH Halley steps with KH series
// terms, then NN Newton steps with KN terms.  KepCountsFixed bakes them in at
// compile time (the integrator); KepCountsRun takes them at run time, uniform
// over a launch (the envelope explorer of App. A).
template <int NH, int NN, int KH, int KN> struct KepCountsFixed {
  __device__ static constexpr int nh() { return NH; }
  __device__ static constexpr int nn() { return NN; }
  template <int N0> __device__ static double series_h(double z) { return stumpff_series<KH, N0>(z); }
  template <int N0> __device__ static double series_n(double z) { return stumpff_series<KN, N0>(z); }
};

// 1/n! for n = 0..31 (exact to n = 18, correctly rounded products beyond).
struct InvFactTable {
  double v[32];
  __host__ __device__ constexpr InvFactTable() : v() {
    for (int n = 0; n < 32; ++n) v[n] = inv_factorial(n);
  }
};
__constant__ constexpr InvFactTable kInvFact{};

template <int N0> __device__ __forceinline__ double stumpff_series_rt(double z, int K) {
  double s = kInvFact.v[N0 + 2 * (K - 1)];
  for (int k = K - 2; k >= 0; --k) s = fma(-z, s, kInvFact.v[N0 + 2 * k]);
  return s;
}

// Run-time counts; limits keep every table index in range.
constexpr int KEP_RT_MAX_NH = 8, KEP_RT_MAX_NN = 8, KEP_RT_MAX_TERMS = 14;
struct KepCountsRun {
  int h, n, kh, kn;
  __device__ int nh() const { return h; }
  __device__ int nn() const { return n; }
  template <int N0> __device__ double series_h(double z) const { return stumpff_series_rt<N0>(z, kh); }
  template <int N0> __device__ double series_n(double z) const { return stumpff_series_rt<N0>(z, kn); }
};

// Kepler drift of one planet over tau about a star with mu = G m0 (Sec. 3.2),
// in universal variables: with r0 = |Q|, eta = Q.V, beta = 2mu/r0 - V^2,
// zeta = mu - beta r0, solve
//   F(X) = r0 X + eta G2(X) + zeta G3(X) - tau = 0,  G_n = X^n c_n(beta X^2),
// with a fixed number of Halley steps then Newton steps (counts and series
// lengths from P), no convergence test and no branch on the data, then form
// the Lagrange coefficients.  Initial guess: X = tau/r0 - eta tau^2 / (2 r0^3).
// g' - 1 is taken from the Wronskian identity f g' - f' g = 1, which keeps
// the discrete map area-preserving to rounding.  Returns the anomaly X.
template <class P>
__device__ __forceinline__ double kepler_coeffs_p(const P& p, double qx, double qy, double qz, double vx, double vy,
                                                  double vz, double mu, double tau, KepDiag& dg, KepCoef& k) {
  double r2 = fma(qx, qx, fma(qy, qy, qz * qz));
  double v2 = fma(vx, vx, fma(vy, vy, vz * vz));
  double eta = fma(qx, vx, fma(qy, vy, qz * vz));
  double ir0 = rsqrt_full(r2);
  double r0 = r2 * ir0;
  double beta = fma(2.0 * mu, ir0, -v2);
  double zeta = fma(-beta, r0, mu);
  dg.bmin = fmin(dg.bmin, beta);
  double a = tau * ir0;
  double X = a * fma(-0.5 * eta * ir0, a, 1.0);
#pragma unroll
  for (int it = 0; it < p.nh(); ++it) {
    double X2 = X * X;
    double z = beta * X2;
    double c2 = p.template series_h<2>(z);
    double c3 = p.template series_h<3>(z);
    double c0 = fma(-z, c2, 1.0);
    double c1 = fma(-z, c3, 1.0);
    double G1 = X * c1, G2 = X2 * c2, G3 = X2 * X * c3;
    double F = fma(r0, X, fma(eta, G2, fma(zeta, G3, -tau)));
    double Fp = fma(eta, G1, fma(zeta, G2, r0));
    double Fpp = fma(eta, c0, zeta * G1);
    // Halley: X -= 2 F F' / (2 F'^2 - F F'')
    double den = fma(-0.5 * F, Fpp, Fp * Fp);
    X = fma(-F * Fp, rcp_seed(den), X);
  }
  // Newton steps.  The G functions of the final anomaly come from those of
  // the last iterate: G_n(X + d) = G_n(X) + d G_{n-1}(X) + O(d^2), and d is at
  // rounding level once the iteration has converged.
  double G1 = 0.0, G2 = 0.0, G3 = 0.0;
#pragma unroll
  for (int it = 0; it < p.nn(); ++it) {
    double X2 = X * X;
    double z = beta * X2;
    if (it == p.nn() - 1) dg.zmax = fmax(dg.zmax, z);
    double c2 = p.template series_n<2>(z);
    double c3 = p.template series_n<3>(z);
    double c1 = fma(-z, c3, 1.0);
    G1 = X * c1; G2 = X2 * c2; G3 = X2 * X * c3;
    double F = fma(r0, X, fma(eta, G2, fma(zeta, G3, -tau)));
    double Fp = fma(eta, G1, fma(zeta, G2, r0));
    double d = -F * rcp_seed(Fp);
    X += d;
    if (it == p.nn() - 1) {
      double G0 = fma(-z, c2, 1.0);
      G3 = fma(d, G2, G3);
      G2 = fma(d, G1, G2);
      G1 = fma(d, G0, G1);
    }
  }
  if (p.nn() == 0) {
    // no Newton step: the G functions are evaluated afresh at the last
    // Halley iterate with the final series length
    double X2 = X * X;
    double z = beta * X2;
    dg.zmax = fmax(dg.zmax, z);
    double c2 = p.template series_n<2>(z);
    double c3 = p.template series_n<3>(z);
    G1 = X * fma(-z, c3, 1.0); G2 = X2 * c2; G3 = X2 * X * c3;
  }
  double r = fma(eta, G1, fma(zeta, G2, r0));
  double ir = rcp_full(r);
  k.fm1 = -mu * G2 * ir0;
  k.g = fma(-mu, G3, tau);
  k.fd = -mu * G1 * ir0 * ir;
  k.gdm1 = fma(k.fd, k.g, -k.fm1) * rcp_full(1.0 + k.fm1);
  return X;
}

template <int NH, int NN, int KH, int KN>
__device__ __forceinline__ double kepler_coeffs(double qx, double qy, double qz, double vx, double vy, double vz,
                                                double mu, double tau, KepDiag& dg, KepCoef& k) {
  return kepler_coeffs_p(KepCountsFixed<NH, NN, KH, KN>{}, qx, qy, qz, vx, vy, vz, mu, tau, dg, k);
}

// Increment a x + b y of one coordinate as an unevaluated sum hi + lo, with
// the rounding errors of the product b y and of the sum kept in lo (b y is
// the larger term: g V for positions, f' Q for velocities).  Contraction is
// off: fusing b*y into p - t would count the product error twice.
__device__ __forceinline__ void lin2_dd(double a, double x, double b, double y, double& hi, double& lo) {
#pragma clang fp contract(off)
  double p = b * y;
  double pe = fma(b, y, -p);
  double t = fma(a, x, p);
  double te = fma(a, x, p - t);
  hi = t;
  lo = pe + te;
}

// Double-double accumulation (s, c) += (d, e), where s + c is the state with
// |c| <= ulp(s)/2: an exact two-sum of s and d, the low parts added, then
// renormalized.
__device__ __forceinline__ void dd_add(double& s, double& c, double d, double e) {
#pragma clang fp contract(off)
  double t = s + d;
  double bp = t - s;
  double err = (s - (t - bp)) + (d - bp);
  double lo = (c + e) + err;
  s = t + lo;
  c = lo - (s - t);
}

// The paper's solver: 2 Halley steps with 4 series terms, 2 Newton steps
// with 8 terms (Sec. 3.2).
constexpr int KEP_NH = 2, KEP_NN = 2, KEP_KH = 4, KEP_KN = 8;

// Count sets of the integrator's solve (wh_config.kepler_counts): 0 the
// paper's; 1 one Halley step with 3 series terms then the paper's two Newton
// steps with 8, the cheapest combination the envelope explorer finds within
// App. A's bound (relative a-error < 1e-13 over 10 years of 5-day steps for
// a test particle at a = 0.387) for every eccentricity up to 0.6.
template <int KC> struct KepSet {
  static constexpr int NH = KEP_NH, NN = KEP_NN, KH = KEP_KH, KN = KEP_KN;
};
template <> struct KepSet<1> {
  static constexpr int NH = 1, NN = 2, KH = 3, KN = 8;
};

// ---------------------------------------------------------------------------
// Interaction kick (Sec. 3.3, acceleration equation) inside a G-lane group,
// using Newton's third law: round k = 1..G/2 pairs lane p with lane
// (p + k) mod G.  For k < G/2 the G pairs of the round are distinct, so the
// lane also computes its partner's reaction and returns it (the partner
// reads it back from lane (p - k) mod G); the round k = G/2 pairs lanes
// symmetrically and each side computes its own half.  Every unordered pair
// is evaluated exactly once per side that needs it, with one reciprocal
// square root per lane per round (G/2 per lane in all, 28 per 8-planet
// system for the two-sided rounds and 4 for the symmetric one).
template <int G> struct GroupTopo {
  int fetch[G / 2 > 0 ? G / 2 : 1];   // byte address of the round-k partner
  int back[G / 2 > 0 ? G / 2 : 1];    // byte address of the lane whose partner I am
  double mp[G / 2 > 0 ? G / 2 : 1];   // partner masses (constant, Sec. 3.5)
};

template <int G> __device__ __forceinline__ void make_topo(GroupTopo<G>& t, int lane, double m) {
#pragma unroll
  for (int k = 1; k <= G / 2; ++k) {
    int base = lane & ~(G - 1);
    int p = lane & (G - 1);
    t.fetch[k - 1] = (base | ((p + k) & (G - 1))) << 2;
    t.back[k - 1] = (base | ((p - k) & (G - 1))) << 2;
    t.mp[k - 1] = bperm(t.fetch[k - 1], m);
  }
}

// Acceleration a_i of the lane's planet from the other planets of its group.
template <int G> __device__ __forceinline__ void interaction_accel(const GroupTopo<G>& t, double qx, double qy,
                                                                   double qz, double m, double& ax, double& ay,
                                                                   double& az) {
  ax = 0.0; ay = 0.0; az = 0.0;
#pragma unroll
  for (int k = 1; k <= G / 2; ++k) {
    double px = bperm(t.fetch[k - 1], qx);
    double py = bperm(t.fetch[k - 1], qy);
    double pz = bperm(t.fetch[k - 1], qz);
    double dx = qx - px, dy = qy - py, dz = qz - pz;
    double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    double ir3 = rsqrt3_full(r2);
    double wj = t.mp[k - 1] * ir3;
    ax = fma(-wj, dx, ax);
    ay = fma(-wj, dy, ay);
    az = fma(-wj, dz, az);
    if (2 * k < G) {
      double wi = m * ir3;   // partner's acceleration is +wi * d
      double rx = bperm(t.back[k - 1], wi * dx);
      double ry = bperm(t.back[k - 1], wi * dy);
      double rz = bperm(t.back[k - 1], wi * dz);
      ax += rx;
      ay += ry;
      az += rz;
    }
  }
}

// ---------------------------------------------------------------------------
// The same kick with every exchange done by DPP row moves (VALU, no LDS
// latency), for groups of 2, 4 or 8 lanes.  Lane p = 4 q + r (quad q,
// position r).  Rounds:
//   R1  partner (r+1) mod 4 in the quad, reaction returned (4 distinct pairs
//       per quad);
//   R2  partner r xor 2 in the quad, each side its own half (2 pairs/quad);
//   R3  partner (r+1) mod 4 of the other quad, reaction returned: quad 0 lane
//       r pairs with quad 1 lane r+1, quad 1 lane r with quad 0 lane r+1, so
//       the 8 pairs are distinct;
//   R4  partner r of the other quad (one-sided), R5 partner r xor 2 of the
//       other quad (one-sided).
// G = 8 uses R1-R5 (12 intra-quad + 16 cross-quad pairs = 28, five reciprocal
// square roots per lane), G = 4 uses R1-R2, G = 2 pairs lanes r xor 1.
// Cross-quad reads are a row_half_mirror (lane p reads 7 - p) followed by a
// quad_perm.
constexpr int QP_NEXT = 0x39;     // quad_perm [1,2,3,0]: r reads (r+1)&3
constexpr int QP_PREV = 0x93;     // quad_perm [3,0,1,2]: r reads (r-1)&3
constexpr int QP_R3 = 0xC6;       // after mirror: other quad's (r+1)&3
constexpr int QP_R3_BACK = 0x6C;  // after mirror: other quad's (r-1)&3
constexpr int QP_R4 = 0x1B;       // after mirror: other quad's r
constexpr int QP_R5 = 0xB1;       // after mirror: other quad's r^2

struct DppMass {
  double m[5];   // partner mass of each round
};

template <int G> __device__ __forceinline__ void make_dpp_mass(DppMass& t, double m) {
  if (G == 2) t.m[0] = dpp<DPP_XOR1>(m);
  if (G >= 4) {
    t.m[0] = dpp<QP_NEXT>(m);
    t.m[1] = dpp<DPP_XOR2>(m);
  }
  if (G == 8) {
    double mm = dpp<DPP_HALF_MIRROR>(m);
    t.m[2] = dpp<QP_R3>(mm);
    t.m[3] = dpp<QP_R4>(mm);
    t.m[4] = dpp<QP_R5>(mm);
  }
}

// One pair: a -= m_j ir^3 d with d = q - p; returns ir^3 (for the reaction).
__device__ __forceinline__ double pair_accel(double qx, double qy, double qz, double px, double py, double pz,
                                             double mj, double& ax, double& ay, double& az, double& dx, double& dy,
                                             double& dz) {
  dx = qx - px; dy = qy - py; dz = qz - pz;
  double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  double ir3 = rsqrt3_full(r2);
  double w = mj * ir3;
  ax = fma(-w, dx, ax);
  ay = fma(-w, dy, ay);
  az = fma(-w, dz, az);
  return ir3;
}

template <int G> __device__ __forceinline__ void interaction_accel_dpp(const DppMass& t, double qx, double qy,
                                                                       double qz, double m, double& ax, double& ay,
                                                                       double& az) {
  ax = 0.0; ay = 0.0; az = 0.0;
  double dx, dy, dz;
  if (G == 2) {
    pair_accel(qx, qy, qz, dpp<DPP_XOR1>(qx), dpp<DPP_XOR1>(qy), dpp<DPP_XOR1>(qz), t.m[0], ax, ay, az, dx, dy, dz);
  }
  if (G >= 4) {
    double ir3 = pair_accel(qx, qy, qz, dpp<QP_NEXT>(qx), dpp<QP_NEXT>(qy), dpp<QP_NEXT>(qz), t.m[0], ax, ay, az,
                            dx, dy, dz);
    double wi = m * ir3;
    ax += dpp<QP_PREV>(wi * dx);
    ay += dpp<QP_PREV>(wi * dy);
    az += dpp<QP_PREV>(wi * dz);
    pair_accel(qx, qy, qz, dpp<DPP_XOR2>(qx), dpp<DPP_XOR2>(qy), dpp<DPP_XOR2>(qz), t.m[1], ax, ay, az, dx, dy, dz);
  }
  if (G == 8) {
    double mx = dpp<DPP_HALF_MIRROR>(qx), my = dpp<DPP_HALF_MIRROR>(qy), mz = dpp<DPP_HALF_MIRROR>(qz);
    double ir3 = pair_accel(qx, qy, qz, dpp<QP_R3>(mx), dpp<QP_R3>(my), dpp<QP_R3>(mz), t.m[2], ax, ay, az, dx,
                            dy, dz);
    double wi = m * ir3;
    ax += dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(wi * dx));
    ay += dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(wi * dy));
    az += dpp<QP_R3_BACK>(dpp<DPP_HALF_MIRROR>(wi * dz));
    pair_accel(qx, qy, qz, dpp<QP_R4>(mx), dpp<QP_R4>(my), dpp<QP_R4>(mz), t.m[3], ax, ay, az, dx, dy, dz);
    pair_accel(qx, qy, qz, dpp<QP_R5>(mx), dpp<QP_R5>(my), dpp<QP_R5>(mz), t.m[4], ax, ay, az, dx, dy, dz);
  }
}

// Jump (Sec. 3.4): every planet of the group moves by (tau/m0) sum_j m_j V_j;
// velocities are unchanged.  Returns the group's total planetary momentum.
template <int G> __device__ __forceinline__ void group_momentum(double m, double vx, double vy, double vz,
                                                                double& sx, double& sy, double& sz) {
  sx = group_sum<G>(m * vx);
  sy = group_sum<G>(m * vy);
  sz = group_sum<G>(m * vz);
}

// GR acceleration -6 mu^2/c^2 * Q/|Q|^4, from the potential -3 mu^2 m/(c^2 |Q|^2)
// centred on the star.  kg = 6 mu^2 / c^2.
__device__ __forceinline__ void gr_accel(double qx, double qy, double qz, double kg, double& ax, double& ay,
                                         double& az) {
  double r2 = fma(qx, qx, fma(qy, qy, qz * qz));
  double ir2 = rcp_full(r2);
  double w = -kg * ir2 * ir2;
  ax = w * qx;
  ay = w * qy;
  az = w * qz;
}

}  // namespace wh
