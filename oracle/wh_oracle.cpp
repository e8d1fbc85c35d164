// ORACLE -- test infrastructure, not part of the product.
//
// A plain, slow CPU reference of the Wisdom-Holman map in democratic
// heliocentric coordinates (WHFast512 paper, Sec. 3).  Only the test suite,
// the smoke check and the CPU-baseline leg of the benchmark load this library.
// It shares no code, header, table or helper with the GPU path.
//
// What it computes (each function cites the passage it follows):
//   * the exact Kepler flow of H_K,i (Sec. 3.2, the per-planet Hamiltonian
//     P^2/2m - G m0 m / Q), solved to convergence in universal variables;
//   * the jump flow of H_J (Sec. 3.4, the jump equation);
//   * the interaction kick of H_I (Sec. 3.3, the acceleration equation);
//   * the 1/r^2 GR kick (Sec. 3.3, last paragraphs; the potential constant is
//     a reading, see gr_kick);
//   * the plain operator composition of Sec. 3.1 (drift-kick-drift, every
//     half step applied separately, nothing merged), and a kick-drift-kick
//     variant;
//   * the energy H = H_K + H_I + H_J (+ H_GR) of Sec. 3.1 and the angular
//     momentum;
//   * the tangent (variational) map, by running the same code on dual numbers;
//   * a fixed-iteration Kepler solver (Sec. 3.2 and App. A) kept apart from
//     the exact one, used only for the App. A experiment and the operation
//     count (with either the direct or the Wronskian form of g');
//   * the SABA_n splittings (Laskar & Robutel 2001; Sec. 3.1 mentions
//     higher-order generalizations of the step) with Gauss-Legendre
//     coefficients;
//   * the Wisdom-Holman map in Jacobi coordinates (Wisdom & Holman 1991; the
//     Sec. 3.5 footnote and Sec. 6 name it for two or four planets), its
//     kick taken as the dual-number gradient of H_I, plus the closed-form
//     Jacobi acceleration for the operation count.
//
// Scalar types: long double (parity reference), double (CPU timing baseline),
// Dual<long double> (tangent map), Counted (operation count).
//
// G = 1 throughout (Sec. 3.5 assumptions).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <omp.h>

namespace {

typedef long double ld;

// ---------------------------------------------------------------------------
// Dual numbers: value + one tangent direction.
template <class R> struct Dual {
  R v, d;
  Dual() : v(0), d(0) {}
  Dual(R x) : v(x), d(0) {}   // NOLINT: implicit on purpose (constants)
  Dual(R x, R dx) : v(x), d(dx) {}
};
template <class R> Dual<R> operator+(Dual<R> a, Dual<R> b) { return {a.v + b.v, a.d + b.d}; }
template <class R> Dual<R> operator-(Dual<R> a, Dual<R> b) { return {a.v - b.v, a.d - b.d}; }
template <class R> Dual<R> operator-(Dual<R> a) { return {-a.v, -a.d}; }
template <class R> Dual<R> operator*(Dual<R> a, Dual<R> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class R> Dual<R> operator/(Dual<R> a, Dual<R> b) {
  R q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class R> Dual<R>& operator+=(Dual<R>& a, Dual<R> b) { a = a + b; return a; }
template <class R> Dual<R>& operator-=(Dual<R>& a, Dual<R> b) { a = a - b; return a; }
template <class R> Dual<R>& operator*=(Dual<R>& a, Dual<R> b) { a = a * b; return a; }
template <class R> Dual<R> sqrt(Dual<R> a) { R s = std::sqrt(a.v); return {s, a.d / (2 * s)}; }
template <class R> Dual<R> cos(Dual<R> a) { return {std::cos(a.v), -std::sin(a.v) * a.d}; }
template <class R> Dual<R> sin(Dual<R> a) { return {std::sin(a.v), std::cos(a.v) * a.d}; }
template <class R> Dual<R> cosh(Dual<R> a) { return {std::cosh(a.v), std::sinh(a.v) * a.d}; }
template <class R> Dual<R> sinh(Dual<R> a) { return {std::sinh(a.v), std::cosh(a.v) * a.d}; }

// ---------------------------------------------------------------------------
// Counted: a double that counts the floating-point operations applied to it.
// add/sub/mul count one flop each, div and sqrt one each (kept apart).
struct OpCount { long add, mul, div, sqrt; };
thread_local OpCount g_ops;
struct Counted {
  double v;
  Counted() : v(0) {}
  Counted(double x) : v(x) {}   // NOLINT
};
inline Counted operator+(Counted a, Counted b) { ++g_ops.add; return a.v + b.v; }
inline Counted operator-(Counted a, Counted b) { ++g_ops.add; return a.v - b.v; }
inline Counted operator-(Counted a) { return -a.v; }
inline Counted operator*(Counted a, Counted b) { ++g_ops.mul; return a.v * b.v; }
inline Counted operator/(Counted a, Counted b) { ++g_ops.div; return a.v / b.v; }
inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
inline Counted& operator*=(Counted& a, Counted b) { a = a * b; return a; }
inline Counted sqrt(Counted a) { ++g_ops.sqrt; return std::sqrt(a.v); }

// real part, for control flow only
inline double val(double x) { return x; }
inline ld val(ld x) { return x; }
template <class R> R val(const Dual<R>& x) { return x.v; }
inline double val(const Counted& x) { return x.v; }

template <class T> struct Real { typedef T type; };
template <class R> struct Real<Dual<R> > { typedef R type; };
template <> struct Real<Counted> { typedef double type; };

template <class R> R eps_of();
template <> double eps_of<double>() { return 2.220446049250313e-16; }
template <> ld eps_of<ld>() { return 1.0842021724855044e-19L; }

// ---------------------------------------------------------------------------
// Stumpff functions c0..c3 of z, evaluated to full precision of T
// (Sec. 3.2 uses them for the universal-variable Kepler solve).
// c_n(z) = sum_k (-z)^k / (n+2k)!; for |z| >= 1 the closed forms in cos/sin
// (z > 0) or cosh/sinh (z < 0) of sqrt(|z|) are used instead.
template <class T> void stumpff_exact(const T& z, T c[4]) {
  typedef typename Real<T>::type R;
  using std::sqrt; using std::cos; using std::sin; using std::cosh; using std::sinh;
  R az = val(z) < 0 ? -val(z) : val(z);
  if (az < 1) {
    // c2 = 1/2! - z/4! + z^2/6! ...   c3 = 1/3! - z/5! + ...
    T t2 = T(R(0.5)), t3 = T(R(1) / R(6));
    T s2 = t2, s3 = t3;
    for (int k = 0; k < 40; ++k) {
      R a2 = R(2 * k + 3) * R(2 * k + 4);
      R a3 = R(2 * k + 4) * R(2 * k + 5);
      t2 = t2 * (-z) / T(a2);
      t3 = t3 * (-z) / T(a3);
      s2 += t2;
      s3 += t3;
      R mag = val(t2) < 0 ? -val(t2) : val(t2);
      if (mag < eps_of<R>() * R(1e-3) * val(s2) && k > 2) break;
    }
    c[2] = s2;
    c[3] = s3;
    c[0] = T(R(1)) - z * s2;
    c[1] = T(R(1)) - z * s3;
  } else if (val(z) > 0) {
    T s = sqrt(z);
    c[0] = cos(s);
    c[1] = sin(s) / s;
    c[2] = (T(R(1)) - c[0]) / z;
    c[3] = (T(R(1)) - c[1]) / z;
  } else {
    T s = sqrt(-z);
    c[0] = cosh(s);
    c[1] = sinh(s) / s;
    c[2] = (T(R(1)) - c[0]) / z;
    c[3] = (T(R(1)) - c[1]) / z;
  }
}

// Kepler's equation in the universal anomaly X (Sec. 3.2):
//   F(X) = r0 X + eta0 G2(X) + zeta0 G3(X) - tau,  G_n = X^n c_n(beta X^2),
//   F'(X) = r(X) = r0 + eta0 G1 + zeta0 G2  (> 0 for every orbit type).
template <class T> struct KepEq {
  T r0, eta0, zeta0, beta, tau;
  void eval(const T& X, T& F, T& dF, T G[4]) const {
    T c[4];
    T X2 = X * X;
    stumpff_exact(beta * X2, c);
    G[0] = c[0];
    G[1] = X * c[1];
    G[2] = X2 * c[2];
    G[3] = X2 * X * c[3];
    F = r0 * X + eta0 * G[2] + zeta0 * G[3] - tau;
    dF = r0 + eta0 * G[1] + zeta0 * G[2];
  }
};

// Converged root of Kepler's equation in the real type: safeguarded Newton
// (bisection whenever a Newton step leaves the bracket [lo, hi]).  F rises
// with X (F' = r > 0) and F(0) = -tau, so the root lies on the side of 0 that
// tau's sign gives; the bracket grows from 0 towards it (tau < 0: a backward
// drift, the exact flow run backwards).
template <class R> R solve_universal(const KepEq<R>& e) {
  R F, dF, G[4];
  R lo = 0, hi = 0;
  if (e.tau >= 0) {
    hi = e.tau / e.r0;
    for (int k = 0; k < 400; ++k) {   // grow the bracket until F(hi) > 0
      e.eval(hi, F, dF, G);
      if (F > 0) break;
      lo = hi;
      hi *= 2;
    }
  } else {
    lo = e.tau / e.r0;
    for (int k = 0; k < 400; ++k) {   // grow it downwards until F(lo) < 0
      e.eval(lo, F, dF, G);
      if (F < 0) break;
      hi = lo;
      lo *= 2;
    }
  }
  R X = e.tau / e.r0;
  if (!(X > lo && X < hi)) X = (lo + hi) / 2;
  for (int it = 0; it < 500; ++it) {
    e.eval(X, F, dF, G);
    if (F < 0) lo = X; else hi = X;
    R Xn = X - F / dF;
    if (!(Xn > lo && Xn < hi)) Xn = (lo + hi) / 2;
    R dx = Xn - X;
    if (dx < 0) dx = -dx;
    R ax = Xn < 0 ? -Xn : Xn;
    X = Xn;
    if (dx <= 4 * eps_of<R>() * ax || hi - lo <= 4 * eps_of<R>() * ax) break;
  }
  return X;
}

// Exact Kepler drift of one particle over tau with mu = G m0 (Sec. 3.2).
// Solves Kepler's equation to convergence, then applies the Lagrange f and g
// functions.  For dual numbers the root is found on the real part and two
// further Newton steps carry the derivative (implicit function theorem).
template <class T> void kepler_exact(T Q[3], T V[3], const T& mu, const T& tau, typename Real<T>::type* Xout) {
  typedef typename Real<T>::type R;
  using std::sqrt;
  T r0 = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
  T v2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
  T eta0 = Q[0] * V[0] + Q[1] * V[1] + Q[2] * V[2];
  T beta = T(R(2)) * mu / r0 - v2;
  T zeta0 = mu - beta * r0;
  KepEq<T> e = {r0, eta0, zeta0, beta, tau};
  KepEq<R> er = {val(r0), val(eta0), val(zeta0), val(beta), val(tau)};
  T X = T(solve_universal(er));
  T F, dF, G[4];
  for (int k = 0; k < 2; ++k) {
    e.eval(X, F, dF, G);
    X = X - F / dF;
  }
  e.eval(X, F, dF, G);
  T r = dF;
  T f = T(R(1)) - mu * G[2] / r0;
  T g = tau - mu * G[3];
  T fd = -mu * G[1] / (r0 * r);
  T gd = T(R(1)) - mu * G[2] / r;
  T Qn[3], Vn[3];
  for (int a = 0; a < 3; ++a) {
    Qn[a] = f * Q[a] + g * V[a];
    Vn[a] = fd * Q[a] + gd * V[a];
  }
  for (int a = 0; a < 3; ++a) { Q[a] = Qn[a]; V[a] = Vn[a]; }
  if (Xout) *Xout = val(X);
}

// ---------------------------------------------------------------------------
// Fixed-iteration Kepler solver of Sec. 3.2 / App. A (sweep and count mode).
// Not used by the exact map above.  The paper counts "terms" of the Stumpff
// series without saying which series; here `terms` terms are summed for
// c_{2+2r} and c_{3+2r} and the rest follows from r downward recurrences
// c_n = 1/n! - z c_{n+2} (r = 0: the plain series of c2 and c3), then
// c0 = 1 - z c2 and c1 = 1 - z c3.
template <class R> R inv_fact(int n) {
  R f = 1;
  for (int k = 2; k <= n; ++k) f /= R(k);
  return f;
}
template <class T> void stumpff_trunc(const T& z, int terms, int recur, T c[4]) {
  typedef typename Real<T>::type R;
  int n2 = 2 + 2 * recur, n3 = 3 + 2 * recur;
  // Horner from the highest retained term down.
  T s2 = T(inv_fact<R>(n2 + 2 * (terms - 1))), s3 = T(inv_fact<R>(n3 + 2 * (terms - 1)));
  for (int k = terms - 2; k >= 0; --k) {
    s2 = T(inv_fact<R>(n2 + 2 * k)) - z * s2;
    s3 = T(inv_fact<R>(n3 + 2 * k)) - z * s3;
  }
  for (int r = recur - 1; r >= 0; --r) {
    s2 = T(inv_fact<R>(2 + 2 * r)) - z * s2;
    s3 = T(inv_fact<R>(3 + 2 * r)) - z * s3;
  }
  c[2] = s2;
  c[3] = s3;
  c[0] = T(R(1)) - z * s2;
  c[1] = T(R(1)) - z * s3;
}

int g_recur = 0;   // series arrangement of the fixed-iteration solver
int g_guess = 0;   // initial guess of the fixed-iteration solver
// Form of g' in the fixed-iteration solver: 0 = its definition 1 - mu G2 / r;
// 1 = from the Wronskian identity f g' - f' g = 1 of the Lagrange
// coefficients, g' = (1 + f' g) / f.  Both equal the exact g' once the solve
// has converged; they differ where it has not (the envelope of Fig. 1).
int g_gd_form = 0;

template <class T> void kep_trunc_eval(const KepEq<T>& e, const T& X, int terms, T& F, T& dF, T& ddF, T G[4],
                                       bool need_dd) {
  T c[4];
  T X2 = X * X;
  stumpff_trunc(e.beta * X2, terms, g_recur, c);
  G[0] = c[0];
  G[1] = X * c[1];
  G[2] = X2 * c[2];
  G[3] = X2 * X * c[3];
  F = e.r0 * X + e.eta0 * G[2] + e.zeta0 * G[3] - e.tau;
  dF = e.r0 + e.eta0 * G[1] + e.zeta0 * G[2];
  if (need_dd) ddF = e.eta0 * G[0] + e.zeta0 * G[1];
}

// Initial guess (the paper does not print one): second-order Taylor expansion
// of X(t), using dX/dt = 1/r and d2X/dt2 = -eta/r^3 (g_guess = 0), or the
// first-order term tau/r0 alone (g_guess = 1, App. A sweep only).
template <class T> void kepler_fixed(T Q[3], T V[3], const T& mu, const T& tau,
                                     int n_halley, int n_newton, int terms_halley, int terms_newton) {
  typedef typename Real<T>::type R;
  using std::sqrt;
  T r0 = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
  T v2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
  T eta0 = Q[0] * V[0] + Q[1] * V[1] + Q[2] * V[2];
  T ir0 = T(R(1)) / r0;
  T beta = T(R(2)) * mu * ir0 - v2;
  T zeta0 = mu - beta * r0;
  KepEq<T> e = {r0, eta0, zeta0, beta, tau};
  T X = tau * ir0;
  if (g_guess == 0) X = X - eta0 * tau * tau * ir0 * ir0 * ir0 * T(R(0.5));
  T F, dF, ddF, G[4];
  for (int k = 0; k < n_halley; ++k) {
    kep_trunc_eval(e, X, terms_halley, F, dF, ddF, G, true);
    X = X - T(R(2)) * F * dF / (T(R(2)) * dF * dF - F * ddF);
  }
  // Newton steps; the G functions at the final anomaly follow from those of
  // the last iterate by G_n(X + d) = G_n(X) + d G_{n-1}(X) (d is at rounding
  // level once converged; with no Newton step they are evaluated afresh).
  for (int k = 0; k < n_newton; ++k) {
    kep_trunc_eval(e, X, terms_newton, F, dF, ddF, G, false);
    T d = -(F / dF);
    X = X + d;
    if (k == n_newton - 1) {
      G[3] = G[3] + d * G[2];
      G[2] = G[2] + d * G[1];
      G[1] = G[1] + d * G[0];
    }
  }
  if (n_newton == 0) kep_trunc_eval(e, X, terms_newton, F, dF, ddF, G, false);
  T r = e.r0 + e.eta0 * G[1] + e.zeta0 * G[2];
  T f = T(R(1)) - mu * G[2] * ir0;
  T g = tau - mu * G[3];
  T ir = T(R(1)) / r;
  T fd = -mu * G[1] * ir0 * ir;
  T gd = g_gd_form == 0 ? T(R(1)) - mu * G[2] * ir : T(R(1)) + (fd * g - (f - T(R(1)))) / f;
  T Qn[3], Vn[3];
  for (int a = 0; a < 3; ++a) {
    Qn[a] = f * Q[a] + g * V[a];
    Vn[a] = fd * Q[a] + gd * V[a];
  }
  for (int a = 0; a < 3; ++a) { Q[a] = Qn[a]; V[a] = Vn[a]; }
}

// ---------------------------------------------------------------------------
// One planetary system: star mass m0 and n <= 8 planets with heliocentric
// positions Q and barycentric velocities V = P/m (Sec. 3.1).
template <class T> struct Sys {
  int n;
  T m0;
  T m[8];
  T Q[8][3];
  T V[8][3];
};

// Jump flow of H_J over tau (Sec. 3.4): every planet moves by
// (tau/m0) * sum_j P_j; momenta are unchanged; the star does not move.
template <class T> void jump(Sys<T>& s, const T& tau) {
  T P[3] = {T(0), T(0), T(0)};
  for (int j = 0; j < s.n; ++j)
    for (int a = 0; a < 3; ++a) P[a] += s.m[j] * s.V[j][a];
  T k = tau / s.m0;
  for (int i = 0; i < s.n; ++i)
    for (int a = 0; a < 3; ++a) s.Q[i][a] += k * P[a];
}

// Interaction kick of H_I over tau (Sec. 3.3, acceleration equation):
//   a_i = - sum_{j != i} G m_j Q_ij / |Q_ij|^3,  V_i += tau a_i.
// Every ordered pair is evaluated on its own (no third-law reuse), j ascending.
template <class T> void interaction(Sys<T>& s, const T& tau) {
  using std::sqrt;
  T acc[8][3];
  for (int i = 0; i < s.n; ++i) {
    T a[3] = {T(0), T(0), T(0)};
    for (int j = 0; j < s.n; ++j) {
      if (j == i) continue;
      T d[3] = {s.Q[i][0] - s.Q[j][0], s.Q[i][1] - s.Q[j][1], s.Q[i][2] - s.Q[j][2]};
      T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      T r = sqrt(r2);
      T w = s.m[j] / (r2 * r);
      for (int c = 0; c < 3; ++c) a[c] -= w * d[c];
    }
    for (int c = 0; c < 3; ++c) acc[i][c] = a[c];
  }
  for (int i = 0; i < s.n; ++i)
    for (int c = 0; c < 3; ++c) s.V[i][c] += tau * acc[i][c];
}

// GR kick over tau (Sec. 3.3, 1/r^2 potential centred on the star).  The
// paper gives no formula; reading: H_GR = - sum_i 3 mu^2 m_i / (c^2 |Q_i|^2)
// with mu = G m0, the potential that reproduces the relativistic perihelion
// precession 6 pi mu / (c^2 a (1-e^2)).  dV_i/dt = -6 mu^2 Q_i / (c^2 |Q_i|^4).
// In these canonical coordinates the star's back reaction is carried by the
// barycentric momenta and needs no separate term.
template <class T> void gr_kick(Sys<T>& s, const T& tau, const T& c) {
  typedef typename Real<T>::type R;
  T mu = s.m0;
  T k = T(R(6)) * mu * mu / (c * c);
  for (int i = 0; i < s.n; ++i) {
    T r2 = s.Q[i][0] * s.Q[i][0] + s.Q[i][1] * s.Q[i][1] + s.Q[i][2] * s.Q[i][2];
    T w = k / (r2 * r2);
    for (int a = 0; a < 3; ++a) s.V[i][a] -= tau * w * s.Q[i][a];
  }
}

template <class T> void kepler_all(Sys<T>& s, const T& tau) {
  for (int i = 0; i < s.n; ++i) kepler_exact(s.Q[i], s.V[i], s.m0, tau, (typename Real<T>::type*)0);
}

// interaction step = H_I kick plus the optional GR kick (both change V only
// and depend on Q only, so they commute).
template <class T> void kick(Sys<T>& s, const T& tau, const T& gr_c, bool gr) {
  interaction(s, tau);
  if (gr) gr_kick(s, tau, gr_c);
}

// One full step (Sec. 3.1 operator composition), every piece applied on its
// own:
//   scheme 0 (drift-kick-drift): K(dt/2) J(dt/2) I(dt) J(dt/2) K(dt/2)
//   scheme 1 (kick-drift-kick):  I(dt/2) J(dt/2) K(dt) J(dt/2) I(dt/2)
// (operators listed in the order they act; both are symmetric.)
template <class T> void step(Sys<T>& s, const T& dt, int scheme, const T& gr_c, bool gr) {
  typedef typename Real<T>::type R;
  T h = dt * T(R(0.5));
  if (scheme == 0) {
    kepler_all(s, h);
    jump(s, h);
    kick(s, dt, gr_c, gr);
    jump(s, h);
    kepler_all(s, h);
  } else {
    kick(s, h, gr_c, gr);
    jump(s, h);
    kepler_all(s, dt);
    jump(s, h);
    kick(s, h, gr_c, gr);
  }
}

// ---------------------------------------------------------------------------
// SABA_n splittings (Laskar & Robutel 2001) for H = A + B with A = the Kepler
// part and B the perturbation:
//   exp(c_1 dt A) exp(d_1 dt B) exp(c_2 dt A) ... exp(d_n dt B) exp(c_{n+1} dt A),
// with d_k the weights of n-point Gauss-Legendre quadrature on [0, 1], c_1
// its first node, c_k the gaps between consecutive nodes and c_{n+1} = 1 -
// the last node.  n = 1 is the drift-kick-drift step.  The error is
// O(eps dt^(2n) + eps^2 dt^2) for a perturbation of relative size eps.
// Schemes 2, 3, 4 of the step functions below are SABA_2, SABA_3, SABA_4.
struct Saba {
  int n;
  ld c[6], d[5];
};

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on the
// Legendre polynomial P_n (three-term recurrence), mapped to [0, 1].
Saba saba_coeffs(int n) {
  Saba q;
  q.n = n;
  ld x[5] = {0, 0, 0, 0, 0}, w[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    ld z = std::cos(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      ld pn = n == 1 ? z : p1, pm = n == 1 ? 1 : p0;    // P_n(z), P_{n-1}(z)
      ld dp = n * (z * pn - pm) / (z * z - 1);
      ld dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) {
        x[i] = z;
        w[i] = 2 / ((1 - z * z) * dp * dp);
        break;
      }
      x[i] = z;
      w[i] = 2 / ((1 - z * z) * dp * dp);
    }
  }
  // ascending nodes on [0, 1]
  ld t[5] = {0, 0, 0, 0, 0}, u[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    t[i] = (1 - x[i]) / 2;   // x descending -> t ascending
    u[i] = w[i] / 2;
  }
  q.c[0] = t[0];
  for (int k = 1; k < n; ++k) q.c[k] = t[k] - t[k - 1];
  q.c[n] = 1 - t[n - 1];
  for (int k = 0; k < n; ++k) q.d[k] = u[k];
  return q;
}

// DHC, no GR: B = H_I + H_J, whose flows commute (the interaction is
// translation invariant), so exp(d dt B) = I(d dt) J(d dt) exactly.
template <class T> void saba_step(Sys<T>& s, const T& dt, const Saba& q) {
  typedef typename Real<T>::type R;
  for (int k = 0; k < q.n; ++k) {
    kepler_all(s, dt * T(R(q.c[k])));
    interaction(s, dt * T(R(q.d[k])));
    jump(s, dt * T(R(q.d[k])));
  }
  kepler_all(s, dt * T(R(q.c[q.n])));
}

// Energy (Sec. 3.1 Hamiltonian, H_0 = 0 in the barycentric frame):
//   sum_i [m_i V_i^2/2 - m0 m_i/|Q_i|] - sum_{i<j} m_i m_j/|Q_ij|
//   + |sum_i m_i V_i|^2 / (2 m0)  [ - sum_i 3 m0^2 m_i / (c^2 |Q_i|^2) ].
template <class T> T energy(const Sys<T>& s, const T& gr_c, bool gr) {
  typedef typename Real<T>::type R;
  using std::sqrt;
  T E = T(0);
  T P[3] = {T(0), T(0), T(0)};
  for (int i = 0; i < s.n; ++i) {
    T v2 = s.V[i][0] * s.V[i][0] + s.V[i][1] * s.V[i][1] + s.V[i][2] * s.V[i][2];
    T r2 = s.Q[i][0] * s.Q[i][0] + s.Q[i][1] * s.Q[i][1] + s.Q[i][2] * s.Q[i][2];
    E += T(R(0.5)) * s.m[i] * v2 - s.m0 * s.m[i] / sqrt(r2);
    if (gr) E -= T(R(3)) * s.m0 * s.m0 * s.m[i] / (gr_c * gr_c * r2);
    for (int a = 0; a < 3; ++a) P[a] += s.m[i] * s.V[i][a];
  }
  for (int i = 0; i < s.n; ++i)
    for (int j = i + 1; j < s.n; ++j) {
      T d[3] = {s.Q[i][0] - s.Q[j][0], s.Q[i][1] - s.Q[j][1], s.Q[i][2] - s.Q[j][2]};
      E -= s.m[i] * s.m[j] / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
  E += (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) / (T(R(2)) * s.m0);
  return E;
}

// --------------------------------------------------------------------------
// array <-> system marshalling. Arrays: Q,V [S][nmax][3], m [S][nmax].
template <class T, class A> void load(Sys<T>& s, int idx, int nmax, const int* np, const A* m0,
                                      const A* m, const A* Q, const A* V) {
  s.n = np[idx];
  s.m0 = T(m0[idx]);
  for (int i = 0; i < s.n; ++i) {
    s.m[i] = T(m[idx * nmax + i]);
    for (int a = 0; a < 3; ++a) {
      s.Q[i][a] = T(Q[(idx * nmax + i) * 3 + a]);
      s.V[i][a] = T(V[(idx * nmax + i) * 3 + a]);
    }
  }
}
template <class T, class A> void store(const Sys<T>& s, int idx, int nmax, A* Q, A* V) {
  for (int i = 0; i < s.n; ++i)
    for (int a = 0; a < 3; ++a) {
      Q[(idx * nmax + i) * 3 + a] = val(s.Q[i][a]);
      V[(idx * nmax + i) * 3 + a] = val(s.V[i][a]);
    }
}

template <class T> void integrate_arrays(int S, int nmax, const int* np, const T* m0, const T* m, T* Q, T* V,
                                         const T* dt, long n_steps, int scheme, T gr_c, int nthreads) {
  bool gr = gr_c > 0;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int k = 0; k < S; ++k) {
    Sys<T> s;
    load(s, k, nmax, np, m0, m, Q, V);
    if (scheme >= 2) {
      Saba q = saba_coeffs(scheme);
      for (long t = 0; t < n_steps; ++t) saba_step(s, dt[k], q);
    } else {
      for (long t = 0; t < n_steps; ++t) step(s, dt[k], scheme, gr_c, gr);
    }
    store(s, k, nmax, Q, V);
  }
}

// ---------------------------------------------------------------------------
// Wisdom-Holman map in Jacobi coordinates (Wisdom & Holman 1991), the
// alternative the paper names for systems of two or four planets (Sec. 3.5,
// footnote on Jacobi coordinates; Sec. 6 outlook).  Bodies 0 (the star) .. n,
// interior masses M_i = m_0 + m_1 + ... + m_i.  Jacobi coordinates of body
// i >= 1 are measured from the centre of mass of the bodies inside it:
//   x'_i = x_i - (m_0 x_0 + ... + m_{i-1} x_{i-1}) / M_{i-1}   (same for v),
// translation invariant, so computable from heliocentric positions Q_j =
// x_j - x_0 (Q_0 = 0) and heliocentric velocities u_j.  With reduced masses
// m'_i = m_i M_{i-1} / M_i the barycentric kinetic energy is
// sum_i m'_i |v'_i|^2 / 2, and the Hamiltonian splits as
//   H_K = sum_i [ m'_i |v'_i|^2 / 2 - G M_i m'_i / |x'_i| ]  (Kepler, mu_i = G M_i)
//   H_I = U + sum_i G M_i m'_i / |x'_i|,
//   U   = - sum_{i>=1} G m_0 m_i / |Q_i| - sum_{1<=i<j} G m_i m_j / |Q_i - Q_j|.
// The kick is v'_i -= tau (1/m'_i) dH_I/dx'_i with the gradient taken by
// dual numbers through this definition of H_I (no hand-derived force).
template <class T> struct JSys {
  int n;
  T m0;
  T m[8];
  T M[9];        // M[i] = m_0 + ... + m_i over bodies 0..n (M[0] = m0)
  T x[8][3];     // Jacobi position of planet k (body k + 1)
  T v[8][3];     // Jacobi velocity
  T gr_c;        // speed of light of the GR term, <= 0: no GR
};

template <class T> void jac_masses(JSys<T>& s) {
  s.M[0] = s.m0;
  for (int k = 0; k < s.n; ++k) s.M[k + 1] = s.M[k] + s.m[k];
}

// Heliocentric -> Jacobi for one vector field (positions or heliocentric
// velocities): x'_k = h_k - (sum_{j<k} m_j h_j) / M_k  (star at h = 0).
template <class T, class A> void helio_to_jacobi(const JSys<T>& s, const A h[8][3], T out[8][3]) {
  T acc[3] = {T(0), T(0), T(0)};
  for (int k = 0; k < s.n; ++k) {
    for (int a = 0; a < 3; ++a) out[k][a] = T(h[k][a]) - acc[a] / s.M[k];
    for (int a = 0; a < 3; ++a) acc[a] += s.m[k] * T(h[k][a]);
  }
}
// Jacobi -> heliocentric: h_k = x'_k + (sum_{j<k} m_j h_j) / M_k.
template <class T, class U> void jacobi_to_helio(const JSys<T>& s, const U xp[8][3], U h[8][3]) {
  U acc[3] = {U(0), U(0), U(0)};
  for (int k = 0; k < s.n; ++k) {
    for (int a = 0; a < 3; ++a) h[k][a] = xp[k][a] + acc[a] / U(s.M[k]);
    for (int a = 0; a < 3; ++a) acc[a] += U(s.m[k]) * h[k][a];
  }
}

// From democratic heliocentric Q (heliocentric) and V (barycentric): the
// star's barycentric velocity is -sum_j m_j V_j / m0, so u_j = V_j + sum m V / m0.
template <class T> void jac_from_dhc(JSys<T>& s, const T Q[8][3], const T V[8][3]) {
  jac_masses(s);
  T P[3] = {T(0), T(0), T(0)};
  for (int k = 0; k < s.n; ++k)
    for (int a = 0; a < 3; ++a) P[a] += s.m[k] * V[k][a];
  T u[8][3];
  for (int k = 0; k < s.n; ++k)
    for (int a = 0; a < 3; ++a) u[k][a] = V[k][a] + P[a] / s.m0;
  helio_to_jacobi(s, Q, s.x);
  helio_to_jacobi(s, u, s.v);
}
// Back: heliocentric Q from x', heliocentric u from v', and V = u + v_0 with
// the star's barycentric velocity v_0 = -sum_j m_j u_j / M_n.
template <class T> void jac_to_dhc(const JSys<T>& s, T Q[8][3], T V[8][3]) {
  jacobi_to_helio(s, s.x, Q);
  T u[8][3];
  jacobi_to_helio(s, s.v, u);
  T P[3] = {T(0), T(0), T(0)};
  for (int k = 0; k < s.n; ++k)
    for (int a = 0; a < 3; ++a) P[a] += s.m[k] * u[k][a];
  for (int k = 0; k < s.n; ++k)
    for (int a = 0; a < 3; ++a) V[k][a] = u[k][a] - P[a] / s.M[s.n];
}

template <class T> T jac_reduced_mass(const JSys<T>& s, int k) { return s.m[k] * s.M[k] / s.M[k + 1]; }

// H_I at Jacobi positions xp (scalar type U: long double, or dual numbers
// for the gradient).
template <class T, class U> U jac_hint(const JSys<T>& s, const U xp[8][3]) {
  using std::sqrt;
  U Q[8][3];
  jacobi_to_helio(s, xp, Q);
  U H = U(0);
  for (int i = 0; i < s.n; ++i) {
    U r = sqrt(Q[i][0] * Q[i][0] + Q[i][1] * Q[i][1] + Q[i][2] * Q[i][2]);
    H -= U(s.m0 * s.m[i]) / r;
    for (int j = i + 1; j < s.n; ++j) {
      U d[3] = {Q[i][0] - Q[j][0], Q[i][1] - Q[j][1], Q[i][2] - Q[j][2]};
      H -= U(s.m[i] * s.m[j]) / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
    U rp = sqrt(xp[i][0] * xp[i][0] + xp[i][1] * xp[i][1] + xp[i][2] * xp[i][2]);
    H += U(s.M[i + 1] * jac_reduced_mass(s, i)) / rp;
    // the GR potential of Sec. 3.3 (reading of gr_kick), a function of the
    // heliocentric positions and so part of the perturbation
    if (val(s.gr_c) > 0) H -= U(T(3.0L) * s.m0 * s.m0 * s.m[i] / (s.gr_c * s.gr_c)) / (r * r);
  }
  return H;
}

template <class T> T jac_hk(const JSys<T>& s) {
  using std::sqrt;
  T H = T(0);
  for (int i = 0; i < s.n; ++i) {
    T mp = jac_reduced_mass(s, i);
    T v2 = s.v[i][0] * s.v[i][0] + s.v[i][1] * s.v[i][1] + s.v[i][2] * s.v[i][2];
    T r = sqrt(s.x[i][0] * s.x[i][0] + s.x[i][1] * s.x[i][1] + s.x[i][2] * s.x[i][2]);
    H += T(0.5L) * mp * v2 - s.M[i + 1] * mp / r;
  }
  return H;
}

// Kick of H_I over tau: one dual-number evaluation of H_I per coordinate.
void jac_kick(JSys<ld>& s, ld tau) {
  typedef Dual<ld> D;
  ld g[8][3];
  for (int i = 0; i < s.n; ++i)
    for (int a = 0; a < 3; ++a) {
      D xp[8][3];
      for (int k = 0; k < s.n; ++k)
        for (int b = 0; b < 3; ++b) xp[k][b] = D(s.x[k][b], (k == i && b == a) ? 1.0L : 0.0L);
      g[i][a] = jac_hint(s, xp).d;
    }
  for (int i = 0; i < s.n; ++i) {
    ld mp = jac_reduced_mass(s, i);
    for (int a = 0; a < 3; ++a) s.v[i][a] -= tau * g[i][a] / mp;
  }
}

// The same kick from the closed form of the gradient (for the operation
// count; a test checks it against the dual-number gradient above):
//   a'_i = a_i - A_{i-1} + G M_i x'_i / |x'_i|^3,
// with a_i the Newtonian acceleration of planet i and A_{i-1} that of the
// centre of mass of the bodies inside it; the mutual forces of those bodies
// cancel, leaving  M_{i-1} A_{i-1} = G m_0 sum_{k>=i} m_k Q_k/|Q_k|^3 +
// sum_{j<i} m_j a^pl_j  (a^pl: the planet-planet part, each pair once).
template <class T> void jac_kick_direct(JSys<T>& s, const T& tau) {
  typedef typename Real<T>::type R;
  using std::sqrt;
  T Q[8][3], apl[8][3], g[8][3];
  jacobi_to_helio(s, s.x, Q);
  for (int i = 0; i < s.n; ++i)
    for (int a = 0; a < 3; ++a) apl[i][a] = T(R(0));
  for (int i = 0; i < s.n; ++i)
    for (int j = i + 1; j < s.n; ++j) {
      T d[3] = {Q[i][0] - Q[j][0], Q[i][1] - Q[j][1], Q[i][2] - Q[j][2]};
      T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      T ir3 = T(R(1)) / (r2 * sqrt(r2));
      T wi = s.m[j] * ir3, wj = s.m[i] * ir3;
      for (int a = 0; a < 3; ++a) { apl[i][a] -= wi * d[a]; apl[j][a] += wj * d[a]; }
    }
  for (int i = 0; i < s.n; ++i) {
    T r2 = Q[i][0] * Q[i][0] + Q[i][1] * Q[i][1] + Q[i][2] * Q[i][2];
    T ir3 = T(R(1)) / (r2 * sqrt(r2));
    for (int a = 0; a < 3; ++a) g[i][a] = Q[i][a] * ir3;
  }
  // running sums: suf[i] = sum_{k>=i} m_k g_k, pre[i] = sum_{j<i} m_j a^pl_j
  T suf[9][3], pre[9][3];
  for (int a = 0; a < 3; ++a) { suf[s.n][a] = T(R(0)); pre[0][a] = T(R(0)); }
  for (int k = s.n - 1; k >= 0; --k)
    for (int a = 0; a < 3; ++a) suf[k][a] = suf[k + 1][a] + s.m[k] * g[k][a];
  for (int j = 0; j < s.n; ++j)
    for (int a = 0; a < 3; ++a) pre[j + 1][a] = pre[j][a] + s.m[j] * apl[j][a];
  for (int i = 0; i < s.n; ++i) {
    T rp2 = s.x[i][0] * s.x[i][0] + s.x[i][1] * s.x[i][1] + s.x[i][2] * s.x[i][2];
    T kp = s.M[i + 1] / (rp2 * sqrt(rp2));
    for (int a = 0; a < 3; ++a) {
      T A = (s.m0 * suf[i][a] + pre[i][a]) / s.M[i];
      s.v[i][a] += tau * (apl[i][a] - s.m0 * g[i][a] - A + kp * s.x[i][a]);
    }
  }
  // GR: the force m_k gr_k on every planet and its reaction on the star give
  // a'_i += gr_i + (sum_{k>=i} m_k gr_k) / M_{i-1}, gr_k = -6 m0^2 Q_k / (c^2 |Q_k|^4)
  if (val(s.gr_c) > 0) {
    T gr[8][3], gsuf[9][3];
    for (int k = 0; k < s.n; ++k) {
      T r2 = Q[k][0] * Q[k][0] + Q[k][1] * Q[k][1] + Q[k][2] * Q[k][2];
      T w = T(R(6)) * s.m0 * s.m0 / (s.gr_c * s.gr_c * r2 * r2);
      for (int a = 0; a < 3; ++a) gr[k][a] = -w * Q[k][a];
    }
    for (int a = 0; a < 3; ++a) gsuf[s.n][a] = T(R(0));
    for (int k = s.n - 1; k >= 0; --k)
      for (int a = 0; a < 3; ++a) gsuf[k][a] = gsuf[k + 1][a] + s.m[k] * gr[k][a];
    for (int i = 0; i < s.n; ++i)
      for (int a = 0; a < 3; ++a) s.v[i][a] += tau * (gr[i][a] + gsuf[i][a] / s.M[i]);
  }
}

void jac_drift(JSys<ld>& s, ld tau) {
  for (int i = 0; i < s.n; ++i) kepler_exact(s.x[i], s.v[i], s.M[i + 1], tau, (ld*)0);
}

// scheme 0: K(dt/2) I(dt) K(dt/2); scheme 1: I(dt/2) K(dt) I(dt/2).
void jac_step(JSys<ld>& s, ld dt, int scheme) {
  if (scheme >= 2) {     // SABA_n with B = H_I
    Saba q = saba_coeffs(scheme);
    for (int k = 0; k < q.n; ++k) {
      jac_drift(s, dt * q.c[k]);
      jac_kick(s, dt * q.d[k]);
    }
    jac_drift(s, dt * q.c[q.n]);
    return;
  }
  ld h = dt * 0.5L;
  if (scheme == 0) {
    jac_drift(s, h);
    jac_kick(s, dt);
    jac_drift(s, h);
  } else {
    jac_kick(s, h);
    jac_drift(s, dt);
    jac_kick(s, h);
  }
}

// The same map on any scalar type (dual numbers for the tangent map), with
// the kick from its closed form (a test pins it to the gradient of H_I).
template <class T> void jac_drift_t(JSys<T>& s, const T& tau) {
  for (int i = 0; i < s.n; ++i) kepler_exact(s.x[i], s.v[i], s.M[i + 1], tau, (typename Real<T>::type*)0);
}
template <class T> void jac_step_t(JSys<T>& s, const T& dt, int scheme) {
  typedef typename Real<T>::type R;
  if (scheme >= 2) {
    Saba q = saba_coeffs(scheme);
    for (int k = 0; k < q.n; ++k) {
      jac_drift_t(s, dt * T(R(q.c[k])));
      jac_kick_direct(s, dt * T(R(q.d[k])));
    }
    jac_drift_t(s, dt * T(R(q.c[q.n])));
    return;
  }
  T h = dt * T(R(0.5));
  if (scheme == 0) {
    jac_drift_t(s, h);
    jac_kick_direct(s, dt);
    jac_drift_t(s, h);
  } else {
    jac_kick_direct(s, h);
    jac_drift_t(s, dt);
    jac_kick_direct(s, h);
  }
}

template <class A> void jac_load(JSys<ld>& s, int idx, int nmax, const int* np, const A* m0, const A* m, const A* Q,
                                 const A* V) {
  s.n = np[idx];
  s.m0 = m0[idx];
  s.gr_c = 0;
  ld q[8][3], vv[8][3];
  for (int i = 0; i < s.n; ++i) {
    s.m[i] = m[idx * nmax + i];
    for (int a = 0; a < 3; ++a) {
      q[i][a] = Q[(idx * nmax + i) * 3 + a];
      vv[i][a] = V[(idx * nmax + i) * 3 + a];
    }
  }
  jac_from_dhc(s, q, vv);
}
template <class A> void jac_store(const JSys<ld>& s, int idx, int nmax, A* Q, A* V) {
  ld q[8][3], vv[8][3];
  jac_to_dhc(s, q, vv);
  for (int i = 0; i < s.n; ++i)
    for (int a = 0; a < 3; ++a) {
      Q[(idx * nmax + i) * 3 + a] = (A)q[i][a];
      V[(idx * nmax + i) * 3 + a] = (A)vv[i][a];
    }
}

// ---- Symplectic correctors for the Jacobi map --------------------------
// (Wisdom, Holman & Touma 1996; derived here, coefficients computed.)
// To first order in the perturbation B = H_I, the drift-kick-drift map of
// step h is the time-h flow of A + F(x) B with A the Kepler part and
// x = h ad_A (the first-order-in-B part of the symmetric BCH formula):
//   drift-kick-drift  F(x) = (x/2) / sinh(x/2),
//   kick-drift-kick   F(x) = (x/2) cosh(x/2) / sinh(x/2).
// A near-identity canonical change of variables generated by h Psi(x) B with
// Psi(x) = (1 - F(x)) / x (odd in x) turns that flow into the flow of A + B,
// up to O(B^2).  The kernel X(a, b): drift a h, kick b h, drift -a h (a kick
// carried by the Kepler flow) and Z(a, b) = X(a, b) then X(-a, -b) generate
// 2 b h sinh(a x) B, so n stages Z(a_i, b_i) with
//   sum_i 2 b_i a_i^(2k-1) / (2k-1)! = sigma [x^(2k-1)] Psi(x),   k = 1..n
// remove the first-order error terms through h^(2n) (a corrector of order
// 2n + 1).  sigma = +1 or -1 fixes which way the change is applied (the
// pins choose it: the corrected energy error must fall).  The a_i are
// i / (2n) (no drift of a stage longer than one step) and the b_i solve the
// n x n system.  Z(a, b)^-1 = Z(-a, b) exactly.
struct Corr {
  int n;
  ld a[8], b[8];
};

// Taylor coefficients f_k of F (F = sum_k f_k x^(2k)), k = 0..kmax, by power
// series division of  y cosh y  (kick-drift-kick) or y  (drift-kick-drift)
// by  sinh y = sum_k y^(2k+1) / (2k+1)!,  then y = x / 2.
void corrector_F_series(int scheme, int kmax, ld* f) {
  ld num[16], den[16], q[16];
  for (int k = 0; k <= kmax; ++k) {
    ld fac2k = 1, fac2k1 = 1;
    for (int j = 2; j <= 2 * k; ++j) fac2k *= j;
    fac2k1 = fac2k * (2 * k + 1);
    den[k] = 1 / fac2k1;                        // sinh(y) / y
    num[k] = scheme == 1 ? 1 / fac2k : (k == 0 ? 1 : 0);   // cosh(y) or 1
  }
  for (int k = 0; k <= kmax; ++k) {             // q = num / den
    ld s = num[k];
    for (int j = 1; j <= k; ++j) s -= den[j] * q[k - j];
    q[k] = s / den[0];
  }
  for (int k = 0; k <= kmax; ++k) f[k] = q[k] / std::pow(2.0L, 2 * k);   // y^(2k) = x^(2k) / 4^k
}

Corr corrector_coeffs(int stages, int scheme, int sigma) {
  Corr c;
  c.n = stages;
  ld f[16];
  corrector_F_series(scheme, stages, f);
  ld M[8][9];
  for (int i = 0; i < stages; ++i) c.a[i] = (ld)(i + 1) / (2 * stages);
  for (int k = 1; k <= stages; ++k) {
    ld fac = 1;
    for (int j = 2; j <= 2 * k - 1; ++j) fac *= j;
    for (int i = 0; i < stages; ++i) M[k - 1][i] = 2 * std::pow(c.a[i], (ld)(2 * k - 1)) / fac;
    M[k - 1][stages] = sigma * (-f[k]);         // [x^(2k-1)] Psi = -f_k
  }
  for (int col = 0; col < stages; ++col) {      // Gauss-Jordan with partial pivoting
    int piv = col;
    for (int r = col + 1; r < stages; ++r)
      if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
    for (int j = 0; j <= stages; ++j) std::swap(M[col][j], M[piv][j]);
    for (int r = 0; r < stages; ++r) {
      if (r == col) continue;
      ld g = M[r][col] / M[col][col];
      for (int j = col; j <= stages; ++j) M[r][j] -= g * M[col][j];
    }
  }
  for (int i = 0; i < stages; ++i) c.b[i] = M[i][stages] / M[i][i];
  return c;
}

void jac_corr_stage(JSys<ld>& s, ld h, ld a, ld b) {     // Z(a, b)
  jac_drift(s, a * h);
  jac_kick(s, b * h);
  jac_drift(s, -2 * a * h);
  jac_kick(s, -b * h);
  jac_drift(s, a * h);
}

// The change of variables C (inverse: C^-1): mapping coordinates -> real
// coordinates.  C applies Z(a_n, b_n) first and Z(a_1, b_1) last.
void jac_corrector(JSys<ld>& s, ld h, const Corr& c, bool inverse) {
  if (!inverse)
    for (int i = c.n - 1; i >= 0; --i) jac_corr_stage(s, h, c.a[i], c.b[i]);
  else
    for (int i = 0; i < c.n; ++i) jac_corr_stage(s, h, -c.a[i], c.b[i]);
}

template <class A> void jac_integrate_arrays(int S, int nmax, const int* np, const A* m0, const A* m, A* Q, A* V,
                                             const A* dt, long n_steps, int scheme, ld gr_c, int nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int k = 0; k < S; ++k) {
    JSys<ld> s;
    jac_load(s, k, nmax, np, m0, m, Q, V);
    s.gr_c = gr_c;
    for (long t = 0; t < n_steps; ++t) jac_step(s, (ld)dt[k], scheme);
    jac_store(s, k, nmax, Q, V);
  }
}

}  // namespace

// ===========================================================================
// C interface (ctypes).  "_ld" = long double arrays, "_d" = double arrays.
extern "C" {

int or_max_threads() { return omp_get_max_threads(); }

// Series arrangement of the fixed-iteration solver (see stumpff_trunc).
void or_set_series_recur(int r) { g_recur = r; }
// Initial guess of the fixed-iteration solver: 0 second order, 1 first order.
void or_set_guess(int g) { g_guess = g; }

void or_set_gd_form(int g) { g_gd_form = g; }

// Exact Kepler drift of n independent particles, in place.
void or_kepler_ld(int n, ld* Q, ld* V, const ld* mu, const ld* tau, ld* X) {
  for (int i = 0; i < n; ++i) kepler_exact<ld>(Q + 3 * i, V + 3 * i, mu[i], tau[i], X ? X + i : 0);
}

// Fixed-iteration Kepler drift (App. A sweep mode), in place, long double.
void or_kepler_fixed_ld(int n, ld* Q, ld* V, const ld* mu, const ld* tau, int nh, int nn, int th, int tn) {
  for (int i = 0; i < n; ++i) kepler_fixed<ld>(Q + 3 * i, V + 3 * i, mu[i], tau[i], nh, nn, th, tn);
}
// Same solver in double arithmetic.
void or_kepler_fixed_d(int n, double* Q, double* V, const double* mu, const double* tau, int nh, int nn, int th,
                       int tn) {
  for (int i = 0; i < n; ++i) kepler_fixed<double>(Q + 3 * i, V + 3 * i, mu[i], tau[i], nh, nn, th, tn);
}

// Single sub-flows on S systems (tau per system), in place.
// which: 0 = Kepler, 1 = jump, 2 = interaction, 3 = GR kick.
void or_substep_ld(int which, int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V,
                   const ld* tau, ld gr_c) {
  for (int k = 0; k < S; ++k) {
    Sys<ld> s;
    load(s, k, nmax, np, m0, m, Q, V);
    if (which == 0) kepler_all(s, tau[k]);
    else if (which == 1) jump(s, tau[k]);
    else if (which == 2) interaction(s, tau[k]);
    else gr_kick(s, tau[k], gr_c);
    store(s, k, nmax, Q, V);
  }
}

// n_steps full steps of the plain composition on S systems, in place.
// scheme 0 = drift-kick-drift, 1 = kick-drift-kick; gr_c <= 0 turns GR off.
void or_integrate_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V, const ld* dt,
                     long n_steps, int scheme, ld gr_c, int nthreads) {
  integrate_arrays<ld>(S, nmax, np, m0, m, Q, V, dt, n_steps, scheme, gr_c, nthreads);
}
void or_integrate_d(int S, int nmax, const int* np, const double* m0, const double* m, double* Q, double* V,
                    const double* dt, long n_steps, int scheme, double gr_c, int nthreads) {
  integrate_arrays<double>(S, nmax, np, m0, m, Q, V, dt, n_steps, scheme, gr_c, nthreads);
}

// SABA_n coefficients: c[0..n], d[0..n-1].
void or_saba_coeffs(int n, ld* c, ld* d) {
  Saba q = saba_coeffs(n);
  for (int k = 0; k <= n; ++k) c[k] = q.c[k];
  for (int k = 0; k < n; ++k) d[k] = q.d[k];
}

// ---- Jacobi-coordinate map (Wisdom & Holman 1991) ----------------------
// DHC in, DHC out; the state is carried in Jacobi coordinates in between.
void or_jacobi_integrate_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V, const ld* dt,
                            long n_steps, int scheme, ld gr_c, int nthreads) {
  jac_integrate_arrays(S, nmax, np, m0, m, Q, V, dt, n_steps, scheme, gr_c, nthreads);
}
void or_jacobi_integrate_d(int S, int nmax, const int* np, const double* m0, const double* m, double* Q, double* V,
                           const double* dt, long n_steps, int scheme, double gr_c, int nthreads) {
  jac_integrate_arrays(S, nmax, np, m0, m, Q, V, dt, n_steps, scheme, (ld)gr_c, nthreads);
}
// Symplectic corrector coefficients (a_i, b_i) of an n-stage corrector
// (order 2n + 1) of scheme 0 (drift-kick-drift) or 1 (kick-drift-kick).
void or_corrector_coeffs(int stages, int scheme, int sigma, ld* a, ld* b) {
  Corr c = corrector_coeffs(stages, scheme, sigma);
  for (int i = 0; i < stages; ++i) { a[i] = c.a[i]; b[i] = c.b[i]; }
}
// Taylor coefficients of F (for the pins).
void or_corrector_F_series(int scheme, int kmax, ld* f) { corrector_F_series(scheme, kmax, f); }
// Apply the corrector C (inverse != 0: C^-1) with step dt[k] to DHC states.
void or_jacobi_corrector_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V, const ld* dt,
                            int stages, int scheme, int sigma, int inverse, ld gr_c, int nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  const Corr c = corrector_coeffs(stages, scheme, sigma);
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int k = 0; k < S; ++k) {
    JSys<ld> s;
    jac_load(s, k, nmax, np, m0, m, Q, V);
    s.gr_c = gr_c;
    jac_corrector(s, dt[k], c, inverse != 0);
    jac_store(s, k, nmax, Q, V);
  }
}

// Jacobi coordinates of DHC states (xp, vp: [S][nmax][3]).
void or_jacobi_from_dhc_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, const ld* Q, const ld* V,
                           ld* xp, ld* vp) {
  for (int k = 0; k < S; ++k) {
    JSys<ld> s;
    jac_load(s, k, nmax, np, m0, m, Q, V);
    for (int i = 0; i < s.n; ++i)
      for (int a = 0; a < 3; ++a) {
        xp[(k * nmax + i) * 3 + a] = s.x[i][a];
        vp[(k * nmax + i) * 3 + a] = s.v[i][a];
      }
  }
}
// DHC states of Jacobi coordinates.
void or_jacobi_to_dhc_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, const ld* xp, const ld* vp,
                         ld* Q, ld* V) {
  for (int k = 0; k < S; ++k) {
    JSys<ld> s;
    s.n = np[k];
    s.m0 = m0[k];
    s.gr_c = 0;
    for (int i = 0; i < s.n; ++i) s.m[i] = m[k * nmax + i];
    jac_masses(s);
    for (int i = 0; i < s.n; ++i)
      for (int a = 0; a < 3; ++a) {
        s.x[i][a] = xp[(k * nmax + i) * 3 + a];
        s.v[i][a] = vp[(k * nmax + i) * 3 + a];
      }
    jac_store(s, k, nmax, Q, V);
  }
}
// The closed-form kick (jac_kick_direct) on DHC states.
void or_jacobi_kick_direct_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V, ld tau,
                              ld gr_c) {
  for (int k = 0; k < S; ++k) {
    JSys<ld> s;
    jac_load(s, k, nmax, np, m0, m, Q, V);
    s.gr_c = gr_c;
    jac_kick_direct(s, tau);
    jac_store(s, k, nmax, Q, V);
  }
}
// Per system: [kinetic energy sum m'|v'|^2/2, H_K, H_I] of DHC states.
void or_jacobi_parts_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, const ld* Q, const ld* V,
                        ld gr_c, ld* out) {
  for (int k = 0; k < S; ++k) {
    JSys<ld> s;
    jac_load(s, k, nmax, np, m0, m, Q, V);
    s.gr_c = gr_c;
    ld T = 0;
    for (int i = 0; i < s.n; ++i)
      T += 0.5L * jac_reduced_mass(s, i) * (s.v[i][0] * s.v[i][0] + s.v[i][1] * s.v[i][1] + s.v[i][2] * s.v[i][2]);
    out[3 * k] = T;
    out[3 * k + 1] = jac_hk(s);
    out[3 * k + 2] = jac_hint(s, s.x);
  }
}
// One kick of H_I over tau applied to DHC states (converted to Jacobi and back).
void or_jacobi_kick_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V, ld tau, ld gr_c) {
  for (int k = 0; k < S; ++k) {
    JSys<ld> s;
    jac_load(s, k, nmax, np, m0, m, Q, V);
    s.gr_c = gr_c;
    jac_kick(s, tau);
    jac_store(s, k, nmax, Q, V);
  }
}

void or_energy_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, const ld* Q, const ld* V, ld gr_c,
                  ld* E) {
  for (int k = 0; k < S; ++k) {
    Sys<ld> s;
    load(s, k, nmax, np, m0, m, Q, V);
    E[k] = energy(s, gr_c, gr_c > 0);
  }
}

// Total angular momentum sum_i m_i Q_i x V_i (barycentric frame).
void or_angmom_ld(int S, int nmax, const int* np, const ld* m, const ld* Q, const ld* V, ld* L) {
  for (int k = 0; k < S; ++k) {
    ld l[3] = {0, 0, 0};
    for (int i = 0; i < np[k]; ++i) {
      const ld* q = Q + (k * nmax + i) * 3;
      const ld* v = V + (k * nmax + i) * 3;
      ld mi = m[k * nmax + i];
      l[0] += mi * (q[1] * v[2] - q[2] * v[1]);
      l[1] += mi * (q[2] * v[0] - q[0] * v[2]);
      l[2] += mi * (q[0] * v[1] - q[1] * v[0]);
    }
    for (int a = 0; a < 3; ++a) L[3 * k + a] = l[a];
  }
}

// Tangent map: integrate the plain composition on dual numbers.  Inputs
// (Q, V, m, m0) carry the direction (dQ, dV, dm, dm0); on return Q, V hold
// the final state and dQ, dV its directional derivative.
void or_tangent_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V, const ld* dt,
                   long n_steps, int scheme, ld gr_c, const ld* dm0, const ld* dm, ld* dQ, ld* dV,
                   int nthreads) {
  typedef Dual<ld> D;
  bool gr = gr_c > 0;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int k = 0; k < S; ++k) {
    Sys<D> s;
    s.n = np[k];
    s.m0 = D(m0[k], dm0[k]);
    for (int i = 0; i < s.n; ++i) {
      int p = k * nmax + i;
      s.m[i] = D(m[p], dm[p]);
      for (int a = 0; a < 3; ++a) {
        s.Q[i][a] = D(Q[3 * p + a], dQ[3 * p + a]);
        s.V[i][a] = D(V[3 * p + a], dV[3 * p + a]);
      }
    }
    D dtk(dt[k]);
    D c(gr_c);
    if (scheme >= 2) {
      Saba q = saba_coeffs(scheme);
      for (long t = 0; t < n_steps; ++t) saba_step(s, dtk, q);
    } else {
      for (long t = 0; t < n_steps; ++t) step(s, dtk, scheme, c, gr);
    }
    for (int i = 0; i < s.n; ++i) {
      int p = k * nmax + i;
      for (int a = 0; a < 3; ++a) {
        Q[3 * p + a] = s.Q[i][a].v;
        V[3 * p + a] = s.V[i][a].v;
        dQ[3 * p + a] = s.Q[i][a].d;
        dV[3 * p + a] = s.V[i][a].d;
      }
    }
  }
}

// Operation count of one step of the method as the paper states it
// (Sec. 3.1-3.4 with the fixed-iteration Kepler solve of Sec. 3.2): combined
// drift K(dt), then the jump(s) and the interaction kick, each planet pair
// evaluated once (third law, Sec. 3.3).  With GR the two half jumps stay
// separate (Sec. 3.1) and the GR kick is added.
// counts[0..3] = add/sub, mul, div, sqrt.
void or_count_ops(int n, int gr, int nh, int nn, int th, int tn, long* counts) {
  typedef Counted C;
  g_ops = OpCount{0, 0, 0, 0};
  Sys<C> s;
  s.n = n;
  s.m0 = C(1.0);
  for (int i = 0; i < n; ++i) {
    s.m[i] = C(1e-5);
    s.Q[i][0] = C(1.0 + i); s.Q[i][1] = C(0.01 * i); s.Q[i][2] = C(0.0);
    s.V[i][0] = C(0.0); s.V[i][1] = C(1.0 / std::sqrt(1.0 + i)); s.V[i][2] = C(0.001);
  }
  C dt(0.01), c(10065.0);
  g_ops = OpCount{0, 0, 0, 0};
  // Kepler drift (combined halves)
  for (int i = 0; i < n; ++i) kepler_fixed<C>(s.Q[i], s.V[i], s.m0, dt, nh, nn, th, tn);
  // jump(s)
  if (gr) jump(s, dt * C(0.5)); else jump(s, dt);
  // interaction kick with each pair once
  {
    C acc[8][3];
    for (int i = 0; i < n; ++i) for (int a = 0; a < 3; ++a) acc[i][a] = C(0.0);
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) {
        C d[3] = {s.Q[i][0] - s.Q[j][0], s.Q[i][1] - s.Q[j][1], s.Q[i][2] - s.Q[j][2]};
        C r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        C ir3 = C(1.0) / (r2 * sqrt(r2));
        C wi = s.m[j] * ir3, wj = s.m[i] * ir3;
        for (int a = 0; a < 3; ++a) { acc[i][a] -= wi * d[a]; acc[j][a] += wj * d[a]; }
      }
    for (int i = 0; i < n; ++i) for (int a = 0; a < 3; ++a) s.V[i][a] += dt * acc[i][a];
  }
  if (gr) { gr_kick(s, dt, c); jump(s, dt * C(0.5)); }
  counts[0] = g_ops.add; counts[1] = g_ops.mul; counts[2] = g_ops.div; counts[3] = g_ops.sqrt;
}


// Operation count of one step of the Jacobi map: the fixed-iteration drift of
// every planet about mu = G M_i and the closed-form kick (no jump).  The
// interior masses are per-system constants and are not counted.
void or_count_ops_jacobi(int n, int gr, int nh, int nn, int th, int tn, long* counts) {
  typedef Counted C;
  JSys<C> s;
  s.n = n;
  s.m0 = C(1.0);
  s.gr_c = C(gr ? 10065.0 : 0.0);
  for (int i = 0; i < n; ++i) {
    s.m[i] = C(1e-5);
    s.x[i][0] = C(1.0 + i); s.x[i][1] = C(0.01 * i); s.x[i][2] = C(0.0);
    s.v[i][0] = C(0.0); s.v[i][1] = C(1.0 / std::sqrt(1.0 + i)); s.v[i][2] = C(0.001);
  }
  jac_masses(s);
  C dt(0.01);
  g_ops = OpCount{0, 0, 0, 0};
  for (int i = 0; i < n; ++i) kepler_fixed<C>(s.x[i], s.v[i], s.M[i + 1], dt, nh, nn, th, tn);
  jac_kick_direct(s, dt);
  counts[0] = g_ops.add; counts[1] = g_ops.mul; counts[2] = g_ops.div; counts[3] = g_ops.sqrt;
}

// Tangent map of the Jacobi-coordinate map, with DHC inputs and outputs as
// or_jacobi_integrate_ld: the transforms, drifts (mu = G M_i) and kicks on
// dual numbers carrying the direction (dQ, dV, dm, dm0).
void or_jacobi_tangent_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V, const ld* dt,
                          long n_steps, int scheme, ld gr_c, const ld* dm0, const ld* dm, ld* dQ, ld* dV,
                          int nthreads) {
  typedef Dual<ld> D;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int k = 0; k < S; ++k) {
    JSys<D> s;
    s.n = np[k];
    s.m0 = D(m0[k], dm0[k]);
    s.gr_c = D(gr_c);
    D q[8][3], v[8][3];
    for (int i = 0; i < s.n; ++i) {
      int p = k * nmax + i;
      s.m[i] = D(m[p], dm[p]);
      for (int a = 0; a < 3; ++a) {
        q[i][a] = D(Q[3 * p + a], dQ[3 * p + a]);
        v[i][a] = D(V[3 * p + a], dV[3 * p + a]);
      }
    }
    jac_from_dhc(s, q, v);
    D dtk(dt[k]);
    for (long t = 0; t < n_steps; ++t) jac_step_t(s, dtk, scheme);
    jac_to_dhc(s, q, v);
    for (int i = 0; i < s.n; ++i) {
      int p = k * nmax + i;
      for (int a = 0; a < 3; ++a) {
        Q[3 * p + a] = q[i][a].v;
        V[3 * p + a] = v[i][a].v;
        dQ[3 * p + a] = q[i][a].d;
        dV[3 * p + a] = v[i][a].d;
      }
    }
  }
}

}  // extern "C"
