// ORACLE PIN -- test infrastructure, not part of the product.
//
// Brute-force reference for the whole Wisdom-Holman map: a Gragg-Bulirsch-
// Stoer integrator (Gragg's modified midpoint rule with polynomial Richardson
// extrapolation in h^2, Bulirsch & Stoer 1966) of the full Newtonian
// (N+1)-body problem in barycentric inertial coordinates, in long double.
// It is not symplectic and shares nothing with the splitting code in
// wh_oracle.cpp; tests use it to check that the splitting map converges to
// the true trajectory at second order as dt -> 0 (Sec. 3.1).
//
// Input and output are democratic heliocentric coordinates (Sec. 3.1):
// Q_i = x_i - x_0 (relative to the star), V_i = barycentric velocity.

#include <cmath>
#include <cstring>

namespace {
typedef long double ld;
const int MAXB = 9;          // star + up to 8 planets
const int KMAX = 14;         // extrapolation levels

struct Body { int nb; ld m[MAXB]; };

// y = [x(nb*3), v(nb*3)]
void deriv(const Body& b, const ld* y, ld* dy) {
  int nb = b.nb;
  const ld* x = y;
  const ld* v = y + 3 * nb;
  for (int i = 0; i < 3 * nb; ++i) dy[i] = v[i];
  ld* a = dy + 3 * nb;
  for (int i = 0; i < 3 * nb; ++i) a[i] = 0;
  for (int i = 0; i < nb; ++i)
    for (int j = i + 1; j < nb; ++j) {
      ld d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
      ld r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      ld ir3 = 1.0L / (r2 * sqrtl(r2));
      for (int c = 0; c < 3; ++c) {
        a[3 * i + c] -= b.m[j] * ir3 * d[c];
        a[3 * j + c] += b.m[i] * ir3 * d[c];
      }
    }
}

// Gragg's modified midpoint over H with n substeps.
void midpoint(const Body& b, const ld* y0, ld H, int n, ld* out) {
  int dim = 6 * b.nb;
  ld h = H / n;
  ld zm[6 * MAXB], z[6 * MAXB], f[6 * MAXB], tmp[6 * MAXB];
  memcpy(zm, y0, sizeof(ld) * dim);
  deriv(b, zm, f);
  for (int i = 0; i < dim; ++i) z[i] = zm[i] + h * f[i];
  for (int k = 1; k < n; ++k) {
    deriv(b, z, f);
    for (int i = 0; i < dim; ++i) {
      tmp[i] = zm[i] + 2 * h * f[i];
      zm[i] = z[i];
      z[i] = tmp[i];
    }
  }
  deriv(b, z, f);
  for (int i = 0; i < dim; ++i) out[i] = 0.5L * (z[i] + zm[i] + h * f[i]);
}

// One macro step with extrapolation; returns the final error estimate.
ld gbs_step(const Body& b, ld* y, ld H) {
  int dim = 6 * b.nb;
  static thread_local ld T[KMAX][KMAX][6 * MAXB];
  ld err = 0;
  int kfin = 0;
  for (int k = 0; k < KMAX; ++k) {
    int nk = 2 * (k + 1);
    midpoint(b, y, H, nk, T[k][0]);
    for (int j = 1; j <= k; ++j) {
      int nkj = 2 * (k - j + 1);
      ld ratio = (ld)nk / nkj;
      ld den = ratio * ratio - 1;
      for (int i = 0; i < dim; ++i) T[k][j][i] = T[k][j - 1][i] + (T[k][j - 1][i] - T[k - 1][j - 1][i]) / den;
    }
    kfin = k;
    if (k >= 2) {
      ld e = 0, s = 0;
      for (int i = 0; i < dim; ++i) {
        ld d = fabsl(T[k][k][i] - T[k][k - 1][i]);
        if (d > e) e = d;
        ld a = fabsl(T[k][k][i]);
        if (a > s) s = a;
      }
      err = e / s;
      if (err < 1e-19L) break;
    }
  }
  memcpy(y, T[kfin][kfin], sizeof(ld) * dim);
  return err;
}
}  // namespace

extern "C" {
// Integrate S systems over time t_total with n_macro macro steps each.
// Arrays as in the oracle: Q, V [S][nmax][3], m [S][nmax]; updated in place.
// Returns the largest per-macro-step error estimate seen.
ld or_gbs_ld(int S, int nmax, const int* np, const ld* m0, const ld* m, ld* Q, ld* V, ld t_total, long n_macro) {
  ld worst = 0;
  for (int k = 0; k < S; ++k) {
    int n = np[k];
    Body b;
    b.nb = n + 1;
    b.m[0] = m0[k];
    ld M = m0[k];
    for (int i = 0; i < n; ++i) { b.m[i + 1] = m[k * nmax + i]; M += b.m[i + 1]; }
    ld y[6 * MAXB];
    ld* x = y;
    ld* v = y + 3 * b.nb;
    // DHC -> barycentric inertial: x0 = -sum m_i Q_i / M, x_i = Q_i + x0,
    // v_i = V_i, v0 = -sum m_i V_i / m0.
    for (int c = 0; c < 3; ++c) {
      ld sq = 0, sv = 0;
      for (int i = 0; i < n; ++i) {
        sq += b.m[i + 1] * Q[(k * nmax + i) * 3 + c];
        sv += b.m[i + 1] * V[(k * nmax + i) * 3 + c];
      }
      x[c] = -sq / M;
      v[c] = -sv / m0[k];
      for (int i = 0; i < n; ++i) {
        x[3 * (i + 1) + c] = Q[(k * nmax + i) * 3 + c] + x[c];
        v[3 * (i + 1) + c] = V[(k * nmax + i) * 3 + c];
      }
    }
    ld H = t_total / n_macro;
    for (long s = 0; s < n_macro; ++s) {
      ld e = gbs_step(b, y, H);
      if (e > worst) worst = e;
    }
    // back to DHC
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) {
        Q[(k * nmax + i) * 3 + c] = x[3 * (i + 1) + c] - x[c];
        V[(k * nmax + i) * 3 + c] = v[3 * (i + 1) + c];
      }
  }
  return worst;
}
}
