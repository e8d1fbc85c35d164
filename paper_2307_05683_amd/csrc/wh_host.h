// Host-side logic of the library that needs no GPU: lane packings, the
// workspace layout, configuration checks, SABA_n coefficients, tape sizes and
// the balanced launch-window planner.  Plain C++ (wh.hip includes it; a
// sanitizer build of the test suite compiles it with g++ alone).
#pragma once
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "wh.h"

namespace wh_host {

// Rows of the state of a lane slot in the workspace: Q, V, m and the
// compensation terms of Q and V.
constexpr int WH_STATE_ROWS = 13;
// Rows of one recorded step in a reverse-mode segment tape: the rounded
// state before the step (Q, V), the Kepler anomaly X, and the velocity after
// the kick.
constexpr int WH_TAPE_ROWS = 10;

// The defaults of wh_config (wh_config_default).
inline void config_defaults(wh_config* cfg, int32_t n_systems) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->n_systems = n_systems;
  cfg->G = 1.0;
  cfg->gr_c = 0.0;
  cfg->scheme = WH_DKD;
  cfg->packing = WH_PACK_AUTO;
  cfg->block_waves = 1;
  cfg->chunk_steps = 4096;
  cfg->graph_launches = 8;
  cfg->z_max = 1.0;
  cfg->exchange = WH_EXCH_AUTO;
  cfg->coords = WH_COORDS_DHC;
  cfg->balance = 0;
  cfg->kepler_counts = 0;
  cfg->corrector = 0;
}

struct Packing {
  bool pair = false;   // WH_PACK_PAIR: two slots (planets) per lane, 128 slots per wave
  bool split = false;  // WH_PACK_SPLIT: two lanes (copies) per planet, 16 lanes per system
  bool serial = false; // WH_PACK_SERIAL: the G8 storage, one thread per system in the step
  bool mixed = false;  // WH_PACK_MIXED: waves [wm, w8) hold two systems per 8-lane group
  int ns = 0, nwaves = 0;
  int w1 = 0, w2 = 0, w4 = 0, wm = 0, w8 = 0;
  int plain_begin[9] = {0}, plain_end[9] = {0};   // G8 packing: waves of each planet count
  std::vector<int32_t> slot_sys, slot_pl;
};

inline int group_size(int n, int packing) {
  if (packing == WH_PACK_G8 || packing == WH_PACK_SERIAL) return 8;
  return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : 8;
}

// Systems that share an 8-lane group in the mixed packing: each 5-planet
// system takes the next unpaired 3-planet one, else the next 2-planet one;
// each 6-planet system the next 2-planet one (index order throughout).  A
// shared group's step costs about 1.12 of a one-system 8-lane group's, less
// than the 2- or 4-lane group the smaller system would otherwise take; a
// 1-planet partner (64 per wave) would not pay.
struct MixedPairs {
  std::vector<int> a, b;          // the groups: larger system a, smaller b
  std::vector<char> paired;       // per system
};
inline MixedPairs mixed_pairs(int S, const int32_t* np) {
  MixedPairs M;
  M.paired.assign(S, 0);
  std::vector<int> by[9];
  for (int s = 0; s < S; ++s) by[np[s]].push_back(s);
  size_t i3 = 0, i2 = 0;
  for (int s : by[5]) {
    int t = -1;
    if (i3 < by[3].size()) t = by[3][i3++];
    else if (i2 < by[2].size()) t = by[2][i2++];
    if (t < 0) break;
    M.a.push_back(s); M.b.push_back(t);
  }
  for (int s : by[6]) {
    if (i2 >= by[2].size()) break;
    M.a.push_back(s); M.b.push_back(by[2][i2++]);
  }
  for (size_t k = 0; k < M.a.size(); ++k) M.paired[M.a[k]] = M.paired[M.b[k]] = 1;
  return M;
}

// Device indexing is 32-bit: row r of a [rows][ns] array sits at r * ns, with
// up to 13 rows (the state), so the lane-slot count is capped at 2^27
// (14 GB of state; 16.7 million eight-planet systems with one planet per
// lane).
constexpr int64_t MAX_SLOTS = int64_t(1) << 27;

// Lane slots a packing needs, counted before any table is built.
inline int64_t slots_needed(int S, const int32_t* np, int packing) {
  int64_t cnt[9] = {0};
  for (int s = 0; s < S; ++s) cnt[np[s]]++;
  auto waves = [](int64_t n, int per_wave) { return (n + per_wave - 1) / per_wave; };
  if (packing == WH_PACK_SPLIT) return waves(S, 4) * 64;
  if (packing == WH_PACK_PAIR)
    return (waves(cnt[1] + cnt[2], 64) + waves(cnt[3] + cnt[4], 32) + waves(cnt[5] + cnt[6] + cnt[7] + cnt[8], 16)) *
           128;
  if (packing == WH_PACK_G8 || packing == WH_PACK_SERIAL) {
    int64_t w = 0;
    for (int n = 1; n <= 8; ++n) w += waves(cnt[n], 8);
    return w * 64;
  }
  if (packing == WH_PACK_MIXED) {
    // the pairing rule of mixed_pairs, on the counts
    const int64_t p53 = std::min(cnt[5], cnt[3]);
    const int64_t p52 = std::min(cnt[5] - p53, cnt[2]);
    const int64_t p62 = std::min(cnt[6], cnt[2] - p52);
    return (waves(cnt[1], 64) + waves(cnt[2] - p52 - p62, 32) + waves(cnt[3] - p53 + cnt[4], 16) +
            waves(cnt[5] - p53 - p52 + cnt[6] - p62 + cnt[7] + cnt[8], 8) + waves(p53 + p52 + p62, 8)) * 64;
  }
  return (waves(cnt[1], 64) + waves(cnt[2], 32) + waves(cnt[3] + cnt[4], 16) +
          waves(cnt[5] + cnt[6] + cnt[7] + cnt[8], 8)) * 64;
}

// Lay systems out on lanes.  Systems of one group size fill whole waves; G8
// packing also keeps each planet count on waves of its own (for the
// per-size reference path).  Within a class systems keep their index order.
inline bool make_packing(int S, const int32_t* np, int packing, Packing& P, std::string* why = nullptr) {
  for (int s = 0; s < S; ++s)
    if (np[s] < 1 || np[s] > 8) {
      if (why) *why = "planet counts must be in 1..8";
      return false;
    }
  if (slots_needed(S, np, packing) > MAX_SLOTS) {
    if (why) *why = "too many systems: the packing needs more than 2^27 lane slots";
    return false;
  }
  auto add_wave_block = [&](const std::vector<int>& systems, int G) {
    int per_wave = 64 / G;
    int nw = ((int)systems.size() + per_wave - 1) / per_wave;
    for (int w = 0; w < nw; ++w)
      for (int j = 0; j < per_wave; ++j) {
        int idx = w * per_wave + j;
        int s = idx < (int)systems.size() ? systems[idx] : -1;
        for (int l = 0; l < G; ++l) {
          P.slot_sys.push_back(s);
          P.slot_pl.push_back(s >= 0 && l < np[s] ? l : -1);
        }
      }
    P.nwaves += nw;
  };
  if (packing == WH_PACK_PAIR) {
    // a system of N planets takes G = 1, 2 or 4 lanes (2G >= N); lane l of a
    // group holds planet l in slot 128 w + (lane) and planet G + l in slot
    // 128 w + 64 + (lane) of its wave w
    int ends[3];
    const int Gs[3] = {1, 2, 4};
    for (int gi = 0; gi < 3; ++gi) {
      const int G = Gs[gi];
      std::vector<int> cls;
      for (int s = 0; s < S; ++s)
        if ((np[s] <= 2 ? 1 : np[s] <= 4 ? 2 : 4) == G) cls.push_back(s);
      const int per_wave = 64 / G;
      const int nw = ((int)cls.size() + per_wave - 1) / per_wave;
      for (int w = 0; w < nw; ++w) {
        int32_t a_sys[64], a_pl[64], b_sys[64], b_pl[64];
        for (int j = 0; j < per_wave; ++j) {
          const int idx = w * per_wave + j;
          const int s = idx < (int)cls.size() ? cls[idx] : -1;
          for (int l = 0; l < G; ++l) {
            const int ln = j * G + l;
            a_sys[ln] = s;
            a_pl[ln] = s >= 0 && l < np[s] ? l : -1;
            b_sys[ln] = s;
            b_pl[ln] = s >= 0 && G + l < np[s] ? G + l : -1;
          }
        }
        P.slot_sys.insert(P.slot_sys.end(), a_sys, a_sys + 64);
        P.slot_pl.insert(P.slot_pl.end(), a_pl, a_pl + 64);
        P.slot_sys.insert(P.slot_sys.end(), b_sys, b_sys + 64);
        P.slot_pl.insert(P.slot_pl.end(), b_pl, b_pl + 64);
      }
      P.nwaves += nw;
      ends[gi] = P.nwaves;
    }
    P.pair = true;
    P.w1 = ends[0]; P.w2 = ends[1]; P.w4 = ends[2]; P.w8 = ends[2];
  } else if (packing == WH_PACK_SPLIT) {
    // every system takes a 16-lane group, four per wave, in index order;
    // planet p (padding beyond N) in lanes 2p and 2p + 1
    const int nw = (S + 3) / 4;
    for (int w = 0; w < nw; ++w)
      for (int j = 0; j < 4; ++j) {
        const int s = w * 4 + j < S ? w * 4 + j : -1;
        for (int l = 0; l < 16; ++l) {
          P.slot_sys.push_back(s);
          P.slot_pl.push_back(s >= 0 && (l >> 1) < np[s] ? l >> 1 : -1);
        }
      }
    P.nwaves = nw;
    P.split = true;
    P.w1 = P.w2 = P.w4 = 0;
    P.w8 = nw;
  } else if (packing == WH_PACK_G8 || packing == WH_PACK_SERIAL) {
    for (int n = 1; n <= 8; ++n) {
      std::vector<int> cls;
      for (int s = 0; s < S; ++s)
        if (np[s] == n) cls.push_back(s);
      P.plain_begin[n] = P.nwaves;
      add_wave_block(cls, 8);
      P.plain_end[n] = P.nwaves;
    }
    P.w1 = P.w2 = P.w4 = 0;
    P.w8 = P.nwaves;
    P.serial = packing == WH_PACK_SERIAL;
  } else {
    MixedPairs M;
    if (packing == WH_PACK_MIXED) M = mixed_pairs(S, np);
    int ends[4];
    const int Gs[4] = {1, 2, 4, 8};
    for (int gi = 0; gi < 4; ++gi) {
      std::vector<int> cls;
      for (int s = 0; s < S; ++s)
        if (group_size(np[s], packing) == Gs[gi] && (M.paired.empty() || !M.paired[s])) cls.push_back(s);
      add_wave_block(cls, Gs[gi]);
      ends[gi] = P.nwaves;
    }
    P.w1 = ends[0]; P.w2 = ends[1]; P.w4 = ends[2]; P.wm = ends[3];
    if (packing == WH_PACK_MIXED) {
      // shared 8-lane groups: system a in lanes 0..Na-1, b in Na..Na+Nb-1,
      // padding lanes after them belong to b (its star and step)
      const int ng = (int)M.a.size(), nw = (ng + 7) / 8;
      for (int g = 0; g < nw * 8; ++g) {
        const int a = g < ng ? M.a[g] : -1, b = g < ng ? M.b[g] : -1;
        for (int l = 0; l < 8; ++l) {
          if (a < 0) {
            P.slot_sys.push_back(-1);
            P.slot_pl.push_back(-1);
          } else if (l < np[a]) {
            P.slot_sys.push_back(a);
            P.slot_pl.push_back(l);
          } else {
            P.slot_sys.push_back(b);
            P.slot_pl.push_back(l - np[a] < np[b] ? l - np[a] : -1);
          }
        }
      }
      P.nwaves += nw;
      P.mixed = true;
    }
    P.w8 = P.nwaves;
  }
  if (!P.mixed) P.wm = P.w8;
  P.ns = P.nwaves * (P.pair ? 128 : 64);
  // every wave holds exactly 64 (pair layout: 128) slots; the device tables are copied at ns
  if ((int)P.slot_sys.size() != P.ns || (int)P.slot_pl.size() != P.ns || P.ns != slots_needed(S, np, packing)) {
    if (why) *why = "internal error: inconsistent lane packing";
    return false;
  }
  return true;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t st, m0s, dts, slot_sys, slot_pl, flags, synced, plan_wave, plan_steps, total;
};

// plan_cap: entries reserved for the balanced launch windows (0 without).
inline Layout make_layout(int S, int ns, size_t plan_cap = 0) {
  Layout L;
  size_t o = 0;
  L.st = o; o = align256(o + sizeof(double) * WH_STATE_ROWS * (size_t)ns);
  L.m0s = o; o = align256(o + sizeof(double) * (size_t)ns);
  L.dts = o; o = align256(o + sizeof(double) * (size_t)ns);
  L.slot_sys = o; o = align256(o + sizeof(int) * (size_t)ns);
  L.slot_pl = o; o = align256(o + sizeof(int) * (size_t)ns);
  L.flags = o; o = align256(o + sizeof(uint32_t) * (size_t)S);
  L.synced = o; o = align256(o + sizeof(int) * (size_t)S);
  L.plan_wave = o; o = align256(o + sizeof(int) * plan_cap);
  L.plan_steps = o; o = align256(o + sizeof(int) * plan_cap);
  L.total = o;
  return L;
}

// Balanced launch windows.  A chunk of R steps is cut so that the heaviest
// wave runs in about PLAN_Q windows of R / PLAN_Q steps.  Every appearance of
// a wave but its last runs at least max(1, floor(R / PLAN_Q)) steps, so a wave
// appears in at most 2 PLAN_Q - 1 windows of a chunk (R < PLAN_Q: R windows;
// PLAN_Q <= R < 2 PLAN_Q: one step each; beyond, floor(R / PLAN_Q) >= 2 and
// R / floor(R / PLAN_Q) < 1.5 PLAN_Q), and 2 PLAN_Q entries per wave bound
// the plan.
constexpr int PLAN_Q = 16;
inline size_t plan_capacity(const wh_config* cfg, const Packing& P) {
  return cfg->balance == 1 && !P.serial ? (size_t)P.nwaves * 2 * PLAN_Q : 0;
}

inline bool config_ok(const wh_config* c, std::string& why) {
  if (!c) { why = "null config"; return false; }
  if (c->n_systems < 1) { why = "n_systems must be >= 1"; return false; }
  if (c->G != 1.0) { why = "G must be 1 (units with G = 1)"; return false; }
  if (c->scheme != WH_DKD && c->scheme != WH_KDK && c->scheme != WH_SABA2 && c->scheme != WH_SABA3 &&
      c->scheme != WH_SABA4) {
    why = "scheme must be WH_DKD, WH_KDK or WH_SABA2..4"; return false;
  }
  if (c->scheme >= WH_SABA2 && c->gr_c > 0 && c->coords != WH_COORDS_JACOBI) {
    why = "SABA_n with GR needs Jacobi coordinates: in DHC the GR and jump flows do not commute"; return false;
  }
  if (c->packing < WH_PACK_AUTO || c->packing > WH_PACK_MIXED) { why = "unknown packing"; return false; }
  if (c->packing == WH_PACK_MIXED &&
      (c->coords != WH_COORDS_DHC || (c->scheme != WH_DKD && c->scheme != WH_KDK) || c->exchange == WH_EXCH_LDS ||
       c->kepler_counts != 0)) {
    why = "the mixed packing runs DHC drift-kick-drift or kick-drift-kick with the DPP exchange and the paper's "
          "Kepler counts";
    return false;
  }
  if (c->block_waves != 0 && c->block_waves != 1 && c->block_waves != 2 && c->block_waves != 4) {
    why = "block_waves must be 0, 1, 2 or 4"; return false;
  }
  if (c->chunk_steps < 0) { why = "chunk_steps must be >= 0"; return false; }
  if (c->balance != 0 && c->balance != 1) { why = "balance must be 0 or 1"; return false; }
  if (c->kepler_counts != 0 && c->kepler_counts != 1) { why = "kepler_counts must be 0 or 1"; return false; }
  if (c->kepler_counts == 1 &&
      (c->coords != WH_COORDS_DHC || (c->scheme != WH_DKD && c->scheme != WH_KDK) ||
       c->packing == WH_PACK_SERIAL || c->exchange == WH_EXCH_LDS)) {
    why = "kepler_counts = 1 runs DHC drift-kick-drift or kick-drift-kick with the DPP exchange in the POW2, G8, "
          "PAIR or SPLIT packing";
    return false;
  }
  if (c->corrector < 0 || c->corrector > 3) { why = "corrector must be 0..3 stages"; return false; }
  if (c->corrector > 0 && (c->coords != WH_COORDS_JACOBI || (c->scheme != WH_DKD && c->scheme != WH_KDK))) {
    why = "symplectic correctors need Jacobi coordinates with WH_DKD or WH_KDK";
    return false;
  }
  if (!(c->z_max >= 0.0)) { why = "z_max must be >= 0"; return false; }
  if (c->exchange < WH_EXCH_AUTO || c->exchange > WH_EXCH_DPP) { why = "unknown exchange"; return false; }
  if (c->coords != WH_COORDS_DHC && c->coords != WH_COORDS_JACOBI) { why = "unknown coordinates"; return false; }
  if ((c->packing == WH_PACK_PAIR || c->packing == WH_PACK_SPLIT || c->packing == WH_PACK_SERIAL) &&
      c->coords != WH_COORDS_DHC) {
    why = "the two-planets-per-lane, two-lanes-per-planet and one-lane-per-system packings run in democratic "
          "heliocentric coordinates only";
    return false;
  }

  if (!(c->gr_c == c->gr_c)) { why = "gr_c is NaN"; return false; }
  return true;
}

inline int eff_packing(const wh_config* c) { return c->packing == WH_PACK_AUTO ? WH_PACK_POW2 : c->packing; }


// SABA_n coefficients from n-point Gauss-Legendre quadrature on [0, 1]:
// d_k the weights, c_1 the first node, c_k the gaps between nodes, c_{n+1}
// = c_1 by symmetry.  Nodes by Newton's method on the Legendre polynomial.
inline void saba_coefficients(int n, double* c, double* d) {
  const double pi = 3.14159265358979323846;
  std::vector<long double> t(n), w(n);
  for (int i = 0; i < n; ++i) {
    long double x = std::cos(pi * (n - i - 0.25) / (n + 0.5));   // ascending root guesses
    long double dp = 1;
    for (int it = 0; it < 60; ++it) {
      long double pm = 1, pc = x;      // P_0, P_1
      for (int k = 2; k <= n; ++k) {
        long double pn = ((2 * k - 1) * x * pc - (k - 1) * pm) / k;
        pm = pc;
        pc = pn;
      }
      if (n == 1) pm = 1;
      dp = n * (x * pc - pm) / (x * x - 1);
      long double step = pc / dp;
      x -= step;
      if (std::fabs((double)step) < 1e-19) break;
    }
    t[i] = (x + 1) / 2;
    w[i] = 1 / ((1 - x * x) * dp * dp);
  }
  c[0] = (double)t[0];
  for (int k = 1; k < n; ++k) c[k] = (double)(t[k] - t[k - 1]);
  c[n] = c[0];
  for (int k = 0; k < n; ++k) d[k] = (double)w[k];
}


// Symplectic corrector of the Jacobi map, n stages (order 2n + 1), scheme
// WH_DKD or WH_KDK.  To first order in the perturbation the map of step h is
// the flow of A + F(h ad_A) B, F(x) = (x/2)/sinh(x/2) (drift-kick-drift) or
// (x/2) cosh(x/2)/sinh(x/2) (kick-drift-kick); a stage Z(a, b) (drift a h,
// kick b h, drift -2a h, kick -b h, drift a h) generates 2 b h sinh(a h ad_A)
// B, so with a_i = i/(2n) the b_i solve
//   sum_i 2 b_i a_i^(2k-1)/(2k-1)! = -f_k,  k = 1..n,
// f_k the coefficient of x^(2k) in F: the change of variables h Psi B,
// Psi = (1 - F(x))/x, that takes the map's flow to that of A + B.
inline void corrector_coefficients(int n, int scheme, double* a, double* b) {
  // F = (x/2) g(x/2)/ (sinh(y)/y) with y = x/2: numerator 1 or cosh y,
  // denominator sinh(y)/y, both as series in y^2; divide term by term.
  double num[8], den[8], q[8];
  double fact = 1.0;                       // (2k)!
  for (int k = 0; k <= n; ++k) {
    if (k > 0) fact *= (2.0 * k - 1.0) * (2.0 * k);
    den[k] = 1.0 / (fact * (2.0 * k + 1.0));
    num[k] = scheme == WH_KDK ? 1.0 / fact : (k == 0 ? 1.0 : 0.0);
  }
  for (int k = 0; k <= n; ++k) {
    double s = num[k];
    for (int j = 1; j <= k; ++j) s -= den[j] * q[k - j];
    q[k] = s / den[0];
  }
  double M[3][4];
  for (int i = 0; i < n; ++i) a[i] = (i + 1.0) / (2.0 * n);
  for (int k = 1; k <= n; ++k) {
    double f = 1.0;                        // (2k-1)!
    for (int j = 2; j <= 2 * k - 1; ++j) f *= j;
    for (int i = 0; i < n; ++i) M[k - 1][i] = 2.0 * std::pow(a[i], 2 * k - 1) / f;
    M[k - 1][n] = -q[k] / std::pow(4.0, k);   // f_k: y^(2k) = x^(2k) / 4^k
  }
  for (int col = 0; col < n; ++col) {      // Gauss-Jordan, partial pivoting
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
    for (int j = 0; j <= n; ++j) std::swap(M[col][j], M[piv][j]);
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double g = M[r][col] / M[col][col];
      for (int j = col; j <= n; ++j) M[r][j] -= g * M[col][j];
    }
  }
  for (int i = 0; i < n; ++i) b[i] = M[i][n] / M[i][i];
}

struct TapeLayout {
  int64_t n_seg = 0;       // segments
  size_t ck = 0;           // checkpoints: (n_seg + 1) x [12][ns]
  size_t seg[2] = {0, 0};  // two segment tapes: ckpt_every x [WH_TAPE_ROWS][ns] each
  size_t grad = 0;         // adjoint state: [8][ns]
  size_t total = 0;
};

// units: tape row sets per step (SABA_n records each of its n drift-kick
// units, the other schemes one).  Every product and sum is checked: a size
// that does not fit in size_t gives T.total = 0 (the callers reject it), so a
// wrapped, too small tape can never pass the size check.
inline TapeLayout tape_layout(int ns, int64_t n_steps, int64_t every, int units) {
  TapeLayout T;
  if (ns < 0 || n_steps < 0 || every < 1 || units < 1) return T;
  T.n_seg = n_steps / every + (n_steps % every != 0 ? 1 : 0);
  bool bad = false;
  auto mul = [&bad](size_t a, size_t b) {
    size_t r;
    if (__builtin_mul_overflow(a, b, &r)) bad = true;
    return r;
  };
  auto add256 = [&bad](size_t a, size_t b) {
    size_t r;
    if (__builtin_add_overflow(a, b, &r) || __builtin_add_overflow(r, (size_t)255, &r)) bad = true;
    return r & ~(size_t)255;
  };
  size_t o = 0;
  T.ck = o;
  o = add256(o, mul(mul(sizeof(double) * 12, (size_t)ns), (size_t)T.n_seg + 1));
  for (int b = 0; b < 2; ++b) {
    T.seg[b] = o;
    o = add256(o, mul(mul(mul(sizeof(double) * WH_TAPE_ROWS, (size_t)ns), (size_t)every), (size_t)units));
  }
  T.grad = o;
  o = add256(o, mul(sizeof(double) * 8, (size_t)ns));
  T.total = bad ? 0 : o;
  return T;
}


// Relative cost of one step of wave w of the packing (gfx950; without and
// with GR; only the proportions matter).  One planet per lane: the measured
// time of a drift-kick-drift step of a wavefront alone on its SIMD, for each
// group size, scaled to the 8-lane group's VALU instructions per lane-step
// (1024 one-size wavefronts: 0.662 / 0.692 / 0.791 of the 8-lane step for
// 1, 2, 4 lanes without GR, 0.627 / 0.698 / 0.790 with; the instruction
// counts, 293 / 326 / 372 / 478, had the 4-lane waves 1.6% too cheap).  Two
// planets per lane: VALU instructions per lane-step.
inline double wave_step_cost(const Packing& P, bool with_gr, int w) {
  const int gr = with_gr ? 1 : 0;
  if (P.split) return 1.0;
  if (P.pair) {
    static const double t[2][3] = {{611, 704, 831}, {653, 755, 891}};
    return t[gr][w < P.w1 ? 0 : w < P.w2 ? 1 : 2];
  }
  static const double t[2][4] = {{316, 331, 378, 478}, {330, 367, 416, 526}};
  static const double mixed[2] = {543, 598};
  if (P.mixed && w >= P.wm) return mixed[gr];
  return t[gr][w < P.w1 ? 0 : w < P.w2 ? 1 : w < P.w4 ? 2 : 3];
}


// Cut one chunk of R steps into launch windows.  cost[w]: relative cost of
// one step of wave w.  While waves have steps left, a window takes the (at
// most slots) waves with the most work left and gives each the steps that
// cost about B = (heaviest wave's cost) x R / Q, so that every SIMD carries
// about the same work in every window and all waves finish the chunk
// together.  Output: window k holds entries [off[k], off[k+1]) of (hw: wave,
// hs: steps); every wave's steps add up to R; a wave appears in at most
// 2 Q - 1 windows (max(1, floor(B / cost)) >= max(1, floor(R / Q)) steps each
// time but the last).
inline void plan_windows(const std::vector<double>& cost, int R, int slots, int Q, std::vector<int>& hw,
                         std::vector<int>& hs, std::vector<int>& off) {
  const int W = (int)cost.size();
  hw.clear();
  hs.clear();
  off.clear();
  if (W == 0 || R < 1 || slots < 1 || Q < 1) return;
  double cmax = 0.0;
  for (double c : cost) cmax = std::max(cmax, c);
  const double B = cmax * R / Q;
  std::vector<int> rem(W, R), order(W);
  for (int w = 0; w < W; ++w) order[w] = w;
  off.push_back(0);
  int left = W;
  while (left > 0) {
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return rem[a] * cost[a] > rem[b] * cost[b]; });
    for (int i = 0, n = 0; i < W && n < slots; ++i, ++n) {
      const int w = order[i];
      if (rem[w] == 0) break;                // sorted: every later wave is done too
      const int s = std::min(rem[w], std::max(1, (int)(B / cost[w])));
      hw.push_back(w);
      hs.push_back(s);
      rem[w] -= s;
      if (rem[w] == 0) --left;
    }
    off.push_back((int)hw.size());
  }
}

}  // namespace wh_host
