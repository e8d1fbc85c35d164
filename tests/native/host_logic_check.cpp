// Checks of the library's host logic (wh_host.h: lane packings, workspace
// layout, configuration checks, SABA_n coefficients, tape sizes, launch
// windows), built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py.  Prints "host logic ok" and exits 0, or reports
// the first failed check and exits 1.
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <random>

#include "wh_host.h"

using namespace wh_host;

static int g_fail = 0;
#define CHECK(cond)                                                            \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);  \
      if (++g_fail > 20) std::exit(1);                                         \
    }                                                                          \
  } while (0)

static void check_packing(const std::vector<int32_t>& np, int packing) {
  const int S = (int)np.size();
  Packing P;
  std::string why;
  const int eff = packing == WH_PACK_AUTO ? WH_PACK_POW2 : packing;
  CHECK(make_packing(S, np.data(), eff, P, &why));
  CHECK(P.ns == (int)P.slot_sys.size() && P.ns == (int)P.slot_pl.size());
  CHECK(P.ns == slots_needed(S, np.data(), eff));
  CHECK(P.ns == P.nwaves * (P.pair ? 128 : 64));
  CHECK(P.w1 <= P.w2 && P.w2 <= P.w4 && P.w4 <= P.wm && P.wm <= P.w8 && P.w8 <= P.nwaves);
  CHECK(P.mixed == (eff == WH_PACK_MIXED));
  CHECK(P.mixed || P.wm == P.w8);
  // every planet of every system sits in exactly one slot (two in the split
  // layout, whose two lanes per planet are copies); padding slots are -1
  std::vector<int> seen((size_t)S * 8, 0);
  for (int i = 0; i < P.ns; ++i) {
    const int s = P.slot_sys[i], p = P.slot_pl[i];
    CHECK(s >= -1 && s < S);
    if (p >= 0) {
      CHECK(s >= 0 && p < np[s]);
      if (s >= 0 && p < 8) seen[(size_t)s * 8 + p]++;
    }
  }
  const int copies = P.split ? 2 : 1;
  for (int s = 0; s < S; ++s)
    for (int p = 0; p < 8; ++p) CHECK(seen[(size_t)s * 8 + p] == (p < np[s] ? copies : 0));
  // a system never straddles a wavefront, and in the one-planet layouts its
  // planets fill an aligned group of group_size lanes from the group's start
  if (!P.pair && !P.split) {
    for (int i = 0; i < P.ns; ++i) {
      const int s = P.slot_sys[i];
      if (s < 0) continue;
      if (P.mixed && i >= P.wm * 64) {
        // a shared 8-lane group: system a from the group's first lane, then
        // system b, then b's padding; a has 5 or 6 planets, b 2 or 3
        const int base = i & ~7;
        const int a = P.slot_sys[base];
        CHECK(a >= 0 && (np[a] == 5 || np[a] == 6));
        if (a < 0) continue;
        const int b = P.slot_sys[base + np[a]];
        CHECK(b >= 0 && b != a && (np[b] == 2 || np[b] == 3) && np[a] + np[b] <= 8);
        if (b < 0) continue;
        const int l = i - base;
        if (l < np[a]) CHECK(s == a && P.slot_pl[i] == l);
        else CHECK(s == b && P.slot_pl[i] == (l - np[a] < np[b] ? l - np[a] : -1));
        continue;
      }
      const int G = group_size(np[s], eff);
      const int base = i & ~(G - 1);
      CHECK(P.slot_sys[base] == s);
      CHECK((i - base) < G);
      if (P.slot_pl[i] >= 0) CHECK(P.slot_pl[i] == i - base);
    }
  }
  // the layout's regions are 256-byte aligned and disjoint
  wh_config cfg;
  config_defaults(&cfg, S);
  cfg.packing = packing;
  cfg.balance = 1;
  const size_t cap = plan_capacity(&cfg, P);
  const Layout L = make_layout(S, P.ns, cap);
  const size_t offs[] = {L.st, L.m0s, L.dts, L.slot_sys, L.slot_pl, L.flags, L.synced, L.plan_wave, L.plan_steps,
                         L.total};
  for (int k = 0; k + 1 < 10; ++k) {
    CHECK(offs[k] % 256 == 0);
    CHECK(offs[k] <= offs[k + 1]);
  }
  CHECK(L.m0s - L.st >= sizeof(double) * WH_STATE_ROWS * (size_t)P.ns);
  CHECK(L.plan_steps - L.plan_wave >= sizeof(int) * cap);
  CHECK(cap == (P.serial ? 0 : (size_t)P.nwaves * 2 * PLAN_Q));
}

static void check_plan(std::mt19937_64& rng) {
  for (int trial = 0; trial < 60; ++trial) {
    const int W = 1 + (int)(rng() % 3000);
    const int slots = 1 + (int)(rng() % 1200);
    // short chunks, chunks from Q to about 3 Q (one or two steps per
    // appearance: the most windows per wave), and long ones
    const int R = trial % 4 == 0   ? 1 + (int)(rng() % 9)
                  : trial % 4 == 1 ? PLAN_Q + (int)(rng() % (2 * PLAN_Q + 8))
                                   : 1 + (int)(rng() % 5000);
    std::vector<double> cost(W);
    static const double classes[] = {293, 326, 372, 478, 611, 704, 831};
    for (auto& c : cost) c = classes[rng() % 7];
    std::vector<int> hw, hs, off;
    plan_windows(cost, R, slots, PLAN_Q, hw, hs, off);
    CHECK(hw.size() == hs.size());
    CHECK(!off.empty() && off.front() == 0 && off.back() == (int)hw.size());
    CHECK(hw.size() <= (size_t)W * 2 * PLAN_Q);
    std::vector<long> total(W, 0);
    std::vector<int> last(W, -1), seen(W, 0);
    double cmax = 0;
    for (double c : cost) cmax = std::max(cmax, c);
    for (size_t k = 0; k + 1 < off.size(); ++k) {
      CHECK(off[k + 1] > off[k]);
      CHECK(off[k + 1] - off[k] <= slots);
      for (int e = off[k]; e < off[k + 1]; ++e) {
        const int w = hw[e];
        CHECK(w >= 0 && w < W);
        if (w < 0 || w >= W) continue;
        CHECK(last[w] != (int)k);         // a wave at most once per window
        last[w] = (int)k;
        CHECK(hs[e] >= 1);
        // a wave's share of a window costs at most the window budget (or
        // one step, when the budget is below a step)
        CHECK(hs[e] == 1 || hs[e] * cost[w] <= cmax * R / PLAN_Q * (1 + 1e-12));
        total[w] += hs[e];
        ++seen[w];
      }
    }
    for (int w = 0; w < W; ++w) CHECK(total[w] == R && seen[w] <= 2 * PLAN_Q - 1);
  }
  // the chunk length with the most windows per wave: every wave at the
  // largest cost and R = 2 Q - 1 (one step per appearance); the old bound of
  // Q + 2 entries per wave did not hold it
  {
    std::vector<double> cost(100, 478.0);
    std::vector<int> hw, hs, off;
    plan_windows(cost, 2 * PLAN_Q - 1, 40, PLAN_Q, hw, hs, off);
    CHECK(hw.size() == cost.size() * (2 * PLAN_Q - 1));
    CHECK(hw.size() <= cost.size() * 2 * PLAN_Q);
  }
  // quality of the plan on an uneven batch in the mixed packing (16384
  // systems of 2..8 planets, 1024 slots, a 4096-step chunk): with one wave
  // per slot a window lasts as long as its longest share, and the windows
  // together stay within 3% of the chunk's work divided evenly over the
  // slots (98.1% measured without GR, 98.3% with)
  for (int gr = 0; gr < 2; ++gr) {
    std::mt19937_64 r2(2024 + gr);
    std::vector<int32_t> np(16384);
    for (auto& n : np) n = 2 + (int)(r2() % 7);
    Packing P;
    std::string why;
    CHECK(make_packing((int)np.size(), np.data(), WH_PACK_MIXED, P, &why));
    std::vector<double> cost(P.nwaves);
    double work = 0.0;
    const int R = 4096, slots = 1024;
    for (int w = 0; w < P.nwaves; ++w) {
      cost[w] = wave_step_cost(P, gr == 1, w);
      work += cost[w] * R;
    }
    std::vector<int> hw, hs, off;
    plan_windows(cost, R, slots, PLAN_Q, hw, hs, off);
    double span = 0.0;
    for (size_t k = 0; k + 1 < off.size(); ++k) {
      double longest = 0.0;
      for (int e = off[k]; e < off[k + 1]; ++e) longest = std::max(longest, hs[e] * cost[hw[e]]);
      span += longest;
    }
    CHECK(span > 0.0 && work / slots / span >= 0.97);
  }
}

int main() {
  std::mt19937_64 rng(12345);
  // configuration checks
  wh_config c;
  config_defaults(&c, 10);
  std::string why;
  CHECK(config_ok(&c, why));
  wh_config bad = c; bad.G = 2.0; CHECK(!config_ok(&bad, why));
  bad = c; bad.n_systems = 0; CHECK(!config_ok(&bad, why));
  bad = c; bad.scheme = 9; CHECK(!config_ok(&bad, why));
  bad = c; bad.packing = 7; CHECK(!config_ok(&bad, why));
  bad = c; bad.packing = WH_PACK_MIXED; CHECK(config_ok(&bad, why));
  bad.scheme = WH_SABA2; CHECK(!config_ok(&bad, why));
  bad = c; bad.packing = WH_PACK_MIXED; bad.coords = WH_COORDS_JACOBI; CHECK(!config_ok(&bad, why));
  bad = c; bad.packing = WH_PACK_MIXED; bad.exchange = WH_EXCH_LDS; CHECK(!config_ok(&bad, why));
  bad = c; bad.packing = WH_PACK_MIXED; bad.kepler_counts = 1; CHECK(!config_ok(&bad, why));
  bad = c; bad.packing = WH_PACK_MIXED + 1; CHECK(!config_ok(&bad, why));
  bad = c; bad.block_waves = 3; CHECK(!config_ok(&bad, why));
  bad = c; bad.balance = 2; CHECK(!config_ok(&bad, why));
  bad = c; bad.scheme = WH_SABA2; bad.gr_c = 10.0; CHECK(!config_ok(&bad, why));
  // packings of random batches
  for (int S : {1, 2, 7, 64, 65, 1000, 4099}) {
    std::vector<int32_t> np(S);
    for (auto& n : np) n = 1 + (int)(rng() % 8);
    for (int pk : {WH_PACK_AUTO, WH_PACK_POW2, WH_PACK_G8, WH_PACK_PAIR, WH_PACK_SPLIT, WH_PACK_SERIAL,
                   WH_PACK_MIXED})
      check_packing(np, pk);
  }
  {
    std::vector<int32_t> np(5, 9);
    Packing P;
    CHECK(!make_packing(5, np.data(), WH_PACK_POW2, P, &why));
    np.assign(5, 0);
    Packing P2;
    CHECK(!make_packing(5, np.data(), WH_PACK_POW2, P2, &why));
  }
  // tape sizes: the formula, and sizes that would wrap size_t give 0
  {
    const TapeLayout T = tape_layout(640, 1000, 100, 1);
    CHECK(T.n_seg == 10);
    CHECK(T.total >= sizeof(double) * (12 * 640 * 11 + 2 * WH_TAPE_ROWS * 640 * 100 + 8 * 640));
    CHECK(tape_layout(640, 1001, 100, 1).n_seg == 11);
    CHECK(tape_layout(640, (int64_t(1) << 62) + 3, 1, 1).total == 0);
    CHECK(tape_layout(1 << 27, INT64_MAX, 2, 1).total == 0);
    CHECK(tape_layout(1 << 27, 10, int64_t(1) << 40, 4).total == 0);
    CHECK(tape_layout(64, 0, 1, 1).n_seg == 0);
  }
  // SABA_n coefficients: drift and kick weights each sum to one, symmetric
  for (int n = 1; n <= 4; ++n) {
    double cc[5], d[4];
    saba_coefficients(n, cc, d);
    double sc = 0, sd = 0;
    for (int k = 0; k <= n; ++k) sc += cc[k];
    for (int k = 0; k < n; ++k) sd += d[k];
    CHECK(std::fabs(sc - 1.0) < 1e-15 && std::fabs(sd - 1.0) < 1e-15);
    for (int k = 0; k < n; ++k) CHECK(std::fabs(d[k] - d[n - 1 - k]) < 1e-15);
  }
  // symplectic corrector coefficients: a_i = i/(2n) and the stages'
  // generator sum_i 2 b_i sinh(a_i x) meets (1 - F(x))/x to order x^(2n-1),
  // so doubling x multiplies the difference by ~2^(2n+1)
  for (int scheme : {WH_DKD, WH_KDK})
    for (int n = 1; n <= 3; ++n) {
      double a[3], b[3];
      corrector_coefficients(n, scheme, a, b);
      double d[2];
      for (int j = 0; j < 2; ++j) {
        const double x = 0.16 * (1 << j), y = x / 2;
        const double F = scheme == WH_DKD ? y / std::sinh(y) : y * std::cosh(y) / std::sinh(y);
        double g = 0;
        for (int i = 0; i < n; ++i) {
          CHECK(std::fabs(a[i] - (i + 1.0) / (2.0 * n)) < 1e-15);
          g += 2 * b[i] * std::sinh(a[i] * x);
        }
        d[j] = std::fabs(g - (1 - F) / x);
      }
      const double r = d[1] / d[0], want = std::pow(2.0, 2 * n + 1);
      CHECK(r > 0.7 * want && r < 1.3 * want);
    }
  // launch windows
  check_plan(rng);
  if (g_fail) return 1;
  std::printf("host logic ok\n");
  return 0;
}
