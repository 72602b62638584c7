// Randomized check of the host SELL-64 layout builder, meant to be built with
// AddressSanitizer and UndefinedBehaviorSanitizer.  Random sorted CSR patterns
// (with and without diagonals, empty rows, long rows, bands wide enough for
// 32-bit deltas) are laid out, and the layout is checked: every entry's slot
// lies in its row's slice and lane and decodes to its column, and every slot
// of a row, padding included, gathers a node inside [0, N).
// Usage: fuzz_sell_layout TRIALS SMALL_N_MAX LARGE_N_MAX LARGE_EVERY
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>
#include "afc_layout.h"

int main(int argc, char** argv) {
  const int trials = argc > 1 ? std::atoi(argv[1]) : 300;
  const int small_n = argc > 2 ? std::atoi(argv[2]) : 300;
  const int large_n = argc > 3 ? std::atoi(argv[3]) : 40000;
  const int large_every = argc > 4 ? std::atoi(argv[4]) : 10;
  std::mt19937_64 rng(12345);
  long checked = 0;
  for (int trial = 0; trial < trials; ++trial) {
    const int N = 1 + (int)(rng() % (trial % large_every == large_every - 1 ? large_n : small_n));
    const int band = 1 + (int)(rng() % (trial % 3 == 0 ? N : std::min(N, 70)));
    std::vector<int> rp(N + 1, 0), col;
    for (int i = 0; i < N; ++i) {
      std::set<int> s;
      const int len = (rng() % 10 == 0) ? 0 : (int)(rng() % (trial % 7 == 0 ? 90 : 28));
      if (rng() % 5) s.insert(i);
      for (int k = 0; k < len; ++k) {
        long j = (long)i + (long)(rng() % (2 * band + 1)) - band;
        if (j >= 0 && j < N) s.insert((int)j);
      }
      for (int j : s) col.push_back(j);
      rp[i + 1] = (int)col.size();
    }
    afc::SellLayout L;
    const std::string err = afc::build_sell_layout(N, rp.data(), col.data(), L);
    if (!err.empty()) { std::printf("trial %d N %d: error %s\n", trial, N, err.c_str()); continue; }
    const int nsl = (N + 63) / 64;
    if ((int)L.slp.size() != nsl + 1 || (int)L.dl.size() != nsl || L.pos.size() != col.size()) { std::printf("size mismatch\n"); return 1; }
    for (int i = 0; i < N; ++i) {
      const int s = i / 64, lane = i % 64;
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int p = L.pos[k];
        if (p < L.slp[s] || p >= L.slp[s + 1] || (p - L.slp[s]) % 64 != lane) { std::printf("bad slot trial %d\n", trial); return 1; }
        const int q = (p - L.slp[s]) / 64;
        int d;
        if (L.dl[s] < 0) d = L.pat[~L.dl[s] + q];
        else d = L.dlt16 ? L.d16[L.dl[s] + 64 * q + lane] : L.d32[L.dl[s] + 64 * q + lane];
        if (i + d != col[k]) { std::printf("bad delta trial %d\n", trial); return 1; }
        ++checked;
      }
      // every slot of the row (padding included) gathers inside [0, N)
      const int Ls = (L.slp[s + 1] - L.slp[s]) / 64;
      for (int q = 0; q < Ls; ++q) {
        int d;
        if (L.dl[s] < 0) d = L.pat[~L.dl[s] + q];
        else d = L.dlt16 ? L.d16[L.dl[s] + 64 * q + lane] : L.d32[L.dl[s] + 64 * q + lane];
        if (i + d < 0 || i + d >= N) { std::printf("padding gather out of range trial %d i %d d %d\n", trial, i, d); return 1; }
      }
    }
  }
  std::printf("ok, %ld entries checked\n", checked);
  return 0;
}
