// Host construction of the SELL-64 layout (see afc_layout.h) and its C entry
// point afc_sell_layout, which needs no GPU.
#include "afc_layout.h"

#include <algorithm>
#include <cstdlib>
#include <limits>
#include <map>
#include <utility>

#include "afc.h"

namespace afc {

std::string build_sell_layout(int N, const int* rp, const int* col, SellLayout& L) {
  const int nsl = (N + 63) / 64;
  L.slp.assign(nsl + 1, 0);
  L.dl.assign(nsl, 0);
  L.pos.assign(rp[N], 0);
  std::vector<int> lane_delta;  // collected as int32, narrowed at the end
  std::map<std::vector<int>, int> patterns;
  std::vector<std::pair<int, int>> sorted;  // (delta, slot) of the candidate pattern
  std::vector<char> used;
  for (int sl = 0; sl < nsl; ++sl) {
    const int r0 = sl * 64, r1 = std::min(N, r0 + 64);
    int len = 0, lr = r0;
    for (int i = r0; i < r1; ++i)
      if (rp[i + 1] - rp[i] > len) {
        len = rp[i + 1] - rp[i];
        lr = i;
      }
    if ((int64_t)L.slp[sl] + 64LL * len >= (int64_t)std::numeric_limits<int>::max())
      return "SELL layout exceeds 2^31 slots";
    L.slp[sl + 1] = L.slp[sl] + 64 * len;
    // candidate pattern
    std::vector<int> P(len);
    sorted.resize(len);
    for (int p = 0; p < len; ++p) {
      P[p] = col[rp[lr] + p] - lr;
      sorted[p] = {P[p], p};
    }
    std::sort(sorted.begin(), sorted.end());
    bool ok = true;
    for (int p = 1; p < len && ok; ++p) ok = sorted[p].first != sorted[p - 1].first;
    used.assign(len, 0);
    for (int i = r0; i < r1 && ok; ++i) {
      std::fill(used.begin(), used.end(), 0);
      for (int k = rp[i]; k < rp[i + 1] && ok; ++k) {
        auto it = std::lower_bound(sorted.begin(), sorted.end(), std::make_pair(col[k] - i, -1));
        if (it == sorted.end() || it->first != col[k] - i || used[it->second]) {
          ok = false;
        } else {
          used[it->second] = 1;
          L.pos[k] = L.slp[sl] + 64 * it->second + (i - r0);
        }
      }
      for (int p = 0; p < len && ok; ++p)
        if (!used[p] && (i + P[p] < 0 || i + P[p] >= N)) ok = false;
    }
    if (ok) {
      auto it = patterns.find(P);
      int off;
      if (it == patterns.end()) {
        if ((int64_t)L.pat.size() + len >= (int64_t)std::numeric_limits<int>::max())
          return "SELL pattern table exceeds 2^31 entries";
        off = (int)L.pat.size();
        L.pat.insert(L.pat.end(), P.begin(), P.end());
        patterns.emplace(P, off);
      } else {
        off = it->second;
      }
      L.dl[sl] = ~off;
      L.uniform += 1;
    } else {
      if ((int64_t)lane_delta.size() + 64LL * len >= (int64_t)std::numeric_limits<int>::max())
        return "SELL delta array exceeds 2^31 entries";
      const int off = (int)lane_delta.size();
      L.dl[sl] = off;
      lane_delta.resize(lane_delta.size() + 64 * (size_t)len, 0);
      for (int i = r0; i < r1; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
          const int q = 64 * (k - rp[i]) + (i - r0);
          L.pos[k] = L.slp[sl] + q;
          lane_delta[off + q] = col[k] - i;
        }
    }
  }
  int maxd = 0;
  for (int d : lane_delta) maxd = std::max(maxd, std::abs(d));
  L.dlt16 = maxd <= 32767;
  if (L.dlt16)
    L.d16.assign(lane_delta.begin(), lane_delta.end());
  else
    L.d32.assign(lane_delta.begin(), lane_delta.end());
  return std::string();
}

}  // namespace afc

extern "C" afc_status afc_sell_layout(int32_t n, const int32_t* row_ptr, const int32_t* col, afc_sell_info* info,
                                      int32_t* slice_ptr, int32_t* slice_delta, int32_t* pattern, int32_t* pos,
                                      int32_t* lane_deltas) {
  if (n < 0 || !row_ptr || !info) return AFC_EINVAL;
  if (row_ptr[0] != 0) return AFC_EINVAL;
  for (int32_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return AFC_EINVAL;
  const int64_t nnz = row_ptr[n];
  if (nnz > 0 && !col) return AFC_EINVAL;
  for (int64_t k = 0; k < nnz; ++k)
    if (col[k] < 0 || col[k] >= n) return AFC_EINVAL;
  afc::SellLayout L;
  if (!afc::build_sell_layout(n, row_ptr, col, L).empty()) return AFC_EINVAL;
  info->slices = (int64_t)L.dl.size();
  info->slots = L.slp.empty() ? 0 : (int64_t)L.slp.back();
  info->uniform_slices = L.uniform;
  info->lane_delta_slots = (int64_t)(L.dlt16 ? L.d16.size() : L.d32.size());
  info->pattern_ints = (int64_t)L.pat.size();
  info->delta_bytes = L.dlt16 ? 2 : 4;
  info->reserved = 0;
  if (slice_ptr) std::copy(L.slp.begin(), L.slp.end(), slice_ptr);
  if (slice_delta) std::copy(L.dl.begin(), L.dl.end(), slice_delta);
  if (pattern) std::copy(L.pat.begin(), L.pat.end(), pattern);
  if (pos) std::copy(L.pos.begin(), L.pos.end(), pos);
  if (lane_deltas) {
    if (L.dlt16)
      std::copy(L.d16.begin(), L.d16.end(), lane_deltas);
    else
      std::copy(L.d32.begin(), L.d32.end(), lane_deltas);
  }
  return AFC_OK;
}
