// Host construction of the SELL-64 layout of a CSR pattern.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace afc {

// SELL-64 layout: slices of 64 consecutive rows padded to the slice's
// longest row.  A slice is "uniform" when one list of column deltas P (taken
// from its first longest row) places every row: each entry j of row i goes to
// the slot p with P[p] = j - i, and every slot a row leaves empty points at an
// existing node (i + P[p] in [0, N)), so the padding (value 0) needs no
// per-row delta.  Uniform slices share deduplicated patterns; the others keep
// one delta per slot in CSR order.
struct SellLayout {
  std::vector<int> slp;      // [nsl + 1] slot offsets
  std::vector<int> dl;       // [nsl] >= 0: lane-delta offset; < 0: ~pattern offset
  std::vector<int> pat;      // pattern table
  std::vector<int> pos;      // [nnz] CSR entry -> slot
  std::vector<int16_t> d16;  // per-lane deltas of non-uniform slices
  std::vector<int32_t> d32;
  bool dlt16 = true;
  int64_t uniform = 0;
};

// Builds L for the N-row CSR pattern (rp, col); returns an error message, or
// an empty string on success.
std::string build_sell_layout(int N, const int* rp, const int* col, SellLayout& L);

}  // namespace afc
