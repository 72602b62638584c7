// Device helpers shared by the HIP translation units of libafc.
#pragma once

#include <hip/hip_runtime.h>

namespace afc {

// Sums / extrema over groups of G consecutive lanes (G divides 64).
template <int G>
static __device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}
template <int G>
static __device__ __forceinline__ float gsumf(float v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}
template <int G>
static __device__ __forceinline__ double gmax(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, G));
  return v;
}
template <int G>
static __device__ __forceinline__ double gmin(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, G));
  return v;
}

// Lane move of a double with one DPP control (both 32-bit halves).
template <int CTRL>
static __device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (every lane active), returned to every lane.
// DPP lane moves build it in lane 63: pairs and quads (quad permutes), rows
// of 16 (row rotates by 4 and 8), then rows 0+1 and 2+3 (broadcast of lane
// 15 into the next row) and all four rows (broadcast of lane 31 into rows 2
// and 3).  A fixed pattern, so the result is deterministic.
static __device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x124>(v);  // row_ror 4
  v += dpp_move<0x128>(v);  // row_ror 8
  v += dpp_move<0x142>(v);  // row_bcast 15
  v += dpp_move<0x143>(v);  // row_bcast 31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// v of lane src (src the same for the whole wave)
static __device__ __forceinline__ double lane_value(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// a + b after an exchange of halves between lanes l and l ^ 32: lanes 0..31
// return a(l) + a(l + 32), lanes 32..63 return b(l - 32) + b(l)
// (v_permlane32_swap, both 32-bit halves)
static __device__ __forceinline__ double swap32_sum(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// the same between lanes l and l ^ 16: even rows of 16 lanes sum a, odd rows b
static __device__ __forceinline__ double swap16_sum(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// Eight sums over the 64 lanes of a wave (every lane active): lane l returns
// the wave total of v[l >> 3].  Three exchange steps (partners l ^ 32, l ^ 16,
// l ^ 8) each keep half of the values a lane holds, summed with its partner's
// copy of the same values; then the eight lanes holding one value add up
// (quad permutes, half-row mirror).  About a fifth of the lane moves of eight
// wave_sum calls.  A fixed pattern, so the result is deterministic.
static __device__ __forceinline__ double wave_sum8(const double (&v)[8]) {
  double u[4], w[2];
#pragma unroll
  for (int m = 0; m < 4; ++m) u[m] = swap32_sum(v[m], v[m + 4]);  // lanes with bit 5 set hold v[4..7]
#pragma unroll
  for (int m = 0; m < 2; ++m) w[m] = swap16_sum(u[m], u[m + 2]);  // bit 4: the upper pair
  const bool b3 = (threadIdx.x & 8) != 0;                          // bit 3: the upper one
  double x = (b3 ? w[1] : w[0]) + dpp_move<0x128>(b3 ? w[0] : w[1]);  // row_ror 8 = lane ^ 8
  x += dpp_move<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_move<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_move<0x141>(x);  // row_half_mirror: lane ^ 7 inside each group of 8
  return x;
}

// Zalesak's R = min(1, m Q / (dt P)), 1 when P = 0 (Sec. 2.1.3, step 3).
static __device__ __forceinline__ double zalesak_R(double mi, double Q, double P, double dt) {
  return P != 0.0 ? fmin(1.0, mi * Q / (dt * P)) : 1.0;
}

static __device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return fmin(a, b);
  if (a < 0.0 && b < 0.0) return fmax(a, b);
  return 0.0;
}

// CN flux r_ij of eq. (12), prelimited by eq. (13) (midpoint reading)
static __device__ __forceinline__ double cn_flux(double mij, double d, double inv_dt, double dui, double duj, double sui,
                                          double suj, double L) {
  double r = mij * inv_dt * (dui - duj) + 0.5 * d * (suj - sui);
  if (L != 0.0) r = minmod(r, L * d * (0.5 * suj - 0.5 * sui));
  return r;
}


}  // namespace afc
