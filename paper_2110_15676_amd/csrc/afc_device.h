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

static __device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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
