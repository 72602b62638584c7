// HIP kernels of the AFC hot path for gfx950 (CDNA4, wave64).
//
// Solver and limiter passes run over a SELL-64 copy of each matrix: one wave
// per 64-row slice, one row per lane, slots column-major inside the slice, so
// every lane streams its own row with coalesced loads and needs no cross-lane
// sum.  Column offsets are shared per slice where one offset pattern places
// every row (read as scalars), else stored per slot (16 or 32 bits).  Each
// workgroup takes a contiguous, balanced range of tiles, and workgroup ids are
// remapped so that each of the 8 XCDs works on one contiguous slab of rows
// (workgroups are dispatched round-robin over XCDs), which keeps the neighbour
// gathers inside that XCD's L2.  The few setup kernels over CSR rows map G
// lanes to a row (G = 8/16/32/64 from the mean row length).
//
// Reductions (norms, dot products) are deterministic: per-workgroup partials
// in fixed slots, summed in a fixed order by a separate small reduce kernel
// that also performs the scalar step of the solver (Givens rotation, BiCGStab
// coefficients, convergence flag), so the host never waits inside a Krylov
// cycle.  No kernel uses floating-point atomics.

#include <algorithm>
#include <cmath>

#include <hip/hip_ext.h>

#include "afc_device.h"
#include "afc_kernels.h"

namespace afc {
namespace {

constexpr int kRowGridCap = 32768;

__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b & 7, k = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return x * per + min(x, rem) + k;
}

// contiguous, balanced share of ntiles for this workgroup (sizes differ by at
// most one), in the XCD-aware order
__device__ __forceinline__ void tile_range(int ntiles, int& t0, int& t1) {
  const int nb = gridDim.x;
  const int b = xcd_block(blockIdx.x, nb);
  t0 = (int)(((int64_t)b * ntiles) / nb);
  t1 = (int)(((int64_t)(b + 1) * ntiles) / nb);
}

// the same shares, each XCD's slab taken from its end: workgroups dispatched
// first get the slab's last tiles
__device__ __forceinline__ void tile_range_rev(int ntiles, int& t0, int& t1) {
  const int nb = gridDim.x;
  const int x = blockIdx.x & 7, k = blockIdx.x >> 3;
  const int per = nb >> 3, rem = nb & 7;
  const int cnt = per + (x < rem ? 1 : 0);
  const int b = x * per + min(x, rem) + (cnt - 1 - k);
  t0 = (int)(((int64_t)b * ntiles) / nb);
  t1 = (int)(((int64_t)(b + 1) * ntiles) / nb);
}

// Block totals of nv per-thread values into partials[q * kRedBlocks + slot].
template <int KMAX>
__device__ void block_partials(const double (&v)[KMAX], int nv, double* partials, int slot) {
  __shared__ double sh[KMAX][kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    if (q < nv) {
      const double s = wave_sum(v[q]);
      if (lane == 0) sh[q][wv] = s;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nv; q += kBlock) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += sh[q][w];
    partials[(size_t)q * kRedBlocks + slot] = s;
  }
}

// Partial rows of the GMRES step: projection partials in rows
// 0..k, the squared norm of the new basis vector in the last row.
constexpr int kNormRow = kMaxRed - 1;
// Start of a Krylov cycle from the squared norm of its residual.
__device__ void cycle_start_dev(KState* ks, int mode, double rr, double tol_abs, double tol_rel) {
  ks->ctol_abs = tol_abs;
  ks->ctol_rel = tol_rel;
  const double beta = sqrt(rr);
  ks->beta = beta;
  ks->res = beta;
  ks->k = 0;
  ks->g[0] = beta;
  ks->tol = fmax(tol_abs, tol_rel * beta);
  ks->flag = isfinite(beta) ? 0 : 2;
  ks->done = (!isfinite(beta) || beta <= ks->tol) ? 1 : 0;
  ks->solved = (!isfinite(beta) || beta <= tol_abs) ? 1 : 0;
  if (mode == 1) ks->sc[0] = beta > 0.0 ? 1.0 / beta : 0.0;
  if (mode == 2) ks->sc[0] = 1.0;
}

// ---------------------------------------------------------------------------
// vector helpers
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_copy(int N, double* __restrict__ d, const double* __restrict__ s) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) d[i] = s[i];
}

__global__ __launch_bounds__(kBlock) void k_set_dirichlet(int N, double* __restrict__ u,
                                                          const uint8_t* __restrict__ is_dir,
                                                          const double* __restrict__ uD) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock)
    if (is_dir[i]) u[i] = uD[i];
}

__global__ __launch_bounds__(kBlock) void k_rhs_dirichlet(int N, double* __restrict__ b, const double* __restrict__ F,
                                                          const uint8_t* __restrict__ is_dir,
                                                          const double* __restrict__ uD) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) b[i] = is_dir[i] ? uD[i] : F[i];
}

__global__ __launch_bounds__(kBlock) void k_fill(int N, double* __restrict__ u, double v) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) u[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_norm2(int N, const double* __restrict__ x, KState* ks, int idx,
                                                  double* partials) {
  double acc[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) acc[0] += x[i] * x[i];
  block_partials<1>(acc, 1, partials, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_relax(int N, double* __restrict__ u, const double* __restrict__ x,
                                                  double omega) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) u[i] += omega * (x[i] - u[i]);
}

// ---------------------------------------------------------------------------
// System matrix scale A_low + M_L/dt (Dirichlet rows identity): the CN matrix
// M_L/dt + A_low/2, or A_low itself (scale 1, no mass term)
// ---------------------------------------------------------------------------

template <int G>
__global__ __launch_bounds__(kBlock) void k_build_cn(int N, const int* __restrict__ rp, const int* __restrict__ col,
                                                     const double* __restrict__ AL, const double* __restrict__ ml,
                                                     const uint8_t* __restrict__ is_dir, double scale,
                                                     double inv_dt, double* __restrict__ Acn,
                                                     double* __restrict__ dinv) {
  constexpr int RPB = kBlock / G;
  const int lane = threadIdx.x % G, sub = threadIdx.x / G;
  int t0, t1;
  tile_range((N + RPB - 1) / RPB, t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int i = t * RPB + sub;
    if (i >= N) continue;
    const bool dir = is_dir[i];
    const int e = rp[i + 1];
    for (int k = rp[i] + lane; k < e; k += G) {
      const int j = col[k];
      double v;
      if (dir) {
        v = (j == i) ? 1.0 : 0.0;
      } else {
        v = scale * AL[k];
        if (j == i) v += ml[i] * inv_dt;
      }
      Acn[k] = v;
      if (j == i) dinv[i] = 1.0 / v;
    }
  }
}


__global__ void k_cycle_start(KState* ks, int mode, int idx, double tol_abs, double tol_rel) {
  if (threadIdx.x == 0 && blockIdx.x == 0) cycle_start_dev(ks, mode, ks->red[idx], tol_abs, tol_rel);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cast_v0(int N, const double* __restrict__ r, T* __restrict__ V0,
                                                    const KState* __restrict__ ks) {
  if (ks->solved) return;
  const double beta = ks->beta;
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) V0[i] = (T)(r[i] * inv);
}

// Givens step for Arnoldi column k, called by every thread of one workgroup:
// the column and the previous rotations are staged in LDS in parallel
// (givens_stage, which needs no reduction result and so can be issued early),
// one thread applies the rotation chain carrying the running entry in a
// register, and the updated column is written back in parallel.
struct GivensLds {
  double col[kMaxRestart + 1], c[kMaxRestart], sgn[kMaxRestart];
};

__device__ void givens_stage(const KState* ks, int k, int m, GivensLds& L) {
  const double* Hk = ks->H + (size_t)k * (m + 1);
  for (int q = threadIdx.x; q <= k; q += blockDim.x) L.col[q] = Hk[q];
  for (int q = threadIdx.x; q < k; q += blockDim.x) {
    L.c[q] = ks->cs[q];
    L.sgn[q] = ks->sn[q];
  }
}

// after givens_stage and a workgroup barrier
__device__ void givens_apply(KState* ks, int k, int m, double hk1sq, GivensLds& L) {
  double* Hk = ks->H + (size_t)k * (m + 1);
  if (threadIdx.x == 0) {
    const double hk1 = sqrt(hk1sq);
    if (!isfinite(hk1)) {
      ks->flag = 2;
      ks->done = 1;
    } else {
      ks->sc[k + 1] = hk1 > 0.0 ? 1.0 / hk1 : 0.0;
      double cur = L.col[0];
      for (int jj = 0; jj < k; ++jj) {
        const double nxt = L.col[jj + 1];
        L.col[jj] = L.c[jj] * cur + L.sgn[jj] * nxt;
        cur = -L.sgn[jj] * cur + L.c[jj] * nxt;
      }
      const double den = hypot(cur, hk1);
      if (den == 0.0) {  // w = 0 in exact arithmetic: the column adds nothing
        ks->done = 1;
        L.col[k] = cur;
        L.col[k + 1] = hk1;
      } else {
        const double cs = cur / den, sn = hk1 / den;
        ks->cs[k] = cs;
        ks->sn[k] = sn;
        L.col[k] = den;
        L.col[k + 1] = 0.0;
        const double gk = ks->g[k];
        ks->g[k + 1] = -sn * gk;
        ks->g[k] = cs * gk;
        ks->k = k + 1;
        ks->iters += 1;
        ks->res = fabs(ks->g[k + 1]);
        if (ks->res <= ks->tol || hk1 == 0.0) ks->done = 1;
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q <= k + 1; q += blockDim.x) Hk[q] = L.col[q];
}

__device__ void givens_step(KState* ks, int k, int m, double hk1sq) {
  __shared__ GivensLds L;
  givens_stage(ks, k, m, L);
  __syncthreads();
  givens_apply(ks, k, m, hk1sq, L);
}

// ---------------------------------------------------------------------------
// SELL-64: one wave per 64-row slice, one row per lane.  Entry p of the
// slice's rows lies at slot base + 64 p + lane, so value loads are contiguous
// across the wave.  Column deltas j - i come in two forms:
//   * uniform slice (sl_dl < 0): every row of the slice uses the same delta
//     for slot p, held once in the shared pattern table at ~sl_dl; the slice
//     index is wave-uniform, so those reads are scalar loads and a wave's
//     gathers x[i + delta] cover 64 consecutive addresses;
//   * other slices: one delta per slot (int16 or int32) at sl_dl + 64 p + lane.
// Padding slots hold value 0 and an in-range delta.  Rows accumulate in
// registers; no LDS and no shuffles.
// ---------------------------------------------------------------------------

struct SellView {
  int N, nsl;
  const int* __restrict__ sl_ptr;
  const int* __restrict__ sl_dl;
  const int* __restrict__ pat;
};

// slice handled by this wave in tile t (wave-uniform by construction)
__device__ __forceinline__ int wave_slice(int t) {
  return t * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// sum_p val[p] * X(i + delta_p) over the row of lane i in slice s
template <int U, typename TI, typename TA, typename XF>
__device__ __forceinline__ TA sell_row(const SellView& S, const TI* __restrict__ dlt, const TA* __restrict__ val,
                                       int s, int i, XF xf) {
  const int b = S.sl_ptr[s];
  const int L = (S.sl_ptr[s + 1] - b) >> 6;
  const int doff = S.sl_dl[s];
  const TA* __restrict__ v = val + b + (i & 63);
  TA acc = TA(0);
  if (doff < 0) {
    const int* __restrict__ pp = S.pat + ~doff;
    int p = 0;
    for (; p + U <= L; p += U) {
      TA a[U], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = v[64 * (p + u)];
        xv[u] = xf(i + pp[p + u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += a[u] * xv[u];
    }
    for (; p < L; ++p) acc += v[64 * p] * xf(i + pp[p]);
  } else {
    const TI* __restrict__ d = dlt + doff + (i & 63);
    int p = 0;
    for (; p + U <= L; p += U) {
      int j[U];
      TA a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        j[u] = i + d[64 * (p + u)];
        a[u] = v[64 * (p + u)];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += a[u] * xf(j[u]);
    }
    for (; p < L; ++p) acc += v[64 * p] * xf(i + d[64 * p]);
  }
  return acc;
}

// Lane shifts with an edge value: lane l takes lane l - 1's value and lane 0
// the edge value (or lane l + 1's and lane 63 the edge).  The edge value is
// put into the lane that wraps around (63, or 0) and the whole wave is rotated
// by one (DPP wave_ror:1 / wave_rol:1), so every lane reads an active lane and
// no select follows the move.  (A select after a shift was lowered by running
// the move with the edge lane masked off; a DPP read from a disabled lane
// counts as out of range, and its neighbour then read 0.)
__device__ __forceinline__ int rot_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x13C, 0xf, 0xf, false); }
__device__ __forceinline__ int rot_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xf, 0xf, false); }
__device__ __forceinline__ double lane_from_prev(double v, double edge, int lane) {  // lane 0: edge
  const long long b = __builtin_bit_cast(long long, lane == 63 ? edge : v);
  const int lo = rot_prev((int)b), hi = rot_prev((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_from_next(double v, double edge, int lane) {  // lane 63: edge
  const long long b = __builtin_bit_cast(long long, lane == 0 ? edge : v);
  const int lo = rot_next((int)b), hi = rot_next((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_double(double v, int l) {  // lane l's value, wave-uniform
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Stencil runs.  A full uniform slice whose 27 offsets are nine runs
// (c - 1, c, c + 1) in slot order (the trilinear stencil with its diagonal)
// forms X(i + c) once per run in each lane and takes the two neighbours'
// values from the adjacent lanes; lane 0's X(i - 1 + c) and lane 63's
// X(i + 1 + c) of the nine runs come from one 18-lane load.  Every index used
// is one of the row's own column indices, which the layout keeps in range for
// every row of a uniform slice.  X is formed as sell_row forms it (x_j, or a
// product such as D^{-1}_j x_j) and products are added in slot order, so the
// sums equal sell_row's bitwise.  The whole wave must be active.
//
// slice_runs27: whether slice s has that form (wave-uniform), and its centres
__device__ __forceinline__ bool slice_runs27(const SellView& S, int s, int (&c)[9]) {
  const int doff = S.sl_dl[s];
  bool runs = doff < 0 && s * 64 + 64 <= S.N && S.sl_ptr[s + 1] - S.sl_ptr[s] == 64 * 27;
  if (runs) {
    const int* __restrict__ pp = S.pat + ~doff;
#pragma unroll
    for (int w = 0; w < 9; ++w) {
      c[w] = pp[3 * w + 1];
      runs = runs && pp[3 * w] == c[w] - 1 && pp[3 * w + 2] == c[w] + 1;
    }
  }
  return runs;
}
// sell_row27_runs: sum_p val[p] X(i + delta_p) for such a slice, vs its first slot
template <typename XF>
__device__ __forceinline__ double sell_row27_runs(const double* __restrict__ vs, const int (&c)[9], int i0, int lane,
                                                    XF xf) {
  int ce = c[0];
#pragma unroll
  for (int w = 1; w < 9; ++w) ce = (lane >> 1) == w ? c[w] : ce;
  double ev = 0.0;
  if (lane < 18) ev = xf(i0 + ce + ((lane & 1) ? 64 : -1));
  double a[27], xc[9];
#pragma unroll
  for (int w = 0; w < 9; ++w) xc[w] = xf(i0 + lane + c[w]);
#pragma unroll
  for (int q = 0; q < 27; ++q) a[q] = vs[(unsigned)(lane + 64 * q)];
  double acc = 0.0;
#pragma unroll
  for (int w = 0; w < 9; ++w) {
    const double el = lane_double(ev, 2 * w), er = lane_double(ev, 2 * w + 1);
    const double l = lane_from_prev(xc[w], el, lane), r = lane_from_next(xc[w], er, lane);
    acc += a[3 * w] * l;
    acc += a[3 * w + 1] * xc[w];
    acc += a[3 * w + 2] * r;
  }
  return acc;
}

// FP32: y = A x (Jacobi-scaled FP32 matrix, unscaled basis vector)
// y = A x - theta x (theta != 0: the shifted powers of s-step GMRES), A the
// Jacobi-scaled matrix stored without its diagonal (all ones): the diagonal
// term is (1 - theta) x_i.  rev = 1 sweeps every XCD's slab backwards:
// back-to-back SpMVs that alternate direction start on the matrix tiles the
// previous one read last, which the memory-side cache still holds.
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_sell_spmv32(SellView S, const TI* __restrict__ dlt,
                                                        const float* __restrict__ val, const float* __restrict__ x,
                                                        const KState* __restrict__ ks, float theta, int rev,
                                                        float* __restrict__ y) {
  if (ks->done) return;
  const int nt = (S.nsl + kBlock / 64 - 1) / (kBlock / 64);
  int t0, t1;
  if (rev)
    tile_range_rev(nt, t0, t1);
  else
    tile_range(nt, t0, t1);
  for (int tt = t0; tt < t1; ++tt) {
    const int t = rev ? t1 - 1 - (tt - t0) : tt;
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int i = s * 64 + (threadIdx.x & 63);
    if (i >= S.N) continue;
    float acc = sell_row<8>(S, dlt, val, s, i, [&](int j) { return x[j]; });
    if (theta != 1.0f) acc += (1.0f - theta) * x[i];
    __builtin_nontemporal_store(acc, y + i);
  }
}

// FP64: y = A (sc .* x); theta != 0: y = A (sc .* x) - theta x (the shifted
// powers of s-step GMRES with sc = D^{-1}); rev as in k_sell_spmv32
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_sell_spmv64(SellView S, const TI* __restrict__ dlt,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ sc, const double* __restrict__ x,
                                                        const KState* __restrict__ ks, double theta, int rev,
                                                        double* __restrict__ y) {
  if (ks->done) return;
  const int nt = (S.nsl + kBlock / 64 - 1) / (kBlock / 64);
  int t0, t1;
  if (rev)
    tile_range_rev(nt, t0, t1);
  else
    tile_range(nt, t0, t1);
  for (int tt = t0; tt < t1; ++tt) {
    const int t = rev ? t1 - 1 - (tt - t0) : tt;
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int i = s * 64 + (threadIdx.x & 63);
    const auto xf = [&](int j) { return sc[j] * x[j]; };
    int c[9];
    double acc;
    if (slice_runs27(S, s, c)) {  // wave-uniform; a full slice, every lane has a row
      acc = sell_row27_runs(val + S.sl_ptr[s], c, s * 64, i & 63, xf);
    } else {
      if (i >= S.N) continue;
      acc = sell_row<8>(S, dlt, val, s, i, xf);
    }
    if (theta != 0.0) acc -= theta * x[i];
    y[i] = acc;
  }
}

// r = b - A x (FP64) with ||r||^2 partials
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_sell_residual(SellView S, const TI* __restrict__ dlt,
                                                          const double* __restrict__ val,
                                                          const double* __restrict__ bvec,
                                                          const double* __restrict__ x, double* __restrict__ r,
                                                          double* partials, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a cycle queued after the solve converged
  double nrm[1] = {0.0};
  int t0, t1;
  tile_range((S.nsl + kBlock / 64 - 1) / (kBlock / 64), t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int i = s * 64 + (threadIdx.x & 63);
    // full uniform slices with the 27-offset run pattern take the x values by
    // runs (every lane of the wave is active there); the rest gathers
    const auto xf = [&](int j) { return x[j]; };
    int c[9];
    double ax;
    if (slice_runs27(S, s, c)) {  // wave-uniform; a full slice, every lane has a row
      ax = sell_row27_runs(val + S.sl_ptr[s], c, s * 64, i & 63, xf);
    } else {
      if (i >= S.N) continue;
      ax = sell_row<8>(S, dlt, val, s, i, xf);
    }
    const double ri = bvec[i] - ax;
    r[i] = ri;
    nrm[0] += ri * ri;
  }
  block_partials<1>(nrm, 1, partials, blockIdx.x);
}

// CSR values -> SELL slots (padding slots were zeroed at allocation)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_sell(int nnz, const int* __restrict__ pos, const T* __restrict__ src,
                                                    T* __restrict__ dst) {
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < nnz; k += gridDim.x * kBlock) dst[pos[k]] = src[k];
}

__global__ __launch_bounds__(kBlock) void k_to_sell_scaled32(int nnz, const int* __restrict__ pos,
                                                             const int* __restrict__ col,
                                                             const double* __restrict__ src,
                                                             const double* __restrict__ dinv,
                                                             float* __restrict__ dst) {
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < nnz; k += gridDim.x * kBlock)
    if (pos[k] >= 0) dst[pos[k]] = (float)(src[k] * dinv[col[k]]);
}

// ---------------------------------------------------------------------------
// GMRES: classical Gram-Schmidt with unnormalized basis vectors V[j] and
// scales sc_j (v_j = sc_j V[j]); Givens rotations on the device.
// ---------------------------------------------------------------------------

// 16-byte vector access with a scalar tail (basis vectors use a padded,
// 16-byte aligned stride ldv; the tail guard keeps every access below N).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
};
template <>
struct Vec16<double> {
  using type = double2;
};

template <typename T>
__device__ __forceinline__ void load16(const T* __restrict__ p, int e, int N, T (&out)[16 / sizeof(T)]) {
  constexpr int VN = 16 / sizeof(T);
  if (e + VN <= N) {
    const typename Vec16<T>::type v = *reinterpret_cast<const typename Vec16<T>::type*>(p + e);
    __builtin_memcpy(out, &v, 16);
  } else {
#pragma unroll
    for (int c = 0; c < VN; ++c) out[c] = (e + c < N) ? p[e + c] : T(0);
  }
}

template <typename T>
__device__ __forceinline__ void store16(T* __restrict__ p, int e, int N, const T (&in)[16 / sizeof(T)]) {
  constexpr int VN = 16 / sizeof(T);
  if (e + VN <= N) {
    typename Vec16<T>::type v;
    __builtin_memcpy(&v, in, 16);
    *reinterpret_cast<typename Vec16<T>::type*>(p + e) = v;
  } else {
#pragma unroll
    for (int c = 0; c < VN; ++c)
      if (e + c < N) p[e + c] = in[c];
  }
}

// Arnoldi step k (classical Gram-Schmidt) as four launches:
//   SpMV      W = A V[k]                          (unscaled basis vector)
//   dots      per-workgroup partials of (V[q], W), q = 0..k
//   reduce    h_{q,k} = sc_q sc_k (V[q], W); workgroup k + 1 also finishes
//             step k - 1 (norm of V[k] -> Givens rotation of column k - 1)
//   update    V[k+1] = sc_k W - sum_q h_{q,k} sc_q V[q] and its squared norm
// The vector kernels use 256-thread workgroups, one 16-byte access per
// thread and vector per chunk, so that a launch fills every SIMD with waves.
// (Projections taken inside the SpMV, slice by slice, measured slower: their
// 4-byte-per-lane basis reads cannot stream like the 16-byte chunks here.)

// Raw projections (V[q], W), q = 0..k: per-wave sums accumulate in LDS
// (double), one partial per workgroup and row.  Eight basis vectors are
// loaded together and their eight products reduced over the wave at once.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gmres_dots(int N, int ldv, const T* __restrict__ V,
                                                     const T* __restrict__ W, int k, const KState* __restrict__ ks,
                                                     double* __restrict__ partials) {
  if (ks->done) return;
  constexpr int VN = 16 / sizeof(T);
  constexpr int CH = kBlock * VN;
  constexpr int NW = kBlock / 64;
  constexpr int QU = 8;  // one eight-value wave reduction per group of basis vectors
  __shared__ double sh[kMaxRestart + 1][NW];
  const int nv = k + 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int p = lane >> 3;  // the vector of the group whose wave total this lane receives
  for (int q = threadIdx.x; q < nv * NW; q += kBlock) sh[q / NW][q % NW] = 0.0;
  __syncthreads();
  for (int base = blockIdx.x * CH; base < N; base += gridDim.x * CH) {
    const int e = base + threadIdx.x * VN;
    T w[VN];
    load16(W, e, N, w);
    for (int q = 0; q < nv; q += QU) {
      T a[QU][VN];
#pragma unroll
      for (int u = 0; u < QU; ++u) {
#pragma unroll
        for (int c = 0; c < VN; ++c) a[u][c] = T(0);
        if (q + u < nv) load16(V + (size_t)(q + u) * ldv, e, N, a[u]);
      }
      double v[QU];
#pragma unroll
      for (int u = 0; u < QU; ++u) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < VN; ++c) t += (double)a[u][c] * (double)w[c];
        v[u] = t;
      }
      const double x = wave_sum8(v);
      if ((lane & 7) == 0 && q + p < nv) sh[q + p][wv] += x;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nv; q += kBlock) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += sh[q][w];
    partials[(size_t)q * kRedBlocks + blockIdx.x] = t;
  }
}

// Fixed-order sums of the nb (<= kRedBlocks) partials of up to two rows by a
// whole workgroup; every load is issued before the first add.  Thread t adds
// slots t, t + kBlock, ... in order, then waves and lanes combine in a fixed
// order, so identical inputs give bitwise identical sums in every workgroup.
template <int NR>
__device__ void block_rows_sum(const double* const (&row)[NR], const int (&nb)[NR], double (&out)[NR]) {
  constexpr int PER = kRedBlocks / kBlock;
  static_assert(PER * kBlock == kRedBlocks, "partials per thread");
  __shared__ double sh[NR][kBlock / 64];
  double v[NR][PER];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = threadIdx.x + i * kBlock;
      v[r][i] = b < nb[r] ? row[r][b] : 0.0;
    }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < PER; ++i) s += v[r][i];
    s = wave_sum(s);
    if (lane == 0) sh[r][wv] = s;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += sh[r][w];
    out[r] = t;
  }
}

// Workgroup q <= k finalizes h_{q,k} = sc_q sc_k (V[q], W); for k > 0 it
// derives sc_k = 1 / ||V[k]|| itself from the norm partials of the previous
// update (same order everywhere, so the same value).  For k > 0 workgroup
// k + 1 applies the Givens rotation of column k - 1 (it stores sc_k and may end
// the cycle).
__global__ __launch_bounds__(kBlock) void k_gmres_reduce(KState* ks, const double* __restrict__ partials,
                                                       int nb_proj, int nb_norm, int k, int m) {
  const double* norm_row = partials + (size_t)kNormRow * kRedBlocks;
  const int q = blockIdx.x;
  if (q == k + 1) {
    __shared__ GivensLds L;
    if (ks->done) return;
    givens_stage(ks, k - 1, m, L);
    const double* const rows[1] = {norm_row};
    const int nbs[1] = {nb_norm};
    double nrm2[1];
    block_rows_sum<1>(rows, nbs, nrm2);
    givens_apply(ks, k - 1, m, nrm2[0], L);
    return;
  }
  // no early exit here: ks->done may change during this launch (workgroup
  // k + 1), and a column past the cycle's end is never read
  const double scq_prev = q < k ? ks->sc[q] : 0.0;
  double sck = ks->sc[0];
  double t;
  if (k > 0) {
    const double* const rows[2] = {norm_row, partials + (size_t)q * kRedBlocks};
    const int nbs[2] = {nb_norm, nb_proj};
    double sums[2];
    block_rows_sum<2>(rows, nbs, sums);
    const double hk = sqrt(sums[0]);
    sck = hk > 0.0 ? 1.0 / hk : 0.0;
    t = sums[1];
  } else {
    const double* const rows[1] = {partials + (size_t)q * kRedBlocks};
    const int nbs[1] = {nb_proj};
    double sums[1];
    block_rows_sum<1>(rows, nbs, sums);
    t = sums[0];
  }
  if (threadIdx.x == 0) {
    const double scq = q == k ? sck : scq_prev;
    const double h = scq * sck * t;
    ks->H[(size_t)k * (m + 1) + q] = h;
    ks->proj[q] = h * scq;
  }
}

// V[k+1] = sc_k W - sum_q proj_q V[q] and the partials of its squared norm.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gmres_update(int N, int ldv, T* __restrict__ V,
                                                       const T* __restrict__ W, int k,
                                                       const KState* __restrict__ ks, double* __restrict__ partials) {
  if (ks->done) return;
  constexpr int VN = 16 / sizeof(T);
  constexpr int CH = kBlock * VN;
  __shared__ double tq[kMaxRestart + 1];
  const int nv = k + 1;
  for (int q = threadIdx.x; q < nv; q += kBlock) tq[q] = ks->proj[q];
  const double sck = ks->sc[k];
  __syncthreads();
  T* __restrict__ out = V + (size_t)(k + 1) * ldv;
  double nrm[1] = {0.0};
  for (int base = blockIdx.x * CH; base < N; base += gridDim.x * CH) {
    const int e = base + threadIdx.x * VN;
    T w[VN];
    load16(W, e, N, w);
    double c[VN];
#pragma unroll
    for (int i = 0; i < VN; ++i) c[i] = sck * (double)w[i];
    int q = 0;
    for (; q + 4 <= nv; q += 4) {
      T a[4][VN];
#pragma unroll
      for (int u = 0; u < 4; ++u) load16(V + (size_t)(q + u) * ldv, e, N, a[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double t = tq[q + u];
#pragma unroll
        for (int i = 0; i < VN; ++i) c[i] -= t * (double)a[u][i];
      }
    }
    for (; q < nv; ++q) {
      T a[VN];
      load16(V + (size_t)q * ldv, e, N, a);
      const double t = tq[q];
#pragma unroll
      for (int i = 0; i < VN; ++i) c[i] -= t * (double)a[i];
    }
    T o[VN];
#pragma unroll
    for (int i = 0; i < VN; ++i) {
      o[i] = (T)c[i];
      nrm[0] += (double)o[i] * (double)o[i];
    }
    store16(out, e, N, o);
  }
  block_partials<1>(nrm, 1, partials + (size_t)kNormRow * kRedBlocks, blockIdx.x);
}

// ---------------------------------------------------------------------------
// s-step GMRES (mixed precision).  A block of s basis vectors comes from the
// shifted powers W_j = (A - theta I) W_{j-1}, W_0 = V[k] (stored at
// V[k+1..k+s]).  One pass over V[0..k] and the block forms C = V^T W and the
// Gram matrix W^T W; G = W^T W - C^T C is the Gram matrix of the projected
// block, whose Cholesky factor R gives the new orthonormal vectors
// Q = (W - V C) R^{-1} in one more pass.  The Hessenberg columns of the
// Arnoldi relation A [V_k, Q_1..Q_{s-1}] = [V, Q] H follow from the change of
// basis.  In exact arithmetic the iterates are those of GMRES.
// ---------------------------------------------------------------------------

// row of the Gram entry (i, j), i <= j < s, after the (k+1) s rows of C
__device__ __forceinline__ int gram_row(int nv, int s, int i, int j) {
  return nv * s + i * s - i * (i - 1) / 2 + (j - i);
}

// Blocks of up to eight vectors: each thread holds the FP64 copies of its
// 16-byte chunk of W_1..W_s in registers; every row V_q and the Gram rows take
// one eight-value wave reduction per chunk, accumulated per wave in LDS.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sstep_dots(int N, int ldv, const T* __restrict__ V, int k, int s,
                                                     const KState* __restrict__ ks, double* __restrict__ partials) {
  if (ks->done) return;
  constexpr int VN = 16 / sizeof(T);
  constexpr int CH = kBlock * VN;
  constexpr int NW = kBlock / 64;
  constexpr int QU = 4;  // basis vectors loaded together (loads in flight)
  constexpr int HC = 8;  // block columns (one eight-value reduction per row)
  extern __shared__ double sh[];  // [row][NW]
  const int nv = k + 1;
  const int nrows = nv * s + s * (s + 1) / 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int p = lane >> 3;  // the product whose wave total this lane receives
  const bool writer = (lane & 7) == 0 && p < s;
  for (int q = threadIdx.x; q < nrows * NW; q += kBlock) sh[q] = 0.0;
  __syncthreads();
  const T* __restrict__ W = V + (size_t)(k + 1) * ldv;
  for (int base = blockIdx.x * CH; base < N; base += gridDim.x * CH) {
    const int e = base + threadIdx.x * VN;
    double w[HC][VN];
#pragma unroll
    for (int j = 0; j < HC; ++j) {
      T t[VN];
#pragma unroll
      for (int c = 0; c < VN; ++c) t[c] = T(0);
      if (j < s) load16(W + (size_t)j * ldv, e, N, t);
#pragma unroll
      for (int c = 0; c < VN; ++c) w[j][c] = (double)t[c];
    }
    // (V_q, W_j), j < s, for every q: one eight-value reduction per q
    for (int q0 = 0; q0 < nv; q0 += QU) {
      T a[QU][VN];
#pragma unroll
      for (int u = 0; u < QU; ++u)
        if (q0 + u < nv) load16(V + (size_t)(q0 + u) * ldv, e, N, a[u]);
#pragma unroll
      for (int u = 0; u < QU; ++u) {
        if (q0 + u < nv) {
          double v[HC];
#pragma unroll
          for (int j = 0; j < HC; ++j) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < VN; ++c) t += (double)a[u][c] * w[j][c];
            v[j] = t;
          }
          const double x = wave_sum8(v);
          if (writer) sh[((q0 + u) * s + p) * NW + wv] += x;
        }
      }
    }
    // Gram entries (W_i, W_j), i <= j < s: one reduction per i
#pragma unroll
    for (int i = 0; i < HC; ++i) {
      if (i < s) {
        double v[HC];
#pragma unroll
        for (int j = 0; j < HC; ++j) {
          double t = 0.0;
          if (j >= i) {
#pragma unroll
            for (int c = 0; c < VN; ++c) t += w[i][c] * w[j][c];
          }
          v[j] = t;
        }
        const double x = wave_sum8(v);
        if (writer && p >= i) sh[gram_row(nv, s, i, p) * NW + wv] += x;
      }
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < nrows; r += kBlock) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += sh[r * NW + w];
    partials[(size_t)r * kRedBlocks + blockIdx.x] = t;
  }
}

// The same projections as one tall-skinny product on the FP64 matrix cores
// (blocks of more than eight vectors): D = R^T [W_0..W_{s-1}] with the rows
// R = [W_0..W_{s-1}, V_0..V_k] in tiles of 16, accumulated over the elements
// by v_mfma_f64_16x16x4f64 (FP32 data converted to FP64: exact products,
// FP64 sums, no cross-lane reductions in the loop).  Lane l feeds row
// 16 t + (l & 15) of tile t and element group l >> 4; with W first, the
// column operand W_{l & 15} is tile 0's own row operand.  Each wave takes a
// contiguous range of 32-element chunks (eight consecutive elements per lane,
// two 16-byte loads per row) and loads the next chunk before multiplying the
// current one.  The four waves' tiles are summed in LDS in a fixed order.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <typename T, int NT>
__global__ __launch_bounds__(kBlock) void k_sstep_dots_mfma(int N, int ldv, const T* __restrict__ V, int k, int s,
                                                           const KState* __restrict__ ks,
                                                           double* __restrict__ partials) {
  if (ks->done) return;
  constexpr int EPL = 8;        // elements per lane and chunk
  constexpr int CE = 4 * EPL;   // elements per chunk
  constexpr int VN = 16 / sizeof(T);
  constexpr int NW = kBlock / 64;
  const int nv = k + 1, nr = nv + s;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const T* __restrict__ W = V + (size_t)(k + 1) * ldv;
  const T* rp[NT];
  bool rv[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = 16 * t + li;
    rv[t] = r < nr;
    rp[t] = r < s ? W + (size_t)r * ldv : (r < nr ? V + (size_t)(r - s) * ldv : V);
  }
  const bool bcol = li < s;
  mfma_d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  const int nch = (N + CE - 1) / CE;
  const int gw = blockIdx.x * NW + wv, nw = gridDim.x * NW;
  const int c0 = (int)((int64_t)gw * nch / nw), c1 = (int)((int64_t)(gw + 1) * nch / nw);
  auto load = [&](int c, T (&a)[NT][EPL]) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int f = 0; f < EPL / VN; ++f) {
        T q[VN];
#pragma unroll
        for (int x = 0; x < VN; ++x) q[x] = T(0);
        if (rv[t] && c < c1) load16(rp[t], c * CE + lk * EPL + VN * f, N, q);
#pragma unroll
        for (int x = 0; x < VN; ++x) a[t][VN * f + x] = q[x];
      }
  };
  T a[NT][EPL];
  load(c0, a);
  for (int c = c0; c < c1; ++c) {
    T an[NT][EPL];
    load(c + 1, an);
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const double b = bcol ? (double)a[0][e] : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[t][e], b, acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < EPL; ++e) a[t][e] = an[t][e];
  }
  // D[16 t + i][j] of this wave: lane j + 16 (i % 4), register i / 4
  __shared__ double sh[NW][NT * 256];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) sh[wv][(16 * t + lk + 4 * v) * 16 + li] = acc[t][v];
  __syncthreads();
  for (int q = threadIdx.x; q < NT * 256; q += kBlock) {
    const int r = q >> 4, j = q & 15;
    if (j >= s || r >= nr || (r < s && r > j)) continue;
    const int row = r < s ? gram_row(nv, s, r, j) : (r - s) * s + j;
    double x = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) x += sh[w][q];
    partials[(size_t)row * kRedBlocks + blockIdx.x] = x;
  }
}

// workgroup r sums partial row r of the block reduction into ks->blk[r]
__global__ __launch_bounds__(kBlock) void k_sstep_sums(KState* ks, const double* __restrict__ partials, int nb) {
  if (ks->done) return;
  const double* const rows[1] = {partials + (size_t)blockIdx.x * kRedBlocks};
  const int nbs[1] = {nb};
  double t[1];
  block_rows_sum<1>(rows, nbs, t);
  if (threadIdx.x == 0) ks->blk[blockIdx.x] = t[0];
}

// Cholesky QR of the projected block, update coefficients, Hessenberg
// columns k..k+s-1 and their Givens rotations (one workgroup).  The three
// chains of the block (Cholesky factor, its inverse, the block's rotations)
// run one column per lane of the first wave, with the pivots broadcast by
// readlane; every entry is formed by the same operations in the same order as
// a column-by-column loop on one thread would use.
template <int SM>
__global__ __launch_bounds__(kBlock) void k_sstep_small(KState* ks, int k, int s, int m, double theta) {
  static_assert(SM <= kSMax, "block size within the device state");
  constexpr int kRows = kMaxRestart + 1;                          // nr = k + 1 + s <= m + 1
  constexpr int kHLd = kMaxRestart * (kMaxRestart + 1);           // staged index range (c, r), r <= k
  constexpr int kHLU = (kHLd + kBlock - 1) / kBlock;
  constexpr int kHL = (kMaxRestart - 1) * (kMaxRestart + 2) / 2;  // banded: column c < k holds rows 0..c+1
  constexpr int kBU = (kBlkRows + kBlock - 1) / kBlock;
  __shared__ double B[kBlkRows];  // the block's reduced rows: C[q s + j] = (V_q, W_{j+1}), then W^T W
  __shared__ double G[SM * SM], R[SM * SM], Ri[SM * SM];
  __shared__ double Z[kRows * (SM + 1)];  // coordinates of W_0..W_s in [V_0..V_k, Q_1..Q_s]
  __shared__ double M1[kRows * SM];
  __shared__ double Hn[kRows * SM];       // new Hessenberg columns k..k+s-1
  __shared__ double HL[kHL];                 // raw Hessenberg columns 0..k-1, column c at c (c + 3) / 2
  __shared__ double gcs[kMaxRestart], gsn[kMaxRestart], gg[kMaxRestart + 1];  // rotations and rhs, staged
  __shared__ double rdiag[SM];               // 1 / R_jj
  __shared__ int ok, ncols, stop, nonfinite;
  const int nv = k + 1, nr = nv + s;
  const int nrows = nv * s + s * (s + 1) / 2;
  const double* C = B;
  {  // every global read of the kernel in flight at once, the done flag included
    const int was_done = ks->done;
    double hv[kHLU], bv[kBU];
#pragma unroll
    for (int u = 0; u < kHLU; ++u) {
      const int t = threadIdx.x + u * kBlock;
      hv[u] = 0.0;
      if (t < k * (k + 1)) {  // column c, rows 0..k
        const int c = t / (k + 1), r = t % (k + 1);
        if (r <= c + 1) hv[u] = ks->Hraw[(size_t)c * (m + 1) + r];
      }
    }
#pragma unroll
    for (int u = 0; u < kBU; ++u) {
      const int t = threadIdx.x + u * kBlock;
      bv[u] = t < nrows ? ks->blk[t] : 0.0;
    }
    const int t = threadIdx.x;
    double cs0 = 0.0, sn0 = 0.0, g0 = 0.0;
    if (t < k) {
      cs0 = ks->cs[t];
      sn0 = ks->sn[t];
    }
    if (t <= k) g0 = ks->g[t];
    __syncthreads();  // every thread has read done before thread 0 may set it below
    if (was_done) {
      if (threadIdx.x == 0) ks->blk_ok = 0;
      return;
    }
#pragma unroll
    for (int u = 0; u < kHLU; ++u) {
      const int t = threadIdx.x + u * kBlock;
      if (t < k * (k + 1)) {
        const int c = t / (k + 1), r = t % (k + 1);
        if (r <= c + 1) HL[c * (c + 3) / 2 + r] = hv[u];
      }
    }
#pragma unroll
    for (int u = 0; u < kBU; ++u)
      if (threadIdx.x + u * kBlock < nrows) B[threadIdx.x + u * kBlock] = bv[u];
    if (t < k) {
      gcs[t] = cs0;
      gsn[t] = sn0;
    }
    if (t <= k) gg[t] = g0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < s * s; t += blockDim.x) {  // G = W^T W - C^T C
    const int i = t / s, j = t % s;
    double g = B[gram_row(nv, s, min(i, j), max(i, j))];
    for (int q = 0; q < nv; ++q) g -= C[q * s + i] * C[q * s + j];
    G[t] = g;
  }
  __syncthreads();
  // G = R^T R with R upper triangular (left-looking), then R^{-1}, in the
  // first wave: lane i holds column i of G and of R.  At step j every lane
  // reads column j of R (rows p < j, written to LDS by the earlier steps) and
  // the pivot G_jj as broadcasts, forms R_jj and 1 / R_jj itself, and lane
  // i > j its entry R_ji; row j of R then goes to LDS.  The wave's LDS
  // accesses take effect in program order, so no barrier is needed between
  // steps.  Lane j then solves for column j of R^{-1} by back substitution
  // with the reciprocal pivots (no division on the chain).
  if (threadIdx.x < 64) {
    const int i = threadIdx.x;
    double gc[SM], rc[SM], dinv[SM];
#pragma unroll
    for (int p = 0; p < SM; ++p) {
      gc[p] = (i < s && p < s) ? G[p * s + i] : 0.0;
      rc[p] = 0.0;
      dinv[p] = 0.0;
    }
    bool good = true;  // the same on every lane: formed from broadcast values only
#pragma unroll
    for (int j = 0; j < SM; ++j) {
      if (j < s) {
        double rpj[SM];
#pragma unroll
        for (int p = 0; p < j; ++p) rpj[p] = R[p * s + j];
        double d = G[j * s + j], v = gc[j];
#pragma unroll
        for (int p = 0; p < j; ++p) {
          d -= rpj[p] * rpj[p];
          v -= rpj[p] * rc[p];
        }
        good = good && d > 0.0 && isfinite(d);
        const double rjj = sqrt(d);
        dinv[j] = 1.0 / rjj;
        rc[j] = i == j ? rjj : (i > j ? v * dinv[j] : 0.0);
        if (i < s) R[j * s + i] = rc[j];
      }
    }
    if (i == 0) ok = good;
    if (good && i == 0) {
#pragma unroll
      for (int p = 0; p < SM; ++p)
        if (p < s) rdiag[p] = dinv[p];
    }
    if (good) {
      // column i of R^{-1}: entries below the diagonal stay 0, entries above
      // by back substitution; rows of R beyond s read as 0
      double ric[SM];
#pragma unroll
      for (int p = 0; p < SM; ++p) ric[p] = p == i ? dinv[p] : 0.0;
#pragma unroll
      for (int r = SM - 2; r >= 0; --r) {
        if (r < s - 1) {
          double v = 0.0;
#pragma unroll
          for (int p = r + 1; p < SM; ++p) v += (p < s ? R[r * s + p] : 0.0) * ric[p];
          ric[r] = r < i ? -v * dinv[r] : ric[r];
        }
      }
      if (i < s) {
#pragma unroll
        for (int r = 0; r < SM; ++r)
          if (r < s) Ri[r * s + i] = ric[r];
      }
    }
  }
  __syncthreads();
  if (!ok) {
    if (threadIdx.x == 0) {
      ks->blk_ok = 0;
      ks->sfail += 1;  // sticky count of failed blocks (the host halves the block size)
      ks->done = 1;
    }
    return;
  }
  // update coefficients: Q = W R^{-1} - V (C R^{-1})
  for (int t = threadIdx.x; t < nv * s; t += blockDim.x) {
    const int q = t / s, j = t % s;
    double v = 0.0;
    for (int i = 0; i <= j; ++i) v += C[q * s + i] * Ri[i * s + j];
    ks->dco[t] = v;
  }
  for (int t = threadIdx.x; t < s * s; t += blockDim.x) ks->rinv[t] = Ri[t];
  for (int t = threadIdx.x; t < nr * (s + 1); t += blockDim.x) {
    const int r = t / (s + 1), c = t % (s + 1);
    double v;
    if (c == 0)
      v = r == k ? 1.0 : 0.0;
    else if (r < nv)
      v = C[r * s + (c - 1)];
    else
      v = R[(r - nv) * s + (c - 1)];
    Z[t] = v;
  }
  __syncthreads();
  // A W_{j} = W_{j+1} + theta W_j: A [V Z_{:, 0..s-1}] = V (Z B); split the
  // left side into A V_{0..k-1} E (known: the raw Hessenberg) and A X T with
  // X = [V_k, Q_1..Q_{s-1}], T = Z[k..k+s-1, 0..s-1] upper triangular
  for (int t = threadIdx.x; t < nr * s; t += blockDim.x) {
    const int r = t / s, j = t % s;
    double v = theta * Z[r * (s + 1) + j] + Z[r * (s + 1) + j + 1];
    if (r <= k)
      for (int c = max(r - 1, 0); c < k; ++c) v -= HL[c * (c + 3) / 2 + r] * Z[c * (s + 1) + j];
    M1[t] = v;
  }
  __syncthreads();
  if (threadIdx.x < nr) {  // Hn = M1 T^{-1}, one row per thread, the row in registers
    const int r = threadIdx.x;
    double h[SM];
#pragma unroll
    for (int j = 0; j < SM; ++j) {
      if (j < s) {
        double v = M1[r * s + j];
#pragma unroll
        for (int i = 0; i < j; ++i) v -= h[i] * Z[(k + i) * (s + 1) + j];
        h[j] = j == 0 ? v : v * rdiag[j - 1];  // T_00 = 1, T_jj = R_{j-1,j-1}
        Hn[r * s + j] = h[j];
      }
    }
  }
  __syncthreads();
  const int ns = min(s, m - k);
  for (int t = threadIdx.x; t < ns * nr; t += blockDim.x) {
    const int j = t / nr, r = t % nr;
    if (r <= k + j + 1) ks->Hraw[(size_t)(k + j) * (m + 1) + r] = Hn[r * s + j];
  }
  __syncthreads();  // the raw columns are stored before the rotations change Hn
  // rotations 0..k-1 of earlier blocks, one thread per new column, eight at a time
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    double* col = Hn + j;  // column j of Hn, stride s
    double cur = col[0];
    int jj = 0;
    for (; jj + 8 <= k; jj += 8) {
      double nx[8], c8[8], s8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        nx[u] = col[(jj + u + 1) * s];
        c8[u] = gcs[jj + u];
        s8[u] = gsn[jj + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        col[(jj + u) * s] = c8[u] * cur + s8[u] * nx[u];
        cur = -s8[u] * cur + c8[u] * nx[u];
      }
    }
    for (; jj < k; ++jj) {
      const double nxt = col[(jj + 1) * s];
      col[jj * s] = gcs[jj] * cur + gsn[jj] * nxt;
      cur = -gsn[jj] * cur + gcs[jj] * nxt;
    }
    col[k * s] = cur;
  }
  __syncthreads();
  // rotations of this block: lane j holds rows k..k+s of new column j; at
  // step t the rotation of column t (lane t's two leading rows, broadcast)
  // is formed, stored, and applied to every later column
  if (threadIdx.x < 64) {
    const int j = threadIdx.x;
    const bool mine = j < ns;
    double v[SM + 1];
#pragma unroll
    for (int r = 0; r <= SM; ++r) v[r] = (mine && k + r < nr) ? Hn[(k + r) * s + j] : 0.0;
    const double tol = ks->tol;
    double gk = gg[k];
    int st = 0, nf = 0, nc = 0;
#pragma unroll
    for (int t = 0; t < SM; ++t) {
      if (t < ns && !st) {
        const double cur = lane_value(v[t], t);
        const double hk1 = lane_value(v[t + 1], t);
        const double den = sqrt(fma(cur, cur, hk1 * hk1));  // |H| entries are O(||A|| beta): no overflow
        if (!isfinite(den)) {
          nf = 1;
          st = 1;
        } else if (den == 0.0) {  // the new direction adds nothing: the column stays as rotated
          st = 1;
        } else {
          const double inv = 1.0 / den;
          const double cs = cur * inv, sn = hk1 * inv;
          const double a = v[t], b = v[t + 1];
          const bool later = j > t && mine;
          v[t] = j == t ? den : (later ? cs * a + sn * b : a);
          v[t + 1] = j == t ? 0.0 : (later ? -sn * a + cs * b : b);
          const double gn = -sn * gk;
          if (j == 0) {
            gcs[k + t] = cs;
            gsn[k + t] = sn;
            gg[k + t + 1] = gn;
            gg[k + t] = cs * gk;
          }
          gk = gn;
          nc = t + 1;
          if (fabs(gn) <= tol) st = 1;
        }
      }
    }
#pragma unroll
    for (int r = 0; r <= SM; ++r)
      if (mine && k + r < nr) Hn[(k + r) * s + j] = v[r];
    if (j == 0) {
      ncols = nc;  // columns completed by this block
      stop = st;
      nonfinite = nf;
    }
  }
  __syncthreads();
  // write back the rotated columns, rotations and right-hand side
  const int nc = ncols;
  for (int t = threadIdx.x; t < nc * nr; t += blockDim.x) {
    const int j = t / nr, r = t % nr;
    if (r <= k + j + 1) ks->H[(size_t)(k + j) * (m + 1) + r] = Hn[r * s + j];
  }
  for (int j = threadIdx.x; j < nc; j += blockDim.x) {
    ks->cs[k + j] = gcs[k + j];
    ks->sn[k + j] = gsn[k + j];
    ks->sc[k + j + 1] = 1.0;
  }
  for (int i = threadIdx.x; i <= k + nc; i += blockDim.x) ks->g[i] = gg[i];
  if (threadIdx.x == 0) {
    ks->blk_ok = 1;
    ks->k = k + nc;
    ks->iters += nc;
    ks->res = fabs(gg[k + nc]);
    if (nonfinite) ks->flag = 2;
    if (stop) ks->done = 1;
  }
}

// Q = W R^{-1} - V (C R^{-1}), in place over the block V[k+1..k+s] (blocks of
// up to eight vectors).  The basis part is summed first and W read last, so
// that W and the accumulators are not live together.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sstep_update(int N, int ldv, T* __restrict__ V, int k, int s,
                                                       const KState* __restrict__ ks) {
  constexpr int VN = 16 / sizeof(T);
  constexpr int CH = kBlock * VN;
  constexpr int QU = 4;  // basis vectors loaded together
  constexpr int HC = 8;  // output columns
  __shared__ double D[(kMaxRestart + 1) * HC], Ri[HC * HC];
  __shared__ int okb;
  if (threadIdx.x == 0) okb = ks->blk_ok;
  __syncthreads();
  if (!okb) return;
  const int nv = k + 1;
  for (int t = threadIdx.x; t < nv * s; t += kBlock) D[t] = ks->dco[t];
  for (int t = threadIdx.x; t < s * s; t += kBlock) Ri[t] = ks->rinv[t];
  __syncthreads();
  T* __restrict__ W = V + (size_t)(k + 1) * ldv;
  for (int base = blockIdx.x * CH; base < N; base += gridDim.x * CH) {
    const int e = base + threadIdx.x * VN;
    double acc[HC][VN];
#pragma unroll
    for (int j = 0; j < HC; ++j)
#pragma unroll
      for (int c = 0; c < VN; ++c) acc[j][c] = 0.0;
    for (int q0 = 0; q0 < nv; q0 += QU) {
      T a[QU][VN];
#pragma unroll
      for (int u = 0; u < QU; ++u)
        if (q0 + u < nv) load16(V + (size_t)(q0 + u) * ldv, e, N, a[u]);
#pragma unroll
      for (int u = 0; u < QU; ++u) {
        if (q0 + u < nv) {
#pragma unroll
          for (int j = 0; j < HC; ++j)
            if (j < s) {
              const double d = D[(q0 + u) * s + j];
#pragma unroll
              for (int c = 0; c < VN; ++c) acc[j][c] -= d * (double)a[u][c];
            }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < HC; ++i)
      if (i < s) {
        T w[VN];
        load16(W + (size_t)i * ldv, e, N, w);
#pragma unroll
        for (int j = 0; j < HC; ++j)
          if (i <= j && j < s) {
            const double r = Ri[i * s + j];
#pragma unroll
            for (int c = 0; c < VN; ++c) acc[j][c] += r * (double)w[c];
          }
      }
#pragma unroll
    for (int j = 0; j < HC; ++j)
      if (j < s) {
        T o[VN];
#pragma unroll
        for (int c = 0; c < VN; ++c) o[c] = (T)acc[j][c];
        store16(W + (size_t)j * ldv, e, N, o);
      }
  }
}

// The same update for blocks of more than eight vectors, on the FP64 matrix
// cores: Q^T = Coef^T [W_0..W_{s-1}, V_0..V_k]^T with Coef = [R^{-1}; -C R^{-1}]
// (K = s + k + 1 rows, taken four at a time by v_mfma_f64_16x16x4f64).  A
// wave takes 64-element tiles; lane l loads four consecutive elements of row
// 4 g + (l >> 4) of each row group g at element 4 (l & 15) (256 contiguous
// bytes per row and load), and the four elements become the four MFMA
// chains x = 0..3, so that lane l ends with Q_{(l >> 4) + 4 v} at elements
// 4 (l & 15) + x and stores them as one 16-byte write per column.  Every row
// of a tile is read before the tile's in-place stores; waves own disjoint
// tiles.
template <typename T, int KG>
__global__ __launch_bounds__(kBlock) void k_sstep_update_mfma(int N, int ldv, T* __restrict__ V, int k, int s,
                                                             const KState* __restrict__ ks) {
  constexpr int NW = kBlock / 64;
  constexpr int VN = 16 / sizeof(T);
  if (!ks->blk_ok) return;
  const int nv = k + 1, K = s + nv;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  T* __restrict__ W = V + (size_t)(k + 1) * ldv;
  // A operand of row group g: Coef[4 g + lk][li]
  double cf[KG];
  const T* rp[KG];
  bool rv[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    const int r = 4 * g + lk;
    double c = 0.0;
    if (r < K && li < s) c = r < s ? (r <= li ? ks->rinv[r * s + li] : 0.0) : -ks->dco[(r - s) * s + li];
    cf[g] = c;
    rv[g] = r < K;
    rp[g] = r < s ? W + (size_t)r * ldv : (r < K ? V + (size_t)(r - s) * ldv : V);
  }
  const int ntile = (N + 63) / 64;
  const int gw = blockIdx.x * NW + wv, nw = gridDim.x * NW;
  const int t0 = (int)((int64_t)gw * ntile / nw), t1 = (int)((int64_t)(gw + 1) * ntile / nw);
  // rows of tile t (zeros past the wave's range); with up to eight row groups
  // the next tile is loaded before the current one is multiplied
  constexpr bool kPrefetch = KG <= 8;
  auto load_tile = [&](int t, T (&a)[KG][4]) {
    const int e = t * 64 + 4 * li;
#pragma unroll
    for (int g = 0; g < KG; ++g) {
#pragma unroll
      for (int x = 0; x < 4; ++x) a[g][x] = T(0);
      if (rv[g] && t < t1) {
#pragma unroll
        for (int f = 0; f < 4 / VN; ++f) {
          T q[VN];
          load16(rp[g], e + VN * f, N, q);
#pragma unroll
          for (int x = 0; x < VN; ++x) a[g][VN * f + x] = q[x];
        }
      }
    }
  };
  T an[KG][4];
  if (kPrefetch) load_tile(t0, an);
  for (int t = t0; t < t1; ++t) {
    const int e = t * 64 + 4 * li;
    T a[KG][4];
    if (kPrefetch) {
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int x = 0; x < 4; ++x) a[g][x] = an[g][x];
      load_tile(t + 1, an);
    } else {
      load_tile(t, a);
    }
    mfma_d4 acc[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) acc[x] = mfma_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < KG; ++g)
#pragma unroll
      for (int x = 0; x < 4; ++x) acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[g], (double)a[g][x], acc[x], 0, 0, 0);
    // lane l holds Q_i, i = lk + 4 v, at elements e .. e + 3
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = lk + 4 * v;
      if (i < s) {
#pragma unroll
        for (int f = 0; f < 4 / VN; ++f) {
          T o[VN];
#pragma unroll
          for (int x = 0; x < VN; ++x) o[x] = (T)acc[VN * f + x][v];
          store16(W + (size_t)i * ldv, e + VN * f, N, o);
        }
      }
    }
  }
}


// back substitution R y = g over the columns completed in the cycle (one
// wave): lane j holds row j of R and g_j; y_i = g_i / R_ii, broadcast from
// lane i, then g_j -= R_ji y_i on the rows above, for i from the last row up
// sb > 0: the cycle ended with an s-step block of sb raw vectors starting at
// kb; lane t then also forms the combined coefficient t of the x update
// (see k_sstep_xupdate) into ks->xco.
__global__ __launch_bounds__(64) void k_gmres_solve(KState* ks, int m, int kb, int sb) {
  static_assert(kMaxRestart <= 64, "one row of R per lane");
  if (ks->solved) return;
  const int kk = ks->k;
  const int j = threadIdx.x;
  double row[kMaxRestart];
#pragma unroll
  for (int c = 0; c < kMaxRestart; ++c)
    row[c] = (j < kk && c < kk && c >= j) ? ks->H[(size_t)c * (m + 1) + j] : 0.0;
  double gj = j < kk ? ks->g[j] : 0.0;
#pragma unroll
  for (int i = kMaxRestart - 1; i >= 0; --i) {
    if (i < kk) {
      const double yi = lane_value(gj, i) / lane_value(row[i], i);
      if (j < i) gj -= row[i] * yi;
      if (j == i) gj = yi;
    }
  }
  const double cj = gj * ks->sc[j < kk ? j : 0];
  if (j < kk) ks->coef[j] = cj;
  if (sb <= 0) return;
  __shared__ double cf[kMaxRestart];
  if (j < kk) cf[j] = cj;
  __syncthreads();
  const int J = min(kk - kb - 1, sb);  // block vectors used by the solution
  const int nq = J > 0 ? kb + 1 : kk, nw = J > 0 ? sb : 0;
  for (int t = j; t < nq + nw; t += 64) {
    double v;
    if (t < nq) {  // a_q = y_q - sum_{i < J} y_{kb+1+i} (C R^{-1})_{q i}
      v = cf[t];
      for (int i = 0; i < J; ++i) v -= cf[kb + 1 + i] * ks->dco[t * sb + i];
    } else {       // b_i = sum_{i <= l < J} y_{kb+1+l} (R^{-1})_{i l}
      const int i = t - nq;
      v = 0.0;
      for (int l = i; l < J; ++l) v += cf[kb + 1 + l] * ks->rinv[i * sb + l];
    }
    ks->xco[t] = v;
  }
  if (j == 0) {
    ks->xnq = nq;
    ks->xnw = nw;
  }
}

// End of an s-step cycle whose last block starts at kb with sb vectors: the
// block is left unorthogonalized (V[kb+1..kb+sb] hold the raw powers W), and
// x += D^{-1} sum_{q < kk} y_q V_q is taken with the block's basis vectors
// written out, Q = W R^{-1} - V_{0..kb} (C R^{-1}):
//   x += D^{-1} (sum_{q <= kb} a_q V_q + sum_{i < sb} b_i W_i),
//   a_q = y_q - sum_{j < J} y_{kb+1+j} (C R^{-1})_{qj},  b_i = sum_{i <= j < J} y_{kb+1+j} (R^{-1})_{ij},
// J = kk - kb - 1 block vectors used by the solution (none: W is not read).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sstep_xupdate(int N, int ldv, const T* __restrict__ V,
                                                        const double* __restrict__ dinv, double* __restrict__ x,
                                                        const KState* __restrict__ ks, int kb, int sb) {
  if (ks->solved) return;
  constexpr int VN = 16 / sizeof(T);
  constexpr int CH = kBlock * VN;
  constexpr int QU = 8;  // basis vectors loaded together
  __shared__ double a[kMaxRestart + 1 + kSMax];
  const int nq = ks->xnq;  // basis vectors V_0.. with coefficients
  const int nw = ks->xnw;  // raw block vectors with coefficients
  for (int q = threadIdx.x; q < nq + nw; q += kBlock) a[q] = ks->xco[q];
  __syncthreads();
  const bool vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(dinv)) & 15) == 0;
  const int nt = nq + nw;  // V_0..V_{nq-1}, then V_{kb+1..kb+nw} (the raw W)
  for (int base = blockIdx.x * CH; base < N; base += gridDim.x * CH) {
    const int e = base + threadIdx.x * VN;
    const bool vx = vec && VN == 4 && e + 4 <= N;
    double2 d0{0.0, 0.0}, d1{0.0, 0.0}, x0{0.0, 0.0}, x1{0.0, 0.0};
    if (vx) {  // x and D^{-1} in flight with the first basis loads
      const double2* dp = reinterpret_cast<const double2*>(dinv + e);
      const double2* xq = reinterpret_cast<const double2*>(x + e);
      d0 = dp[0];
      d1 = dp[1];
      x0 = xq[0];
      x1 = xq[1];
    }
    double acc[VN];
#pragma unroll
    for (int c = 0; c < VN; ++c) acc[c] = 0.0;
    for (int t0 = 0; t0 < nt; t0 += QU) {
      T v[QU][VN];
#pragma unroll
      for (int u = 0; u < QU; ++u) {
        const int t = t0 + u;
        if (t < nt) load16(V + (size_t)(t < nq ? t : kb + 1 + (t - nq)) * ldv, e, N, v[u]);
      }
#pragma unroll
      for (int u = 0; u < QU; ++u) {
        if (t0 + u < nt) {
          const double cq = a[t0 + u];
#pragma unroll
          for (int c = 0; c < VN; ++c) acc[c] += cq * (double)v[u][c];
        }
      }
    }
    if (vx) {  // two 16-byte accesses per array
      double2* xp = reinterpret_cast<double2*>(x + e);
      x0.x += d0.x * acc[0];
      x0.y += d0.y * acc[1 % VN];
      x1.x += d1.x * acc[2 % VN];
      x1.y += d1.y * acc[3 % VN];
      xp[0] = x0;
      xp[1] = x1;
    } else {
#pragma unroll
      for (int c = 0; c < VN; ++c)
        if (e + c < N) x[e + c] += dinv[e + c] * acc[c];
    }
  }
}

// x += D^{-1} sum_q coef_q V[q]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gmres_xupdate(int N, int ldv, const T* __restrict__ V,
                                                          const double* __restrict__ dinv, double* __restrict__ x,
                                                          const KState* __restrict__ ks) {
  if (ks->solved) return;
  constexpr int VN = 16 / sizeof(T);
  constexpr int CH = kBlock * VN;
  __shared__ double coef[kMaxRestart + 1];
  const int kk = ks->k;
  for (int q = threadIdx.x; q < kk; q += kBlock) coef[q] = ks->coef[q];
  __syncthreads();
  for (int base = blockIdx.x * CH; base < N; base += gridDim.x * CH) {
    const int e0 = base + threadIdx.x * VN;
    double acc[VN];
#pragma unroll
    for (int c = 0; c < VN; ++c) acc[c] = 0.0;
    for (int q = 0; q < kk; ++q) {
      T a[VN];
      load16(V + (size_t)q * ldv, e0, N, a);
      const double cq = coef[q];
#pragma unroll
      for (int c = 0; c < VN; ++c) acc[c] += cq * (double)a[c];
    }
#pragma unroll
    for (int c = 0; c < VN; ++c)
      if (e0 + c < N) x[e0 + c] += dinv[e0 + c] * acc[c];
  }
}

// ---------------------------------------------------------------------------
// Reduction finish: one workgroup sums the per-workgroup partials of the
// preceding kernel in a fixed order (wave q-strided, lanes block-strided) into
// ks->red and takes the solver's scalar step.  Being a separate kernel, it
// sees the partials through the kernel boundary; the producing kernels need
// no device-scope fence.
// ---------------------------------------------------------------------------

enum FinishAct {
  ACT_STORE = 0,   // red[off..off+nv) only
  ACT_DOTS,        // Arnoldi column: H[q,k] = sc_q red[q]
  ACT_GIVENS,      // norm of the new basis vector + Givens rotation
  ACT_CYCLE,       // residual norm -> Krylov cycle start (mode 1 / 2)
  ACT_BICG_INIT,
  ACT_BICG_ALPHA,
  ACT_BICG_S,
  ACT_BICG_OMEGA,
  ACT_BICG_RHO
};

constexpr int kFinish = 1024;

__global__ __launch_bounds__(kFinish) void k_finish(KState* ks, const double* __restrict__ partials, int nb, int nv,
                                                    int act, int red_off, int k, int m, int mode, double p1,
                                                    double p2, int prow) {
  if (act == ACT_CYCLE && mode != 0 && ks->solved) return;  // restart of a cycle queued after convergence
  switch (act) {
    case ACT_DOTS:
    case ACT_GIVENS:
    case ACT_BICG_ALPHA:
    case ACT_BICG_S:
    case ACT_BICG_RHO:
      if (ks->done) return;
      break;
    case ACT_BICG_OMEGA:
      if (ks->done || ks->half) return;
      break;
    default:
      break;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double* red = ks->red + red_off;
  if (nv == 1) {  // one row: every wave takes a strided share, then the wave totals in order
    __shared__ double sw[kFinish / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kFinish) s += partials[(size_t)prow * kRedBlocks + b];
    s = wave_sum(s);
    if (lane == 0) sw[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kFinish / 64; ++w) t += sw[w];
      red[0] = t;
    }
  } else {
    for (int q = wv; q < nv; q += kFinish / 64) {
      double s = 0.0;
      for (int b = lane; b < nb; b += 64) s += partials[(size_t)(prow + q) * kRedBlocks + b];
      s = wave_sum(s);
      if (lane == 0) red[q] = s;
    }
  }
  __syncthreads();
  if (act == ACT_DOTS) {
    double* Hk = ks->H + (size_t)k * (m + 1);
    for (int q = threadIdx.x; q < nv; q += kFinish) Hk[q] = ks->sc[q] * red[q];
    return;
  }
  if (act == ACT_GIVENS) {
    givens_step(ks, k, m, red[0]);
    return;
  }
  if (threadIdx.x != 0) return;
  switch (act) {
    case ACT_CYCLE:  // tolerances as set by the solve's first cycle_start
      if (mode != 0) cycle_start_dev(ks, mode, red[0], ks->ctol_abs, ks->ctol_rel);
      break;
    case ACT_BICG_INIT: {
      const double rr = red[0];
      ks->rho = rr;
      ks->alpha = 1.0;
      ks->omega = 1.0;
      ks->bcg_beta = 0.0;
      ks->res = sqrt(rr);
      ks->tol = p1;
      ks->half = 0;
      ks->flag = isfinite(rr) ? 0 : 2;
      ks->done = (!isfinite(rr) || ks->res <= p1) ? 1 : 0;
      break;
    }
    case ACT_BICG_ALPHA: {
      const double rv = red[0];
      ks->half = 0;
      if (rv == 0.0 || !isfinite(rv)) {
        ks->flag = isfinite(rv) ? 1 : 2;
        ks->done = 1;
      } else {
        ks->alpha = ks->rho / rv;
      }
      break;
    }
    case ACT_BICG_S:
      if (sqrt(red[0]) <= ks->tol) {
        ks->half = 1;
        ks->omega = 0.0;
      }
      break;
    case ACT_BICG_OMEGA: {
      const double ts = red[0], tt = red[1];
      ks->omega = tt != 0.0 ? ts / tt : 0.0;
      if (!isfinite(ks->omega)) {
        ks->flag = 2;
        ks->done = 1;
      }
      break;
    }
    case ACT_BICG_RHO: {
      const double rho_new = red[0];
      const double res = sqrt(red[1]);
      ks->iters += 1;
      ks->res = res;
      if (!isfinite(res)) {
        ks->flag = 2;
        ks->done = 1;
      } else if (res <= ks->tol) {
        ks->done = 1;
      } else if (rho_new == 0.0 || ks->omega == 0.0) {
        ks->flag = 1;
        ks->done = 1;
      } else {
        ks->bcg_beta = (rho_new / ks->rho) * (ks->alpha / ks->omega);
        ks->rho = rho_new;
      }
      break;
    }
    default:
      break;
  }
}

// ---------------------------------------------------------------------------
// BiCGStab (van der Vorst), right Jacobi preconditioning, FP64.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_bicg_init(int N, const double* __restrict__ r, double* __restrict__ rhat,
                                                      double* __restrict__ p, double* __restrict__ v, KState* ks,
                                                      double* partials, double tol) {
  double acc[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    const double ri = r[i];
    rhat[i] = ri;
    p[i] = ri;
    v[i] = 0.0;
    acc[0] += ri * ri;
  }
  block_partials<1>(acc, 1, partials, blockIdx.x);
}

// v = A D^{-1} p ; alpha = rho / (rhat, v)   (A in SELL order)
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_bicg_v(SellView S, const TI* __restrict__ dlt,
                                                   const double* __restrict__ A, const double* __restrict__ dinv,
                                                   const double* __restrict__ p, const double* __restrict__ rhat,
                                                   double* __restrict__ v, KState* ks, double* partials) {
  if (ks->done) return;
  double acc[1] = {0.0};
  int t0, t1;
  tile_range((S.nsl + kBlock / 64 - 1) / (kBlock / 64), t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int i = s * 64 + (threadIdx.x & 63);
    const auto xf = [&](int j) { return dinv[j] * p[j]; };
    int c[9];
    double q;
    if (slice_runs27(S, s, c)) {  // wave-uniform; a full slice, every lane has a row
      q = sell_row27_runs(A + S.sl_ptr[s], c, s * 64, i & 63, xf);
    } else {
      if (i >= S.N) continue;
      q = sell_row<8>(S, dlt, A, s, i, xf);
    }
    v[i] = q;
    acc[0] += rhat[i] * q;
  }
  block_partials<1>(acc, 1, partials, blockIdx.x);
}

// s = r - alpha v ; stop early when ||s|| <= tol
__global__ __launch_bounds__(kBlock) void k_bicg_s(int N, const double* __restrict__ r, const double* __restrict__ v,
                                                   double* __restrict__ s, KState* ks, double* partials) {
  if (ks->done) return;
  const double alpha = ks->alpha;
  double acc[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    const double si = r[i] - alpha * v[i];
    s[i] = si;
    acc[0] += si * si;
  }
  block_partials<1>(acc, 1, partials, blockIdx.x);
}

// t = A D^{-1} s ; omega = (t, s) / (t, t)   (A in SELL order)
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_bicg_t(SellView S, const TI* __restrict__ dlt,
                                                   const double* __restrict__ A, const double* __restrict__ dinv,
                                                   const double* __restrict__ sv, double* __restrict__ tv, KState* ks,
                                                   double* partials) {
  if (ks->done || ks->half) return;
  double acc[2] = {0.0, 0.0};
  int t0, t1;
  tile_range((S.nsl + kBlock / 64 - 1) / (kBlock / 64), t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int i = s * 64 + (threadIdx.x & 63);
    const auto xf = [&](int j) { return dinv[j] * sv[j]; };
    int c[9];
    double q;
    if (slice_runs27(S, s, c)) {  // wave-uniform; a full slice, every lane has a row
      q = sell_row27_runs(A + S.sl_ptr[s], c, s * 64, i & 63, xf);
    } else {
      if (i >= S.N) continue;
      q = sell_row<8>(S, dlt, A, s, i, xf);
    }
    tv[i] = q;
    acc[0] += q * sv[i];
    acc[1] += q * q;
  }
  block_partials<2>(acc, 2, partials, blockIdx.x);
}

// x += alpha D^{-1} p + omega D^{-1} s ; r = s - omega t ; rho_new = (rhat, r)
__global__ __launch_bounds__(kBlock) void k_bicg_xr(int N, const double* __restrict__ dinv,
                                                    const double* __restrict__ p, const double* __restrict__ s,
                                                    const double* __restrict__ tv, const double* __restrict__ rhat,
                                                    double* __restrict__ x, double* __restrict__ r, KState* ks,
                                                    double* partials) {
  if (ks->done) return;
  const double alpha = ks->alpha, omega = ks->omega;
  const bool half = ks->half != 0;
  double acc[2] = {0.0, 0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    const double di = dinv[i];
    double ri;
    if (half) {
      x[i] += alpha * (di * p[i]);
      ri = s[i];
    } else {
      x[i] += alpha * (di * p[i]) + omega * (di * s[i]);
      ri = s[i] - omega * tv[i];
    }
    r[i] = ri;
    acc[0] += rhat[i] * ri;
    acc[1] += ri * ri;
  }
  block_partials<2>(acc, 2, partials, blockIdx.x);
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(kBlock) void k_bicg_p(int N, const double* __restrict__ r, const double* __restrict__ v,
                                                   double* __restrict__ p, const KState* __restrict__ ks) {
  if (ks->done) return;
  const double beta = ks->bcg_beta, omega = ks->omega;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock)
    p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// ---------------------------------------------------------------------------
// Zalesak FCT, explicit SSP stage (eqs. (18)-(21), limiter steps 1-4)
// ---------------------------------------------------------------------------

// Three passes per stage over the SELL-64 rows (one row per lane, values in
// slot order, stored slots marked in `mask`; see the MCL passes below):
//   lowrate  udot = M_L^{-1} (F - A_low u) (0 on Dirichlet nodes), ut = u + dt udot (u_D)
//   limit_R  P+-, Q+- (from ut) and R+- of r_ij = m_ij (udot_i - udot_j) + d_ij (u_j - u_i)
//   apply    F*_i = sum_j alpha_ij r_ij ; out = c0 * base + c1 * (ut + dt F* / m)
__device__ __forceinline__ int sell_delta_any(const SellView& S, const void* dlt, bool d16, int doff, int p,
                                              int lane) {
  if (doff < 0) return S.pat[~doff + p];
  return d16 ? (int)static_cast<const int16_t*>(dlt)[doff + 64 * p + lane]
             : static_cast<const int*>(dlt)[doff + 64 * p + lane];
}

// rows of a SELL launch: slice s of this wave, row i of this lane
#define AFC_SELL_ROWS(S, s, i)                                                        \
  int t0_, t1_;                                                                       \
  tile_range(((S).nsl + kBlock / 64 - 1) / (kBlock / 64), t0_, t1_);                  \
  for (int t_ = t0_; t_ < t1_; ++t_)                                                  \
    if (const int s = wave_slice(t_); s < (S).nsl)                                    \
      if (const int i = s * 64 + (int)(threadIdx.x & 63); i < (S).N)

__global__ __launch_bounds__(kBlock) void k_ssp_lowrate_sell(SellView S, const void* __restrict__ dlt, int d16,
                                                             const uint32_t* __restrict__ mask,
                                                             const double* __restrict__ Sal,
                                                             const double* __restrict__ u,
                                                             const double* __restrict__ F,
                                                             const double* __restrict__ ml,
                                                             const uint8_t* __restrict__ is_dir,
                                                             const double* __restrict__ uD, double dt,
                                                             double* __restrict__ udot, double* __restrict__ ut) {
  int t0, t1;
  tile_range((S.nsl + kBlock / 64 - 1) / (kBlock / 64), t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int lane = threadIdx.x & 63;
    const int i = s * 64 + lane;
    if (i >= S.N) continue;
    if (is_dir[i]) {
      udot[i] = 0.0;
      ut[i] = uD[i];
      continue;
    }
    const int base = S.sl_ptr[s];
    const int L = (S.sl_ptr[s + 1] - base) >> 6;
    const int doff = S.sl_dl[s];
    uint32_t msk = 0u;
    double acc = 0.0;
#pragma unroll 4
    for (int p = 0; p < L; ++p) {
      if ((p & 31) == 0) msk = mask[(size_t)(p >> 5) * S.N + i];
      if (!((msk >> (p & 31)) & 1u)) continue;
      acc += Sal[(size_t)base + 64 * p + lane] * u[i + sell_delta_any(S, dlt, d16, doff, p, lane)];
    }
    const double ud = (F[i] - acc) / ml[i];
    udot[i] = ud;
    ut[i] = u[i] + dt * ud;
  }
}

__global__ __launch_bounds__(kBlock) void k_ssp_limit_R_sell(SellView S, const void* __restrict__ dlt, int d16,
                                                             const uint32_t* __restrict__ mask,
                                                             const double* __restrict__ Smij,
                                                             const double* __restrict__ Sdp,
                                                             const double* __restrict__ u,
                                                             const double* __restrict__ udot,
                                                             const double* __restrict__ ut,
                                                             const double* __restrict__ ml,
                                                             const uint8_t* __restrict__ is_dir, double dt,
                                                             double* __restrict__ Rp, double* __restrict__ Rm) {
  int t0, t1;
  tile_range((S.nsl + kBlock / 64 - 1) / (kBlock / 64), t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int lane = threadIdx.x & 63;
    const int i = s * 64 + lane;
    if (i >= S.N) continue;
    if (is_dir[i]) {
      Rp[i] = Rm[i] = 1.0;
      continue;
    }
    const int base = S.sl_ptr[s];
    const int L = (S.sl_ptr[s + 1] - base) >> 6;
    const int doff = S.sl_dl[s];
    const double ui = u[i], udi = udot[i], uti = ut[i];
    uint32_t msk = 0u;
    double pp = 0.0, pm = 0.0, qp = 0.0, qm = 0.0;
#pragma unroll 2
    for (int p = 0; p < L; ++p) {
      if ((p & 31) == 0) msk = mask[(size_t)(p >> 5) * S.N + i];
      if (!((msk >> (p & 31)) & 1u)) continue;
      const int dj = sell_delta_any(S, dlt, d16, doff, p, lane);
      if (dj == 0) continue;
      const int j = i + dj;
      const size_t v = (size_t)base + 64 * p + lane;
      const double r = Smij[v] * (udi - udot[j]) - Sdp[v] * (u[j] - ui);
      pp += fmax(r, 0.0);
      pm += fmin(r, 0.0);
      const double du = ut[j] - uti;
      qp = fmax(qp, du);
      qm = fmin(qm, du);
    }
    Rp[i] = zalesak_R(ml[i], qp, pp, dt);
    Rm[i] = zalesak_R(ml[i], qm, pm, dt);
  }
}

__global__ __launch_bounds__(kBlock) void k_ssp_apply_sell(
    SellView S, const void* __restrict__ dlt, int d16, const uint32_t* __restrict__ mask,
    const double* __restrict__ Smij, const double* __restrict__ Sdp, const double* __restrict__ u,
    const double* __restrict__ udot, const double* __restrict__ ut, const double* __restrict__ Rp,
    const double* __restrict__ Rm, const double* __restrict__ ml, const uint8_t* __restrict__ is_dir,
    const double* __restrict__ uD, double dt, int alpha_mode, const double* __restrict__ base_v, double c0, double c1,
    double* __restrict__ out) {
  int t0, t1;
  tile_range((S.nsl + kBlock / 64 - 1) / (kBlock / 64), t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int lane = threadIdx.x & 63;
    const int i = s * 64 + lane;
    if (i >= S.N) continue;
    if (is_dir[i]) {
      out[i] = uD[i];
      continue;
    }
    double fs = 0.0;
    if (alpha_mode != AFC_ALPHA_ZERO) {
      const int base = S.sl_ptr[s];
      const int L = (S.sl_ptr[s + 1] - base) >> 6;
      const int doff = S.sl_dl[s];
      const double ui = u[i], udi = udot[i], rpi = Rp[i], rmi = Rm[i];
      uint32_t msk = 0u;
#pragma unroll 2
      for (int p = 0; p < L; ++p) {
        if ((p & 31) == 0) msk = mask[(size_t)(p >> 5) * S.N + i];
        if (!((msk >> (p & 31)) & 1u)) continue;
        const int dj = sell_delta_any(S, dlt, d16, doff, p, lane);
        if (dj == 0) continue;
        const int j = i + dj;
        const size_t v = (size_t)base + 64 * p + lane;
        const double uj = u[j], udj = udot[j], rpj = Rp[j], rmj = Rm[j];  // every gather issued at once
        const double r = Smij[v] * (udi - udj) - Sdp[v] * (uj - ui);
        double a = 1.0;
        if (alpha_mode == AFC_ALPHA_LIMITED) a = r > 0.0 ? fmin(rpi, rmj) : fmin(rmi, rpj);
        fs += a * r;
      }
    }
    const double unew = ut[i] + dt * fs / ml[i];
    out[i] = (c0 == 0.0) ? c1 * unew : c0 * base_v[i] + c1 * unew;
  }
}

// ---------------------------------------------------------------------------
// Zalesak FCT, Crank-Nicolson (eqs. (11)-(14))
// ---------------------------------------------------------------------------

// ut = u_old - dt/2 M_L^{-1} (A_low u_old - F_old) ; g = (M_L/dt - A_low/2) u_old + (F_old + F_new)/2
// Linear Zal+CN (Sec. 2.1.1): u* = 2 u~ - u^{n-1} stands for u^n in the
// fluxes of eq. (12); u_D at Dirichlet nodes.
__global__ __launch_bounds__(kBlock) void k_cn_extrapolate(int N, const double* __restrict__ ut,
                                                           const double* __restrict__ uo,
                                                           const uint8_t* __restrict__ is_dir,
                                                           const double* __restrict__ uD, double* __restrict__ us) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock)
    us[i] = is_dir[i] ? uD[i] : 2.0 * ut[i] - uo[i];
}


// Q+-_i = max/min(0, ext_{j != i} (ut_j - ut_i))


// b = g + F*(u), r = b - A_cn u ; reductions: R^2 (free rows), ||b||^2, ||r||^2

// The Crank-Nicolson passes over the SELL-64 rows (one row per lane, values
// in slot order, stored slots marked in `mask`).
struct FctSell {
  SellView S;
  const void* dlt;
  int d16;
  const uint32_t* mask;
  const double *Smij, *Sdp, *Sal;
};

#define AFC_FCT_SLOTS(F, s, i, p, dj, v)                                                  \
  const int base_ = (F).S.sl_ptr[s];                                                      \
  const int L_ = ((F).S.sl_ptr[s + 1] - base_) >> 6;                                      \
  const int doff_ = (F).S.sl_dl[s];                                                       \
  uint32_t msk_ = 0u;                                                                     \
  for (int p = 0; p < L_; ++p)                                                            \
    if (((p & 31) == 0 ? (msk_ = (F).mask[(size_t)(p >> 5) * (F).S.N + i]) : msk_),       \
        ((msk_ >> (p & 31)) & 1u))                                                        \
      if (const int dj = sell_delta_any((F).S, (F).dlt, (F).d16, doff_, p, i & 63); true) \
        if (const size_t v = (size_t)base_ + 64 * p + (i & 63); true)

// ut = u_old - dt/2 M_L^{-1} (A_low u_old - F_old) (eq. (14));
// g = (M_L/dt - A_low/2) u_old + (F_old + F_new)/2 (right-hand side of eq. (11))
__global__ __launch_bounds__(kBlock) void k_cn_predict(FctSell F, const double* __restrict__ uo,
                                                       const double* __restrict__ Fo, const double* __restrict__ Fn,
                                                       const double* __restrict__ ml,
                                                       const uint8_t* __restrict__ is_dir,
                                                       const double* __restrict__ uD, double dt,
                                                       double* __restrict__ ut, double* __restrict__ g) {
  AFC_SELL_ROWS(F.S, s, i) {
    if (is_dir[i]) {
      ut[i] = g[i] = uD[i];
      continue;
    }
    double y = 0.0;
    AFC_FCT_SLOTS(F, s, i, p, dj, v) y += F.Sal[v] * uo[i + dj];
    const double mi = ml[i];
    ut[i] = uo[i] - 0.5 * dt * (y - Fo[i]) / mi;
    g[i] = mi / dt * uo[i] - 0.5 * y + 0.5 * (Fo[i] + Fn[i]);
  }
}

// Q+-_i = max/min(0, ext_{j != i} (ut_j - ut_i))
__global__ __launch_bounds__(kBlock) void k_zalesak_Q(FctSell F, const double* __restrict__ ut,
                                                      double* __restrict__ Qp, double* __restrict__ Qm) {
  AFC_SELL_ROWS(F.S, s, i) {
    const double uti = ut[i];
    double qp = 0.0, qm = 0.0;
    AFC_FCT_SLOTS(F, s, i, p, dj, v) {
      if (dj == 0) continue;
      const double du = ut[i + dj] - uti;
      qp = fmax(qp, du);
      qm = fmin(qm, du);
    }
    Qp[i] = qp;
    Qm[i] = qm;
  }
}

// P+- of the (prelimited) CN fluxes of eqs. (12), (13) and R+-
__global__ __launch_bounds__(kBlock) void k_cn_limit_R(FctSell F, const double* __restrict__ u,
                                                       const double* __restrict__ uo, const double* __restrict__ Qp,
                                                       const double* __restrict__ Qm, const double* __restrict__ ml,
                                                       const uint8_t* __restrict__ is_dir, double dt, double L,
                                                       double* __restrict__ Rp, double* __restrict__ Rm) {
  const double inv_dt = 1.0 / dt;
  AFC_SELL_ROWS(F.S, s, i) {
    if (is_dir[i]) {
      Rp[i] = Rm[i] = 1.0;
      continue;
    }
    const double dui = u[i] - uo[i], sui = u[i] + uo[i];
    double pp = 0.0, pm = 0.0;
    AFC_FCT_SLOTS(F, s, i, p, dj, v) {
      if (dj == 0) continue;
      const int j = i + dj;
      const double uj = u[j], uoj = uo[j];
      const double r = cn_flux(F.Smij[v], -F.Sdp[v], inv_dt, dui, uj - uoj, sui, uj + uoj, L);
      pp += fmax(r, 0.0);
      pm += fmin(r, 0.0);
    }
    Rp[i] = zalesak_R(ml[i], Qp[i], pp, dt);
    Rm[i] = zalesak_R(ml[i], Qm[i], pm, dt);
  }
}

// b = g + F*(u), r = b - A_cn u (A_cn in slot order); reductions: R^2 (free rows), ||b||^2, ||r||^2
__global__ __launch_bounds__(kBlock) void k_cn_apply(FctSell F, const double* __restrict__ Scn,
                                                     const double* __restrict__ u, const double* __restrict__ uo,
                                                     const double* __restrict__ Rp, const double* __restrict__ Rm,
                                                     const double* __restrict__ g,
                                                     const uint8_t* __restrict__ is_dir,
                                                     const double* __restrict__ uD, double dt, double L,
                                                     int alpha_mode, double* __restrict__ b, double* __restrict__ r,
                                                     double* partials) {
  const double inv_dt = 1.0 / dt;
  double acc[3] = {0.0, 0.0, 0.0};
  AFC_SELL_ROWS(F.S, s, i) {
    if (is_dir[i]) {
      const double bi = uD[i], ri = uD[i] - u[i];
      b[i] = bi;
      r[i] = ri;
      acc[1] += bi * bi;
      acc[2] += ri * ri;
      continue;
    }
    const double dui = u[i] - uo[i], sui = u[i] + uo[i], rpi = Rp[i], rmi = Rm[i];
    double fs = 0.0, au = 0.0;
    AFC_FCT_SLOTS(F, s, i, p, dj, v) {
      const int j = i + dj;
      const double uj = u[j];
      au += Scn[v] * uj;
      if (dj == 0 || alpha_mode == AFC_ALPHA_ZERO) continue;
      const double uoj = uo[j], rpj = Rp[j], rmj = Rm[j];  // every gather issued at once
      const double rf = cn_flux(F.Smij[v], -F.Sdp[v], inv_dt, dui, uj - uoj, sui, uj + uoj, L);
      double a = 1.0;
      if (alpha_mode == AFC_ALPHA_LIMITED) a = rf > 0.0 ? fmin(rpi, rmj) : fmin(rmi, rpj);
      fs += a * rf;
    }
    const double bi = g[i] + fs, ri = bi - au;
    b[i] = bi;
    r[i] = ri;
    acc[0] += ri * ri;
    acc[1] += bi * bi;
    acc[2] += ri * ri;
  }
  block_partials<3>(acc, 3, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Monolithic convex limiter (eqs. (22)-(23), (25), Remark 1)
// ---------------------------------------------------------------------------

// Both passes run over the SELL-64 rows: one row per lane, no column array,
// no cross-lane sums.  Bit p % 32 of mask[(p / 32) N + i] marks slot p of
// row i as a stored entry: padding slots of a uniform slice can point at
// nodes outside N_i, so they must not enter u^max / u^min or the fluxes.

// u^max_i, u^min_i: extremes of u over N_i (i included)

__global__ __launch_bounds__(kBlock) void k_mcl_bounds_sell(SellView S, const void* __restrict__ dlt, int d16,
                                                            const uint32_t* __restrict__ mask,
                                                            const double* __restrict__ u, double* __restrict__ umax,
                                                            double* __restrict__ umin) {
  int t0, t1;
  tile_range((S.nsl + kBlock / 64 - 1) / (kBlock / 64), t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int lane = threadIdx.x & 63;
    const int i = s * 64 + lane;
    if (i >= S.N) continue;
    const int L = (S.sl_ptr[s + 1] - S.sl_ptr[s]) >> 6;
    const int doff = S.sl_dl[s];
    uint32_t msk = 0u;
    double mx = -INFINITY, mn = INFINITY;
#pragma unroll 4
    for (int p = 0; p < L; ++p) {
      if ((p & 31) == 0) msk = mask[(size_t)(p >> 5) * S.N + i];
      const int j = i + sell_delta_any(S, dlt, d16, doff, p, lane);
      if ((msk >> (p & 31)) & 1u) {
        const double uj = u[j];
        mx = fmax(mx, uj);
        mn = fmin(mn, uj);
      }
    }
    umax[i] = mx;
    umin[i] = mn;
  }
}

// r*_ij from d_ij = -max(c_ij, 0, c_ji) and the bar states in product form
// 2 d_ij ubar_ij = d_ij (u_i + u_j) + c_ij (u_j - u_i); F*_i = sum_j r*_ij;
// b = F + F*, r = b - A_low u; reductions: R^2 (free rows), ||b||^2, ||r||^2.
// A_low, c_ij and c_ji come in SELL slot order (Sal, Scc, SccT).  Those three
// streams are read once, with nontemporal loads, so that they do not push the
// gathered node vectors (u, u^max, u^min of the neighbour planes) out of L2.
__global__ __launch_bounds__(kBlock) void k_mcl_apply_sell(
    SellView S, const void* __restrict__ dlt, int d16, const uint32_t* __restrict__ mask,
    const double* __restrict__ Scc, const double* __restrict__ SccT, const double* __restrict__ Sal,
    const double* __restrict__ u, const double* __restrict__ umax, const double* __restrict__ umin,
    const double* __restrict__ F, const uint8_t* __restrict__ is_dir, const double* __restrict__ uD, int alpha_mode,
    double* __restrict__ b, double* __restrict__ r, double* partials) {
  double acc[3] = {0.0, 0.0, 0.0};
  int t0, t1;
  tile_range((S.nsl + kBlock / 64 - 1) / (kBlock / 64), t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int s = wave_slice(t);
    if (s >= S.nsl) continue;
    const int lane = threadIdx.x & 63;
    const int i = s * 64 + lane;
    if (i >= S.N) continue;
    if (is_dir[i]) {
      const double bi = uD[i], ri = uD[i] - u[i];
      b[i] = bi;
      r[i] = ri;
      acc[1] += bi * bi;
      acc[2] += ri * ri;
      continue;
    }
    const int base = S.sl_ptr[s];
    const int L = (S.sl_ptr[s + 1] - base) >> 6;
    const int doff = S.sl_dl[s];
    uint32_t msk = 0u;
    const double ui = u[i], umaxi = umax[i], umini = umin[i];
    double fs = 0.0, au = 0.0;
#pragma unroll 2
    for (int p = 0; p < L; ++p) {
      if ((p & 31) == 0) msk = mask[(size_t)(p >> 5) * S.N + i];
      if (!((msk >> (p & 31)) & 1u)) continue;
      const int dj = sell_delta_any(S, dlt, d16, doff, p, lane);
      const int j = i + dj;
      const size_t v = (size_t)base + 64 * p + lane;
      const double uj = u[j];
      au += __builtin_nontemporal_load(Sal + v) * uj;
      if (dj == 0 || alpha_mode == AFC_ALPHA_ZERO) continue;
      const double c = __builtin_nontemporal_load(Scc + v), ct = __builtin_nontemporal_load(SccT + v);
      const double d = -fmax(fmax(c, 0.0), ct);
      if (d == 0.0) continue;
      const double rf = d * (uj - ui);
      if (alpha_mode == AFC_ALPHA_ONE) {
        fs += rf;
        continue;
      }
      const double sij = d * (ui + uj) + c * (uj - ui);
      const double sji = d * (ui + uj) + ct * (ui - uj);
      const double two_d = 2.0 * d;
      double rs;
      if (rf > 0.0)
        rs = fmin(rf, fmin(sij - two_d * umaxi, two_d * umin[j] - sji));
      else
        rs = fmax(rf, fmax(sij - two_d * umini, two_d * umax[j] - sji));
      fs += rs;
    }
    const double bi = F[i] + fs, ri = bi - au;
    b[i] = bi;
    r[i] = ri;
    acc[0] += ri * ri;
    acc[1] += bi * bi;
    acc[2] += ri * ri;
  }
  block_partials<3>(acc, 3, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Time-dependent monolithic convex limiting (Sec. 2.2): the fluxes of eq. (20),
// r_ij = m_ij (udot_i - udot_j) + d_ij (u_j - u_i), d_ij = -max(c_ij, 0, c_ji)
// from the convective part (Remark 1), clipped by eq. (22) with the bar states
// of the current state u (r* = 0 where d_ij = 0)
// ---------------------------------------------------------------------------

// SELL view of the MC data (m_ij and the convective a_ij, a_ji in slot order)
struct McSell {
  SellView S;
  const void* dlt;
  int d16;
  const uint32_t* mask;
  const double *Smij, *Scc, *SccT;
};

// F*_i = sum_j r*_ij over the SELL row of lane i in slice s (slot order)
__device__ __forceinline__ double mc_row_fstar(const McSell& M, int s, int i, const double* __restrict__ u,
                                               const double* __restrict__ udot, const double* __restrict__ umax,
                                               const double* __restrict__ umin, int alpha_mode) {
  if (alpha_mode == AFC_ALPHA_ZERO) return 0.0;
  const int lane = i & 63;
  const int base = M.S.sl_ptr[s];
  const int L = (M.S.sl_ptr[s + 1] - base) >> 6;
  const int doff = M.S.sl_dl[s];
  const double ui = u[i], udi = udot[i], umaxi = umax[i], umini = umin[i];
  uint32_t msk = 0u;
  double fs = 0.0;
  for (int p = 0; p < L; ++p) {
    if ((p & 31) == 0) msk = M.mask[(size_t)(p >> 5) * M.S.N + i];
    if (!((msk >> (p & 31)) & 1u)) continue;
    const int dj = sell_delta_any(M.S, M.dlt, M.d16, doff, p, lane);
    if (dj == 0) continue;
    const int j = i + dj;
    const size_t v = (size_t)base + 64 * p + lane;
    const double uj = u[j], udj = udot[j], umaxj = umax[j], uminj = umin[j];  // gathers issued together
    const double c = M.Scc[v], ct = M.SccT[v];
    const double d = -fmax(fmax(c, 0.0), ct);
    const double rf = M.Smij[v] * (udi - udj) + d * (uj - ui);
    if (alpha_mode == AFC_ALPHA_ONE) {
      fs += rf;
      continue;
    }
    if (d == 0.0) continue;
    const double sij = d * (ui + uj) + c * (uj - ui);
    const double sji = d * (ui + uj) + ct * (ui - uj);
    const double two_d = 2.0 * d;
    if (rf > 0.0)
      fs += fmin(rf, fmin(sij - two_d * umaxi, two_d * uminj - sji));
    else
      fs += fmax(rf, fmax(sij - two_d * umini, two_d * umaxj - sji));
  }
  return fs;
}

// MC forward-Euler stage of eq. (18): out = c0 u0 + c1 (u + dt (udot + F*/m)),
// u_D at Dirichlet nodes (udot from the MC low-order operator)
__global__ __launch_bounds__(kBlock) void k_mc_stage(McSell M, const double* __restrict__ ml,
                                                     const uint8_t* __restrict__ is_dir,
                                                     const double* __restrict__ uD, const double* __restrict__ u,
                                                     const double* __restrict__ udot,
                                                     const double* __restrict__ umax,
                                                     const double* __restrict__ umin, double dt,
                                                     const double* __restrict__ u0, double c0, double c1,
                                                     int alpha_mode, double* __restrict__ out) {
  AFC_SELL_ROWS(M.S, s, i) {
    if (is_dir[i]) {
      out[i] = c0 * u0[i] + c1 * uD[i];
      continue;
    }
    const double fs = mc_row_fstar(M, s, i, u, udot, umax, umin, alpha_mode);
    out[i] = c0 * u0[i] + c1 * (u[i] + dt * (udot[i] + fs / ml[i]));
  }
}

// MC+CN right-hand side without the new-level correction:
// g = M_L/dt u^{n-1} - A_low u^{n-1}/2 + (F^{n-1} + F^n)/2 + F*(u^{n-1})/2, with
// A_low u^{n-1} = F^{n-1} - M_L udot^{n-1} on free rows; u_D on Dirichlet rows
__global__ __launch_bounds__(kBlock) void k_mc_cn_g(McSell M, const double* __restrict__ ml,
                                                    const uint8_t* __restrict__ is_dir,
                                                    const double* __restrict__ uD, const double* __restrict__ uo,
                                                    const double* __restrict__ udot,
                                                    const double* __restrict__ umax,
                                                    const double* __restrict__ umin, const double* __restrict__ Fn,
                                                    double inv_dt, int alpha_mode, double* __restrict__ g) {
  AFC_SELL_ROWS(M.S, s, i) {
    if (is_dir[i]) {
      g[i] = uD[i];
      continue;
    }
    const double fs = mc_row_fstar(M, s, i, uo, udot, umax, umin, alpha_mode);
    const double mi = ml[i];
    g[i] = mi * inv_dt * uo[i] + 0.5 * mi * udot[i] + 0.5 * Fn[i] + 0.5 * fs;
  }
}

// MC+CN fixed-point residual: b = g + F*(u)/2, r = b - A_cn u (A_cn in SELL
// slot order); reductions R^2 (free rows), ||b||^2, ||r||^2
__global__ __launch_bounds__(kBlock) void k_mc_cn_apply(McSell M, const double* __restrict__ Scn,
                                                        const double* __restrict__ u,
                                                        const double* __restrict__ udot,
                                                        const double* __restrict__ umax,
                                                        const double* __restrict__ umin,
                                                        const double* __restrict__ g,
                                                        const uint8_t* __restrict__ is_dir,
                                                        const double* __restrict__ uD, int alpha_mode,
                                                        double* __restrict__ b, double* __restrict__ r,
                                                        double* partials) {
  double acc[3] = {0.0, 0.0, 0.0};
  AFC_SELL_ROWS(M.S, s, i) {
    if (is_dir[i]) {
      const double bi = uD[i], ri = uD[i] - u[i];
      b[i] = bi;
      r[i] = ri;
      acc[1] += bi * bi;
      acc[2] += ri * ri;
      continue;
    }
    const double fs = mc_row_fstar(M, s, i, u, udot, umax, umin, alpha_mode);
    const int lane = i & 63;
    const int base = M.S.sl_ptr[s];
    const int L = (M.S.sl_ptr[s + 1] - base) >> 6;
    const int doff = M.S.sl_dl[s];
    uint32_t msk = 0u;
    double au = 0.0;
    for (int p = 0; p < L; ++p) {
      if ((p & 31) == 0) msk = M.mask[(size_t)(p >> 5) * M.S.N + i];
      if (!((msk >> (p & 31)) & 1u)) continue;
      au += Scn[(size_t)base + 64 * p + lane] * u[i + sell_delta_any(M.S, M.dlt, M.d16, doff, p, lane)];
    }
    const double bi = g[i] + 0.5 * fs, ri = bi - au;
    b[i] = bi;
    r[i] = ri;
    acc[0] += ri * ri;
    acc[1] += bi * bi;
    acc[2] += ri * ri;
  }
  block_partials<3>(acc, 3, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Monolithic upwind limiter (Sec. 3.2) of r^ss_ij = d_ij (u_j - u_i),
// d_ij = -d+_ij from the matrix A (eq. (5)); own[k] orients each edge
// (1: a_ji < a_ij, node i; 2: a_ji > a_ij, node j; 0: both)
// ---------------------------------------------------------------------------

// P+-_i over the edges node i owns, Q+-_i over all its fluxes, R+-_i (SELL rows;
// Sown: own[k] in slot order)
__global__ __launch_bounds__(kBlock) void k_mu_R(FctSell F, const uint8_t* __restrict__ Sown,
                                                 const double* __restrict__ u, const uint8_t* __restrict__ is_dir,
                                                 double* __restrict__ Rp, double* __restrict__ Rm) {
  AFC_SELL_ROWS(F.S, s, i) {
    if (is_dir[i]) {
      Rp[i] = Rm[i] = 1.0;
      continue;
    }
    const double ui = u[i];
    double pp = 0.0, pm = 0.0, qp = 0.0, qm = 0.0;
    AFC_FCT_SLOTS(F, s, i, p, dj, v) {
      if (dj == 0) continue;
      const double rf = -F.Sdp[v] * (u[i + dj] - ui);
      const double rpos = fmax(rf, 0.0), rneg = fmin(rf, 0.0);
      if (Sown[v] != 2) {
        pp += rpos;
        pm += rneg;
      }
      qp -= rneg;
      qm -= rpos;
    }
    Rp[i] = pp != 0.0 ? fmin(1.0, qp / pp) : 1.0;
    Rm[i] = pm != 0.0 ? fmin(1.0, qm / pm) : 1.0;
  }
}

// alpha_ij = alpha_ji from the owning node (the smaller of both when equal),
// F*_i = sum_j alpha_ij r_ij; b = F + F*, r = b - A u (A in slot order);
// reductions R^2 (free rows), ||b||^2, ||r||^2
__global__ __launch_bounds__(kBlock) void k_mu_apply(FctSell F, const uint8_t* __restrict__ Sown,
                                                     const double* __restrict__ Sa, const double* __restrict__ u,
                                                     const double* __restrict__ Rp, const double* __restrict__ Rm,
                                                     const double* __restrict__ Fv,
                                                     const uint8_t* __restrict__ is_dir,
                                                     const double* __restrict__ uD, int alpha_mode,
                                                     double* __restrict__ b, double* __restrict__ r,
                                                     double* partials) {
  double acc[3] = {0.0, 0.0, 0.0};
  AFC_SELL_ROWS(F.S, s, i) {
    if (is_dir[i]) {
      const double bi = uD[i], ri = uD[i] - u[i];
      b[i] = bi;
      r[i] = ri;
      acc[1] += bi * bi;
      acc[2] += ri * ri;
      continue;
    }
    const double ui = u[i], rpi = Rp[i], rmi = Rm[i];
    double fs = 0.0, au = 0.0;
    AFC_FCT_SLOTS(F, s, i, p, dj, v) {
      const int j = i + dj;
      const double uj = u[j];
      au += Sa[v] * uj;
      if (dj == 0 || alpha_mode == AFC_ALPHA_ZERO) continue;
      const double rf = -F.Sdp[v] * (uj - ui);
      double a = 1.0;
      if (alpha_mode == AFC_ALPHA_LIMITED) {
        const double rpj = Rp[j], rmj = Rm[j];
        const double ai = rf > 0.0 ? rpi : (rf < 0.0 ? rmi : 1.0);  // node i, flux r_ij
        const double aj = rf < 0.0 ? rpj : (rf > 0.0 ? rmj : 1.0);  // node j, flux r_ji = -r_ij
        const int o = Sown[v];
        a = o == 1 ? ai : (o == 2 ? aj : fmin(ai, aj));
      }
      fs += a * rf;
    }
    const double bi = Fv[i] + fs, ri = bi - au;
    b[i] = bi;
    r[i] = ri;
    acc[0] += ri * ri;
    acc[1] += bi * bi;
    acc[2] += ri * ri;
  }
  block_partials<3>(acc, 3, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------

int row_grid(const H* h, bool reduce) {
  const int rpb = kBlock / h->G;
  const int nt = (h->N + rpb - 1) / rpb;
  return std::max(1, std::min(nt, reduce ? kRedBlocks : kRowGridCap));
}

int vec_grid(const H* h) { return std::max(1, std::min((h->N + kBlock - 1) / kBlock, kRedBlocks)); }

#define AFC_DISPATCH_G(h, KERNEL, GRID, ...)                                                   \
  do {                                                                                           \
    switch ((h)->G) {                                                                            \
      case 8: KERNEL<8><<<(GRID), kBlock, 0, (h)->stream>>>(__VA_ARGS__); break;                 \
      case 16: KERNEL<16><<<(GRID), kBlock, 0, (h)->stream>>>(__VA_ARGS__); break;               \
      case 32: KERNEL<32><<<(GRID), kBlock, 0, (h)->stream>>>(__VA_ARGS__); break;               \
      default: KERNEL<64><<<(GRID), kBlock, 0, (h)->stream>>>(__VA_ARGS__); break;               \
    }                                                                                            \
  } while (0)

}  // namespace

namespace {

void take_events(afc_handle_s* h, hipEvent_t* a, hipEvent_t* b) {
  if (h->ev_pool.size() >= 2) {
    *a = h->ev_pool.back();
    h->ev_pool.pop_back();
    *b = h->ev_pool.back();
    h->ev_pool.pop_back();
  } else {
    (void)hipEventCreate(a);
    (void)hipEventCreate(b);
  }
}

// Launch on the handle's stream.  With per-kernel timing on, the start and
// stop events ride on the dispatch itself (hipExtLaunchKernel), so the time
// folded into the totals is the kernel's own execution, with no gap from
// separately recorded event packets.
template <typename... KArgs, typename... Args>
void launch_shm(H* h, int kid, void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shm, Args... args) {
  if (!h->opt.profile) {
    kernel<<<grid, block, shm, h->stream>>>(args...);
    return;
  }
  hipEvent_t a, b;
  take_events(h, &a, &b);
  hipExtLaunchKernelGGL(kernel, grid, block, shm, h->stream, a, b, 0, static_cast<KArgs>(args)...);
  h->ev_pending.push_back({a, b, kid});
}

template <typename... KArgs, typename... Args>
void launch(H* h, int kid, void (*kernel)(KArgs...), dim3 grid, dim3 block, Args... args) {
  launch_shm(h, kid, kernel, grid, block, 0, args...);
}

}  // namespace

#define AFC_DISPATCH_G_TIMED(h, KID, KERNEL, GRID, ...)                         \
  do {                                                                          \
    switch ((h)->G) {                                                           \
      case 8: launch((h), (KID), KERNEL<8>, (GRID), kBlock, __VA_ARGS__); break;   \
      case 16: launch((h), (KID), KERNEL<16>, (GRID), kBlock, __VA_ARGS__); break; \
      case 32: launch((h), (KID), KERNEL<32>, (GRID), kBlock, __VA_ARGS__); break; \
      default: launch((h), (KID), KERNEL<64>, (GRID), kBlock, __VA_ARGS__); break; \
    }                                                                           \
  } while (0)

void prof_collect(afc_handle_s* h) {
  for (auto& e : h->ev_pending) {
    (void)hipEventSynchronize(e.b);
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      h->prof_ms[e.kid] += ms;
      h->prof_n[e.kid] += 1;
    }
    h->ev_pool.push_back(e.a);
    h->ev_pool.push_back(e.b);
  }
  h->ev_pending.clear();
}

namespace {
// bytes of the SELL matrix stream: values, per-row offsets, patterns, headers
double sell_matrix_bytes(const H* h, int value_bytes) {
  return (double)value_bytes * (double)h->sell_slots + (h->dlt16 ? 2.0 : 4.0) * (double)h->sell_lane_deltas +
         4.0 * (double)h->sell_pat_ints + 8.0 * (double)h->nslices + 4.0;
}

// the FP32 Krylov matrix (off-diagonal layout)
double krylov_matrix_bytes(const H* h) {
  return 4.0 * (double)h->ks_slots + (h->ks_dlt16 ? 2.0 : 4.0) * (double)h->ks_lane_deltas +
         4.0 * (double)h->ks_pat_ints + 8.0 * (double)h->nslices + 4.0;
}
}  // namespace

void prof_release(afc_handle_s* h) {
  prof_collect(h);
  for (auto e : h->ev_pool) (void)hipEventDestroy(e);
  h->ev_pool.clear();
}

void finish_from(H* h, const double* partials, int nb, int nv, int act, int red_off = 0, int k = 0, int m = 0,
                 int mode = 0, double p1 = 0.0, double p2 = 0.0, int prow = 0) {
  launch(h, AFC_KERNEL_FINISH, k_finish, 1, kFinish, h->ks, partials, nb, nv, act, red_off, k, m, mode, p1, p2, prow);
}

void finish(H* h, int nb, int nv, int act, int red_off = 0, int k = 0, int m = 0, int mode = 0, double p1 = 0.0,
            double p2 = 0.0, int prow = 0) {
  finish_from(h, h->partials, nb, nv, act, red_off, k, m, mode, p1, p2, prow);
}

void copy(H* h, double* dst, const double* src) { k_copy<<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, dst, src); }

void set_dirichlet(H* h, double* u) {
  k_set_dirichlet<<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, u, h->is_dir, h->uD);
}

void rhs_dirichlet(H* h, double* b, const double* F) {
  k_rhs_dirichlet<<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, b, F, h->is_dir, h->uD);
}

void fill(H* h, double* u, double v) { k_fill<<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, u, v); }

void norm2(H* h, const double* x, int red_idx) {
  const int nb = vec_grid(h);
  k_norm2<<<nb, kBlock, 0, h->stream>>>(h->N, x, h->ks, red_idx, h->partials);
  finish(h, nb, 1, ACT_STORE, red_idx);
}

void relax(H* h, double* u, const double* x, double omega) {
  k_relax<<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, u, x, omega);
}



int vec16_grid(const H* h, int elems_per_block) {
  return std::max(1, std::min((h->N + elems_per_block - 1) / elems_per_block, kRedBlocks));
}

int sell_grid(const H* h, bool reduce) {
  const int nt = (h->nslices + kBlock / 64 - 1) / (kBlock / 64);
  return std::max(1, std::min(nt, reduce ? kRedBlocks : kRowGridCap));
}

SellView sell_view(const H* h) { return SellView{h->N, h->nslices, h->sl_ptr, h->sl_dl, h->sl_pat}; }

// one workgroup per tile of slices, with partials of its own (one per workgroup)
void residual(H* h, const double* A, const double* b, const double* x, double* r, int mode) {
  const int nb = sell_grid(h, false);
  if (h->opt.profile) {
    h->prof_bytes[AFC_KERNEL_RESIDUAL] += sell_matrix_bytes(h, 8) + 24.0 * h->N + 8.0 * nb;
    h->prof_work[AFC_KERNEL_RESIDUAL] += 1;
  }
  // inside a Krylov cycle (mode 1 / 2) the residual and its restart are
  // skipped once the solve has converged
  const int* skip = mode != 0 ? &h->ks->solved : nullptr;
  if (h->dlt16)
    launch(h, AFC_KERNEL_RESIDUAL, k_sell_residual<int16_t>, nb, kBlock, sell_view(h),
           static_cast<const int16_t*>(h->sl_dlt), A, b, x, r, h->partials_res, skip);
  else
    launch(h, AFC_KERNEL_RESIDUAL, k_sell_residual<int32_t>, nb, kBlock, sell_view(h),
           static_cast<const int32_t*>(h->sl_dlt), A, b, x, r, h->partials_res, skip);
  finish_from(h, h->partials_res, nb, 1, ACT_CYCLE, 0, 0, 0, mode);
}

void to_sell8(H* h, const uint8_t* csr, uint8_t* sell) {
  k_to_sell<uint8_t><<<vec_grid(h), kBlock, 0, h->stream>>>((int)h->nnz, h->sell_pos, csr, sell);
}

void to_sell64(H* h, const double* csr, double* sell) {
  k_to_sell<double><<<vec_grid(h), kBlock, 0, h->stream>>>((int)h->nnz, h->sell_pos, csr, sell);
}

void to_sell32_scaled(H* h, const double* csr, const double* dinv, float* sell) {
  k_to_sell_scaled32<<<vec_grid(h), kBlock, 0, h->stream>>>((int)h->nnz, h->kpos, h->col, csr, dinv, sell);
}

void cycle_start(H* h, int mode, int red_idx, double tol_abs, double tol_rel) {
  k_cycle_start<<<1, 64, 0, h->stream>>>(h->ks, mode, red_idx, tol_abs, tol_rel);
}

void cast_v0(H* h, const double* r, bool fp64) {
  if (fp64)
    k_cast_v0<double><<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, r, h->V64, h->ks);
  else
    k_cast_v0<float><<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, r, h->V32, h->ks);
}

// workgroups of the GMRES vector kernels: one 16-byte access per thread and
// vector per chunk, at most kRedBlocks partials per row
int gmres_grid(const H* h, bool fp32) { return vec16_grid(h, kBlock * (fp32 ? 4 : 2)); }

void spmv64(H* h, const double* A, const double* dinv, const double* x, double theta, int rev, double* y) {
  if (h->dlt16)
    launch(h, AFC_KERNEL_SPMV64, k_sell_spmv64<int16_t>, sell_grid(h, false), kBlock, sell_view(h),
           static_cast<const int16_t*>(h->sl_dlt), A, dinv, x, (const KState*)h->ks, theta, rev, y);
  else
    launch(h, AFC_KERNEL_SPMV64, k_sell_spmv64<int32_t>, sell_grid(h, false), kBlock, sell_view(h),
           static_cast<const int32_t*>(h->sl_dlt), A, dinv, x, (const KState*)h->ks, theta, rev, y);
}

void gmres_spmv64(H* h, const double* A, const double* dinv, int k) {
  spmv64(h, A, dinv, h->V64 + (size_t)k * h->ldv, 0.0, 0, h->w[0]);
}

void spmv32(H* h, const float* A32, const float* x, float theta, int rev, float* y) {
  const SellView S{h->N, h->nslices, h->ks_ptr, h->ks_dl, h->ks_pat};
  if (h->ks_dlt16)
    launch(h, AFC_KERNEL_SPMV32, k_sell_spmv32<int16_t>, sell_grid(h, false), kBlock, S,
           static_cast<const int16_t*>(h->ks_dlt), A32, x, (const KState*)h->ks, theta, rev, y);
  else
    launch(h, AFC_KERNEL_SPMV32, k_sell_spmv32<int32_t>, sell_grid(h, false), kBlock, S,
           static_cast<const int32_t*>(h->ks_dlt), A32, x, (const KState*)h->ks, theta, rev, y);
}

void gmres_spmv32(H* h, const float* A32, int k) {
  spmv32(h, A32, h->V32 + (size_t)k * h->ldv, 0.0f, 0, reinterpret_cast<float*>(h->w[0]));
}

void gmres_dots(H* h, bool fp32, int k) {
  const int nb = gmres_grid(h, fp32);
  if (fp32)
    launch(h, AFC_KERNEL_DOTS, k_gmres_dots<float>, nb, kBlock, h->N, h->ldv, (const float*)h->V32,
           reinterpret_cast<const float*>(h->w[0]), k, (const KState*)h->ks, h->partials);
  else
    launch(h, AFC_KERNEL_DOTS, k_gmres_dots<double>, nb, kBlock, h->N, h->ldv, (const double*)h->V64,
           (const double*)h->w[0], k, (const KState*)h->ks, h->partials);
}

void gmres_reduce(H* h, bool fp32, int k, int m) {
  launch(h, AFC_KERNEL_FINISH, k_gmres_reduce, k + (k > 0 ? 2 : 1), kBlock, h->ks, (const double*)h->partials,
         gmres_grid(h, fp32), gmres_grid(h, fp32), k, m);
}

void gmres_update(H* h, bool fp32, int k) {
  const int nb = gmres_grid(h, fp32);
  if (fp32)
    launch(h, AFC_KERNEL_UPDATE, k_gmres_update<float>, nb, kBlock, h->N, h->ldv, h->V32,
           reinterpret_cast<const float*>(h->w[0]), k, (const KState*)h->ks, h->partials);
  else
    launch(h, AFC_KERNEL_UPDATE, k_gmres_update<double>, nb, kBlock, h->N, h->ldv, h->V64,
           (const double*)h->w[0], k, (const KState*)h->ks, h->partials);
}

void gmres_last_givens(H* h, bool fp32, int k, int m) {
  finish(h, gmres_grid(h, fp32), 1, ACT_GIVENS, 0, k, m, 0, 0.0, 0.0, kNormRow);
}

// workgroups of the s-step projections (one 16-byte chunk per thread and
// vector per pass): at most 1024, as many as stay resident at four waves per
// SIMD, so that no workgroup starts late and runs its chunk alone at the end
int sstep_grid(const H* h) { return std::min(vec16_grid(h, kBlock * 4), 1024); }

// blocks of up to eight vectors: wave reductions (LDS holds the output rows of
// every wave); larger blocks: the FP64 matrix cores, in row tiles of 16
template <typename T>
void sstep_dots_t(H* h, const T* V, int k, int s) {
  if (s <= 8) {
    const size_t shm = sizeof(double) * ((size_t)(k + 1) * s + s * (s + 1) / 2) * (kBlock / 64);
    const int nb = std::min(vec16_grid(h, kBlock * (int)(16 / sizeof(T))), 1024);
    launch_shm(h, AFC_KERNEL_DOTS, k_sstep_dots<T>, nb, kBlock, shm, h->N, h->ldv, V, k, s, (const KState*)h->ks,
               h->partials_blk);
    return;
  }
  const int nt = (k + 1 + s + 15) / 16;
#define AFC_DOTS_MFMA(NT)                                                                                       \
  launch(h, AFC_KERNEL_DOTS, k_sstep_dots_mfma<T, NT>, sstep_grid(h), kBlock, h->N, h->ldv, V, k, s, \
         (const KState*)h->ks, h->partials_blk)
  static_assert(kMaxRestart + 1 <= 5 * 16, "row tiles of the largest block");
  switch (nt) {
    case 1: AFC_DOTS_MFMA(1); break;
    case 2: AFC_DOTS_MFMA(2); break;
    case 3: AFC_DOTS_MFMA(3); break;
    case 4: AFC_DOTS_MFMA(4); break;
    default: AFC_DOTS_MFMA(5); break;
  }
#undef AFC_DOTS_MFMA
}

// partial slots per output row of the projections just launched
int sstep_dots_grid(const H* h, int s, bool fp64) {
  return s <= 8 ? std::min(vec16_grid(h, kBlock * (fp64 ? 2 : 4)), 1024) : sstep_grid(h);
}

void sstep_dots(H* h, int k, int s, bool fp64) {
  if (fp64)
    sstep_dots_t<double>(h, h->V64, k, s);
  else
    sstep_dots_t<float>(h, h->V32, k, s);
}

void sstep_reduce(H* h, int k, int s, int m, double theta, bool fp64) {
  const int nrows = (k + 1) * s + s * (s + 1) / 2;
  launch(h, AFC_KERNEL_FINISH, k_sstep_sums, nrows, kBlock, h->ks, (const double*)h->partials_blk,
         sstep_dots_grid(h, s, fp64));
  if (s <= 8)
    launch(h, AFC_KERNEL_FINISH, k_sstep_small<8>, 1, kBlock, h->ks, k, s, m, theta);
  else
    launch(h, AFC_KERNEL_FINISH, k_sstep_small<kSMax>, 1, kBlock, h->ks, k, s, m, theta);
}

// blocks of up to eight vectors: FP64 FMAs per element; larger blocks: the
// FP64 matrix cores, in row groups of four (K = s + k + 1 <= m rows)
template <typename T>
void sstep_update_t(H* h, T* V, int k, int s) {
  if (s <= 8) {
    launch(h, AFC_KERNEL_UPDATE, k_sstep_update<T>, gmres_grid(h, sizeof(T) == 4), kBlock, h->N, h->ldv, V, k, s,
           (const KState*)h->ks);
    return;
  }
  const int kg = (k + 1 + s + 3) / 4;
  const int nb = sstep_grid(h);
  static_assert(kMaxRestart <= 4 * 16, "row groups of the largest updated block");
  if (kg <= 4)
    launch(h, AFC_KERNEL_UPDATE, k_sstep_update_mfma<T, 4>, nb, kBlock, h->N, h->ldv, V, k, s, (const KState*)h->ks);
  else if (kg <= 8)
    launch(h, AFC_KERNEL_UPDATE, k_sstep_update_mfma<T, 8>, nb, kBlock, h->N, h->ldv, V, k, s, (const KState*)h->ks);
  else if (kg <= 12)
    launch(h, AFC_KERNEL_UPDATE, k_sstep_update_mfma<T, 12>, nb, kBlock, h->N, h->ldv, V, k, s,
           (const KState*)h->ks);
  else
    launch(h, AFC_KERNEL_UPDATE, k_sstep_update_mfma<T, 16>, nb, kBlock, h->N, h->ldv, V, k, s,
           (const KState*)h->ks);
}

void sstep_update(H* h, int k, int s, bool fp64) {
  if (fp64)
    sstep_update_t<double>(h, h->V64, k, s);
  else
    sstep_update_t<float>(h, h->V32, k, s);
}

void gmres_solve(H* h, int m, int kb, int sb) { k_gmres_solve<<<1, 64, 0, h->stream>>>(h->ks, m, kb, sb); }

void sstep_xupdate(H* h, int kb, int sb, const double* dinv, double* x, bool fp64) {
  if (fp64)
    k_sstep_xupdate<double><<<vec16_grid(h, kBlock * 2), kBlock, 0, h->stream>>>(h->N, h->ldv, h->V64, dinv, x,
                                                                                  h->ks, kb, sb);
  else
    k_sstep_xupdate<float><<<vec16_grid(h, kBlock * 4), kBlock, 0, h->stream>>>(h->N, h->ldv, h->V32, dinv, x,
                                                                                 h->ks, kb, sb);
}

void gmres_xupdate(H* h, bool fp32, const double* dinv, double* x) {
  if (fp32)
    k_gmres_xupdate<float><<<vec16_grid(h, kBlock * 4), kBlock, 0, h->stream>>>(h->N, h->ldv, h->V32, dinv, x,
                                                                                h->ks);
  else
    k_gmres_xupdate<double><<<vec16_grid(h, kBlock * 2), kBlock, 0, h->stream>>>(h->N, h->ldv, h->V64, dinv, x,
                                                                                 h->ks);
}

// One application of a Krylov operator of the stationary MCL system (A_low,
// D = diag(A_low)) by the solvers' own SELL kernels: op 0 y := y - A x (the
// FP64 residual kernel), 1 y = A D^{-1} x (FP64 SpMV of the FP64 GMRES), 2 the
// same in FP32 (the Jacobi-scaled FP32 copy and the FP32 SpMV of the mixed
// GMRES, x and y converted), 3 y = A D^{-1} x by the BiCGStab SpMV.  tmp
// holds ldv doubles (op 0: a copy of the input y, taken by the caller, as the
// kernel's b; op 2: the two FP32 vectors).  The SpMV kernels skip their work once a solve is flagged done,
// so the flag is cleared first.
__global__ void k_to_f32(int N, const double* __restrict__ x, float* __restrict__ y) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) y[i] = (float)x[i];
}
__global__ void k_to_f64(int N, const float* __restrict__ x, double* __restrict__ y) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) y[i] = (double)x[i];
}
__global__ void k_clear_done(KState* ks) { ks->done = 0; }

void apply_operator(H* h, int op, const double* x, double* y, double* tmp) {
  float* tmp32 = reinterpret_cast<float*>(tmp);
  k_clear_done<<<1, 1, 0, h->stream>>>(h->ks);
  const int nb = sell_grid(h, false);
  if (op == 0) {
    if (h->dlt16)
      k_sell_residual<int16_t><<<nb, kBlock, 0, h->stream>>>(sell_view(h), static_cast<const int16_t*>(h->sl_dlt),
                                                              h->S64_mcl, tmp, x, y, h->partials_res, nullptr);
    else
      k_sell_residual<int32_t><<<nb, kBlock, 0, h->stream>>>(sell_view(h), static_cast<const int32_t*>(h->sl_dlt),
                                                              h->S64_mcl, tmp, x, y, h->partials_res, nullptr);
  } else if (op == 1) {
    spmv64(h, h->S64_mcl, h->dinv_mcl, x, 0.0, 0, y);
  } else if (op == 2) {
    k_to_f32<<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, x, tmp32);
    spmv32(h, h->S32_mcl, tmp32, 0.0f, 0, tmp32 + h->ldv);
    k_to_f64<<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, tmp32 + h->ldv, y);
  } else {
    const int nr = sell_grid(h, true);
    if (h->dlt16)
      k_bicg_v<int16_t><<<nr, kBlock, 0, h->stream>>>(sell_view(h), static_cast<const int16_t*>(h->sl_dlt),
                                                       h->S64_mcl, h->dinv_mcl, x, x, y, h->ks, h->partials);
    else
      k_bicg_v<int32_t><<<nr, kBlock, 0, h->stream>>>(sell_view(h), static_cast<const int32_t*>(h->sl_dlt),
                                                       h->S64_mcl, h->dinv_mcl, x, x, y, h->ks, h->partials);
  }
}

void bicg_init(H* h, const BicgVec& b, double tol) {
  const int nb = vec_grid(h);
  k_bicg_init<<<nb, kBlock, 0, h->stream>>>(h->N, b.r, b.rhat, b.p, b.v, h->ks, h->partials, tol);
  finish(h, nb, 1, ACT_BICG_INIT, 0, 0, 0, 0, tol);
}

void bicg_iter(H* h, const double* A, const double* dinv, const BicgVec& b) {
  const int nr = sell_grid(h, true), nv = vec_grid(h);
  if (h->dlt16)
    k_bicg_v<int16_t><<<nr, kBlock, 0, h->stream>>>(sell_view(h), static_cast<const int16_t*>(h->sl_dlt), A, dinv,
                                                     b.p, b.rhat, b.v, h->ks, h->partials);
  else
    k_bicg_v<int32_t><<<nr, kBlock, 0, h->stream>>>(sell_view(h), static_cast<const int32_t*>(h->sl_dlt), A, dinv,
                                                     b.p, b.rhat, b.v, h->ks, h->partials);
  finish(h, nr, 1, ACT_BICG_ALPHA);
  k_bicg_s<<<nv, kBlock, 0, h->stream>>>(h->N, b.r, b.v, b.s, h->ks, h->partials);
  finish(h, nv, 1, ACT_BICG_S);
  if (h->dlt16)
    k_bicg_t<int16_t><<<nr, kBlock, 0, h->stream>>>(sell_view(h), static_cast<const int16_t*>(h->sl_dlt), A, dinv,
                                                     b.s, b.t, h->ks, h->partials);
  else
    k_bicg_t<int32_t><<<nr, kBlock, 0, h->stream>>>(sell_view(h), static_cast<const int32_t*>(h->sl_dlt), A, dinv,
                                                     b.s, b.t, h->ks, h->partials);
  finish(h, nr, 2, ACT_BICG_OMEGA);
  k_bicg_xr<<<nv, kBlock, 0, h->stream>>>(h->N, dinv, b.p, b.s, b.t, b.rhat, b.x, b.r, h->ks, h->partials);
  finish(h, nv, 2, ACT_BICG_RHO);
  k_bicg_p<<<nv, kBlock, 0, h->stream>>>(h->N, b.r, b.v, b.p, h->ks);
}

static FctSell fct_sell(const H* h) {
  return FctSell{sell_view(h), h->sl_dlt, (int)h->dlt16, h->sl_mask, h->S_mij, h->S_dp, h->S_alf};
}

void mu_R(H* h, const double* u, double* Rp, double* Rm) {
  launch(h, AFC_KERNEL_MCL, k_mu_R, sell_grid(h, false), kBlock, fct_sell(h), (const uint8_t*)h->S_own, u,
         (const uint8_t*)h->is_dir, Rp, Rm);
}

void mu_apply(H* h, const double* u, const double* Rp, const double* Rm, const double* F, double* b, double* r) {
  const int nb = sell_grid(h, true);
  launch(h, AFC_KERNEL_MCL, k_mu_apply, nb, kBlock, fct_sell(h), (const uint8_t*)h->S_own, (const double*)h->S64_cn,
         u, Rp, Rm, F, (const uint8_t*)h->is_dir, (const double*)h->uD, h->opt.alpha_mode, b, r, h->partials);
  finish(h, nb, 3, ACT_STORE);
}

void mc_lowrate(H* h, const double* u, const double* F, double* udot, double* scratch) {
  k_ssp_lowrate_sell<<<sell_grid(h, false), kBlock, 0, h->stream>>>(
      sell_view(h), (const void*)h->sl_dlt, (int)h->dlt16, (const uint32_t*)h->sl_mask, (const double*)h->S64_mcl, u, F,
      (const double*)h->ml, (const uint8_t*)h->is_dir, (const double*)h->uD, 0.0, udot, scratch);
}

static McSell mc_sell(const H* h) {
  return McSell{sell_view(h), h->sl_dlt, (int)h->dlt16, h->sl_mask, h->S_mij, h->Scc, h->SccT};
}

void mc_stage(H* h, const double* u, const double* udot, const double* umax, const double* umin, double dt,
              const double* u0, double c0, double c1, double* out) {
  k_mc_stage<<<sell_grid(h, false), kBlock, 0, h->stream>>>(mc_sell(h), h->ml, h->is_dir, h->uD, u, udot, umax, umin,
                                                             dt, u0, c0, c1, h->opt.alpha_mode, out);
}

void mc_cn_g(H* h, const double* uo, const double* udot, const double* umax, const double* umin, const double* Fn,
             double dt, double* g) {
  k_mc_cn_g<<<sell_grid(h, false), kBlock, 0, h->stream>>>(mc_sell(h), h->ml, h->is_dir, h->uD, uo, udot, umax, umin,
                                                            Fn, 1.0 / dt, h->opt.alpha_mode, g);
}

void mc_cn_apply(H* h, const double* u, const double* udot, const double* umax, const double* umin, const double* g,
                 double* b, double* r) {
  const int nb = sell_grid(h, true);
  k_mc_cn_apply<<<nb, kBlock, 0, h->stream>>>(mc_sell(h), h->S64_cn, u, udot, umax, umin, g, h->is_dir, h->uD,
                                               h->opt.alpha_mode, b, r, h->partials);
  finish(h, nb, 3, ACT_STORE);
}

void ssp_lowrate(H* h, const double* u, const double* F, double dt, double* udot, double* ut) {
  k_ssp_lowrate_sell<<<sell_grid(h, false), kBlock, 0, h->stream>>>(sell_view(h), (const void*)h->sl_dlt, (int)h->dlt16,
         (const uint32_t*)h->sl_mask, (const double*)h->S_alf, u, F, (const double*)h->ml, (const uint8_t*)h->is_dir,
         (const double*)h->uD, dt, udot, ut);
}

void ssp_limit_R(H* h, const double* u, const double* udot, const double* ut, double dt, double* Rp, double* Rm) {
  k_ssp_limit_R_sell<<<sell_grid(h, false), kBlock, 0, h->stream>>>(sell_view(h), (const void*)h->sl_dlt, (int)h->dlt16,
         (const uint32_t*)h->sl_mask, (const double*)h->S_mij, (const double*)h->S_dp, u, udot, ut,
         (const double*)h->ml, (const uint8_t*)h->is_dir, dt, Rp, Rm);
}

void ssp_apply(H* h, const double* u, const double* udot, const double* ut, const double* Rp, const double* Rm,
               double dt, const double* base, double c0, double c1, double* out) {
  k_ssp_apply_sell<<<sell_grid(h, false), kBlock, 0, h->stream>>>(sell_view(h), (const void*)h->sl_dlt, (int)h->dlt16,
         (const uint32_t*)h->sl_mask, (const double*)h->S_mij, (const double*)h->S_dp, u, udot, ut, Rp, Rm,
         (const double*)h->ml, (const uint8_t*)h->is_dir, (const double*)h->uD, dt, h->opt.alpha_mode, base, c0, c1,
         out);
}


void cn_predict(H* h, const double* u_old, const double* F_old, const double* F_new, double dt, double* ut,
                double* g) {
  k_cn_predict<<<sell_grid(h, false), kBlock, 0, h->stream>>>(fct_sell(h), u_old, F_old, F_new, h->ml, h->is_dir,
                                                               h->uD, dt, ut, g);
}

void cn_extrapolate(H* h, const double* ut, const double* uo, double* us) {
  k_cn_extrapolate<<<vec_grid(h), kBlock, 0, h->stream>>>(h->N, ut, uo, h->is_dir, h->uD, us);
}

void zalesak_Q(H* h, const double* ut, double* Qp, double* Qm) {
  k_zalesak_Q<<<sell_grid(h, false), kBlock, 0, h->stream>>>(fct_sell(h), ut, Qp, Qm);
}

void cn_limit_R(H* h, const double* u, const double* u_old, const double* Qp, const double* Qm, double dt,
                double* Rp, double* Rm) {
  k_cn_limit_R<<<sell_grid(h, false), kBlock, 0, h->stream>>>(fct_sell(h), u, u_old, Qp, Qm, h->ml, h->is_dir, dt,
                                                               h->opt.prelimit, Rp, Rm);
}

void cn_apply(H* h, const double* u, const double* u_old, const double* Rp, const double* Rm, const double* g,
              double dt, double* b, double* r) {
  const int nb = sell_grid(h, true);
  k_cn_apply<<<nb, kBlock, 0, h->stream>>>(fct_sell(h), h->S64_cn, u, u_old, Rp, Rm, g, h->is_dir, h->uD, dt,
                                           h->opt.prelimit, h->opt.alpha_mode, b, r, h->partials);
  finish(h, nb, 3, ACT_STORE);
}

// bytes of the SELL slice headers, patterns and per-lane deltas
static double sell_index_bytes(const H* h) {
  return (double)h->sell_pat_ints * 4.0 + (double)h->sell_lane_deltas * (h->dlt16 ? 2.0 : 4.0) +
         8.0 * h->nslices + 4.0;
}

void mcl_bounds(H* h, const double* u, double* umax, double* umin) {
  if (h->opt.profile) {  // slice index, masks, u, u^max, u^min
    h->prof_bytes[AFC_KERNEL_MCL] += sell_index_bytes(h) + 4.0 * h->mask_words * h->N + 24.0 * h->N;
    h->prof_work[AFC_KERNEL_MCL] += 1;
  }
  launch(h, AFC_KERNEL_MCL, k_mcl_bounds_sell, sell_grid(h, false), kBlock, sell_view(h), (const void*)h->sl_dlt,
         (int)h->dlt16, (const uint32_t*)h->sl_mask, u, umax, umin);
}

void mcl_apply(H* h, const double* u, const double* umax, const double* umin, const double* F, double* b, double* r) {
  const int nb = sell_grid(h, true);
  if (h->opt.profile) {  // slice index, masks, A_low, c_ij, c_ji slots; u, bounds, F, u_D, flags; b, r, partials
    h->prof_bytes[AFC_KERNEL_MCL] +=
        sell_index_bytes(h) + 4.0 * h->mask_words * h->N + 24.0 * h->sell_slots + 57.0 * h->N + 24.0 * nb;
    h->prof_work[AFC_KERNEL_MCL] += 1;
  }
  launch(h, AFC_KERNEL_MCL, k_mcl_apply_sell, nb, kBlock, sell_view(h), (const void*)h->sl_dlt, (int)h->dlt16,
         (const uint32_t*)h->sl_mask, (const double*)h->Scc, (const double*)h->SccT, (const double*)h->S64_mcl, u,
         umax, umin, F, (const uint8_t*)h->is_dir, (const double*)h->uD, h->opt.alpha_mode, b, r, h->partials);
  finish(h, nb, 3, ACT_STORE);
}

void build_cn_matrix(H* h, const double* AL, double dt) {
  const double scale = dt > 0.0 ? 0.5 : 1.0, inv_dt = dt > 0.0 ? 1.0 / dt : 0.0;
  AFC_DISPATCH_G(h, k_build_cn, row_grid(h, false), h->N, h->row_ptr, h->col, AL, h->ml, h->is_dir, scale, inv_dt,
                 h->A_cn, h->dinv_cn);
  to_sell64(h, h->A_cn, h->S64_cn);
  to_sell32_scaled(h, h->A_cn, h->dinv_cn, h->S32_cn);
}

void prof_gmres_cycle(afc_handle_s* h, bool fp32, int m, int kk) {
  if (!h->opt.profile) return;
  const double vb = fp32 ? 4.0 : 8.0;
  const double N = (double)h->N;
  const int kid = fp32 ? AFC_KERNEL_SPMV32 : AFC_KERNEL_SPMV64;
  const double nbv = (double)gmres_grid(h, fp32);
  // SpMV and projections of step k did work for k <= kk (the step after the
  // last completed column still runs: that column's Givens comes after it)
  const int nspmv = std::min(kk + 1, m);
  for (int k = 0; k < nspmv; ++k) {
    // matrix, x = V[k] (FP64: and the Jacobi scales), y
    h->prof_bytes[kid] += (fp32 ? krylov_matrix_bytes(h) : sell_matrix_bytes(h, 8)) + vb * N * (fp32 ? 1.0 : 2.0) + vb * N;
    h->prof_work[kid] += 1;
    // V[0..k], W, partials
    h->prof_bytes[AFC_KERNEL_DOTS] += vb * N * (k + 2) + 8.0 * nbv * (k + 1);
    h->prof_work[AFC_KERNEL_DOTS] += 1;
  }
  // update of step k did work for k < kk
  for (int k = 0; k < std::min(kk, m); ++k) {
    h->prof_bytes[AFC_KERNEL_UPDATE] += vb * N * (k + 1) + 2.0 * vb * N + 8.0 * nbv;
    h->prof_work[AFC_KERNEL_UPDATE] += 1;
  }
}

void prof_sstep_cycle(afc_handle_s* h, int m, int s, int kk, bool fp64) {
  if (!h->opt.profile) return;
  const double N = (double)h->N;
  const double vb = fp64 ? 8.0 : 4.0;
  const int kid = fp64 ? AFC_KERNEL_SPMV64 : AFC_KERNEL_SPMV32;
  // blocks that ran: up to the one holding column kk (a converged block still
  // orthonormalizes its vectors)
  for (int k = 0; k < m && k <= kk; k += s) {
    const int sb = std::min(s, m - k);
    const double nbv = (double)sstep_dots_grid(h, sb, fp64);
    // matrix, x = V[k+j] (FP32: its diagonal term feeds the shift too; FP64:
    // and the Jacobi scales), y
    h->prof_bytes[kid] += sb * (fp64 ? sell_matrix_bytes(h, 8) + 3.0 * vb * N : krylov_matrix_bytes(h) + 2.0 * vb * N);
    h->prof_work[kid] += sb;
    h->prof_bytes[AFC_KERNEL_DOTS] += vb * N * (k + 1 + sb) + 8.0 * nbv * ((k + 1) * sb + sb * (sb + 1) / 2);
    h->prof_work[AFC_KERNEL_DOTS] += 1;
    if (k + sb < m) {  // the last block is not orthogonalized in place (sstep_xupdate reads it raw)
      h->prof_bytes[AFC_KERNEL_UPDATE] += vb * N * (k + 1 + 2 * sb);
      h->prof_work[AFC_KERNEL_UPDATE] += 1;
    }
    if (k + sb >= kk && kk < m) break;
  }
}

}  // namespace afc
