// Batched Crank-Nicolson FCT: many independent CDR instances advanced by one
// persistent launch (Sec. 2.1.1 scheme, Sec. 2.1.3 limiter, Sec. 4 fixed-point
// iteration with BiCGStab-Jacobi).
//
// All instances live in one packed device layout (SELL-64 entry order, the
// diagonal first in every row).  Each workgroup of NT
// threads repeatedly takes the next instance from an atomic queue (instances
// ordered by decreasing nonzero count) and runs every time step of it: the
// CN matrix for its dt, the low-order predictor, the limiter passes, the
// nonlinear residual and the BiCGStab solves.  Phases are separated by
// workgroup barriers and all reductions are LDS sums in a fixed order, so an
// instance's result does not depend on which workgroup ran it or on what else
// is in the batch.  The queue ends the loop of every workgroup.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

#include "afc_batch_internal.h"
#include "afc_device.h"

namespace afc {
namespace {

// Reductions follow one canonical order whatever the workgroup size: rows are
// visited as if by kVW waves (virtual wave v takes slices v, v + kVW, ...;
// lane l the row 64 s + l), each virtual wave accumulates per lane in slice
// order, and the kVW wave totals are added in virtual-wave order.  A workgroup
// of NT threads runs its NT/64 real waves over virtual waves w, w + NT/64, ...
// with one accumulator set per virtual wave, so every schedule (workgroup size,
// number of workgroups) gives bitwise identical results.
constexpr int kVW = 16;

template <int NT>
struct Sched {
  static constexpr int NW = NT / 64;
  static constexpr int PER = kVW / NW;  // virtual waves per real wave
  static_assert(NW * PER == kVW, "workgroup size must divide 16 waves");
};

enum BatchWork { BW_UOLD = 0, BW_UT, BW_G, BW_QP, BW_QM, BW_RP, BW_RM, BW_B, BW_R, BW_X, BW_RHAT, BW_P, BW_V, BW_S,
                 BW_T, BW_PH, BW_SH, BW_COUNT };

// Totals of NV sums accumulated per virtual wave (acc[c] belongs to virtual
// wave w + c NW); every thread receives them.
template <int NT, int NV>
__device__ void wg_sum(const double (&acc)[Sched<NT>::PER][NV], double (&out)[NV]) {
  constexpr int NW = Sched<NT>::NW, PER = Sched<NT>::PER;
  __shared__ double sh[NV][kVW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < PER; ++c)
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double s = wave_sum(acc[c][q]);
      if (lane == 0) sh[q][wv + c * NW] = s;
    }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = 0.0;
#pragma unroll
    for (int v = 0; v < kVW; ++v) t += sh[q][v];
    out[q] = t;
  }
  __syncthreads();
}

struct InstView {
  int N, nsl;
  const int* slp;
  const int16_t* dlt;
  const double *mij, *dp, *AL, *ml, *uD;
  const uint8_t* isd;
  double *Acn, *dinv;
  double* w[BW_COUNT];
  double* u;
  const double* F;
};

// Row loops in the canonical order: C is the index of the running virtual
// wave among this real wave's (accumulator set acc[C]); lane l owns row
// 64 s + l and walks its slots p = 0..L-1 (p = 0 is the diagonal; padding
// slots point at the row itself with zero values).
#define AFC_ROWS(I, NT, C)                                                                          \
  _Pragma("unroll") for (int C = 0; C < Sched<NT>::PER; ++C)                                        \
    for (int s_ = (int)(threadIdx.x >> 6) + C * Sched<NT>::NW; s_ < (I).nsl; s_ += kVW)              \
      if (const int i = s_ * 64 + (int)(threadIdx.x & 63); i < (I).N)

struct RowSpan {
  int base, L;
};
__device__ __forceinline__ RowSpan row_span(const InstView& I, int i) {
  const int s = i >> 6;
  const int b = I.slp[s];
  return {b + (i & 63), (I.slp[s + 1] - b) >> 6};
}

// y_i = sum_j A_ij xh_j with xh = D^{-1} x already formed; returns sum_i z_i y_i
template <int NT>
__device__ double wg_spmv_prec(const InstView& I, const double* A, const double* xh, double* y, const double* z) {
  double acc[Sched<NT>::PER][1] = {};
  AFC_ROWS(I, NT, c) {
    const RowSpan rs = row_span(I, i);
    double sacc = 0.0;
#pragma unroll 4
    for (int p = 0; p < rs.L; ++p) {
      const int k = rs.base + 64 * p;
      sacc += A[k] * xh[i + I.dlt[k]];
    }
    y[i] = sacc;
    acc[c][0] += z[i] * sacc;
  }
  double out[1];
  wg_sum<NT, 1>(acc, out);
  return out[0];
}

// r = b - A x over the instance; returns ||r||^2
template <int NT>
__device__ double wg_residual(const InstView& I, const double* A, const double* b, const double* x, double* r) {
  double acc[Sched<NT>::PER][1] = {};
  AFC_ROWS(I, NT, c) {
    const RowSpan rs = row_span(I, i);
    double sacc = 0.0;
#pragma unroll 4
    for (int p = 0; p < rs.L; ++p) {
      const int k = rs.base + 64 * p;
      sacc += A[k] * x[i + I.dlt[k]];
    }
    const double ri = b[i] - sacc;
    r[i] = ri;
    acc[c][0] += ri * ri;
  }
  double out[1];
  wg_sum<NT, 1>(acc, out);
  return out[0];
}

// BiCGStab (van der Vorst, right Jacobi) on A_cn x = b inside one workgroup.
// r holds b - A x on entry (squared norm rr).  Returns the iterations done;
// *status is 0, AFC_ENOCONV, AFC_EBREAKDOWN or AFC_ENAN; *res the final true
// residual norm.
template <int NT>
__device__ int wg_bicgstab(const InstView& I, const double* b, double* x, double rr, double tol, int maxit,
                           int* status, double* res) {
  double* r = I.w[BW_R];
  double* rhat = I.w[BW_RHAT];
  double* p = I.w[BW_P];
  double* v = I.w[BW_V];
  double* s = I.w[BW_S];
  double* t = I.w[BW_T];
  double* ph = I.w[BW_PH];  // D^{-1} p and D^{-1} s, formed where p and s are
  double* sh = I.w[BW_SH];
  const double* A = I.Acn;
  const int N = I.N;
  int it = 0, restarts = 0;
  *status = 0;
  while (true) {
    for (int i = threadIdx.x; i < N; i += NT) {
      rhat[i] = r[i];
      p[i] = r[i];
      ph[i] = I.dinv[i] * r[i];
      v[i] = 0.0;
    }
    __syncthreads();
    double rho = rr, alpha = 1.0, omega = 1.0;
    double cur = sqrt(rr);
    bool breakdown = false, converged = !(cur > tol);
    if (!isfinite(cur)) {
      *status = AFC_ENAN;
      *res = cur;
      return it;
    }
    while (!converged && it < maxit) {
      double q1[1] = {wg_spmv_prec<NT>(I, A, ph, v, rhat)};
      if (q1[0] == 0.0 || !isfinite(q1[0])) {
        breakdown = true;
        break;
      }
      alpha = rho / q1[0];
      double a2[Sched<NT>::PER][1] = {};
      AFC_ROWS(I, NT, c) {
        const double si = r[i] - alpha * v[i];
        s[i] = si;
        sh[i] = I.dinv[i] * si;
        a2[c][0] += si * si;
      }
      double q2[1];
      wg_sum<NT, 1>(a2, q2);
      ++it;
      if (sqrt(q2[0]) <= tol) {
        for (int i = threadIdx.x; i < N; i += NT) {
          x[i] += alpha * ph[i];
          r[i] = s[i];
        }
        __syncthreads();
        converged = true;
        break;
      }
      double a3[Sched<NT>::PER][2] = {};
      AFC_ROWS(I, NT, c) {
        const RowSpan rs = row_span(I, i);
        double a = 0.0;
#pragma unroll 4
        for (int pp = 0; pp < rs.L; ++pp) {
          const int k = rs.base + 64 * pp;
          a += A[k] * sh[i + I.dlt[k]];
        }
        t[i] = a;
        a3[c][0] += a * s[i];
        a3[c][1] += a * a;
      }
      double q3[2];
      wg_sum<NT, 2>(a3, q3);
      omega = q3[1] != 0.0 ? q3[0] / q3[1] : 0.0;
      double a4[Sched<NT>::PER][2] = {};
      AFC_ROWS(I, NT, c) {
        x[i] += alpha * ph[i] + omega * sh[i];
        const double ri = s[i] - omega * t[i];
        r[i] = ri;
        a4[c][0] += rhat[i] * ri;
        a4[c][1] += ri * ri;
      }
      double q4[2];
      wg_sum<NT, 2>(a4, q4);
      cur = sqrt(q4[1]);
      if (!isfinite(cur)) {
        *status = AFC_ENAN;
        *res = cur;
        return it;
      }
      if (cur <= tol) {
        converged = true;
        break;
      }
      if (q4[0] == 0.0 || omega == 0.0) {
        breakdown = true;
        break;
      }
      const double beta = (q4[0] / rho) * (alpha / omega);
      rho = q4[0];
      for (int i = threadIdx.x; i < N; i += NT) {
        const double pi = r[i] + beta * (p[i] - omega * v[i]);
        p[i] = pi;
        ph[i] = I.dinv[i] * pi;
      }
      __syncthreads();
    }
    // confirm on the true residual
    double q5[1] = {wg_residual<NT>(I, A, b, x, r)};
    *res = sqrt(q5[0]);
    if (!isfinite(*res)) {
      *status = AFC_ENAN;
      return it;
    }
    if (*res <= tol) return it;
    if (breakdown && ++restarts > 1) {
      *status = AFC_EBREAKDOWN;
      return it;
    }
    if (it >= maxit) {
      *status = AFC_ENOCONV;
      return it;
    }
    rr = q5[0];
  }
}

// True once the wall clock has passed `deadline` (< 0: never); the same
// answer for every thread of the workgroup.
__device__ bool past_deadline(int64_t deadline) {
  __shared__ int flag;
  if (deadline < 0) return false;
  if (threadIdx.x == 0) flag = (int64_t)wall_clock64() > deadline ? 1 : 0;
  __syncthreads();
  const bool r = flag != 0;
  __syncthreads();
  return r;
}

// Damping rule of the fixed point (reading of Sec. 4): halve omega (not below
// 1/64) when the residual grew, else omega <- min(1, 1.25 omega).
__device__ __forceinline__ double next_omega(const BatchOpts& o, const SState& st, double R) {
  if (!o.dynamic_damping || !st.have_prev) return st.omega;
  return (R > st.R_prev) ? fmax(st.omega * 0.5, 1.0 / 64.0) : fmin(1.0, st.omega * 1.25);
}

// One fixed-point update of Sec. 4 after the residual R of the current
// iterate: linear solve of A x = b from x = u (BiCGStab-Jacobi, stopping at
// max(atol, rtol ||b||, lin_eta R)), then u <- u + omega (x - u).  r holds
// b - A u (squared norm rr).  Returns false on a solver error (in st.status).
template <int NT>
__device__ bool fp_update(const InstView& I, const BatchOpts& o, SState& st, double R, double bn, double rr) {
  st.omega = next_omega(o, st, R);
  const bool relax = st.omega != 1.0;
  double* u = I.u;
  double* x = u;
  if (relax) {
    x = I.w[BW_X];
    for (int i = threadIdx.x; i < I.N; i += NT) x[i] = u[i];
    __syncthreads();
  }
  const double tol = fmax(fmax(o.lin_atol, o.lin_rtol * bn), o.lin_eta * R);
  int lst = 0;
  st.kry += wg_bicgstab<NT>(I, I.w[BW_B], x, rr, tol, o.lin_maxit, &lst, &st.lin_res);
  if (lst == AFC_ENAN || lst == AFC_EBREAKDOWN) {
    st.status = lst;
    return false;
  }
  if (relax) {
    const double om = st.omega;
    for (int i = threadIdx.x; i < I.N; i += NT) u[i] += om * (x[i] - u[i]);
  }
  __syncthreads();
  st.R_prev = R;
  st.have_prev = 1;
  ++st.nu;
  return true;
}

// Bookkeeping after the residual R (||b||: bn) of iterate nu: returns true
// when the fixed point stops here (converged, capped or non-finite).
__device__ __forceinline__ bool fp_stop(const BatchOpts& o, SState& st, int N, double R, double bn, bool first_of_run) {
  if (!isfinite(R) || !isfinite(bn)) {
    st.status = AFC_ENAN;
    return true;
  }
  if (st.nu == 0) st.R0 = R;
  if (first_of_run) st.res0 = R;
  st.res = R;
  const bool conv = (o.fp_tol_mode == AFC_TOL_ABS_SQRTN) ? (R < sqrt((double)N) * o.fp_tol) : (R <= o.fp_tol * st.R0);
  if (R == 0.0 || conv) return true;
  if (st.nu >= o.fp_maxit) {
    st.status = st.status > 0 ? st.status : AFC_WMAXIT;
    return true;
  }
  return false;
}

// CN-FCT steps of one instance (eqs. (11)-(14), Zalesak's limiter, the Sec. 4
// fixed point), resumable: returns when st.done is set or, after at least
// one fixed-point iteration of this call, at the top of an iteration once
// the wall clock passes `deadline`.
template <int NT>
__device__ void run_cn(const InstView& I, double dt, int steps, const BatchOpts& o, SState& st, int64_t deadline) {
  const int N = I.N;
  const double inv_dt = 1.0 / dt;
  double* u = I.u;
  double* uo = I.w[BW_UOLD];
  double* ut = I.w[BW_UT];
  double* g = I.w[BW_G];
  double* Qp = I.w[BW_QP];
  double* Qm = I.w[BW_QM];
  double* Rp = I.w[BW_RP];
  double* Rm = I.w[BW_RM];
  double* b = I.w[BW_B];
  double* r = I.w[BW_R];

  if (st.phase < 0) {
    // CN matrix M_L/dt + A_low/2 with Dirichlet identity rows, and its inverse diagonal
    AFC_ROWS(I, NT, c_) {
      const RowSpan rs = row_span(I, i);
      const bool dir = I.isd[i];
      for (int p = 0; p < rs.L; ++p) {
        const int k = rs.base + 64 * p;
        double v;
        if (dir)
          v = (p == 0) ? 1.0 : 0.0;
        else
          v = 0.5 * I.AL[k] + ((p == 0) ? I.ml[i] * inv_dt : 0.0);
        I.Acn[k] = v;
        if (p == 0) I.dinv[i] = 1.0 / v;
      }
    }
    __syncthreads();
    st.phase = 0;
  }
  int iters = 0;  // fixed-point iterations of this call
  while (st.step < steps && st.status >= 0) {
    if (st.phase == 0) {
      // predictor of eq. (14) and the right-hand side of eq. (11)
      AFC_ROWS(I, NT, c_) {
        const double ui = u[i];
        uo[i] = ui;
        if (I.isd[i]) {
          ut[i] = g[i] = I.uD[i];
          continue;
        }
        const RowSpan rs = row_span(I, i);
        double y = 0.0;
#pragma unroll 4
        for (int p = 0; p < rs.L; ++p) {
          const int k = rs.base + 64 * p;
          y += I.AL[k] * u[i + I.dlt[k]];
        }
        const double mi = I.ml[i];
        ut[i] = ui - 0.5 * dt * (y - I.F[i]) / mi;
        // (F^{n-1} + F^n) / 2 with a time-independent load
        g[i] = mi * inv_dt * ui - 0.5 * y + 0.5 * (I.F[i] + I.F[i]);
      }
      __syncthreads();
      // Q+- from the predictor (Sec. 2.1.3 step 2)
      AFC_ROWS(I, NT, c_) {
        const RowSpan rs = row_span(I, i);
        const double uti = ut[i];
        double qp = 0.0, qm = 0.0;
#pragma unroll 4
        for (int p = 1; p < rs.L; ++p) {
          const double du = ut[i + I.dlt[rs.base + 64 * p]] - uti;
          qp = fmax(qp, du);
          qm = fmin(qm, du);
        }
        Qp[i] = qp;
        Qm[i] = qm;
      }
      __syncthreads();
      // Dirichlet values into u (after every predictor read of u)
      AFC_ROWS(I, NT, c_) {
        if (I.isd[i]) u[i] = I.uD[i];
      }
      __syncthreads();
      st.R0 = st.R_prev = 0.0;
      st.omega = o.omega;
      st.have_prev = 0;
      st.nu = 0;
      st.phase = 1;
    }
    while (true) {
      if (iters > 0 && past_deadline(deadline)) return;
      // P+-, R+- of the prelimited CN fluxes (eqs. (12), (13))
      AFC_ROWS(I, NT, c_) {
        if (I.isd[i]) {
          Rp[i] = Rm[i] = 1.0;
          continue;
        }
        const RowSpan rs = row_span(I, i);
        const double dui = u[i] - uo[i], sui = u[i] + uo[i];
        double pp = 0.0, pm = 0.0;
#pragma unroll 4
        for (int p = 1; p < rs.L; ++p) {
          const int k = rs.base + 64 * p;
          const int j = i + I.dlt[k];
          const double rf = cn_flux(I.mij[k], -I.dp[k], inv_dt, dui, u[j] - uo[j], sui, u[j] + uo[j], o.prelimit);
          pp += fmax(rf, 0.0);
          pm += fmin(rf, 0.0);
        }
        Rp[i] = zalesak_R(I.ml[i], Qp[i], pp, dt);
        Rm[i] = zalesak_R(I.ml[i], Qm[i], pm, dt);
      }
      __syncthreads();
      // b = g + F*, r = b - A_cn u ; R^2 (free rows), ||b||^2, ||r||^2
      double acc[Sched<NT>::PER][3] = {};
      AFC_ROWS(I, NT, c) {
        if (I.isd[i]) {
          const double bi = I.uD[i], ri = I.uD[i] - u[i];
          b[i] = bi;
          r[i] = ri;
          acc[c][1] += bi * bi;
          acc[c][2] += ri * ri;
          continue;
        }
        const RowSpan rs = row_span(I, i);
        const double ui = u[i];
        const double dui = ui - uo[i], sui = ui + uo[i], rpi = Rp[i], rmi = Rm[i];
        double fs = 0.0, au = I.Acn[rs.base] * ui;
#pragma unroll 4
        for (int p = 1; p < rs.L; ++p) {
          const int k = rs.base + 64 * p;
          const int j = i + I.dlt[k];
          const double uj = u[j], uoj = uo[j], rpj = Rp[j], rmj = Rm[j];  // every gather issued at once
          au += I.Acn[k] * uj;
          if (o.alpha_mode == AFC_ALPHA_ZERO) continue;
          const double rf = cn_flux(I.mij[k], -I.dp[k], inv_dt, dui, uj - uoj, sui, uj + uoj, o.prelimit);
          double a = 1.0;
          if (o.alpha_mode == AFC_ALPHA_LIMITED) a = rf > 0.0 ? fmin(rpi, rmj) : fmin(rmi, rpj);
          fs += a * rf;
        }
        const double bi = g[i] + fs, ri = bi - au;
        b[i] = bi;
        r[i] = ri;
        acc[c][0] += ri * ri;
        acc[c][1] += bi * bi;
        acc[c][2] += ri * ri;
      }
      double red[3];
      wg_sum<NT, 3>(acc, red);
      const double R = sqrt(red[0]), bn = sqrt(red[1]);
      if (fp_stop(o, st, N, R, bn, st.step == 0 && st.nu == 0)) break;
      if (!fp_update<NT>(I, o, st, R, bn, red[2])) break;
      ++iters;
    }
    st.fp_total += st.nu;
    ++st.step;
    st.phase = 0;
  }
  st.done = 1;
}

// Stationary MCL solve of one instance (Sec. 3.1, eqs. (22)-(23), Remark 1,
// the Sec. 4 fixed point), resumable like run_cn.  A = A_low of the MCL
// scheme with Dirichlet identity rows; cc, ccT: the convective a_ij, a_ji in
// slot order.  init_low: start from the low-order solution A u = F (from
// zero), else from the caller's u.
template <int NT>
__device__ void run_mcl(const InstView& I, const double* cc, const double* ccT, int init_low, const BatchOpts& o,
                        SState& st, int64_t deadline) {
  const int N = I.N;
  double* u = I.u;
  double* umax = I.w[BW_QP];
  double* umin = I.w[BW_QM];
  double* b = I.w[BW_B];
  double* r = I.w[BW_R];
  const double* A = I.Acn;
  if (st.phase < 0) {
    if (init_low) {
      double acc[Sched<NT>::PER][1] = {};
      AFC_ROWS(I, NT, c) {
        const double bi = I.isd[i] ? I.uD[i] : I.F[i];
        b[i] = bi;
        u[i] = I.isd[i] ? I.uD[i] : 0.0;
        acc[c][0] += bi * bi;
      }
      double bn2[1];
      wg_sum<NT, 1>(acc, bn2);
      const double rr = wg_residual<NT>(I, A, b, u, r);
      const double tol = fmax(o.lin_atol, o.lin_rtol * sqrt(bn2[0]));
      int lst = 0;
      st.kry += wg_bicgstab<NT>(I, b, u, rr, tol, o.lin_maxit, &lst, &st.lin_res);
      if (lst == AFC_ENAN) {
        st.status = lst;
        st.done = 1;
        return;
      }
    } else {
      AFC_ROWS(I, NT, c_) {
        if (I.isd[i]) u[i] = I.uD[i];
      }
      __syncthreads();
    }
    st.R0 = st.R_prev = 0.0;
    st.omega = o.omega;
    st.have_prev = 0;
    st.nu = 0;
    st.phase = 1;
  }
  int iters = 0;
  while (true) {
    if (iters > 0 && past_deadline(deadline)) return;
    // local bounds u^max_i, u^min_i over N_i, i included (eq. (23))
    AFC_ROWS(I, NT, c_) {
      const RowSpan rs = row_span(I, i);
      double mx = u[i], mn = u[i];
#pragma unroll 4
      for (int p = 1; p < rs.L; ++p) {
        const double uj = u[i + I.dlt[rs.base + 64 * p]];
        mx = fmax(mx, uj);
        mn = fmin(mn, uj);
      }
      umax[i] = mx;
      umin[i] = mn;
    }
    __syncthreads();
    // clipped fluxes (eq. (22), bar states in product form), b = F + F*,
    // r = b - A u ; R^2 (free rows), ||b||^2, ||r||^2
    double acc[Sched<NT>::PER][3] = {};
    AFC_ROWS(I, NT, c) {
      if (I.isd[i]) {
        const double bi = I.uD[i], ri = I.uD[i] - u[i];
        b[i] = bi;
        r[i] = ri;
        acc[c][1] += bi * bi;
        acc[c][2] += ri * ri;
        continue;
      }
      const RowSpan rs = row_span(I, i);
      const double ui = u[i], umaxi = umax[i], umini = umin[i];
      double fs = 0.0, au = A[rs.base] * ui;
#pragma unroll 2
      for (int p = 1; p < rs.L; ++p) {
        const int k = rs.base + 64 * p;
        const int dj = I.dlt[k];
        const int j = i + dj;
        const double uj = u[j];
        au += A[k] * uj;
        if (dj == 0 || o.alpha_mode == AFC_ALPHA_ZERO) continue;
        const double c = cc[k], ct = ccT[k];
        const double d = -fmax(fmax(c, 0.0), ct);
        if (d == 0.0) continue;
        const double rf = d * (uj - ui);
        if (o.alpha_mode == AFC_ALPHA_ONE) {
          fs += rf;
          continue;
        }
        const double sij = d * (ui + uj) + c * (uj - ui);
        const double sji = d * (ui + uj) + ct * (ui - uj);
        const double two_d = 2.0 * d;
        double rs_;
        if (rf > 0.0)
          rs_ = fmin(rf, fmin(sij - two_d * umaxi, two_d * umin[j] - sji));
        else
          rs_ = fmax(rf, fmax(sij - two_d * umini, two_d * umax[j] - sji));
        fs += rs_;
      }
      const double bi = I.F[i] + fs, ri = bi - au;
      b[i] = bi;
      r[i] = ri;
      acc[c][0] += ri * ri;
      acc[c][1] += bi * bi;
      acc[c][2] += ri * ri;
    }
    double red[3];
    wg_sum<NT, 3>(acc, red);
    const double R = sqrt(red[0]), bn = sqrt(red[1]);
    if (fp_stop(o, st, N, R, bn, st.nu == 0)) break;
    if (!fp_update<NT>(I, o, st, R, bn, red[2])) break;
    ++iters;
  }
  st.fp_total = st.nu;
  st.done = 1;
}

__device__ __forceinline__ SState fresh_state() {
  SState st;
  st.phase = -1;
  st.step = st.nu = st.have_prev = st.status = st.done = st.fp_total = st.pad_ = 0;
  st.kry = 0;
  st.R0 = st.R_prev = st.res0 = st.res = st.lin_res = 0.0;
  st.omega = 1.0;
  return st;
}

template <int NT>
__device__ void run_instance(const BInst& in, const BatchDev& D, const BatchOpts& o, int steps, double* ug,
                             const double* Fg, BStat* stat) {
  InstView I;
  I.N = in.N;
  I.nsl = in.nsl;
  I.slp = D.slp + in.sl_off;
  I.dlt = D.dlt + in.slot_off;
  I.mij = D.mij + in.slot_off;
  I.dp = D.dp + in.slot_off;
  I.AL = D.AL + in.slot_off;
  I.Acn = D.Acn + in.slot_off;
  I.ml = D.ml + in.node_off;
  I.uD = D.uD + in.node_off;
  I.isd = D.is_dir + in.node_off;
  I.dinv = D.dinv + in.node_off;
  for (int q = 0; q < BW_COUNT; ++q) I.w[q] = D.work + (size_t)q * D.total_nodes + in.node_off;
  I.u = ug + in.node_off;
  I.F = Fg + in.node_off;
  SState st = fresh_state();
  run_cn<NT>(I, in.dt, steps, o, st, -1);
  if (threadIdx.x == 0) {
    stat->status = st.status;
    stat->fp_iters = st.fp_total;
    stat->krylov_iters = st.kry;
    stat->res0 = st.res0;
    stat->res = st.res;
    stat->lin_res = st.lin_res;
  }
  __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void k_batch_cn(const BInst* __restrict__ insts, const int* __restrict__ order,
                                                 int count, int* queue, int steps, BatchDev D, BatchOpts o,
                                                 double* u, const double* F, BStat* stats) {
  __shared__ int slot;
  while (true) {
    if (threadIdx.x == 0) slot = atomicAdd(queue, 1);
    __syncthreads();
    const int q = slot;
    __syncthreads();
    if (q >= count) break;
    const int id = order[q];
    run_instance<NT>(insts[id], D, o, steps, u, F, stats + id);
  }
}

// One round of the served loop: each workgroup takes requests from the
// round's queue and advances each by one quantum (resumable state in
// `states`); the queue ends every workgroup's loop.
template <int NT>
__global__ __launch_bounds__(NT) void k_serve_round(const SReq* __restrict__ reqs, SState* states,
                                                    const int* __restrict__ list, int count, int* queue,
                                                    int64_t quantum) {
  __shared__ int slot;
  __shared__ int64_t t0;
  while (true) {
    if (threadIdx.x == 0) {
      slot = atomicAdd(queue, 1);
      t0 = (int64_t)wall_clock64();
    }
    __syncthreads();
    const int q = slot;
    const int64_t deadline = quantum > 0 ? t0 + quantum : -1;
    __syncthreads();
    if (q >= count) break;
    const int id = list[q];
    const SReq& R = reqs[id];
    InstView I;
    I.N = R.N;
    I.nsl = R.nsl;
    I.slp = R.slp;
    I.dlt = R.dlt;
    I.mij = R.mij;
    I.dp = R.dp;
    I.AL = R.AL;
    I.ml = R.ml;
    I.uD = R.uD;
    I.isd = R.isd;
    I.Acn = R.A;
    I.dinv = R.dinv;
    for (int w = 0; w < BW_COUNT; ++w) I.w[w] = R.work + (size_t)w * (size_t)R.ldw;
    I.u = R.u;
    I.F = R.F;
    SState st = states[id];
    if (!st.done) {
      if (R.kind == AFC_REQ_CN)
        run_cn<NT>(I, R.dt, R.steps, R.o, st, deadline);
      else
        run_mcl<NT>(I, R.cc, R.ccT, R.init_low, R.o, st, deadline);
    }
    __syncthreads();
    if (threadIdx.x == 0) states[id] = st;
    __syncthreads();
  }
}

}  // namespace

void batch_launch(afc_batch_s* b, double* u, const double* F, int steps, int threads, int grid) {
  switch (threads) {
    case 256:
      k_batch_cn<256><<<grid, 256, 0, b->stream>>>(b->insts, b->order, b->count, b->queue, steps, b->dev, b->bopt, u,
                                                    F, b->stats_d);
      break;
    case 512:
      k_batch_cn<512><<<grid, 512, 0, b->stream>>>(b->insts, b->order, b->count, b->queue, steps, b->dev, b->bopt, u,
                                                    F, b->stats_d);
      break;
    default:
      k_batch_cn<1024><<<grid, 1024, 0, b->stream>>>(b->insts, b->order, b->count, b->queue, steps, b->dev, b->bopt,
                                                      u, F, b->stats_d);
      break;
  }
}

int batch_work_vectors() { return BW_COUNT; }

int serve_work_vectors() { return BW_COUNT; }

void serve_round_launch(const SReq* reqs, SState* states, const int* list, int count, int* queue, int64_t quantum,
                        int threads, int grid, hipStream_t stream) {
  switch (threads) {
    case 256:
      k_serve_round<256><<<grid, 256, 0, stream>>>(reqs, states, list, count, queue, quantum);
      break;
    case 512:
      k_serve_round<512><<<grid, 512, 0, stream>>>(reqs, states, list, count, queue, quantum);
      break;
    default:
      k_serve_round<1024><<<grid, 1024, 0, stream>>>(reqs, states, list, count, queue, quantum);
      break;
  }
}

}  // namespace afc
