// Launch wrappers of the HIP kernels (defined in afc_kernels.hip).
#pragma once

#include "afc_internal.h"

namespace afc {

using H = afc_handle_s;

// --- plain vector helpers ---------------------------------------------------
void copy(H* h, double* dst, const double* src);
void set_dirichlet(H* h, double* u);                        // u_i = u_D,i on Dirichlet nodes
void rhs_dirichlet(H* h, double* b, const double* F);       // b = F, b_i = u_D,i on Dirichlet nodes
void relax(H* h, double* u, const double* x, double omega); // u += omega (x - u)
void fill(H* h, double* u, double v);
void norm2(H* h, const double* x, int red_idx);             // ||x||^2 into ks->red[red_idx]

// --- setup --------------------------------------------------------------------
// A_cn = M_L/dt + AL/2 for AL = A_low of the FCT (AL_fct) or MC (AL_mcl) scheme
// (+ dinv, SELL FP64 and scaled FP32 copies)
void build_cn_matrix(H* h, const double* AL, double dt);
void to_sell64(H* h, const double* csr, double* sell);
void to_sell8(H* h, const uint8_t* csr, uint8_t* sell);                      // uint8 CSR values -> SELL slots                       // CSR values -> SELL slots
void to_sell32_scaled(H* h, const double* csr, const double* dinv, float* sell);  // (a_ij dinv_j) in FP32

// workgroups of a launch over the SELL tiles (reduce: capped at the partial slots)
int sell_grid(const H* h, bool reduce);

// --- residual of a linear system (FP64 SpMV) -----------------------------------
// r = b - A x (A in SELL order) and ||r||^2 into ks->red[0]; mode selects the cycle start that
// the reduction finish performs (0: none, 1: GMRES FP64 restart into V64[0],
// 2: GMRES mixed restart, V32[0] cast done by cast_v0), with the tolerances
// that the solve's cycle_start stored in the device state.
void residual(H* h, const double* A, const double* b, const double* x, double* r, int mode);
void cycle_start(H* h, int mode, int red_idx, double tol_abs, double tol_rel);  // from a finished reduction
void cast_v0(H* h, const double* r, bool fp64 = false);  // V[0] = r / beta in the basis precision

// --- GMRES (right Jacobi), FP64 or FP32 Arnoldi --------------------------------
// Arnoldi step k = spmv + dots + reduce (finalizes the projections and the
// Givens rotation of step k-1) + update; the last step of a cycle is
// finished by gmres_last_givens.
void gmres_spmv64(H* h, const double* A, const double* dinv, int k);
void gmres_spmv32(H* h, const float* A32, int k);
void gmres_dots(H* h, bool fp32, int k);
void gmres_reduce(H* h, bool fp32, int k, int m);
void gmres_update(H* h, bool fp32, int k);
void gmres_last_givens(H* h, bool fp32, int k, int m);
// s-step GMRES block (FP32 basis in mixed precision, FP64 basis in FP64 mode):
// the shifted powers are spmv32 / spmv64 calls into
// V[k+1..k+s]; then projections + Gram, the block reduction (Cholesky QR,
// Hessenberg columns, Givens) and the in-place orthonormalization
void spmv32(H* h, const float* A32, const float* x, float theta, int rev, float* y);
// y = A (dinv .* x) - theta x (FP64; the SELL FP64 system matrix)
void apply_operator(H* h, int op, const double* x, double* y, double* tmp);
void spmv64(H* h, const double* A, const double* dinv, const double* x, double theta, int rev, double* y);
void sstep_dots(H* h, int k, int s, bool fp64 = false);
void sstep_reduce(H* h, int k, int s, int m, double theta, bool fp64 = false);
void sstep_update(H* h, int k, int s, bool fp64 = false);
void gmres_solve(H* h, int m, int kb = 0, int sb = 0);  // sb > 0: also the x-update coefficients of an s-step cycle
void gmres_xupdate(H* h, bool fp32, const double* dinv, double* x);
// end of an s-step cycle whose last block (start kb, sb vectors) was not orthogonalized in place
void sstep_xupdate(H* h, int kb, int sb, const double* dinv, double* x, bool fp64 = false);

// --- BiCGStab (right Jacobi, FP64) ----------------------------------------------
struct BicgVec { double *x, *r, *rhat, *p, *v, *s, *t; };
void bicg_init(H* h, const BicgVec& b, double tol);
void bicg_iter(H* h, const double* A_sell, const double* dinv, const BicgVec& b);  // A in SELL order

// --- Zalesak FCT, explicit SSP stage -------------------------------------------
void ssp_lowrate(H* h, const double* u, const double* F, double dt, double* udot, double* ut);

// --- MU limiter (Sec. 3.2); the system matrix is in the CN storage (A_cn = A_low) ---
void mu_R(H* h, const double* u, double* Rp, double* Rm);
void mu_apply(H* h, const double* u, const double* Rp, const double* Rm, const double* F, double* b, double* r);

// --- time-dependent MC limiting (Sec. 2.2) ----------------------------------------
void mc_lowrate(H* h, const double* u, const double* F, double* udot, double* scratch);  // udot = (F - A_low^mc u)/m
void mc_stage(H* h, const double* u, const double* udot, const double* umax, const double* umin, double dt,
              const double* u0, double c0, double c1, double* out);
void mc_cn_g(H* h, const double* uo, const double* udot, const double* umax, const double* umin, const double* Fn,
             double dt, double* g);
void mc_cn_apply(H* h, const double* u, const double* udot, const double* umax, const double* umin, const double* g,
                 double* b, double* r);
void ssp_limit_R(H* h, const double* u, const double* udot, const double* ut, double dt, double* Rp, double* Rm);
void ssp_apply(H* h, const double* u, const double* udot, const double* ut, const double* Rp, const double* Rm,
               double dt, const double* base, double c0, double c1, double* out);

// --- Zalesak FCT, Crank-Nicolson --------------------------------------------------
void cn_predict(H* h, const double* u_old, const double* F_old, const double* F_new, double dt, double* ut,
                double* g);
void zalesak_Q(H* h, const double* ut, double* Qp, double* Qm);
void cn_limit_R(H* h, const double* u, const double* u_old, const double* Qp, const double* Qm, double dt,
                double* Rp, double* Rm);
void cn_extrapolate(H* h, const double* ut, const double* uo, double* us);  // u* = 2 u~ - u_old (linear Zal+CN)
void cn_apply(H* h, const double* u, const double* u_old, const double* Rp, const double* Rm, const double* g,
              double dt, double* b, double* r);

// --- monolithic convex limiter, stationary ------------------------------------------
void mcl_bounds(H* h, const double* u, double* umax, double* umin);
void mcl_apply(H* h, const double* u, const double* umax, const double* umin, const double* F, double* b,
               double* r);

}  // namespace afc
