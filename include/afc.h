/*
 * afc.h -- C ABI of the MI355X algebraic flux correction (AFC) library.
 *
 * The library advances P1/Q1 finite element discretizations of the
 * convection-diffusion-reaction (CDR) equation with algebraic flux correction
 * as defined in Jha, Partl, Ahmed, Kuzmin, "An Assessment of Solvers for
 * Algebraically Stabilized Discretizations of Convection-Diffusion-Reaction
 * Equations" (arXiv 2110.15676):
 *   - Zalesak's FCT limiter with the explicit SSP scheme (Sec. 2.1.2, 2.1.3),
 *   - Zalesak's FCT limiter with Crank-Nicolson, nonlinear form solved by
 *     fixed-point iteration (Sec. 2.1.1, Sec. 4),
 *   - the monolithic convex limiter (MCL) for the stationary problem
 *     (Sec. 3.1, Sec. 2.2 eqs. (22)-(23), Remark 1), fixed-point iteration,
 *   - BiCGStab and restarted GMRES with Jacobi preconditioning (Sec. 4,
 *     solver and preconditioner tables), optionally FP32-inner / FP64-outer.
 *
 * Conventions
 *   The semi-discrete problem is M_C du/dt = K u + F, i.e. K = -A where A is
 *   the paper's matrix a_ij of eq. (4).  The graph viscosity used internally is
 *   d+_ij = max(-k_ij, 0, -k_ji) = -d_ij (eq. (5)).
 *   All matrices share one CSR pattern: int32 row_ptr[N+1], int32 col_idx[nnz],
 *   columns sorted ascending within a row, diagonal stored, pattern
 *   structurally symmetric.  Values are float64 in CSR order.
 *
 * Memory and streams
 *   afc_create copies everything it needs into device memory it owns; the
 *   caller's arrays may be freed after it returns.  Vectors passed to the
 *   step/solve calls (u, F, ...) are DEVICE pointers to N float64 values that
 *   the library borrows for the duration of the call; they must be usable on
 *   the stream given in afc_options.stream (NULL = the default stream).  Every
 *   call is synchronous on return (it needs convergence information).
 *   A handle is not thread safe: use one handle per host thread/stream.
 *
 * Errors
 *   Functions return afc_status; nothing is thrown across the ABI.  Negative
 *   values are errors, positive values warnings with a usable result.
 *   afc_last_error(h) returns a description of the last error on h.
 */
#ifndef AFC_H_
#define AFC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct afc_handle_s afc_handle;

typedef enum {
  AFC_OK = 0,
  AFC_WMAXIT = 1,        /* iteration cap reached; u holds the last iterate  */
  AFC_EINVAL = -1,       /* invalid argument / malformed CSR                  */
  AFC_ENOMEM = -2,       /* device allocation failed                          */
  AFC_ENOCONV = -3,      /* linear solver did not converge within its cap     */
  AFC_EBREAKDOWN = -4,   /* BiCGStab breakdown (rho or omega = 0) twice       */
  AFC_ENAN = -5,         /* a norm became non-finite                          */
  AFC_EDEVICE = -6,      /* HIP runtime error                                 */
  AFC_ECANCELED = -7     /* request dropped by afc_server_destroy             */
} afc_status;

enum { AFC_MEM_HOST = 0, AFC_MEM_DEVICE = 1 };
/* alpha_mode: LIMITED applies the limiter; ONE gives the Galerkin scheme
 * (alpha_ij = 1), ZERO the low-order scheme (alpha_ij = 0) (Sec. 2, eq. (10)). */
enum { AFC_ALPHA_LIMITED = 0, AFC_ALPHA_ONE = 1, AFC_ALPHA_ZERO = 2 };
enum { AFC_KRYLOV_BICGSTAB = 0, AFC_KRYLOV_GMRES = 1 };
/* MIXED: Krylov SpMVs/vectors in FP32 inside FP64 iterative refinement;
 * limiter, bounds, flux sums and nonlinear/outer residuals stay FP64. */
enum { AFC_PREC_FP64 = 0, AFC_PREC_MIXED = 1 };
/* Nonlinear stopping: ABS_SQRTN is R < sqrt(N) * fp_tol (eq. (28));
 * REL is R <= fp_tol * R_0.  R is the Euclidean norm of the nonlinear
 * residual over non-Dirichlet rows. */
enum { AFC_TOL_ABS_SQRTN = 0, AFC_TOL_REL = 1 };

/* Limiter of the stationary scheme (afc_solve_stationary). */
enum { AFC_LIMITER_MCL = 0, /* monolithic convex limiter, Sec. 3.1 (D, bar states from K_conv)   */
       AFC_LIMITER_MU = 1   /* monolithic upwind limiter, Sec. 3.2 (D and the edge orientation
                               a_ji <= a_ij from the full matrix A = -K)                       */
};

typedef struct {
  int32_t n;                /* number of nodes N (> 0)                         */
  int64_t nnz;              /* number of stored entries (< 2^31)               */
  int32_t mem_space;        /* AFC_MEM_HOST or AFC_MEM_DEVICE for all arrays   */
  const int32_t *row_ptr;   /* [N+1], row_ptr[0] = 0, row_ptr[N] = nnz         */
  const int32_t *col_idx;   /* [nnz], sorted per row, diagonal present         */
  const double *M;          /* [nnz] consistent mass m_ij (symmetric)          */
  const double *K;          /* [nnz] K = -A (eq. (4) with opposite sign)       */
  const double *K_conv;     /* [nnz] optional convective part of K; MCL builds
                               its graph viscosity and bar states from it
                               (Remark 1).  NULL: use K.                       */
  const double *ML;         /* [N] optional lumped mass m_i > 0; NULL: row sums
                               of M (eq. (5))                                  */
  int32_t n_dir;            /* number of Dirichlet nodes                       */
  const int32_t *dir_idx;   /* [n_dir] distinct node indices                   */
  const double *dir_val;    /* [n_dir] Dirichlet values u_D (time independent) */
} afc_problem;

typedef struct {
  int32_t alpha_mode;       /* AFC_ALPHA_*                                     */
  int32_t krylov;           /* AFC_KRYLOV_*                                    */
  int32_t restart;          /* GMRES restart length m, 1..64 (default 30)      */
  int32_t precision;        /* AFC_PREC_*                                      */
  double lin_atol;          /* linear stop: ||b - A x|| <= max(atol, rtol*||b||) */
  double lin_rtol;
  int32_t lin_maxit;        /* Krylov iteration cap per linear solve           */
  double inner_rtol;        /* MIXED: a sweep's FP32 GMRES cycle stops early
                               once its residual estimate falls by this factor */
  int32_t inner_maxit;      /* MIXED: FP32 steps per sweep (<= restart)        */
  int32_t refine_maxit;     /* MIXED: cap on FP64 refinement sweeps            */
  double fp_tol;            /* nonlinear tolerance (see fp_tol_mode)           */
  int32_t fp_tol_mode;      /* AFC_TOL_*                                       */
  int32_t fp_maxit;         /* cap on fixed-point linear solves                */
  double prelimit;          /* CN prelimiting constant L of eq. (13); 0 = off  */
  double omega;             /* fixed-point relaxation, (0, 1]                   */
  int32_t dynamic_damping;  /* 1: halve omega on residual growth, else grow    */
  int32_t ssp_stages;       /* 3: Shu-Osher SSP-RK3; 2: Heun (paper); 1: one
                               forward-Euler stage of eq. (18)                 */
  int32_t lanes_per_row;    /* 0 = automatic; else 8, 16, 32 or 64             */
  int32_t profile;          /* 1: time every launch of the hot kernels with HIP
                               events on the handle's stream (afc_kernel_time) */
  int32_t limiter;          /* AFC_LIMITER_* of afc_solve_stationary          */
  int32_t sstep;            /* GMRES (FP64 and mixed): 0 = one basis vector per
                               step (classical Gram-Schmidt); s = 2..16 = blocks
                               of s vectors from shifted matrix powers
                               (A - I)^j v, orthonormalized together (block
                               Gram-Schmidt + Cholesky QR), in the basis
                               precision of the mode.  Same Krylov space and
                               minimal-residual iterate as GMRES in exact
                               arithmetic; a block whose QR fails halves s for
                               the handle's later cycles and solves (s = 0
                               below 2) until afc_set_options is called; a
                               solve following one of at most 4 (8) Krylov
                               iterations uses blocks of 4 (8).                */
  double sstep_shift;       /* theta of the shifted powers (default 1: the
                               Jacobi-scaled matrix has unit diagonal)         */
  int32_t graphs;           /* 1 (default): each GMRES cycle is captured once
                               as a HIP graph and replayed (same kernels, same
                               results); 0: plain launches.  Not used while
                               profile = 1.                                    */
  double lin_eta;           /* inexact fixed point (not in the paper): each
                               linear solve of the Sec. 4 iteration may also
                               stop once ||b - A x|| <= lin_eta * R, where R is
                               the current nonlinear residual (the solve starts
                               from u^nu, so R is its initial residual).  The
                               iterates change, the fixed point does not.
                               0 (default) = off; must lie in [0, 1).  The
                               batched launch requires 0.                      */
  void *stream;             /* hipStream_t; NULL = default stream              */
} afc_options;

/* Kernel classes timed when afc_options.profile is set. */
enum {
  AFC_KERNEL_SPMV32 = 0,    /* FP32 SELL-64 SpMV of the mixed-precision GMRES  */
  AFC_KERNEL_SPMV64 = 1,    /* FP64 SELL-64 SpMV (Jacobi-scaled) of FP64 GMRES */
  AFC_KERNEL_DOTS = 2,      /* GMRES Gram-Schmidt projection partials          */
  AFC_KERNEL_UPDATE = 3,    /* GMRES orthogonalization update + norm           */
  AFC_KERNEL_RESIDUAL = 4,  /* FP64 residual b - A x                           */
  AFC_KERNEL_MCL = 5,       /* MCL bounds + limited fluxes + residual          */
  AFC_KERNEL_FINISH = 6,    /* reduction finishes (GMRES projections + Givens, */
                            /* scalar solver steps)                            */
  AFC_KERNEL_COUNT = 7
};

typedef struct {
  int32_t status;           /* same as the return value                        */
  int32_t fp_iters;         /* fixed-point linear solves performed             */
  int64_t krylov_iters;     /* total Krylov iterations (FP64 + FP32 inner)     */
  int64_t inner_iters;      /* FP32 inner iterations (MIXED)                   */
  int32_t refine_sweeps;    /* FP64 refinement sweeps (MIXED)                  */
  double res0;              /* first nonlinear residual norm                   */
  double res;               /* last nonlinear residual norm                    */
  double lin_res;           /* last linear true residual norm                  */
} afc_stats;

/* Fill *opt with defaults: LIMITED, GMRES(30), FP64, lin_atol 1e-12,
 * lin_rtol 0, lin_maxit 10000, inner_rtol 1e-5, inner_maxit 300,
 * refine_maxit 1000, fp_tol 1e-12 ABS_SQRTN, fp_maxit 50, prelimit 2,
 * omega 1, no dynamic damping, ssp_stages 3, automatic lanes, NULL stream. */
void afc_default_options(afc_options *opt);

/* Create a handle: validates the CSR data (EINVAL on a malformed pattern,
 * non-positive lumped mass, out-of-range Dirichlet index), precomputes the
 * graph viscosities d+_ij of eq. (5) from K (FCT) and from K_conv (MCL), the
 * low-order operators A + D of eq. (6) with Dirichlet rows replaced by identity
 * rows, and the FP32 Jacobi-scaled copies; uploads everything to the current
 * HIP device.  *out is NULL on failure.  opt may be NULL (defaults). */
afc_status afc_create(const afc_problem *prob, const afc_options *opt, afc_handle **out);

/* Replace the options of an existing handle (same validation as afc_create). */
afc_status afc_set_options(afc_handle *h, const afc_options *opt);

/* One explicit time step of length dt (Sec. 2.1.2): forward-Euler stages of
 * eq. (18), each limited by Zalesak's algorithm (Sec. 2.1.3) with the
 * predictor of eq. (19) and the fluxes of eqs. (20)-(21); composed as
 * Shu-Osher SSP-RK3 (ssp_stages = 3), Heun (2) or a single stage (1).
 * u: in u^{n-1}, out u^n (device).  F: load vector (device), constant in the
 * step.  stats may be NULL. */
afc_status afc_step_ssprk3(afc_handle *h, double *u, const double *F, double dt, afc_stats *stats);

/* Size of the fixed device array behind afc_step_ssprk3_noalloc: 64 MiB on
 * every GPU the library is loaded on, held until the process ends. */
#define AFC_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step of
 * afc_step_ssprk3, with the same arguments, kernels and results, whose six
 * per-call work vectors (two stage states, the low-order rate, the predictor,
 * Zalesak's R+ and R-) live in a fixed device array of
 * AFC_NOALLOC_SCRATCH_BYTES instead of memory the handle allocates on first
 * use.  It calls no hipMalloc, hipFree or other allocating routine.
 * Limits and errors (EINVAL, u unchanged, afc_last_error says which):
 *   - 6 * ceil(N / 64) * 64 * 8 bytes must fit the array (N <= 1,398,080);
 *   - the handle's slot-order explicit-stage coefficients must exist: they are
 *     built by the first afc_step_ssprk3, afc_step_mc_ssprk3 or CN call on the
 *     handle, which this entry point never makes for the caller;
 *   - options.profile must be 0.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call writes every element it reads, so nothing needs
 * clearing): calls that overlap on one GPU (several host threads or streams)
 * race and must be serialized by the caller. */
afc_status afc_step_ssprk3_noalloc(afc_handle *h, double *u, const double *F, double dt, afc_stats *stats);

/* One Crank-Nicolson FCT step, eq. (11) with fluxes eq. (12), prelimiting
 * eq. (13) and the predictor eq. (14), solved by the fixed-point iteration of
 * Sec. 4 with matrix M_L/dt + A_low/2.  u: in u^{n-1}, out u^n (device).
 * F_old, F_new: load vectors at t_{n-1}, t_n (device).  Returns WMAXIT when
 * fp_maxit solves did not reach fp_tol (u holds the last iterate). */
afc_status afc_step_cn(afc_handle *h, double *u, const double *F_old, const double *F_new, double dt,
                       afc_stats *stats);

/* One linear Zal+CN step (Sec. 2.1.1, the linearized variant of eq. (11)):
 * u^n in the fluxes of eq. (12) is replaced by u* = 2 u~ - u^{n-1}, with u~
 * the predictor of eq. (14) and u_D at Dirichlet nodes.  The fluxes
 * (prelimited by eq. (13)), Zalesak's limiter and F* are then evaluated once,
 * and eq. (11) is one linear system, solved from x0 = u* with the handle's
 * Krylov options.  Same arguments and ownership as afc_step_cn; stats report
 * fp_iters = 1 and res0 = res = the residual of eq. (11) at u*.  Returns the
 * linear solver's status (ENOCONV, EBREAKDOWN, ENAN) or EINVAL. */
afc_status afc_step_cn_linear(afc_handle *h, double *u, const double *F_old, const double *F_new, double dt,
                              afc_stats *stats);

/* Time-dependent monolithic convex limiting (Sec. 2.2).  Both use the
 * semi-discrete fluxes of eq. (20), r_ij = m_ij (udot_i - udot_j) +
 * d_ij (u_j - u_i) with udot the low-order rate of eq. (21), limited by
 * eq. (22) with the bar states and local bounds of the state the fluxes are
 * evaluated at.  As for afc_solve_stationary, D and the bar states come from
 * the convective matrix K_conv (Remark 1) and A_low = A + D^conv.
 *
 * afc_step_mc_ssprk3: forward-Euler stages of eq. (18) with F* = sum_j r*_ij,
 * composed as options.ssp_stages (3 Shu-Osher, 2 Heun, 1 single stage); same
 * arguments as afc_step_ssprk3.
 *
 * afc_step_mc_cn: eq. (11) with A_low^conv and the correction
 * F* = (F*(u^n) + F*(u^{n-1}))/2 (each with udot at its own time level, from
 * F_new resp. F_old), solved by the fixed point of Sec. 4 from u^{n-1}; same
 * arguments, options and statuses as afc_step_cn. */
afc_status afc_step_mc_ssprk3(afc_handle *h, double *u, const double *F, double dt, afc_stats *stats);
afc_status afc_step_mc_cn(afc_handle *h, double *u, const double *F_old, const double *F_new, double dt,
                          afc_stats *stats);

/* Stationary AFC scheme: fixed-point iteration of Sec. 4 for
 * A_low u = F + F*(u), where F* sums the fluxes r^ss_ij = d_ij (u_j - u_i)
 * of eq. (25) limited by options.limiter: the MC limiter of eq. (22)
 * (Sec. 3.1; D and the bar states from K_conv, Remark 1) or the MU limiter
 * of Sec. 3.2 (D from A = -K; node i owns edge (i, j) when a_ji <= a_ij,
 * and when a_ji = a_ij the smaller of both nodes' factors is used).
 * u: in initial guess, out solution (device).  If init_low_order is nonzero
 * the guess is first replaced by the low-order solution A_low u = F.
 * F: load vector (device). */
afc_status afc_solve_stationary(afc_handle *h, double *u, const double *F, int32_t init_low_order,
                                afc_stats *stats);

/* Accumulated HIP-event time (milliseconds) and launch count of one kernel
 * class since the handle was created or the last reset (reset != 0 clears
 * the counters after reading).  Only launches made while options.profile was
 * set are counted.  Returns EINVAL for an unknown kernel id. */
afc_status afc_kernel_time(afc_handle *h, int32_t kernel, double *total_ms, int64_t *launches, int32_t reset);

/* Algorithmic HBM bytes (each array element the kernels must read or write,
 * counted once per launch) and the number of launches that did work, over
 * the same profiled launches as afc_kernel_time (and cleared by its reset).
 * GMRES launches issued after a cycle converged return at once; they count
 * as launches in afc_kernel_time but do no work.  Accounted for the SPMV32,
 * SPMV64, DOTS, UPDATE, RESIDUAL and MCL classes; 0 for FINISH.  Returns EINVAL for an unknown kernel id. */
afc_status afc_kernel_work(afc_handle *h, int32_t kernel, double *bytes, int64_t *launches_with_work);

/* One application of the stationary MCL system's operators by the solvers'
 * own SELL-64 kernels, for tests that check those kernels element by element.
 * A is the low-order operator A_low of eq. (5) that the stationary solve
 * iterates with (Sec. 4), D = diag(A).  op:
 *   AFC_APPLY_RESIDUAL (0)  y := y - A x   (FP64, the refinement residual)
 *   AFC_APPLY_SCALED64 (1)  y = A D^{-1} x (FP64 SpMV of the FP64 GMRES)
 *   AFC_APPLY_SCALED32 (2)  y = A D^{-1} x with the FP32 Jacobi-scaled copy
 *                           and the FP32 SpMV of the mixed GMRES (x rounded to
 *                           FP32, y the FP32 result widened)
 *   AFC_APPLY_BICG     (3)  y = A D^{-1} x by the BiCGStab SpMV (FP64)
 * x and y are device pointers to n doubles on the handle's device and must not
 * overlap.  Runs on the handle's stream and waits for it.  A scratch vector
 * is allocated on the first call (freed by afc_destroy).  EINVAL for a null or
 * aliased pointer or an unknown op; EDEVICE / ENOMEM on a HIP error. */
enum {
  AFC_APPLY_RESIDUAL = 0,
  AFC_APPLY_SCALED64 = 1,
  AFC_APPLY_SCALED32 = 2,
  AFC_APPLY_BICG = 3
};
afc_status afc_apply_operator(afc_handle *h, int32_t op, const double *x, double *y);

/* Storage of the SELL-64 copy of the Krylov system matrices (sizes only).
 * Rows are taken in slices of 64 consecutive rows, each padded to its longest
 * row; a slice whose rows all fit one shared list of column offsets j - i
 * ("uniform") stores no per-row offsets.  Read to price the SpMV's memory
 * traffic: per launch the FP32 SpMV reads 4 * slots value bytes,
 * delta_bytes * lane_delta_slots offset bytes, 4 * pattern_ints pattern
 * bytes and 8 * slices + 4 slice-header bytes, besides x and y. */
typedef struct {
  int64_t slices;            /* ceil(N / 64) */
  int64_t slots;             /* value slots over all slices (64 x padded length) */
  int64_t uniform_slices;    /* slices stored with a shared offset pattern */
  int64_t lane_delta_slots;  /* per-row offsets stored for the other slices */
  int64_t pattern_ints;      /* 32-bit entries of the shared pattern table */
  int32_t delta_bytes;       /* bytes of one per-row offset: 2 or 4 */
  int32_t reserved;
} afc_sell_info;

/* Fill *out for handle h.  Returns EINVAL if h or out is NULL. */
afc_status afc_get_sell_info(const afc_handle *h, afc_sell_info *out);

/* The same for the FP32 Jacobi-scaled Krylov matrices of the mixed-precision
 * solve (GMRES inner iterations, Sec. 4): their layout holds the system
 * pattern without its diagonal, because every scaled diagonal entry is 1 and
 * the SpMV applies it as x_i.  Equal to afc_sell_layout of the pattern with
 * the diagonal entries removed.  Returns EINVAL if h or out is NULL. */
afc_status afc_get_krylov_sell_info(const afc_handle *h, afc_sell_info *out);

/* The same SELL-64 layout computed on the host for an n-row CSR pattern
 * (row_ptr[n + 1], col[row_ptr[n]], 0-based, host memory); needs no GPU.
 * Fills *info; each array pointer may be NULL (call once with NULLs to learn
 * the sizes), else it must hold: slice_ptr info->slices + 1 slot offsets,
 * slice_delta info->slices entries (>= 0: offset of the slice's per-row
 * offsets in lane_deltas, slot p of row lane l at + 64 p + l; < 0: the slice
 * is uniform and ~value is the offset of its pattern in pattern[]), pattern
 * info->pattern_ints, pos row_ptr[n] (slot of each CSR entry; entry p of
 * row lane l of slice s lies at slice_ptr[s] + 64 p + l), lane_deltas
 * info->lane_delta_slots (widened to 32 bits).  Returns EINVAL for a
 * malformed pattern or a layout beyond 2^31 slots. */
afc_status afc_sell_layout(int32_t n, const int32_t *row_ptr, const int32_t *col, afc_sell_info *info,
                           int32_t *slice_ptr, int32_t *slice_delta, int32_t *pattern, int32_t *pos,
                           int32_t *lane_deltas);

/* Nonlinear residuals R (Euclidean norm over non-Dirichlet rows, Sec. 4 and
 * eq. (28)) of the last fixed-point call on h (afc_step_cn, afc_step_mc_cn,
 * afc_solve_stationary): one value per evaluation, R_0 first, the value that
 * ended the loop last.  Copies min(count, cap) values into out (host memory,
 * may be NULL when cap = 0) and stores the full count in *count.  The history
 * is kept until the next fixed-point call on h.  EINVAL on a NULL h or count,
 * or cap < 0. */
afc_status afc_residual_history(const afc_handle *h, double *out, int32_t cap, int32_t *count);

/* Release every device and host resource of h (NULL is ignored). */
void afc_destroy(afc_handle *h);

/* ---- Batched Crank-Nicolson FCT ------------------------------------------
 * Many independent instances (each its own CSR pattern, coefficients and dt)
 * advanced by one persistent launch: every workgroup takes whole instances
 * from a device queue (largest first) and runs all their CN steps (eqs. (11)-
 * (14), Zalesak's limiter, fixed-point iteration with BiCGStab-Jacobi) with
 * workgroup-local barriers only.  An instance's result does not depend on the
 * other instances in the batch.  Vectors are packed: instance k occupies
 * entries [offsets[k], offsets[k+1]) of u and F (afc_batch_offsets). */
typedef struct afc_batch_s afc_batch;

/* Create from count problems (same rules as afc_create).  The options must
 * select BiCGStab and FP64; the other fields apply to every instance. */
afc_status afc_batch_create(int32_t count, const afc_problem *probs, const afc_options *opt, afc_batch **out);

/* offsets: host array of count + 1 entries; offsets[count] is the packed length. */
afc_status afc_batch_offsets(const afc_batch *b, int64_t *offsets);

/* Advance every instance by `steps` CN-FCT steps of its own dt (host array of
 * count entries) with the time-independent load F (packed, device).  u:
 * packed device vector, in u^{n}, out u^{n+steps}.  stats: NULL or a host
 * array of count entries (fp_iters and krylov_iters summed over the steps).
 * Returns the most severe per-instance status. */
afc_status afc_batch_step_cn(afc_batch *b, double *u, const double *F, const double *dt, int32_t steps,
                             afc_stats *stats);

/* Description of the last error on b (b may be NULL: last creation error). */
const char *afc_batch_last_error(const afc_batch *b);

/* Schedule of the persistent batch launch: threads per workgroup (256, 512 or
 * 1024) and the number of workgroups pulling instances from the queue (0 =
 * twice the compute units; never more than the instances).  Every reduction
 * of an instance follows one fixed order whatever the schedule, so results
 * are bitwise identical under every schedule. */
typedef struct {
  int32_t threads;
  int32_t workgroups;
} afc_batch_schedule;

afc_status afc_batch_set_schedule(afc_batch *b, const afc_batch_schedule *s);
afc_status afc_batch_get_schedule(const afc_batch *b, afc_batch_schedule *s);

/* Autotuner: times trial_steps CN steps of the whole batch (from a scratch
 * copy of u; u and the batch's results are untouched) under each candidate
 * schedule (threads 256/512/1024 x 1, 2 or 4 workgroups per compute unit,
 * duplicates dropped), keeps the fastest as the batch's schedule and returns
 * it in *chosen (if not NULL).  trial_ms (if not NULL) receives up to
 * max_trials timings in candidate order, *n_trials (if not NULL) their
 * number.  u, F: device, packed as for afc_batch_step_cn; dt: host, one per
 * instance.  Returns EINVAL for bad arguments, EDEVICE/ENOMEM on HIP errors. */
afc_status afc_batch_autotune(afc_batch *b, const double *u, const double *F, const double *dt, int32_t trial_steps,
                              afc_batch_schedule *chosen, double *trial_ms, int32_t max_trials, int32_t *n_trials);

/* Release the batch (NULL is ignored). */
void afc_batch_destroy(afc_batch *b);

/* ---- Request server (continuous batching) ---------------------------------
 * Requests are copied at submission and served on the current device by two
 * lanes that run concurrently.
 *   Fused lane (N <= fuse_max_nodes; CN, or stationary MCL): host setup
 *   threads build the request's operators (eqs. (4)-(6)) and SELL layout and
 *   upload them into a device block of its own.  A round thread then runs the
 *   active requests in rounds: each round is one launch in which every active
 *   request advances by up to quantum_ms (at least one fixed-point iteration)
 *   in a workgroup of its own, resuming from the state it left in device
 *   memory.  Requests that become ready join the next round; finished ones
 *   leave.  This lane runs BiCGStab-Jacobi in FP64 whatever options.krylov
 *   and options.precision say; tolerances, iteration caps, alpha_mode,
 *   prelimit, omega, dynamic_damping and lin_eta are honoured.
 *   Dedicated lane (larger requests, and the MU limiter): `slots` worker
 *   threads, each with its own stream, run one request at a time end to end
 *   on a handle of its own with the request's options.
 * Admission is per lane in arrival order while the device footprint of the
 * admitted requests fits hbm_budget_bytes (and, for the dedicated lane, a slot
 * is free).  A request's result does not depend on the other requests in
 * flight, on the quantum or on the workgroup that ran it (fixed reduction
 * orders). */
enum { AFC_REQ_CN = 0, AFC_REQ_STATIONARY = 1 };

typedef struct {
  int32_t kind;          /* AFC_REQ_CN: `steps` CN-FCT steps of length dt;
                            AFC_REQ_STATIONARY: stationary solve (options.
                            limiter: MCL or MU)                              */
  afc_problem problem;   /* host arrays (mem_space must be AFC_MEM_HOST)     */
  const double *u0;      /* host [N]: CN initial state (required); stationary
                            initial guess, NULL = the low-order solution     */
  const double *F;       /* host [N] load vector, constant in time           */
  double dt;             /* CN step length                                   */
  int32_t steps;         /* CN steps                                         */
  afc_options opt;       /* solver options; the stream field is ignored      */
} afc_request;

typedef struct afc_server_s afc_server;

typedef struct {
  int32_t slots;            /* dedicated-lane slots (streams), 1..64         */
  int64_t hbm_budget_bytes; /* admission budget over both lanes (> 0)        */
  int32_t fuse_max_nodes;   /* requests with N <= this use the fused lane;
                               0 = every request is dedicated               */
  int32_t loop_threads;     /* fused-lane workgroup size: 256, 512 or 1024   */
  int32_t loop_workgroups;  /* workgroups per round; 0 = one per compute unit */
  int32_t setup_threads;    /* host threads preparing fused requests, 1..32  */
  int32_t max_active;       /* fused requests in flight at most, 1..65536    */
  double quantum_ms;        /* time slice of a request in one round (>= 0;
                               0 = run each request to completion)          */
} afc_server_config;

/* Defaults: 4 slots, 64 GiB budget, fuse_max_nodes 20000, 1024 threads, one
 * workgroup per compute unit, 4 setup threads, 512 active, 2 ms quantum. */
void afc_server_default_config(afc_server_config *cfg);

/* Start a server with the given configuration on the current device.
 * EINVAL for a configuration outside the ranges above. */
afc_status afc_server_create_cfg(const afc_server_config *cfg, afc_server **out);

/* Start a server with the default configuration and `slots` dedicated slots
 * (1..64) within hbm_budget_bytes. */
afc_status afc_server_create(int32_t slots, int64_t hbm_budget_bytes, afc_server **out);

/* Modelled device bytes a dedicated-lane request of this size keeps resident. */
int64_t afc_footprint_bytes(int32_t n, int64_t nnz, int32_t kind, const afc_options *opt);

/* Queue a request (inputs are copied; returns at once); *id identifies it. */
afc_status afc_server_submit(afc_server *s, const afc_request *req, int64_t *id);

/* Block until request id has finished.  u_out: NULL or host [N] for the
 * result; stats: NULL or its statistics; times: NULL or 3 doubles (seconds
 * from submission to admission, seconds of setup and service, submit-to-
 * completion latency).  Returns the request's status (AFC_ECANCELED if
 * afc_server_destroy dropped it).  Each id can be waited for once; a second
 * wait or poll on it returns AFC_EINVAL. */
afc_status afc_server_wait(afc_server *s, int64_t id, double *u_out, afc_stats *stats, double *times);

/* Non-blocking completion check: *done = 1 once request id has finished
 * (afc_server_wait then returns at once), 0 while it is queued or running.
 * AFC_EINVAL for an unknown id or one already waited for. */
afc_status afc_server_poll(afc_server *s, int64_t id, int32_t *done);

/* Rounds run by the fused lane so far, the requests those rounds carried
 * (summed over rounds: divided by the rounds, the mean number of requests
 * per fused launch) and the footprint admitted now.  Any pointer may be NULL. */
afc_status afc_server_info(const afc_server *s, int64_t *rounds, int64_t *request_rounds, int64_t *in_use_bytes);

/* Message of the last failed request or call (empty if none). */
const char *afc_server_last_error(const afc_server *s);

/* Stop the server: admitted requests finish, requests not yet admitted end
 * with AFC_ECANCELED, threads blocked in afc_server_wait return, then s is
 * freed.  No submit, wait or poll may start once this call has begun. */
void afc_server_destroy(afc_server *s);

/* Static description of a status code. */
const char *afc_status_str(int32_t status);

/* Description of the last error on h (empty string if none; h may be NULL). */
const char *afc_last_error(const afc_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* AFC_H_ */
