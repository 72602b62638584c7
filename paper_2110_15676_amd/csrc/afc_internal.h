// Internal definitions shared by the HIP translation units of libafc.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/afc.h"

namespace afc {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kMaxRestart = 64;    // GMRES restart cap (Hessenberg lives on device)
constexpr int kMaxRed = 72;        // values a single fused reduction may produce
constexpr int kRedBlocks = 2048;   // cap on workgroups of reduction kernels
constexpr int kSMax = 16;          // largest s-step GMRES block (two halves of eight columns)
// values of one s-step block reduction: C = V^T W ((m+1) x s) and the Gram W^T W (s(s+1)/2)
constexpr int kBlkRows = (kMaxRestart + 1) * kSMax + kSMax * (kSMax + 1) / 2;

// Device-resident scalars of the Krylov solvers (one per handle).  Every
// scalar decision (step lengths, Givens rotations, convergence) is taken on
// the device so that the host only synchronises once per chunk or cycle.
struct KState {
  // decision scalars first: the host copies this head after each chunk/cycle
  double tol;       // absolute tolerance of the running cycle/solve
  double beta;      // norm of the cycle's start residual
  double res;       // latest residual (estimate) norm
  double rho, alpha, omega, bcg_beta;  // BiCGStab scalars
  double pad_d;
  int m;            // restart length of the running cycle
  int k;            // Arnoldi columns completed in the cycle
  int done;         // converged or stopped: kernels of the chunk become no-ops
  int flag;         // 1 breakdown, 2 non-finite, 3 s-step block QR failed
  int iters;        // Krylov iterations, cumulative over the handle's life
  int half;         // BiCGStab: ||s|| already below tol in this iteration
  int sfail;        // s-step blocks whose QR failed (sticky count)
  int solved;       // the solve's own tolerance holds: every kernel of a cycle queued after it returns at once
  double red[kMaxRed];                        // last finalized reduction
  double H[(kMaxRestart + 1) * kMaxRestart];  // Hessenberg, column k at H[k*(m+1)]
  double cs[kMaxRestart], sn[kMaxRestart];    // Givens rotations
  double g[kMaxRestart + 1];                  // rotated right-hand side
  double sc[kMaxRestart + 1];                 // basis scales: v_j = sc_j * V[j]
  double coef[kMaxRestart + 1];               // update coefficients y_j * sc_j
  double proj[kMaxRestart + 1];               // running Arnoldi step: h_{q,k} sc_q
  double ctol_abs, ctol_rel;                  // cycle restart tolerances of the running solve
  // s-step GMRES (mixed precision): Arnoldi Hessenberg before rotation, block sums,
  // update coefficients D = C R^{-1} and R^{-1} of the running block
  double Hraw[(kMaxRestart + 1) * kMaxRestart];
  double blk[kBlkRows];
  double dco[(kMaxRestart + 1) * kSMax];
  double rinv[kSMax * kSMax];
  int blk_ok;                                 // the running block's QR succeeded
  // x update of an s-step cycle: combined coefficients of V_0..V_{xnq-1}, then
  // of the xnw raw vectors of the last block (written by the back substitution)
  int xnq, xnw;
  double xco[kMaxRestart + 1 + kSMax];
};

// bytes of KState copied back to the host: scalars + red[0..7]
constexpr size_t kStatusBytes = 8 * sizeof(double) + 8 * sizeof(int) + 8 * sizeof(double);

}  // namespace afc

struct afc_handle_s {
  // problem
  int N = 0;
  int64_t nnz = 0;
  int G = 32;  // lanes per row
  int n_dir = 0;
  afc_options opt{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::string last_error;
  std::vector<double> res_hist;  // nonlinear residuals of the last fixed-point call

  // pattern and node data (device)
  int* row_ptr = nullptr;
  int* col = nullptr;
  uint8_t* is_dir = nullptr;
  double* uD = nullptr;     // u_D on Dirichlet nodes, 0 elsewhere
  double* ml = nullptr;     // lumped mass m_i

  // FCT data: m_ij, d+_ij from K, A_low = A + D (Dirichlet rows = identity)
  double* mij = nullptr;
  double* dp_fct = nullptr;
  double* AL_fct = nullptr;
  uint8_t* mu_own = nullptr;  // MU edge orientation per CSR entry (1: a_ji < a_ij, 2: a_ji > a_ij, 0: equal)

  // MCL data: convective c_ij, c_ji (transposed, CSR order), A_low from K_conv
  double* cc = nullptr;
  double* ccT = nullptr;
  double* AL_mcl = nullptr;
  double* dinv_mcl = nullptr;

  // SELL-64 layout of the Krylov system matrices (one 64-row slice per wave,
  // entries column-major in a slice, column deltas j - i); padding entries
  // have value 0 and an in-range delta.  sell_pos maps each CSR entry to its
  // slot.
  int nslices = 0;
  int* sl_ptr = nullptr;      // [nslices + 1] slot offsets (multiples of 64)
  int* sl_dl = nullptr;       // per slice: >= 0 offset of per-lane deltas, < 0 ~offset into sl_pat
  int* sl_pat = nullptr;      // shared delta patterns of uniform slices
  int64_t sell_uniform = 0;   // slices with one delta pattern
  int64_t sell_lane_deltas = 0;  // per-lane deltas stored (other slices)
  int64_t sell_pat_ints = 0;  // entries of sl_pat
  void* sl_dlt = nullptr;     // per-lane deltas: int16 when every |j - i| <= 32767, else int32
  uint32_t* sl_mask = nullptr;  // bit p % 32 of word [p / 32][row]: slot p of the row holds a stored entry
  int mask_words = 1;           // 32-slot words per row
  double* Scc = nullptr;        // c_ij in SELL slot order (MCL)
  double* SccT = nullptr;       // c_ji in SELL slot order (MCL)
  double* S_mij = nullptr;      // m_ij, d+_ij and A_low (FCT) in SELL slot order (SSP stages; built on first use)
  double* S_dp = nullptr;
  double* S_alf = nullptr;
  uint8_t* S_own = nullptr;     // MU edge owner in slot order
  bool dlt16 = true;
  int* sell_pos = nullptr;    // [nnz]
  double* S64_mcl = nullptr;  // A_low (MCL) in SELL order
  double* S64_cn = nullptr;
  int64_t sell_slots = 0;

  // The FP32 Jacobi-scaled Krylov matrices A D^{-1} in a SELL-64 layout of
  // their own: the same pattern without the diagonal, whose scaled value is 1
  // (the SpMV applies it as x_i).  kpos maps each CSR entry to its slot, -1
  // for the diagonal.
  int* ks_ptr = nullptr;
  int* ks_dl = nullptr;
  int* ks_pat = nullptr;
  void* ks_dlt = nullptr;
  bool ks_dlt16 = true;
  int* kpos = nullptr;        // [nnz]
  int64_t ks_slots = 0, ks_uniform = 0, ks_lane_deltas = 0, ks_pat_ints = 0;
  float* S32_mcl = nullptr;   // A_low D^{-1} (MCL), off-diagonal slots, FP32
  float* S32_cn = nullptr;

  // CN system M_L/dt + A_low/2 (built for the last dt used)
  double cn_dt = 0.0;
  const double* cn_src = nullptr;  // A_low the CN matrix was built from (AL_fct or AL_mcl)
  double* A_cn = nullptr;
  double* dinv_cn = nullptr;

  // work vectors (FP64, N each)
  std::vector<double*> w;
  double* V64 = nullptr;  // (m+1) x N
  float* V32 = nullptr;   // (m+1) x N
  double* apply_tmp = nullptr;  // ldv doubles for afc_apply_operator (allocated on first use)
  int Vm = 0;
  int ldv = 0;  // basis / work vector stride: N rounded up to 64 (16-byte aligned rows)
  int bicg_last = 2;  // BiCGStab iterations of the handle's last solve (first chunk size)
  int sstep_cap = afc::kMaxRestart;  // s-step block size cap: halved by a failed block QR, reset by afc_set_options
  int gmres_last = 1 << 30;          // Krylov iterations of the handle's last GMRES solve (block size choice)
  double* partials = nullptr;  // kMaxRed * kRedBlocks
  double* partials_res = nullptr;  // one per workgroup of the FP64 SELL residual
  double* partials_blk = nullptr;  // kBlkRows * kRedBlocks (s-step GMRES, allocated on first use)
  afc::KState* ks = nullptr;
  afc::KState* host_status = nullptr;  // pinned copy of the KState head
  char* ring = nullptr;                // pinned status copies of the two cycles a GMRES solve keeps queued
  hipEvent_t ring_ev[2] = {nullptr, nullptr};

  // launch sequences replayed as HIP graphs (options.graphs): a GMRES cycle,
  // a chunk of BiCGStab iterations.  Captured on a private stream, each keyed
  // by every pointer and size it baked in; a few are kept (oldest dropped).
  hipStream_t cap_stream = nullptr;
  std::vector<std::pair<std::vector<const void*>, hipGraphExec_t>> graphs;

  // optional per-kernel timing (options.profile)
  struct ProfEv {
    hipEvent_t a, b;
    int kid;
  };
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfEv> ev_pending;
  double prof_ms[AFC_KERNEL_COUNT] = {};
  int64_t prof_n[AFC_KERNEL_COUNT] = {};
  double prof_bytes[AFC_KERNEL_COUNT] = {};  // algorithmic bytes of launches that did work
  int64_t prof_work[AFC_KERNEL_COUNT] = {};  // launches that did work
};

namespace afc {
// Algorithmic HBM bytes of one GMRES cycle whose Arnoldi process completed kk
// columns out of m, added to the per-kernel work counters (profiling only).
void prof_gmres_cycle(afc_handle_s* h, bool fp32, int m, int kk);
void prof_sstep_cycle(afc_handle_s* h, int m, int s, int kk, bool fp64);  // the same for an s-step cycle
void prof_collect(afc_handle_s* h);  // fold completed event pairs into the totals
void prof_release(afc_handle_s* h);
}  // namespace afc
