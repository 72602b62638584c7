// Internal definitions of the batched CN-FCT launch (afc_batch_*).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/afc.h"

namespace afc {

// One instance inside the packed layout.
// Entry arrays of an instance are stored in SELL-64 order: slices of 64 rows
// padded to the slice's longest row, slot (slice s, entry p, lane l) at
// sl_ptr[s] + 64 p + l, column as a delta j - i; padding slots have delta 0
// and value 0.
struct BInst {
  int N;
  int nnz;
  int nsl;           // slices
  int64_t node_off;  // offset into packed node arrays (and packed u, F)
  int64_t slot_off;  // offset into packed slot arrays
  int64_t sl_off;    // offset into the packed slice pointers (nsl + 1 per instance)
  double dt;
};

// Per-instance result of one afc_batch_step_cn call.
struct BStat {
  int status;
  int fp_iters;
  long long krylov_iters;
  double res0, res, lin_res;
};

// Options the persistent kernel needs (copied from afc_options).
struct BatchOpts {
  int alpha_mode;
  int fp_tol_mode;
  int fp_maxit;
  int lin_maxit;
  int dynamic_damping;
  double fp_tol;
  double lin_atol, lin_rtol;
  double prelimit;
  double omega;
  double lin_eta;
};

// Resumable state of one instance inside the workgroup-per-instance kernels
// (every thread of the workgroup holds the same values).  A run can stop at
// the top of a fixed-point iteration and continue later from this state and
// the instance's device vectors; the arithmetic is the same either way.
struct SState {
  int phase;      // -1: nothing done; 0: at the start of a CN step; 1: inside the fixed point
  int step;       // CN steps finished
  int nu;         // fixed-point iterations of the current step / solve
  int have_prev;  // a previous residual exists (damping rule)
  int status;     // afc_status so far
  int done;       // 1 once the instance has finished
  int fp_total;   // fixed-point iterations over all steps
  int pad_;
  long long kry;  // Krylov iterations
  double R0, R_prev, omega, res0, res, lin_res;
};

// One request of the served loop (device memory).  Every pointer is device
// memory owned by the request: SELL-64 layout with the diagonal first in each
// row; CN uses mij, dp, AL (A_low of the FCT scheme) and builds A = M_L/dt +
// A_low/2 itself; the stationary MCL solve uses cc, ccT (convective a_ij and
// a_ji) and A = A_low of the MCL scheme, both with Dirichlet identity rows.
struct SReq {
  int kind;       // AFC_REQ_CN or AFC_REQ_STATIONARY
  int N, nsl, steps, init_low, pad_;
  double dt;
  BatchOpts o;
  const int* slp;
  const int16_t* dlt;
  const double *mij, *dp, *AL, *ml, *uD, *cc, *ccT;
  const uint8_t* isd;
  double *A, *dinv, *work, *u;
  const double* F;
  int64_t ldw;    // stride of the work vectors
};

// Packed device arrays (passed by value to the kernel).
struct BatchDev {
  const int* slp;       // slice pointers, relative to the instance's slot_off
  const int16_t* dlt;   // column deltas j - i
  const double *mij, *dp, *AL, *ml, *uD;
  const uint8_t* is_dir;
  double* Acn;     // CN matrix values (SELL order), rebuilt for each call's dt
  double* dinv;
  double* work;    // work vectors, [vector][total_nodes]
  int64_t total_nodes;
};

int batch_work_vectors();

}  // namespace afc

struct afc_batch_s {
  int count = 0;
  int G = 16;
  int device = 0;
  int64_t total_nodes = 0, total_nnz = 0, total_slots = 0;
  afc_options opt{};
  afc::BatchOpts bopt{};
  hipStream_t stream = nullptr;
  int threads = 1024;   // schedule of the persistent launch (results do not depend on it)
  int workgroups = 0;   // 0: twice the compute units, at most count
  std::string last_error;
  std::vector<afc::BInst> host_insts;
  std::vector<int> host_order;
  afc::BInst* insts = nullptr;
  int* order = nullptr;
  int* queue = nullptr;
  afc::BStat* stats_d = nullptr;
  afc::BatchDev dev{};
  // owned device buffers
  int* slp = nullptr;
  int16_t* dlt = nullptr;
  double *mij = nullptr, *dp = nullptr, *AL = nullptr, *ml = nullptr, *uD = nullptr;
  uint8_t* is_dir = nullptr;
  double *Acn = nullptr, *dinv = nullptr, *work = nullptr;
};

namespace afc {
// one persistent launch of `grid` workgroups of `threads` (256, 512 or 1024)
void batch_launch(afc_batch_s* b, double* u, const double* F, int steps, int threads, int grid);
// one round of the served loop: workgroups take the `count` requests of
// `list` from `queue` and advance each by at most `quantum` wall-clock ticks
// (at least one fixed-point iteration; quantum <= 0: to completion)
void serve_round_launch(const SReq* reqs, SState* states, const int* list, int count, int* queue, int64_t quantum,
                        int threads, int grid, hipStream_t stream);
int serve_work_vectors();

// Host image of one request of the served loop: every input array in SELL-64
// order (diagonal first), packed at 256-byte aligned offsets of one device
// block, followed by the request's scratch (CN matrix, work vectors).
struct ServeImage {
  int N = 0, nsl = 0;
  int64_t slots = 0, ldw = 0;
  size_t upload_bytes = 0;  // leading bytes of the block that hold inputs
  size_t block_bytes = 0;   // whole block
  std::vector<unsigned char> bytes;  // the first upload_bytes of the block
  size_t off_slp = 0, off_dlt = 0, off_mij = 0, off_dp = 0, off_AL = 0, off_ml = 0, off_cc = 0, off_ccT = 0,
         off_A = 0, off_dinv = 0, off_uD = 0, off_isd = 0, off_F = 0, off_u = 0, off_work = 0;
};

// Device block size of a request (N nodes, CSR row pointers rp) in the
// served loop, without building it.
size_t serve_block_bytes(int N, const int32_t* rp, int kind);

// Builds the image of a request: the operators of eqs. (4)-(6) (FCT data for
// CN, MCL data for the stationary solve), its SELL layout and its vectors
// (u0: NULL = zero).  Returns AFC_OK or an error status with *err set.
afc_status serve_prepare(const afc_problem* p, int kind, const double* u0, const double* F, ServeImage& img,
                         std::string* err);
}
