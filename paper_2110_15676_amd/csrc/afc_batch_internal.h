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
}
