// C ABI of libafc: validation, setup of the AFC operators, Krylov drivers
// and the time-step / stationary drivers.  The drivers only enqueue kernels;
// the host waits once per fixed-point iteration (nonlinear residual) and once
// per Krylov chunk (BiCGStab) or cycle (GMRES).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "afc_batch_internal.h"
#include "afc_kernels.h"
#include "afc_layout.h"

using afc::KState;
using afc::kMaxRestart;
using afc::kRedBlocks;
using afc::kMaxRed;

namespace {

// work vector slots
enum Slot { W_ARN = 0, W_B, W_R, W_X, W_A, W_B2, W_RP, W_RM, W_UOLD, W_UT, W_G, W_S1, W_S2,
            W_RHAT, W_P, W_V, W_S, W_T, W_COUNT };

struct Fail {
  afc_status st;
  std::string msg;
};

#define HIP_OK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      const std::string m_ = std::string(#expr) + ": " + hipGetErrorString(e_);          \
      if (h) h->last_error = m_;                                                         \
      throw Fail{AFC_EDEVICE, m_};                                                       \
    }                                                                                    \
  } while (0)

[[noreturn]] void fail(afc_handle* h, afc_status st, const std::string& msg) {
  if (h) h->last_error = msg;
  throw Fail{st, msg};
}

thread_local std::string g_create_error;  // errors of afc_create before a handle exists

afc_status check_options(const afc_options& o, std::string& why) {
  if (o.alpha_mode < 0 || o.alpha_mode > 2) return why = "alpha_mode", AFC_EINVAL;
  if (o.krylov != AFC_KRYLOV_BICGSTAB && o.krylov != AFC_KRYLOV_GMRES) return why = "krylov", AFC_EINVAL;
  if (o.restart < 1 || o.restart > kMaxRestart) return why = "restart must be in 1..64", AFC_EINVAL;
  if (o.precision != AFC_PREC_FP64 && o.precision != AFC_PREC_MIXED) return why = "precision", AFC_EINVAL;
  if (o.precision == AFC_PREC_MIXED && o.krylov != AFC_KRYLOV_GMRES)
    return why = "mixed precision is implemented with GMRES", AFC_EINVAL;
  if (!(o.lin_atol >= 0) || !(o.lin_rtol >= 0) || !(o.inner_rtol >= 0) || !(o.fp_tol >= 0))
    return why = "tolerances must be >= 0", AFC_EINVAL;
  if (o.lin_maxit < 1 || o.inner_maxit < 1 || o.refine_maxit < 1 || o.fp_maxit < 0)
    return why = "iteration caps", AFC_EINVAL;
  if (o.fp_tol_mode != AFC_TOL_ABS_SQRTN && o.fp_tol_mode != AFC_TOL_REL) return why = "fp_tol_mode", AFC_EINVAL;
  if (!(o.prelimit >= 0) || !std::isfinite(o.prelimit)) return why = "prelimit", AFC_EINVAL;
  if (!(o.omega > 0 && o.omega <= 1)) return why = "omega must be in (0, 1]", AFC_EINVAL;
  if (o.ssp_stages < 1 || o.ssp_stages > 3) return why = "ssp_stages must be 1, 2 or 3", AFC_EINVAL;
  if (o.profile != 0 && o.profile != 1) return why = "profile must be 0 or 1", AFC_EINVAL;
  if (o.graphs != 0 && o.graphs != 1) return why = "graphs must be 0 or 1", AFC_EINVAL;
  if (o.limiter != AFC_LIMITER_MCL && o.limiter != AFC_LIMITER_MU) return why = "limiter", AFC_EINVAL;
  if (o.sstep != 0 && (o.sstep < 2 || o.sstep > afc::kSMax)) return why = "sstep must be 0 or 2..16", AFC_EINVAL;
  if (!std::isfinite(o.sstep_shift)) return why = "sstep_shift must be finite", AFC_EINVAL;
  if (!(o.lin_eta >= 0 && o.lin_eta < 1)) return why = "lin_eta must be in [0, 1)", AFC_EINVAL;
  if (o.lanes_per_row != 0 && o.lanes_per_row != 8 && o.lanes_per_row != 16 && o.lanes_per_row != 32 &&
      o.lanes_per_row != 64)
    return why = "lanes_per_row must be 0, 8, 16, 32 or 64", AFC_EINVAL;
  return AFC_OK;
}

template <typename T>
std::vector<T> fetch(afc_handle* h, const T* p, size_t n, int mem_space) {
  std::vector<T> v(n);
  if (n == 0) return v;
  if (mem_space == AFC_MEM_DEVICE)
    HIP_OK(hipMemcpy(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost));
  else
    std::memcpy(v.data(), p, n * sizeof(T));
  return v;
}

// Device copy of a host vector, ordered on stream st (the caller synchronizes
// st before the host vector goes away).
template <typename T>
T* upload(afc_handle* h, const std::vector<T>& v, hipStream_t st) {
  T* d = nullptr;
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  if (hipMalloc(&d, bytes) != hipSuccess) fail(h, AFC_ENOMEM, "hipMalloc failed during afc_create");
  if (!v.empty()) HIP_OK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return d;
}

template <typename T>
T* dalloc(afc_handle* h, size_t n) {
  T* d = nullptr;
  if (hipMalloc(&d, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess) fail(h, AFC_ENOMEM, "hipMalloc failed");
  return d;
}

int pick_lanes(int64_t nnz, int N, int forced) {
  if (forced) return forced;
  const double avg = double(nnz) / double(N);
  if (avg <= 8.0) return 8;
  if (avg <= 16.0) return 16;
  if (avg <= 32.0) return 32;
  return 64;
}

void free_all(afc_handle* h) {
  auto f = [](auto*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
  };
  f(h->row_ptr); f(h->col); f(h->is_dir); f(h->uD); f(h->ml);
  f(h->mij); f(h->dp_fct); f(h->AL_fct); f(h->mu_own);
  f(h->cc); f(h->ccT); f(h->AL_mcl); f(h->dinv_mcl);
  f(h->A_cn); f(h->dinv_cn);
  f(h->sl_ptr); f(h->sl_dl); f(h->sl_pat); f(h->sl_dlt); f(h->sell_pos); f(h->sl_mask); f(h->Scc); f(h->SccT); f(h->S_mij); f(h->S_dp); f(h->S_alf); f(h->S_own); f(h->S64_mcl); f(h->S32_mcl); f(h->S64_cn); f(h->S32_cn);
  f(h->ks_ptr); f(h->ks_dl); f(h->ks_pat); f(h->ks_dlt); f(h->kpos);
  for (auto*& p : h->w) f(p);
  h->w.clear();
  f(h->V64); f(h->V32); f(h->apply_tmp);
  f(h->partials); f(h->partials_res); f(h->partials_blk); f(h->ks);
  if (h->host_status) (void)hipHostFree(h->host_status);
  h->host_status = nullptr;
  if (h->ring) (void)hipHostFree(h->ring);
  h->ring = nullptr;
  for (auto& e : h->ring_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  afc::prof_release(h);
  for (auto& e : h->graphs) (void)hipGraphExecDestroy(e.second);
  h->graphs.clear();
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  h->cap_stream = nullptr;
}

void sync_status(afc_handle* h) {
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(h->host_status, h->ks, afc::kStatusBytes, hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  if (!h->ev_pending.empty()) afc::prof_collect(h);
}

// m_ij, d+_ij and A_low (FCT) in SELL slot order, for the explicit stages and
// the MC passes over the SELL rows; built on first use
void ensure_fct_sell(afc_handle* h) {
  if (h->S_mij) return;
  const size_t slots = (size_t)h->sell_slots;
  h->S_mij = dalloc<double>(h, slots);
  h->S_dp = dalloc<double>(h, slots);
  h->S_alf = dalloc<double>(h, slots);
  HIP_OK(hipMemsetAsync(h->S_mij, 0, slots * sizeof(double), h->stream));
  HIP_OK(hipMemsetAsync(h->S_dp, 0, slots * sizeof(double), h->stream));
  HIP_OK(hipMemsetAsync(h->S_alf, 0, slots * sizeof(double), h->stream));
  afc::to_sell64(h, h->mij, h->S_mij);
  afc::to_sell64(h, h->dp_fct, h->S_dp);
  afc::to_sell64(h, h->AL_fct, h->S_alf);
  h->S_own = dalloc<uint8_t>(h, slots);
  HIP_OK(hipMemsetAsync(h->S_own, 0, slots, h->stream));
  afc::to_sell8(h, h->mu_own, h->S_own);
}

void ensure_ring(afc_handle* h) {
  if (h->ring) return;
  HIP_OK(hipHostMalloc((void**)&h->ring, 2 * afc::kStatusBytes, hipHostMallocDefault));
  for (auto& e : h->ring_ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

void ensure_basis(afc_handle* h, int m, bool fp32) {
  if (h->Vm < m) {
    if (h->V64) (void)hipFree(h->V64);
    if (h->V32) (void)hipFree(h->V32);
    h->V64 = nullptr;
    h->V32 = nullptr;
    h->Vm = m;
  }
  const size_t n = (size_t)(h->Vm + 1) * (size_t)h->ldv;
  if (fp32 && !h->V32) {
    h->V32 = dalloc<float>(h, n);
    HIP_OK(hipMemsetAsync(h->V32, 0, n * sizeof(float), h->stream));
  }
  if (!fp32 && !h->V64) {
    h->V64 = dalloc<double>(h, n);
    HIP_OK(hipMemsetAsync(h->V64, 0, n * sizeof(double), h->stream));
  }
}

struct SysMat {
  const double* A;    // CSR values (BiCGStab)
  const double* dinv; // inverse diagonal (right Jacobi)
  const double* S64;  // same matrix in SELL order (GMRES FP64, residuals)
  const float* S32;   // Jacobi-scaled FP32 copy in SELL order (mixed GMRES)
};

struct SolveOut {
  afc_status st = AFC_OK;
  int64_t iters = 0;
  int64_t inner = 0;
  int sweeps = 0;
  double res = 0.0;
};

// The graph of the launches that `issue` makes on the handle's stream, keyed
// by `key`: replayed from the handle's cache, or captured on the handle's
// private capture stream.  At most kGraphCache are kept; a hit moves its entry
// to the back and a capture drops the least recently used one, so the graphs
// that one solve looks up back to back (GMRES holds two) stay alive.
constexpr size_t kGraphCache = 8;
static_assert(kGraphCache >= 2, "a GMRES solve holds two cached graphs at once");

template <typename F>
hipGraphExec_t cached_graph(afc_handle* h, const std::vector<const void*>& key, F&& issue) {
  for (size_t k = 0; k < h->graphs.size(); ++k)
    if (h->graphs[k].first == key) {
      auto e = std::move(h->graphs[k]);
      h->graphs.erase(h->graphs.begin() + (std::ptrdiff_t)k);
      h->graphs.push_back(std::move(e));
      return h->graphs.back().second;
    }
  if (h->graphs.size() >= kGraphCache) {
    (void)hipGraphExecDestroy(h->graphs.front().second);
    h->graphs.erase(h->graphs.begin());
  }
  if (!h->cap_stream) HIP_OK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  hipStream_t user = h->stream;
  h->stream = h->cap_stream;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    issue();
    e = hipStreamEndCapture(h->cap_stream, &g);
  }
  h->stream = user;
  HIP_OK(e);
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIP_OK(e);
  h->graphs.emplace_back(key, exec);
  return exec;
}

const void* key_int(int64_t v) { return reinterpret_cast<const void*>((intptr_t)v); }

// GMRES(m), right Jacobi.  x: in x0, out solution; r: b - A x0 on entry, with
// ||r||^2 in ks->red[red_idx].  FP64 mode runs the Arnoldi process in FP64;
// MIXED runs it in FP32 on the Jacobi-scaled FP32 matrix and recomputes the
// FP64 residual after every cycle (iterative refinement, one sweep per cycle).
SolveOut solve_gmres(afc_handle* h, const SysMat& S, const double* b, double* x, double* r, int red_idx,
                     double tol) {
  SolveOut o;
  const bool mixed = h->opt.precision == AFC_PREC_MIXED;
  // MIXED: one refinement sweep = one FP32 cycle of at most min(restart, inner_maxit) steps
  const int m = mixed ? std::min(h->opt.restart, h->opt.inner_maxit) : h->opt.restart;
  const double inner_rel = mixed ? h->opt.inner_rtol : 0.0;
  const int64_t cap = h->opt.lin_maxit;
  // s-step blocks (both precisions): blocks of s basis vectors from the
  // shifted powers (A - theta I)^j (default theta = 1, the centre of the
  // Gershgorin discs of the Jacobi-scaled matrix).  A cycle whose status
  // shows a failed block QR makes later cycles, in this and later solves on
  // the handle, use half the block size (one vector per step below 2) until
  // the options are set again.
  int s = std::min(h->opt.sstep, h->sstep_cap);
  // A solve expected to take fewer iterations than a block (the handle's
  // previous solve, e.g. inexact fixed-point solves) uses blocks of 4 or 8,
  // whichever first covers them, so that a block computes few powers beyond
  // the solve's end; two extra sizes keep the graph cache small.
  for (int q = 4; q <= 8; q *= 2)
    if (h->gmres_last <= q && q < s) {
      s = q;
      break;
    }
  if (s < 2) s = 0;
  ensure_basis(h, m, mixed);
  // start vector: normalized in the basis precision (mixed, and FP64 s-step
  // cycles), or FP64 r with its scale 1/beta (FP64 one-vector cycles)
  if (mixed || s) {
    afc::cycle_start(h, 2, red_idx, tol, inner_rel);
    afc::cast_v0(h, r, !mixed);
  } else {
    afc::copy(h, h->V64, r);
    afc::cycle_start(h, 1, red_idx, tol, 0.0);
  }
  sync_status(h);
  const int it0 = h->host_status->iters;
  double res = h->host_status->beta;
  if (!std::isfinite(res)) {
    o.st = AFC_ENAN;
    o.res = res;
    return o;
  }
  // one cycle: m Arnoldi steps, back substitution, x update, FP64 residual
  // and the restart (no host decision inside, so it can be replayed)
  auto cycle = [&]() {
    for (int k = 0; k < m; ++k) {
      if (mixed)
        afc::gmres_spmv32(h, S.S32, k);
      else
        afc::gmres_spmv64(h, S.S64, S.dinv, k);
      afc::gmres_dots(h, mixed, k);
      afc::gmres_reduce(h, mixed, k, m);
      afc::gmres_update(h, mixed, k);
    }
    afc::gmres_last_givens(h, mixed, m - 1, m);
    afc::gmres_solve(h, m);
    afc::gmres_xupdate(h, mixed, S.dinv, x);
    if (mixed) {
      afc::residual(h, S.S64, b, x, r, 2);
      afc::cast_v0(h, r);
    } else {
      afc::residual(h, S.S64, b, x, h->V64, 1);
    }
  };
  const double theta = h->opt.sstep_shift;
  // The last block is not orthogonalized in place: no later step reads its
  // vectors, and the x update takes them raw with their coefficients.
  auto cycle_sstep = [&]() {
    int kb = 0, sbl = 0;
    for (int k = 0; k < m; k += s) {
      const int sb = std::min(s, m - k);
      for (int j = 1; j <= sb; ++j) {  // alternating sweep directions (cache reuse between the SpMVs)
        const size_t src = (size_t)(k + j - 1) * h->ldv, dst = (size_t)(k + j) * h->ldv;
        if (mixed)
          afc::spmv32(h, S.S32, h->V32 + src, (float)theta, (j + 1) & 1, h->V32 + dst);
        else
          afc::spmv64(h, S.S64, S.dinv, h->V64 + src, theta, (j + 1) & 1, h->V64 + dst);
      }
      afc::sstep_dots(h, k, sb, !mixed);
      afc::sstep_reduce(h, k, sb, m, theta, !mixed);
      if (k + sb < m) afc::sstep_update(h, k, sb, !mixed);
      kb = k;
      sbl = sb;
    }
    afc::gmres_solve(h, m, kb, sbl);
    afc::sstep_xupdate(h, kb, sbl, S.dinv, x, !mixed);
    afc::residual(h, S.S64, b, x, r, 2);
    afc::cast_v0(h, r, !mixed);
  };
  if (s && !h->partials_blk) {
    h->partials_blk = dalloc<double>(h, (size_t)afc::kBlkRows * afc::kRedBlocks);
    HIP_OK(hipMemsetAsync(h->partials_blk, 0, sizeof(double) * afc::kBlkRows * afc::kRedBlocks, h->stream));
  }
  const int fails0 = h->host_status->sfail;
  uint64_t theta_bits = 0;
  std::memcpy(&theta_bits, &theta, sizeof(theta_bits));
  const bool graphs = h->opt.graphs && !h->opt.profile;
  // graphs are looked up right before their launch, so a capture for a new
  // block size cannot have evicted the one being launched
  auto issue = [&]() {
    if (s) {
      if (graphs)
        HIP_OK(hipGraphLaunch(cached_graph(h, {key_int(3), S.S32, S.S64, S.dinv, b, x, r, h->V32, h->V64,
                                               key_int(m), key_int(mixed), key_int(s), key_int(h->ldv),
                                               key_int((int64_t)theta_bits)},
                                           cycle_sstep),
                              h->stream));
      else
        cycle_sstep();
    } else if (graphs) {
      HIP_OK(hipGraphLaunch(cached_graph(h, {key_int(1), S.S32, S.S64, S.dinv, b, x, r, h->V32, h->V64, h->w[0],
                                             key_int(m), key_int(mixed), key_int(h->ldv)},
                                         cycle),
                            h->stream));
    } else {
      cycle();
    }
  };
  int fails_seen = fails0;
  // after the status of a cycle run with block size s_used: a new failure halves it
  auto after_status = [&](int sfail, int s_used) {
    if (sfail != fails_seen) {
      fails_seen = sfail;
      if (s_used) {
        s = std::min(s, s_used / 2 >= 2 ? s_used / 2 : 0);
        h->sstep_cap = std::min(h->sstep_cap, std::max(s, 1));
      }
    }
  };
  if (h->opt.profile) {  // one cycle at a time, so that each cycle's work can be accounted
    int cycle_it0 = it0;
    while (res > tol) {
      const int s_used = s;
      issue();
      o.sweeps += 1;
      sync_status(h);
      if (s_used) {
        afc::prof_sstep_cycle(h, m, s_used, h->host_status->iters - cycle_it0, !mixed);
        after_status(h->host_status->sfail, s_used);
      } else {
        afc::prof_gmres_cycle(h, mixed, m, h->host_status->iters - cycle_it0);
      }
      cycle_it0 = h->host_status->iters;
      res = h->host_status->beta;
      const int64_t its = h->host_status->iters - it0;
      if (!std::isfinite(res)) {
        o.st = AFC_ENAN;
        break;
      }
      if (its >= cap || (mixed && o.sweeps >= h->opt.refine_maxit)) {
        if (res > tol) o.st = AFC_ENOCONV;
        break;
      }
    }
  } else if (res > tol) {
    // Cycles (replayed graphs, or the same launches issued directly) are kept
    // one ahead: the next cycle is queued before the host waits for the
    // status of the one in flight, when that cycle is not expected to
    // converge and the next one stays within the iteration and sweep caps.
    // This hides the host's round trip between cycles.  A cycle that starts
    // after the solve converged finds ks->solved set, and every kernel of it
    // returns at once.  A failed s-step block halves the block size from the
    // first cycle queued after its status is seen; since graphs and direct
    // launches take the same queueing decisions, both give the same iterates.
    ensure_ring(h);
    int queued = 0, seen = 0;  // cycles issued; cycles whose status was read
    int slot_s[2] = {0, 0};    // block size each ring slot's cycle ran with
    int64_t its = 0;
    // residual factor expected of one cycle: the inner tolerance bounds a
    // mixed-precision sweep; unknown (no look-ahead) before the first FP64 cycle
    double rate = mixed ? inner_rel : 0.0;
    auto queue = [&]() {
      const int slot = queued & 1;
      slot_s[slot] = s;
      issue();
      HIP_OK(hipMemcpyAsync(h->ring + slot * afc::kStatusBytes, h->ks, afc::kStatusBytes, hipMemcpyDeviceToHost,
                            h->stream));
      HIP_OK(hipEventRecord(h->ring_ev[slot], h->stream));
      ++queued;
    };
    queue();
    for (;;) {
      const bool allowed = its + 2 * (int64_t)m <= cap && (!mixed || seen + 2 <= h->opt.refine_maxit);
      if (queued - seen == 1 && allowed && res * rate > 2.0 * tol) queue();
      const int slot = seen & 1;
      HIP_OK(hipEventSynchronize(h->ring_ev[slot]));
      const afc::KState* st = reinterpret_cast<const afc::KState*>(h->ring + slot * afc::kStatusBytes);
      ++seen;
      o.sweeps += 1;
      after_status(st->sfail, slot_s[slot]);
      const double prev = res;
      res = st->beta;
      its = st->iters - it0;
      if (!std::isfinite(res)) {
        o.st = AFC_ENAN;
        break;
      }
      if (res <= tol) break;
      if (its >= cap || (mixed && o.sweeps >= h->opt.refine_maxit)) {
        o.st = AFC_ENOCONV;
        break;
      }
      if (prev > 0.0) rate = res / prev;
      if (queued == seen) queue();
    }
    sync_status(h);  // drains the queue: host_status holds the final state
  }
  o.iters = h->host_status->iters - it0;
  if (mixed) o.inner = o.iters;
  o.res = res;
  h->gmres_last = (int)std::min<int64_t>(o.iters, 1 << 30);
  return o;
}

// BiCGStab, right Jacobi, FP64.  Same contract as solve_gmres.
SolveOut solve_bicgstab(afc_handle* h, const SysMat& S, const double* b, double* x, double* r, double tol) {
  SolveOut o;
  afc::BicgVec v{x, r, h->w[W_RHAT], h->w[W_P], h->w[W_V], h->w[W_S], h->w[W_T]};
  // no status read here: only Krylov kernels change the device's iteration
  // count and every solve ends with a status read, so the host copy is current
  const int it0 = h->host_status->iters;
  int restarts = 0;
  // iterations of the first chunk: about what the previous solve on this
  // handle took (a power of two in 2..16); iterations past convergence find
  // the state done and return at once
  int first = 2;
  while (first < std::min(h->bicg_last, 16)) first *= 2;
  while (true) {
    // no wait after the start: a non-finite start marks the state done, so
    // the chunk's iterations return at once and the status read after the
    // chunk reports it
    afc::bicg_init(h, v, tol);
    int chunk = first;
    do {
      const int n = std::min<int>(chunk, h->opt.lin_maxit - (h->host_status->iters - it0));
      // the chunk's iterations, then the true residual b - A x of its iterate
      // into t (every iteration writes t before reading it) with its norm
      auto iters = [&]() {
        for (int c = 0; c < n; ++c) afc::bicg_iter(h, S.S64, S.dinv, v);
        afc::residual(h, S.S64, b, x, v.t, 0);
      };
      if (h->opt.graphs && !h->opt.profile)
        HIP_OK(hipGraphLaunch(cached_graph(h, {key_int(4), S.S64, S.dinv, b, x, r, key_int(n)}, iters), h->stream));
      else
        iters();
      sync_status(h);
      chunk = std::min(chunk * 2, 16);
    } while (!h->host_status->done && h->host_status->iters - it0 < h->opt.lin_maxit);
    h->bicg_last = h->host_status->iters - it0;
    if (h->host_status->flag == 2) {
      o.st = AFC_ENAN;
      o.res = h->host_status->res;
      break;
    }
    const bool breakdown = h->host_status->flag == 1;
    const double res = std::sqrt(h->host_status->red[0]);  // the true residual of the last iterate
    o.res = res;
    if (!std::isfinite(res)) {
      o.st = AFC_ENAN;
      break;
    }
    if (res <= tol) break;
    if (breakdown && ++restarts > 1) {
      o.st = AFC_EBREAKDOWN;
      break;
    }
    if (h->host_status->iters - it0 >= h->opt.lin_maxit) {
      o.st = AFC_ENOCONV;
      break;
    }
    afc::residual(h, S.S64, b, x, r, 0);  // restart from the true residual
  }
  o.iters = h->host_status->iters - it0;
  return o;
}

SolveOut linear_solve(afc_handle* h, const SysMat& S, const double* b, double* x, double* r, int red_idx,
                      double tol) {
  if (h->opt.krylov == AFC_KRYLOV_GMRES) return solve_gmres(h, S, b, x, r, red_idx, tol);
  return solve_bicgstab(h, S, b, x, r, tol);
}

void add_solve(afc_stats* st, const SolveOut& o) {
  if (!st) return;
  st->krylov_iters += o.iters;
  st->inner_iters += o.inner;
  st->refine_sweeps += o.sweeps;
  st->lin_res = o.res;
}

bool fp_converged(const afc_handle* h, double R, double R0) {
  if (h->opt.fp_tol_mode == AFC_TOL_ABS_SQRTN) return R < std::sqrt((double)h->N) * h->opt.fp_tol;
  return R <= h->opt.fp_tol * R0;
}

double next_omega(const afc_handle* h, double omega, double R, double R_prev, bool have_prev) {
  if (!h->opt.dynamic_damping || !have_prev) return omega;
  if (R > R_prev) return std::max(omega * 0.5, 1.0 / 64.0);
  return std::min(1.0, omega * 1.25);
}

// Fixed-point loop of Sec. 4 shared by the CN and stationary drivers.
// `eval` enqueues the limiter + residual kernels writing b, r and the
// reductions R^2, ||b||^2, ||r||^2 into ks->red[0..2].
template <typename Eval>
afc_status fixed_point(afc_handle* h, double* u, const SysMat& S, Eval eval, afc_stats* st) {
  double* b = h->w[W_B];
  double* r = h->w[W_R];
  double R0 = 0.0, R_prev = 0.0;
  bool have_prev = false;
  double omega = h->opt.omega;
  afc_status status = AFC_OK;
  int nu = 0;
  h->res_hist.clear();
  while (true) {
    eval(u, b, r);
    sync_status(h);
    const double R = std::sqrt(h->host_status->red[0]);
    h->res_hist.push_back(R);
    const double bn = std::sqrt(h->host_status->red[1]);
    if (!std::isfinite(R) || !std::isfinite(bn)) {
      status = AFC_ENAN;
      h->last_error = "non-finite nonlinear residual";
      break;
    }
    if (nu == 0) R0 = R;
    if (st) {
      if (nu == 0) st->res0 = R;
      st->res = R;
    }
    if (R == 0.0 || fp_converged(h, R, R0)) break;
    if (nu >= h->opt.fp_maxit) {
      status = AFC_WMAXIT;
      break;
    }
    omega = next_omega(h, omega, R, R_prev, have_prev);
    const bool relax = omega != 1.0;
    double* x = u;
    if (relax) {
      x = h->w[W_X];
      afc::copy(h, x, u);
    }
    const double tol = std::max(std::max(h->opt.lin_atol, h->opt.lin_rtol * bn), h->opt.lin_eta * R);
    const SolveOut o = linear_solve(h, S, b, x, r, 2, tol);
    add_solve(st, o);
    if (o.st == AFC_ENAN || o.st == AFC_EBREAKDOWN) {
      status = o.st;
      h->last_error = o.st == AFC_ENAN ? "non-finite linear residual" : "BiCGStab breakdown";
      break;
    }
    if (relax) afc::relax(h, u, x, omega);
    R_prev = R;
    have_prev = true;
    ++nu;
  }
  if (st) st->fp_iters = nu;
  return status;
}

void ensure_work(afc_handle* h) {
  if ((int)h->w.size() == W_COUNT) return;
  h->w.assign(W_COUNT, nullptr);
  for (int s = 0; s < W_COUNT; ++s) {
    h->w[s] = dalloc<double>(h, (size_t)h->ldv);
    HIP_OK(hipMemsetAsync(h->w[s], 0, (size_t)h->ldv * sizeof(double), h->stream));
  }
}

// Host-side setup shared by afc_create and afc_batch_create: fetch, validate,
// and build the AFC operators of eqs. (4)-(6).
struct HostOps {
  int N = 0;
  int64_t nnz = 0;
  std::vector<int> rp, col, diag, tpos;
  std::vector<double> M, K, Kc, ml, uD;
  std::vector<uint8_t> is_dir;
  std::vector<double> dp, AL;              // FCT: d+ from K, A_low (Dirichlet rows identity)
  std::vector<double> c, cT, ALc, dinv;    // MCL: convective c, c^T, A_low from it, 1/diag
  std::vector<uint8_t> mu_own;             // MU: 1 if a_ji < a_ij, 2 if a_ji > a_ij, 0 if equal
};

void check_problem(const afc_problem* p) {
  if (p->n <= 0 || p->nnz <= 0 || p->nnz >= (int64_t)std::numeric_limits<int>::max())
    throw Fail{AFC_EINVAL, "need n > 0 and 0 < nnz < 2^31"};
  if (p->mem_space != AFC_MEM_HOST && p->mem_space != AFC_MEM_DEVICE) throw Fail{AFC_EINVAL, "mem_space"};
  if (!p->row_ptr || !p->col_idx || !p->M || !p->K || (p->n_dir > 0 && (!p->dir_idx || !p->dir_val)) ||
      p->n_dir < 0)
    throw Fail{AFC_EINVAL, "null array"};
}

void prepare_ops(afc_handle* h, const afc_problem* p, HostOps& o) {
  check_problem(p);
  const int N = p->n;
  const int64_t nnz = p->nnz;
  const int ms = p->mem_space;
  o.N = N;
  o.nnz = nnz;
  std::vector<int>& rp = o.rp;
  std::vector<int>& col = o.col;
  std::vector<double>& M = o.M;
  std::vector<double>& K = o.K;
  std::vector<double>& Kc = o.Kc;
  std::vector<double>& ml = o.ml;
  o.rp = fetch(h, p->row_ptr, (size_t)N + 1, ms);
  o.col = fetch(h, p->col_idx, (size_t)nnz, ms);
  o.M = fetch(h, p->M, (size_t)nnz, ms);
  o.K = fetch(h, p->K, (size_t)nnz, ms);
  o.Kc = p->K_conv ? fetch(h, p->K_conv, (size_t)nnz, ms) : std::vector<double>();
  o.ml = p->ML ? fetch(h, p->ML, (size_t)N, ms) : std::vector<double>();
  const std::vector<int> didx = fetch(h, p->dir_idx, (size_t)p->n_dir, ms);
  const std::vector<double> dval = fetch(h, p->dir_val, (size_t)p->n_dir, ms);

  // --- pattern checks -------------------------------------------------------
  if (rp[0] != 0 || rp[N] != nnz) fail(h, AFC_EINVAL, "row_ptr[0] must be 0 and row_ptr[N] = nnz");
  std::vector<int>& diag = o.diag;
  diag.assign(N, -1);
  for (int i = 0; i < N; ++i) {
    if (rp[i + 1] < rp[i]) fail(h, AFC_EINVAL, "row_ptr not monotone");
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int j = col[k];
      if (j < 0 || j >= N) fail(h, AFC_EINVAL, "column index out of range");
      if (k > rp[i] && col[k - 1] >= j) fail(h, AFC_EINVAL, "columns not strictly ascending in a row");
      if (j == i) diag[i] = k;
    }
    if (diag[i] < 0) fail(h, AFC_EINVAL, "missing diagonal entry in row " + std::to_string(i));
  }
  std::vector<int>& tpos = o.tpos;
  tpos.assign((size_t)nnz, 0);
  for (int i = 0; i < N; ++i) {
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int j = col[k];
      const int* b0 = col.data() + rp[j];
      const int* b1 = col.data() + rp[j + 1];
      const int* f = std::lower_bound(b0, b1, i);
      if (f == b1 || *f != i) fail(h, AFC_EINVAL, "pattern is not structurally symmetric");
      tpos[k] = (int)(f - col.data());
    }
  }
  for (int64_t k = 0; k < nnz; ++k)
    if (!std::isfinite(M[k]) || !std::isfinite(K[k]) || (!Kc.empty() && !std::isfinite(Kc[k])))
      fail(h, AFC_ENAN, "non-finite matrix entry");
  // lumped mass m_i = sum_j m_ij (eq. (5))
  if (ml.empty()) {
    ml.assign(N, 0.0);
    for (int i = 0; i < N; ++i)
      for (int k = rp[i]; k < rp[i + 1]; ++k) ml[i] += M[k];
  }
  for (int i = 0; i < N; ++i)
    if (!(ml[i] > 0.0) || !std::isfinite(ml[i])) fail(h, AFC_EINVAL, "lumped mass must be positive");
  std::vector<uint8_t>& is_dir = o.is_dir;
  std::vector<double>& uD = o.uD;
  is_dir.assign(N, 0);
  uD.assign(N, 0.0);
  for (int q = 0; q < p->n_dir; ++q) {
    const int i = didx[q];
    if (i < 0 || i >= N) fail(h, AFC_EINVAL, "Dirichlet index out of range");
    if (is_dir[i]) fail(h, AFC_EINVAL, "duplicate Dirichlet index");
    if (!std::isfinite(dval[q])) fail(h, AFC_ENAN, "non-finite Dirichlet value");
    is_dir[i] = 1;
    uD[i] = dval[q];
  }

  // --- AFC operators -----------------------------------------------------------
  // a_ij = -k_ij (eq. (4)); d+_ij = max(a_ij, 0, a_ji) = -d_ij (eq. (5));
  // A_low = A + D (eq. (6)) with Dirichlet rows replaced by identity rows.
  auto build_low = [&](const std::vector<double>& a_src, std::vector<double>& dp, std::vector<double>& AL) {
    dp.assign((size_t)nnz, 0.0);
    AL.assign((size_t)nnz, 0.0);
    for (int i = 0; i < N; ++i) {
      double dsum = 0.0;
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        if (col[k] == i) continue;
        dp[k] = std::max(std::max(a_src[k], 0.0), a_src[tpos[k]]);
        dsum += dp[k];
      }
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const double aik = -K[k];
        AL[k] = col[k] == i ? aik + dsum : aik - dp[k];
        if (is_dir[i]) AL[k] = col[k] == i ? 1.0 : 0.0;
      }
    }
  };
  std::vector<double> a((size_t)nnz);
  for (int64_t k = 0; k < nnz; ++k) a[k] = -K[k];
  build_low(a, o.dp, o.AL);
  // MU (Sec. 3.2): which node of the edge counts it in P_i (a_ji <= a_ij)
  o.mu_own.assign((size_t)nnz, 0);
  for (int64_t k = 0; k < nnz; ++k) {
    const double aij = a[k], aji = a[tpos[k]];
    o.mu_own[k] = aji < aij ? 1 : (aji > aij ? 2 : 0);
  }
  // MCL: c = -K_conv (or a), c^T in CSR order, A_low from the convective D (Remark 1)
  std::vector<double>& c = o.c;
  c = a;
  if (!Kc.empty())
    for (int64_t k = 0; k < nnz; ++k) c[k] = -Kc[k];
  std::vector<double>& cT = o.cT;
  cT.assign((size_t)nnz, 0.0);
  for (int64_t k = 0; k < nnz; ++k) cT[k] = c[tpos[k]];
  std::vector<double> dpc;
  build_low(c, dpc, o.ALc);
  const std::vector<double>& ALc = o.ALc;
  std::vector<double>& dinv = o.dinv;
  dinv.assign(N, 0.0);
  for (int i = 0; i < N; ++i) {
    const double d = ALc[diag[i]];
    if (!(d != 0.0) || !std::isfinite(d)) fail(h, AFC_EINVAL, "zero diagonal in the low-order operator");
    dinv[i] = 1.0 / d;
  }
}

afc_status guard(afc_handle* h, afc_stats* st, afc_status (*body)(afc_handle*, void*), void* ctx) {
  if (!h) return AFC_EINVAL;
  h->last_error.clear();
  if (st) std::memset(st, 0, sizeof(*st));
  afc_status s;
  try {
    HIP_OK(hipSetDevice(h->device));
    ensure_work(h);
    s = body(h, ctx);
  } catch (const Fail& f) {
    s = f.st;
  } catch (...) {
    h->last_error = "unexpected host exception";
    s = AFC_EDEVICE;
  }
  if (st) st->status = s;
  return s;
}

struct SspArgs {
  double* u;
  const double* F;
  double dt;
};

// The stages of one explicit step (Shu-Osher RK3, Heun or one forward-Euler
// stage of eq. (18), Zalesak-limited), with the six per-call work vectors
// given by the caller: s1, s2 (stage states), udot, ut (low-order rate and
// predictor), Rp, Rm (Zalesak's R+-).  Needs the slot-order coefficients.
void ssp_stages(afc_handle* h, const SspArgs& a, double* s1, double* s2, double* udot, double* ut, double* Rp,
                double* Rm) {
  struct Stage {
    const double* in;
    double* out;
    double c0, c1;
  };
  Stage stages[3];
  int ns = 0;
  if (h->opt.ssp_stages == 3) {  // Shu-Osher SSP-RK3
    stages[ns++] = {a.u, s1, 0.0, 1.0};
    stages[ns++] = {s1, s2, 0.75, 0.25};
    stages[ns++] = {s2, a.u, 1.0 / 3.0, 2.0 / 3.0};
  } else if (h->opt.ssp_stages == 2) {  // Heun, u^n = (u^{n,0} + u^{n,2}) / 2
    stages[ns++] = {a.u, s1, 0.0, 1.0};
    stages[ns++] = {s1, a.u, 0.5, 0.5};
  } else {
    stages[ns++] = {a.u, s1, 0.0, 1.0};
  }
  for (int s = 0; s < ns; ++s) {
    afc::ssp_lowrate(h, stages[s].in, a.F, a.dt, udot, ut);
    afc::ssp_limit_R(h, stages[s].in, udot, ut, a.dt, Rp, Rm);
    afc::ssp_apply(h, stages[s].in, udot, ut, Rp, Rm, a.dt, a.u, stages[s].c0, stages[s].c1, stages[s].out);
  }
  if (ns == 1) afc::copy(h, a.u, s1);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(h->stream));
}

// ---------------------------------------------------------------------------
// afc_step_ssprk3_noalloc: the explicit step with its work vectors in a fixed
// per-device array instead of the handle's lazily allocated ones.
// ---------------------------------------------------------------------------

constexpr size_t kNoallocScratchBytes = size_t(AFC_NOALLOC_SCRATCH_BYTES);
constexpr int kNoallocVectors = 6;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// The array of the allocation-free entry point.  In host code this name is
// only a stand-in: its device address comes from hipGetSymbolAddress, once
// per device (noalloc_scratch), and only that address is ever used.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

// Device address of `scratch` on the current device `dev` (looked up on the
// first call per device and kept).
void* noalloc_scratch(afc_handle* h, int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(h, AFC_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(h, AFC_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace



// ---------------------------------------------------------------------------
// Host setup of a request of the served loop (see afc_batch_internal.h)
// ---------------------------------------------------------------------------

namespace afc {

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct BlockLayout {
  int64_t slots = 0, ldw = 0;
  size_t off[15] = {};
  size_t upload = 0, total = 0;
};

// Offsets of the arrays inside a request block, in upload order.
BlockLayout block_layout(int N, int64_t slots, int kind) {
  BlockLayout L;
  L.slots = slots;
  L.ldw = (N + 31) / 32 * 32;
  const int nsl = (N + 63) / 64;
  const bool cn = kind == AFC_REQ_CN;
  size_t at = 0;
  auto put = [&](int idx, size_t bytes) {
    L.off[idx] = at;
    at = align256(at + std::max<size_t>(bytes, 1));
  };
  put(0, sizeof(int) * (size_t)(nsl + 1));         // slp
  put(1, sizeof(int16_t) * (size_t)slots);         // dlt
  if (cn) {
    put(2, 8 * (size_t)slots);                     // mij
    put(3, 8 * (size_t)slots);                     // dp
    put(4, 8 * (size_t)slots);                     // AL
    put(5, 8 * (size_t)N);                         // ml
  } else {
    put(6, 8 * (size_t)slots);                     // cc
    put(7, 8 * (size_t)slots);                     // ccT
    put(8, 8 * (size_t)slots);                     // A (A_low of MCL)
    put(9, 8 * (size_t)N);                         // dinv
  }
  put(10, 8 * (size_t)N);                          // uD
  put(11, (size_t)N);                              // isd
  put(12, 8 * (size_t)N);                          // F
  put(13, 8 * (size_t)N);                          // u
  L.upload = at;
  if (cn) {
    put(8, 8 * (size_t)slots);                     // A: CN matrix, built on the device
    put(9, 8 * (size_t)N);                         // dinv
  }
  put(14, 8 * (size_t)L.ldw * (size_t)serve_work_vectors());  // work vectors
  L.total = at;
  return L;
}

int64_t sell_slots(int N, const int32_t* rp) {
  int64_t slots = 0;
  for (int s0 = 0; s0 < N; s0 += 64) {
    int L = 0;
    for (int i = s0; i < std::min(N, s0 + 64); ++i) L = std::max(L, rp[i + 1] - rp[i]);
    slots += 64 * (int64_t)L;
  }
  return slots;
}

}  // namespace

size_t serve_block_bytes(int N, const int32_t* rp, int kind) {
  return block_layout(N, sell_slots(N, rp), kind).total;
}

afc_status serve_prepare(const afc_problem* p, int kind, const double* u0, const double* F, ServeImage& img,
                         std::string* err) {
  afc_handle* h = nullptr;  // fail() records messages only in the thrown Fail
  try {
    HostOps ops;
    prepare_ops(h, p, ops);
    const int N = ops.N;
    const int nsl = (N + 63) / 64;
    const bool cn = kind == AFC_REQ_CN;
    const BlockLayout L = block_layout(N, sell_slots(N, ops.rp.data()), kind);
    img.N = N;
    img.nsl = nsl;
    img.slots = L.slots;
    img.ldw = L.ldw;
    img.upload_bytes = L.upload;
    img.block_bytes = L.total;
    img.off_slp = L.off[0];
    img.off_dlt = L.off[1];
    img.off_mij = L.off[2];
    img.off_dp = L.off[3];
    img.off_AL = L.off[4];
    img.off_ml = L.off[5];
    img.off_cc = L.off[6];
    img.off_ccT = L.off[7];
    img.off_A = L.off[8];
    img.off_dinv = L.off[9];
    img.off_uD = L.off[10];
    img.off_isd = L.off[11];
    img.off_F = L.off[12];
    img.off_u = L.off[13];
    img.off_work = L.off[14];
    img.bytes.assign(L.upload, 0);
    unsigned char* base = img.bytes.data();
    auto arr = [&](size_t off) { return base + off; };
    int* slp = reinterpret_cast<int*>(arr(L.off[0]));
    int16_t* dlt = reinterpret_cast<int16_t*>(arr(L.off[1]));
    slp[0] = 0;
    for (int sl = 0; sl < nsl; ++sl) {
      int Lr = 0;
      for (int i = sl * 64; i < std::min(N, sl * 64 + 64); ++i) Lr = std::max(Lr, ops.rp[i + 1] - ops.rp[i]);
      slp[sl + 1] = slp[sl] + 64 * Lr;
    }
    double* v0 = reinterpret_cast<double*>(arr(cn ? L.off[2] : L.off[6]));  // mij | cc
    double* v1 = reinterpret_cast<double*>(arr(cn ? L.off[3] : L.off[7]));  // dp  | ccT
    double* v2 = reinterpret_cast<double*>(arr(cn ? L.off[4] : L.off[8]));  // AL  | A_low (MCL)
    for (int i = 0; i < N; ++i) {
      const int sl = i / 64, lane = i % 64;
      int pcount = 1;
      for (int k = ops.rp[i]; k < ops.rp[i + 1]; ++k) {
        const int j = ops.col[k];
        const int pos = (j == i) ? 0 : pcount++;
        const size_t slot = (size_t)slp[sl] + 64 * (size_t)pos + lane;
        if (std::abs(j - i) > 32767) throw Fail{AFC_EINVAL, "request bandwidth exceeds 16-bit column deltas"};
        dlt[slot] = (int16_t)(j - i);
        if (cn) {
          v0[slot] = ops.M[k];
          v1[slot] = ops.dp[k];
          v2[slot] = ops.AL[k];
        } else {
          v0[slot] = ops.c[k];
          v1[slot] = ops.cT[k];
          v2[slot] = ops.ALc[k];
        }
      }
    }
    if (cn)
      std::memcpy(arr(L.off[5]), ops.ml.data(), 8 * (size_t)N);
    else
      std::memcpy(arr(L.off[9]), ops.dinv.data(), 8 * (size_t)N);
    std::memcpy(arr(L.off[10]), ops.uD.data(), 8 * (size_t)N);
    std::memcpy(arr(L.off[11]), ops.is_dir.data(), (size_t)N);
    for (int i = 0; i < N; ++i)
      if (!std::isfinite(F[i]) || (u0 && !std::isfinite(u0[i]))) throw Fail{AFC_ENAN, "non-finite F or u0"};
    std::memcpy(arr(L.off[12]), F, 8 * (size_t)N);
    if (u0) std::memcpy(arr(L.off[13]), u0, 8 * (size_t)N);
  } catch (const Fail& f) {
    if (err) *err = f.msg;
    return f.st;
  } catch (...) {
    if (err) *err = "host allocation failed";
    return AFC_ENOMEM;
  }
  return AFC_OK;
}

}  // namespace afc

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void afc_default_options(afc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->alpha_mode = AFC_ALPHA_LIMITED;
  o->krylov = AFC_KRYLOV_GMRES;
  o->restart = 30;
  o->precision = AFC_PREC_FP64;
  o->lin_atol = 1e-12;
  o->lin_rtol = 0.0;
  o->lin_maxit = 10000;
  o->inner_rtol = 1e-5;
  o->inner_maxit = 300;
  o->refine_maxit = 1000;
  o->fp_tol = 1e-12;
  o->fp_tol_mode = AFC_TOL_ABS_SQRTN;
  o->fp_maxit = 50;
  o->prelimit = 2.0;
  o->omega = 1.0;
  o->dynamic_damping = 0;
  o->ssp_stages = 3;
  o->lanes_per_row = 0;
  o->graphs = 1;
  o->sstep = 0;
  o->sstep_shift = 1.0;
  o->stream = nullptr;
}

const char* afc_status_str(int32_t s) {
  switch (s) {
    case AFC_OK: return "ok";
    case AFC_WMAXIT: return "iteration cap reached";
    case AFC_EINVAL: return "invalid argument";
    case AFC_ENOMEM: return "out of device memory";
    case AFC_ENOCONV: return "linear solver did not converge";
    case AFC_EBREAKDOWN: return "BiCGStab breakdown";
    case AFC_ENAN: return "non-finite value";
    case AFC_EDEVICE: return "HIP runtime error";
    case AFC_ECANCELED: return "request cancelled";
    default: return "unknown status";
  }
}

const char* afc_last_error(const afc_handle* h) { return h ? h->last_error.c_str() : g_create_error.c_str(); }

afc_status afc_set_options(afc_handle* h, const afc_options* opt) {
  if (!h || !opt) return AFC_EINVAL;
  std::string why;
  const afc_status s = check_options(*opt, why);
  if (s != AFC_OK) {
    h->last_error = "invalid options: " + why;
    return s;
  }
  h->opt = *opt;
  h->stream = static_cast<hipStream_t>(opt->stream);
  h->G = pick_lanes(h->nnz, h->N, opt->lanes_per_row);
  h->sstep_cap = afc::kMaxRestart;
  h->gmres_last = 1 << 30;
  return AFC_OK;
}

afc_status afc_create(const afc_problem* p, const afc_options* opt, afc_handle** out) {
  g_create_error.clear();
  if (out) *out = nullptr;
  if (!p || !out) return g_create_error = "null argument", AFC_EINVAL;
  afc_options o;
  afc_default_options(&o);
  if (opt) o = *opt;
  std::string why;
  if (check_options(o, why) != AFC_OK) return g_create_error = "invalid options: " + why, AFC_EINVAL;

  afc_handle* h = new afc_handle();
  try {
    h->opt = o;
    h->stream = static_cast<hipStream_t>(o.stream);
    h->N = p->n;
    h->ldv = (p->n + 63) / 64 * 64;
    h->nnz = p->nnz;
    h->n_dir = p->n_dir;
    h->G = pick_lanes(p->nnz, p->n, o.lanes_per_row);
    HostOps ops;
    prepare_ops(h, p, ops);
    const int N = ops.N;
    const int64_t nnz = ops.nnz;
    const std::vector<int>& rp = ops.rp;
    const std::vector<int>& col = ops.col;
    HIP_OK(hipGetDevice(&h->device));
    h->row_ptr = upload(h, ops.rp, h->stream);
    h->col = upload(h, ops.col, h->stream);
    h->is_dir = upload(h, ops.is_dir, h->stream);
    h->uD = upload(h, ops.uD, h->stream);
    h->ml = upload(h, ops.ml, h->stream);
    h->mij = upload(h, ops.M, h->stream);
    h->dp_fct = upload(h, ops.dp, h->stream);
    h->AL_fct = upload(h, ops.AL, h->stream);
    h->mu_own = upload(h, ops.mu_own, h->stream);
    h->cc = upload(h, ops.c, h->stream);
    h->ccT = upload(h, ops.cT, h->stream);
    h->AL_mcl = upload(h, ops.ALc, h->stream);
    h->dinv_mcl = upload(h, ops.dinv, h->stream);
    // CN system storage (values built per dt on the device)
    h->A_cn = dalloc<double>(h, (size_t)nnz);
    h->dinv_cn = dalloc<double>(h, (size_t)N);
    // SELL-64 layout of the Krylov matrices
    {
      afc::SellLayout L;
      const std::string err = afc::build_sell_layout(N, rp.data(), col.data(), L);
      if (!err.empty()) fail(h, AFC_EINVAL, err.c_str());
      const size_t slots = (size_t)L.slp.back();
      h->nslices = (int)L.dl.size();
      h->sell_slots = (int64_t)slots;
      h->sell_uniform = L.uniform;
      h->sell_lane_deltas = (int64_t)(L.dlt16 ? L.d16.size() : L.d32.size());
      h->sell_pat_ints = (int64_t)L.pat.size();
      h->dlt16 = L.dlt16;
      if (L.pat.empty()) L.pat.push_back(0);
      if (L.d16.empty()) L.d16.push_back(0);
      if (L.d32.empty()) L.d32.push_back(0);
      h->sl_ptr = upload(h, L.slp, h->stream);
      h->sl_dl = upload(h, L.dl, h->stream);
      h->sl_pat = upload(h, L.pat, h->stream);
      h->sell_pos = upload(h, L.pos, h->stream);
      if (h->dlt16)
        h->sl_dlt = upload(h, L.d16, h->stream);
      else
        h->sl_dlt = upload(h, L.d32, h->stream);
      h->S64_mcl = dalloc<double>(h, slots);
      h->S64_cn = dalloc<double>(h, slots);
      // zero the padding slots in stream order before the conversion kernels
      HIP_OK(hipMemsetAsync(h->S64_mcl, 0, slots * sizeof(double), h->stream));
      HIP_OK(hipMemsetAsync(h->S64_cn, 0, slots * sizeof(double), h->stream));
      afc::to_sell64(h, h->AL_mcl, h->S64_mcl);
      // FP32 Krylov layout: the pattern without its diagonal (every row stores
      // one, checked above)
      {
        std::vector<int> rpo(N + 1, 0), colo, kmap(nnz, -1);
        colo.reserve((size_t)(nnz - N));
        for (int i = 0; i < N; ++i) {
          for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] != i) {
              kmap[k] = (int)colo.size();
              colo.push_back(col[k]);
            }
          rpo[i + 1] = (int)colo.size();
        }
        afc::SellLayout Lk;
        const std::string e2 = afc::build_sell_layout(N, rpo.data(), colo.data(), Lk);
        if (!e2.empty()) fail(h, AFC_EINVAL, e2.c_str());
        std::vector<int> kpos(nnz, -1);
        for (int64_t k = 0; k < nnz; ++k)
          if (kmap[k] >= 0) kpos[k] = Lk.pos[kmap[k]];
        const size_t kslots = (size_t)Lk.slp.back();
        h->ks_slots = (int64_t)kslots;
        h->ks_uniform = Lk.uniform;
        h->ks_lane_deltas = (int64_t)(Lk.dlt16 ? Lk.d16.size() : Lk.d32.size());
        h->ks_pat_ints = (int64_t)Lk.pat.size();
        h->ks_dlt16 = Lk.dlt16;
        if (Lk.pat.empty()) Lk.pat.push_back(0);
        if (Lk.d16.empty()) Lk.d16.push_back(0);
        if (Lk.d32.empty()) Lk.d32.push_back(0);
        h->ks_ptr = upload(h, Lk.slp, h->stream);
        h->ks_dl = upload(h, Lk.dl, h->stream);
        h->ks_pat = upload(h, Lk.pat, h->stream);
        h->kpos = upload(h, kpos, h->stream);
        if (h->ks_dlt16)
          h->ks_dlt = upload(h, Lk.d16, h->stream);
        else
          h->ks_dlt = upload(h, Lk.d32, h->stream);
        h->S32_mcl = dalloc<float>(h, std::max<size_t>(kslots, 1));
        h->S32_cn = dalloc<float>(h, std::max<size_t>(kslots, 1));
        HIP_OK(hipMemsetAsync(h->S32_mcl, 0, std::max<size_t>(kslots, 1) * sizeof(float), h->stream));
        HIP_OK(hipMemsetAsync(h->S32_cn, 0, std::max<size_t>(kslots, 1) * sizeof(float), h->stream));
      }
      afc::to_sell32_scaled(h, h->AL_mcl, h->dinv_mcl, h->S32_mcl);
      // MCL bounds and fluxes over the SELL rows: masks of the stored slots and
      // c_ij, c_ji in slot order
      int maxlen = 1;
      for (size_t sl = 0; sl + 1 < L.slp.size(); ++sl) maxlen = std::max(maxlen, (L.slp[sl + 1] - L.slp[sl]) / 64);
      h->mask_words = (maxlen + 31) / 32;
      std::vector<uint32_t> mask((size_t)h->mask_words * N, 0u);
      for (int i = 0; i < N; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
          const int p = (L.pos[k] - L.slp[i / 64]) / 64;
          mask[(size_t)(p / 32) * N + i] |= 1u << (p % 32);
        }
      h->sl_mask = upload(h, mask, h->stream);
      h->Scc = dalloc<double>(h, slots);
      h->SccT = dalloc<double>(h, slots);
      HIP_OK(hipMemsetAsync(h->Scc, 0, slots * sizeof(double), h->stream));
      HIP_OK(hipMemsetAsync(h->SccT, 0, slots * sizeof(double), h->stream));
      afc::to_sell64(h, h->cc, h->Scc);
      afc::to_sell64(h, h->ccT, h->SccT);
    }
    // solver state
    h->partials = dalloc<double>(h, (size_t)kMaxRed * kRedBlocks);
    h->partials_res = dalloc<double>(h, (size_t)std::max(1, afc::sell_grid(h, false)));
    h->ks = dalloc<KState>(h, 1);
    HIP_OK(hipMemsetAsync(h->ks, 0, sizeof(KState), h->stream));
    if (hipHostMalloc((void**)&h->host_status, sizeof(KState), hipHostMallocDefault) != hipSuccess)
      fail(h, AFC_ENOMEM, "hipHostMalloc failed");
    std::memset(h->host_status, 0, sizeof(KState));
    HIP_OK(hipStreamSynchronize(h->stream));
  } catch (const Fail& f) {
    g_create_error = f.msg;
    free_all(h);
    delete h;
    return f.st;
  } catch (...) {
    g_create_error = "host allocation failed";
    free_all(h);
    delete h;
    return AFC_ENOMEM;
  }
  *out = h;
  return AFC_OK;
}

afc_status afc_kernel_time(afc_handle* h, int32_t kernel, double* total_ms, int64_t* launches, int32_t reset) {
  if (!h || kernel < 0 || kernel >= AFC_KERNEL_COUNT) return AFC_EINVAL;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  afc::prof_collect(h);
  if (total_ms) *total_ms = h->prof_ms[kernel];
  if (launches) *launches = h->prof_n[kernel];
  if (reset) {
    h->prof_ms[kernel] = 0.0;
    h->prof_n[kernel] = 0;
    h->prof_bytes[kernel] = 0.0;
    h->prof_work[kernel] = 0;
  }
  return AFC_OK;
}

afc_status afc_kernel_work(afc_handle* h, int32_t kernel, double* bytes, int64_t* launches_with_work) {
  if (!h || kernel < 0 || kernel >= AFC_KERNEL_COUNT) return AFC_EINVAL;
  if (bytes) *bytes = h->prof_bytes[kernel];
  if (launches_with_work) *launches_with_work = h->prof_work[kernel];
  return AFC_OK;
}

afc_status afc_apply_operator(afc_handle* h, int32_t op, const double* x, double* y) {
  if (!h || !x || !y || x == y || op < 0 || op > 3) return AFC_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    if (!h->apply_tmp) h->apply_tmp = dalloc<double>(h, (size_t)h->ldv);
    if (op == 0)
      HIP_OK(hipMemcpyAsync(h->apply_tmp, y, sizeof(double) * h->N, hipMemcpyDeviceToDevice, h->stream));
    afc::apply_operator(h, op, x, y, h->apply_tmp);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(h->stream));
  } catch (const Fail& f) {
    return f.st;
  } catch (...) {
    h->last_error = "unexpected host exception";
    return AFC_EDEVICE;
  }
  return AFC_OK;
}

afc_status afc_get_krylov_sell_info(const afc_handle* h, afc_sell_info* out) {
  if (!h || !out) return AFC_EINVAL;
  out->slices = h->nslices;
  out->slots = h->ks_slots;
  out->uniform_slices = h->ks_uniform;
  out->lane_delta_slots = h->ks_lane_deltas;
  out->pattern_ints = h->ks_pat_ints;
  out->delta_bytes = h->ks_dlt16 ? 2 : 4;
  out->reserved = 0;
  return AFC_OK;
}

afc_status afc_get_sell_info(const afc_handle* h, afc_sell_info* out) {
  if (!h || !out) return AFC_EINVAL;
  out->slices = h->nslices;
  out->slots = h->sell_slots;
  out->uniform_slices = h->sell_uniform;
  out->lane_delta_slots = h->sell_lane_deltas;
  out->pattern_ints = h->sell_pat_ints;
  out->delta_bytes = h->dlt16 ? 2 : 4;
  out->reserved = 0;
  return AFC_OK;
}

afc_status afc_residual_history(const afc_handle* h, double* out, int32_t cap, int32_t* count) {
  if (!h || !count || cap < 0 || (cap > 0 && !out)) return AFC_EINVAL;
  const size_t n = h->res_hist.size();
  *count = (int32_t)std::min<size_t>(n, (size_t)std::numeric_limits<int32_t>::max());
  const size_t m = std::min<size_t>(n, (size_t)cap);
  if (m) std::memcpy(out, h->res_hist.data(), m * sizeof(double));
  return AFC_OK;
}

void afc_destroy(afc_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
}

afc_status afc_step_ssprk3(afc_handle* h, double* u, const double* F, double dt, afc_stats* st) {
  if (!h) return AFC_EINVAL;
  if (!u || !F || !(dt > 0) || !std::isfinite(dt)) {
    h->last_error = "afc_step_ssprk3: need device u, F and dt > 0";
    return AFC_EINVAL;
  }
  SspArgs a{u, F, dt};
  return guard(
      h, st,
      [](afc_handle* h, void* ctx) -> afc_status {
        const SspArgs& a = *static_cast<SspArgs*>(ctx);
        ensure_fct_sell(h);
        ssp_stages(h, a, h->w[W_S1], h->w[W_S2], h->w[W_G], h->w[W_UT], h->w[W_RP], h->w[W_RM]);
        afc::prof_collect(h);
        return AFC_OK;
      },
      &a);
}

afc_status afc_step_ssprk3_noalloc(afc_handle* h, double* u, const double* F, double dt, afc_stats* st) {
  if (!h) return AFC_EINVAL;
  h->last_error.clear();
  if (st) std::memset(st, 0, sizeof(*st));
  afc_status s = AFC_OK;
  if (!u || !F || !(dt > 0) || !std::isfinite(dt)) {
    h->last_error = "afc_step_ssprk3_noalloc: need device u, F and dt > 0";
    s = AFC_EINVAL;
  } else if ((size_t)kNoallocVectors * (size_t)h->ldv * sizeof(double) > kNoallocScratchBytes) {
    h->last_error = "afc_step_ssprk3_noalloc: N = " + std::to_string(h->N) + " needs " +
                    std::to_string((size_t)kNoallocVectors * (size_t)h->ldv * sizeof(double)) +
                    " bytes of work space, above the fixed " + std::to_string(kNoallocScratchBytes);
    s = AFC_EINVAL;
  } else if (!h->S_mij) {
    h->last_error = "afc_step_ssprk3_noalloc: the handle's explicit-stage coefficients are not built yet "
                    "(one afc_step_ssprk3, afc_step_mc_ssprk3 or CN call on the handle builds them)";
    s = AFC_EINVAL;
  } else if (h->opt.profile) {
    h->last_error = "afc_step_ssprk3_noalloc: profiling (options.profile) is not available here";
    s = AFC_EINVAL;
  }
  if (s == AFC_OK) {
    try {
      HIP_OK(hipSetDevice(h->device));
      double* base = static_cast<double*>(noalloc_scratch(h, h->device));
      const size_t ld = (size_t)h->ldv;
      SspArgs a{u, F, dt};
      ssp_stages(h, a, base, base + ld, base + 2 * ld, base + 3 * ld, base + 4 * ld, base + 5 * ld);
    } catch (const Fail& f) {
      s = f.st;
    } catch (...) {
      h->last_error = "unexpected host exception";
      s = AFC_EDEVICE;
    }
  }
  if (st) st->status = s;
  return s;
}

// System matrix kept in the handle's CN storage: M_L/dt + AL/2 for a CN step
// (dt > 0), or AL itself for a stationary solve (dt = 0); rebuilt when dt or
// the low-order operator changes
void ensure_cn_matrix(afc_handle* h, const double* AL, double dt) {
  if (h->cn_dt == dt && h->cn_src == AL) return;
  afc::build_cn_matrix(h, AL, dt);
  h->cn_dt = dt;
  h->cn_src = AL;
}

struct CnArgs {
  double* u;
  const double* Fo;
  const double* Fn;
  double dt;
  afc_stats* st;
};

afc_status afc_step_cn(afc_handle* h, double* u, const double* F_old, const double* F_new, double dt,
                       afc_stats* st) {
  if (!h) return AFC_EINVAL;
  if (!u || !F_old || !F_new || !(dt > 0) || !std::isfinite(dt)) {
    h->last_error = "afc_step_cn: need device u, F_old, F_new and dt > 0";
    return AFC_EINVAL;
  }
  CnArgs a{u, F_old, F_new, dt, st};
  return guard(
      h, st,
      [](afc_handle* h, void* ctx) -> afc_status {
        const CnArgs& a = *static_cast<CnArgs*>(ctx);
        ensure_cn_matrix(h, h->AL_fct, a.dt);
        ensure_fct_sell(h);
        double* uo = h->w[W_UOLD];
        double* ut = h->w[W_UT];
        double* g = h->w[W_G];
        double* Qp = h->w[W_A];
        double* Qm = h->w[W_B2];
        double* Rp = h->w[W_RP];
        double* Rm = h->w[W_RM];
        afc::copy(h, uo, a.u);
        afc::cn_predict(h, uo, a.Fo, a.Fn, a.dt, ut, g);  // eq. (14) and the right-hand side of eq. (11)
        afc::zalesak_Q(h, ut, Qp, Qm);
        afc::set_dirichlet(h, a.u);
        const SysMat S{h->A_cn, h->dinv_cn, h->S64_cn, h->S32_cn};
        const double dt = a.dt;
        auto eval = [&](double* u, double* b, double* r) {
          afc::cn_limit_R(h, u, uo, Qp, Qm, dt, Rp, Rm);
          afc::cn_apply(h, u, uo, Rp, Rm, g, dt, b, r);
        };
        return fixed_point(h, a.u, S, eval, a.st);
      },
      &a);
}

afc_status afc_step_cn_linear(afc_handle* h, double* u, const double* F_old, const double* F_new, double dt,
                              afc_stats* st) {
  if (!h) return AFC_EINVAL;
  if (!u || !F_old || !F_new || !(dt > 0) || !std::isfinite(dt)) {
    h->last_error = "afc_step_cn_linear: need device u, F_old, F_new and dt > 0";
    return AFC_EINVAL;
  }
  CnArgs a{u, F_old, F_new, dt, st};
  return guard(
      h, st,
      [](afc_handle* h, void* ctx) -> afc_status {
        const CnArgs& a = *static_cast<CnArgs*>(ctx);
        ensure_cn_matrix(h, h->AL_fct, a.dt);
        ensure_fct_sell(h);
        double* uo = h->w[W_UOLD];
        double* ut = h->w[W_UT];
        double* g = h->w[W_G];
        double* Qp = h->w[W_A];
        double* Qm = h->w[W_B2];
        double* Rp = h->w[W_RP];
        double* Rm = h->w[W_RM];
        double* b = h->w[W_B];
        double* r = h->w[W_R];
        afc::copy(h, uo, a.u);
        afc::cn_predict(h, uo, a.Fo, a.Fn, a.dt, ut, g);  // eq. (14) and the right-hand side of eq. (11)
        afc::zalesak_Q(h, ut, Qp, Qm);
        afc::cn_extrapolate(h, ut, uo, a.u);  // u <- u* = 2 u~ - u^{n-1}
        afc::cn_limit_R(h, a.u, uo, Qp, Qm, a.dt, Rp, Rm);
        afc::cn_apply(h, a.u, uo, Rp, Rm, g, a.dt, b, r);  // b = g + F*(u*), r = b - A_cn u*
        sync_status(h);
        const double R = std::sqrt(h->host_status->red[0]);
        const double bn = std::sqrt(h->host_status->red[1]);
        if (a.st) {
          a.st->res0 = R;
          a.st->res = R;
          a.st->fp_iters = 1;
        }
        if (!std::isfinite(R) || !std::isfinite(bn)) {
          h->last_error = "non-finite residual";
          return AFC_ENAN;
        }
        const SysMat S{h->A_cn, h->dinv_cn, h->S64_cn, h->S32_cn};
        const double tol = std::max(h->opt.lin_atol, h->opt.lin_rtol * bn);
        const SolveOut o = linear_solve(h, S, b, a.u, r, 2, tol);
        add_solve(a.st, o);
        if (o.st == AFC_ENAN) h->last_error = "non-finite linear residual";
        if (o.st == AFC_EBREAKDOWN) h->last_error = "BiCGStab breakdown";
        return o.st;
      },
      &a);
}

afc_status afc_step_mc_ssprk3(afc_handle* h, double* u, const double* F, double dt, afc_stats* st) {
  if (!h) return AFC_EINVAL;
  if (!u || !F || !(dt > 0) || !std::isfinite(dt)) {
    h->last_error = "afc_step_mc_ssprk3: need device u, F and dt > 0";
    return AFC_EINVAL;
  }
  SspArgs a{u, F, dt};
  return guard(
      h, st,
      [](afc_handle* h, void* ctx) -> afc_status {
        const SspArgs& a = *static_cast<SspArgs*>(ctx);
        double* s1 = h->w[W_S1];
        double* s2 = h->w[W_S2];
        double* udot = h->w[W_G];
        double* scratch = h->w[W_UT];
        double* umax = h->w[W_A];
        double* umin = h->w[W_B2];
        struct Stage {
          const double* in;
          double* out;
          double c0, c1;
        };
        Stage stages[3];
        int ns = 0;
        if (h->opt.ssp_stages == 3) {  // Shu-Osher SSP-RK3
          stages[ns++] = {a.u, s1, 0.0, 1.0};
          stages[ns++] = {s1, s2, 0.75, 0.25};
          stages[ns++] = {s2, a.u, 1.0 / 3.0, 2.0 / 3.0};
        } else if (h->opt.ssp_stages == 2) {  // Heun
          stages[ns++] = {a.u, s1, 0.0, 1.0};
          stages[ns++] = {s1, a.u, 0.5, 0.5};
        } else {
          stages[ns++] = {a.u, s1, 0.0, 1.0};
        }
        ensure_fct_sell(h);
        for (int s = 0; s < ns; ++s) {
          afc::mc_lowrate(h, stages[s].in, a.F, udot, scratch);
          afc::mcl_bounds(h, stages[s].in, umax, umin);
          afc::mc_stage(h, stages[s].in, udot, umax, umin, a.dt, a.u, stages[s].c0, stages[s].c1, stages[s].out);
        }
        if (ns == 1) afc::copy(h, a.u, s1);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(h->stream));
        afc::prof_collect(h);
        return AFC_OK;
      },
      &a);
}

afc_status afc_step_mc_cn(afc_handle* h, double* u, const double* F_old, const double* F_new, double dt,
                          afc_stats* st) {
  if (!h) return AFC_EINVAL;
  if (!u || !F_old || !F_new || !(dt > 0) || !std::isfinite(dt)) {
    h->last_error = "afc_step_mc_cn: need device u, F_old, F_new and dt > 0";
    return AFC_EINVAL;
  }
  CnArgs a{u, F_old, F_new, dt, st};
  return guard(
      h, st,
      [](afc_handle* h, void* ctx) -> afc_status {
        const CnArgs& a = *static_cast<CnArgs*>(ctx);
        ensure_cn_matrix(h, h->AL_mcl, a.dt);
        ensure_fct_sell(h);
        double* uo = h->w[W_UOLD];
        double* g = h->w[W_G];
        double* udot = h->w[W_S1];
        double* scratch = h->w[W_UT];
        double* umax = h->w[W_A];
        double* umin = h->w[W_B2];
        afc::copy(h, uo, a.u);
        afc::mc_lowrate(h, uo, a.Fo, udot, scratch);
        afc::mcl_bounds(h, uo, umax, umin);
        afc::mc_cn_g(h, uo, udot, umax, umin, a.Fn, a.dt, g);
        afc::set_dirichlet(h, a.u);
        const SysMat S{h->A_cn, h->dinv_cn, h->S64_cn, h->S32_cn};
        auto eval = [&](double* u, double* b, double* r) {
          afc::mc_lowrate(h, u, a.Fn, udot, scratch);
          afc::mcl_bounds(h, u, umax, umin);
          afc::mc_cn_apply(h, u, udot, umax, umin, g, b, r);
        };
        return fixed_point(h, a.u, S, eval, a.st);
      },
      &a);
}

struct StatArgs {
  double* u;
  const double* F;
  int init_low;
  afc_stats* st;
};

afc_status afc_solve_stationary(afc_handle* h, double* u, const double* F, int32_t init_low_order,
                                afc_stats* st) {
  if (!h) return AFC_EINVAL;
  if (!u || !F) {
    h->last_error = "afc_solve_stationary: need device u and F";
    return AFC_EINVAL;
  }
  StatArgs a{u, F, init_low_order, st};
  return guard(
      h, st,
      [](afc_handle* h, void* ctx) -> afc_status {
        const StatArgs& a = *static_cast<StatArgs*>(ctx);
        const bool mu = h->opt.limiter == AFC_LIMITER_MU;
        // MCL: A_low from the convective D (Remark 1); MU: A_low = A + D from A,
        // assembled into the handle's CN storage
        if (mu) {
          ensure_cn_matrix(h, h->AL_fct, 0.0);
          ensure_fct_sell(h);
        }
        const SysMat S = mu ? SysMat{h->A_cn, h->dinv_cn, h->S64_cn, h->S32_cn}
                            : SysMat{h->AL_mcl, h->dinv_mcl, h->S64_mcl, h->S32_mcl};
        double* b = h->w[W_B];
        double* r = h->w[W_R];
        if (a.init_low) {  // low-order solution A_low u = F (alpha = 0), from zero
          afc::rhs_dirichlet(h, b, a.F);
          afc::fill(h, a.u, 0.0);
          afc::set_dirichlet(h, a.u);
          afc::norm2(h, b, 1);
          afc::residual(h, S.S64, b, a.u, r, 0);
          sync_status(h);
          const double tol = std::max(h->opt.lin_atol, h->opt.lin_rtol * std::sqrt(h->host_status->red[1]));
          const SolveOut o = linear_solve(h, S, b, a.u, r, 0, tol);
          add_solve(a.st, o);
          if (o.st == AFC_ENAN) {
            h->last_error = "non-finite residual in the low-order solve";
            return AFC_ENAN;
          }
        }
        afc::set_dirichlet(h, a.u);
        double* umax = h->w[W_A];
        double* umin = h->w[W_B2];
        auto eval = [&](double* u, double* bb, double* rr) {
          if (mu) {
            afc::mu_R(h, u, umax, umin);  // R+ and R- of Sec. 3.2 in the same two vectors
            afc::mu_apply(h, u, umax, umin, a.F, bb, rr);
          } else {
            afc::mcl_bounds(h, u, umax, umin);
            afc::mcl_apply(h, u, umax, umin, a.F, bb, rr);
          }
        };
        return fixed_point(h, a.u, S, eval, a.st);
      },
      &a);
}


// ---------------------------------------------------------------------------
// batched CN-FCT
// ---------------------------------------------------------------------------

static thread_local std::string g_batch_error;

afc_status afc_batch_create(int32_t count, const afc_problem* probs, const afc_options* opt, afc_batch** out) {
  g_batch_error.clear();
  if (out) *out = nullptr;
  if (count <= 0 || !probs || !out) return g_batch_error = "need count > 0, probs and out", AFC_EINVAL;
  afc_options o;
  afc_default_options(&o);
  if (opt) o = *opt;
  std::string why;
  if (check_options(o, why) != AFC_OK) return g_batch_error = "invalid options: " + why, AFC_EINVAL;
  if (o.krylov != AFC_KRYLOV_BICGSTAB || o.precision != AFC_PREC_FP64)
    return g_batch_error = "the batched launch runs BiCGStab in FP64", AFC_EINVAL;
  if (o.lin_eta != 0.0) return g_batch_error = "the batched launch has no inexact solves (lin_eta = 0)", AFC_EINVAL;
  afc_batch* b = new afc_batch();
  afc_handle* h = nullptr;  // HIP_OK / fail record messages only in the thrown Fail
  try {
    b->count = count;
    b->opt = o;
    b->stream = static_cast<hipStream_t>(o.stream);
    b->bopt = afc::BatchOpts{o.alpha_mode, o.fp_tol_mode, o.fp_maxit, o.lin_maxit, o.dynamic_damping,
                             o.fp_tol, o.lin_atol, o.lin_rtol, o.prelimit, o.omega, o.lin_eta};
    std::vector<int> slp;
    std::vector<int16_t> dlt;
    std::vector<double> mij, dp, AL, ml, uD;
    std::vector<uint8_t> is_dir;
    b->host_insts.resize(count);
    int64_t node_off = 0, slot_off = 0, sl_off = 0, nnz_tot = 0;
    for (int q = 0; q < count; ++q) {
      HostOps ops;
      try {
        prepare_ops(h, &probs[q], ops);
      } catch (const Fail& f) {
        throw Fail{f.st, "instance " + std::to_string(q) + ": " + f.msg};
      }
      const int N = ops.N;
      const int nsl = (N + 63) / 64;
      afc::BInst& in = b->host_insts[q];
      in.N = N;
      in.nnz = (int)ops.nnz;
      in.nsl = nsl;
      in.node_off = node_off;
      in.slot_off = slot_off;
      in.sl_off = sl_off;
      in.dt = 0.0;
      // SELL-64 with the diagonal in slot 0 of every row
      std::vector<int> lp(nsl + 1, 0);
      for (int sl = 0; sl < nsl; ++sl) {
        int L = 0;
        for (int i = sl * 64; i < std::min(N, sl * 64 + 64); ++i) L = std::max(L, ops.rp[i + 1] - ops.rp[i]);
        lp[sl + 1] = lp[sl] + 64 * L;
      }
      const size_t slots = (size_t)lp[nsl];
      const size_t s0 = dlt.size();
      dlt.resize(s0 + slots, 0);
      mij.resize(s0 + slots, 0.0);
      dp.resize(s0 + slots, 0.0);
      AL.resize(s0 + slots, 0.0);
      for (int i = 0; i < N; ++i) {
        const int sl = i / 64, lane = i % 64;
        int p = 1;
        for (int k = ops.rp[i]; k < ops.rp[i + 1]; ++k) {
          const int j = ops.col[k];
          const int pos = (j == i) ? 0 : p++;
          const size_t slot = s0 + (size_t)lp[sl] + 64 * (size_t)pos + lane;
          if (std::abs(j - i) > 32767) throw Fail{AFC_EINVAL, "batched instance bandwidth exceeds 16-bit deltas"};
          dlt[slot] = (int16_t)(j - i);
          mij[slot] = ops.M[k];
          dp[slot] = ops.dp[k];
          AL[slot] = ops.AL[k];
        }
      }
      slp.insert(slp.end(), lp.begin(), lp.end());
      ml.insert(ml.end(), ops.ml.begin(), ops.ml.end());
      uD.insert(uD.end(), ops.uD.begin(), ops.uD.end());
      is_dir.insert(is_dir.end(), ops.is_dir.begin(), ops.is_dir.end());
      node_off += N;
      slot_off += (int64_t)slots;
      sl_off += nsl + 1;
      nnz_tot += ops.nnz;
      if (slot_off >= (int64_t)std::numeric_limits<int>::max()) throw Fail{AFC_EINVAL, "batch too large"};
    }
    b->total_slots = slot_off;
    b->total_nodes = node_off;
    b->total_nnz = nnz_tot;
    // workgroups take the largest instances first
    b->host_order.resize(count);
    std::iota(b->host_order.begin(), b->host_order.end(), 0);
    std::stable_sort(b->host_order.begin(), b->host_order.end(),
                     [&](int a, int c) { return b->host_insts[a].nnz > b->host_insts[c].nnz; });
    HIP_OK(hipGetDevice(&b->device));
    b->slp = upload(h, slp, b->stream);
    b->dlt = upload(h, dlt, b->stream);
    b->mij = upload(h, mij, b->stream);
    b->dp = upload(h, dp, b->stream);
    b->AL = upload(h, AL, b->stream);
    b->ml = upload(h, ml, b->stream);
    b->uD = upload(h, uD, b->stream);
    b->is_dir = upload(h, is_dir, b->stream);
    b->Acn = dalloc<double>(h, (size_t)slot_off);
    b->dinv = dalloc<double>(h, (size_t)node_off);
    b->work = dalloc<double>(h, (size_t)afc::batch_work_vectors() * (size_t)node_off);
    b->insts = upload(h, b->host_insts, b->stream);
    b->order = upload(h, b->host_order, b->stream);
    b->queue = dalloc<int>(h, 1);
    b->stats_d = dalloc<afc::BStat>(h, (size_t)count);
    b->dev = afc::BatchDev{b->slp, b->dlt, b->mij, b->dp, b->AL, b->ml, b->uD, b->is_dir, b->Acn, b->dinv, b->work,
                           node_off};
    HIP_OK(hipStreamSynchronize(b->stream));
  } catch (const Fail& f) {
    g_batch_error = f.msg;
    afc_batch_destroy(b);
    return f.st;
  } catch (...) {
    g_batch_error = "host allocation failed";
    afc_batch_destroy(b);
    return AFC_ENOMEM;
  }
  *out = b;
  return AFC_OK;
}

afc_status afc_batch_offsets(const afc_batch* b, int64_t* offsets) {
  if (!b || !offsets) return AFC_EINVAL;
  for (int q = 0; q < b->count; ++q) offsets[q] = b->host_insts[q].node_off;
  offsets[b->count] = b->total_nodes;
  return AFC_OK;
}

static int severity(int s) { return s < 0 ? 100 - s : s; }

// per-call instance data (dt) and the work queue, in stream order
void batch_prepare(afc_handle* h, afc_batch* b, const double* dt) {
  for (int q = 0; q < b->count; ++q) b->host_insts[q].dt = dt[q];
  HIP_OK(hipMemcpyAsync(b->insts, b->host_insts.data(), sizeof(afc::BInst) * b->count, hipMemcpyHostToDevice,
                        b->stream));
  HIP_OK(hipMemsetAsync(b->queue, 0, sizeof(int), b->stream));
}

// workgroups of the persistent launch: `want`, or twice the compute units;
// never more than the instances
int batch_grid(afc_handle* h, const afc_batch* b, int want) {
  int cus = 0;
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
  return std::max(1, std::min(b->count, want > 0 ? want : 2 * cus));
}

afc_status afc_batch_step_cn(afc_batch* b, double* u, const double* F, const double* dt, int32_t steps,
                             afc_stats* stats) {
  if (!b) return AFC_EINVAL;
  b->last_error.clear();
  if (!u || !F || !dt || steps < 0) {
    b->last_error = "afc_batch_step_cn: need device u, F, host dt and steps >= 0";
    return AFC_EINVAL;
  }
  for (int q = 0; q < b->count; ++q)
    if (!(dt[q] > 0) || !std::isfinite(dt[q])) {
      b->last_error = "dt must be positive for every instance";
      return AFC_EINVAL;
    }
  afc_handle* h = nullptr;
  try {
    HIP_OK(hipSetDevice(b->device));
    batch_prepare(h, b, dt);
    afc::batch_launch(b, u, F, steps, b->threads, batch_grid(h, b, b->workgroups));
    HIP_OK(hipGetLastError());
    std::vector<afc::BStat> hs(b->count);
    HIP_OK(hipMemcpyAsync(hs.data(), b->stats_d, sizeof(afc::BStat) * b->count, hipMemcpyDeviceToHost, b->stream));
    HIP_OK(hipStreamSynchronize(b->stream));
    int worst = AFC_OK;
    for (int q = 0; q < b->count; ++q) {
      if (severity(hs[q].status) > severity(worst)) worst = hs[q].status;
      if (stats) {
        std::memset(&stats[q], 0, sizeof(afc_stats));
        stats[q].status = hs[q].status;
        stats[q].fp_iters = hs[q].fp_iters;
        stats[q].krylov_iters = hs[q].krylov_iters;
        stats[q].res0 = hs[q].res0;
        stats[q].res = hs[q].res;
        stats[q].lin_res = hs[q].lin_res;
      }
    }
    if (worst < 0) b->last_error = std::string("an instance failed: ") + afc_status_str(worst);
    return (afc_status)worst;
  } catch (const Fail& f) {
    b->last_error = f.msg;
    return f.st;
  }
}

afc_status afc_batch_set_schedule(afc_batch* b, const afc_batch_schedule* sch) {
  if (!b || !sch) return AFC_EINVAL;
  if ((sch->threads != 256 && sch->threads != 512 && sch->threads != 1024) || sch->workgroups < 0) {
    b->last_error = "schedule: threads must be 256, 512 or 1024 and workgroups >= 0";
    return AFC_EINVAL;
  }
  b->threads = sch->threads;
  b->workgroups = sch->workgroups;
  return AFC_OK;
}

afc_status afc_batch_get_schedule(const afc_batch* b, afc_batch_schedule* sch) {
  if (!b || !sch) return AFC_EINVAL;
  sch->threads = b->threads;
  sch->workgroups = b->workgroups;
  return AFC_OK;
}

afc_status afc_batch_autotune(afc_batch* b, const double* u, const double* F, const double* dt, int32_t trial_steps,
                              afc_batch_schedule* chosen, double* trial_ms, int32_t max_trials,
                              int32_t* n_trials) {
  if (!b) return AFC_EINVAL;
  b->last_error.clear();
  if (!u || !F || !dt || trial_steps < 1 || (trial_ms && max_trials < 0)) {
    b->last_error = "afc_batch_autotune: need device u, F, host dt and trial_steps >= 1";
    return AFC_EINVAL;
  }
  for (int q = 0; q < b->count; ++q)
    if (!(dt[q] > 0) || !std::isfinite(dt[q])) {
      b->last_error = "dt must be positive for every instance";
      return AFC_EINVAL;
    }
  afc_handle* h = nullptr;
  double* scratch = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    HIP_OK(hipSetDevice(b->device));
    int cus = 0;
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    HIP_OK(hipMalloc(&scratch, sizeof(double) * std::max<int64_t>(1, b->total_nodes)));
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    std::vector<afc_batch_schedule> cand;
    for (int t : {256, 512, 1024})
      for (int mult : {1, 2, 4}) {
        const int g = batch_grid(h, b, mult * cus);
        bool dup = false;
        for (auto& c : cand) dup = dup || (c.threads == t && c.workgroups == g);
        if (!dup) cand.push_back({t, g});
      }
    double best = 0.0;
    afc_batch_schedule pick = {b->threads, b->workgroups};
    int nt = 0;
    for (const auto& c : cand) {
      HIP_OK(hipMemcpyAsync(scratch, u, sizeof(double) * b->total_nodes, hipMemcpyDeviceToDevice, b->stream));
      batch_prepare(h, b, dt);
      HIP_OK(hipEventRecord(e0, b->stream));
      afc::batch_launch(b, scratch, F, trial_steps, c.threads, c.workgroups);
      HIP_OK(hipGetLastError());
      HIP_OK(hipEventRecord(e1, b->stream));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      if (trial_ms && nt < max_trials) trial_ms[nt] = ms;
      ++nt;
      if (nt == 1 || ms < best) {
        best = ms;
        pick = c;
      }
    }
    b->threads = pick.threads;
    b->workgroups = pick.workgroups;
    if (chosen) *chosen = pick;
    if (n_trials) *n_trials = nt;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    return AFC_OK;
  } catch (const Fail& f) {
    b->last_error = f.msg;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (scratch) {
      (void)hipStreamSynchronize(b->stream);
      (void)hipFree(scratch);
    }
    return f.st;
  }
}

const char* afc_batch_last_error(const afc_batch* b) { return b ? b->last_error.c_str() : g_batch_error.c_str(); }

void afc_batch_destroy(afc_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  auto f = [](auto*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
  };
  f(b->slp); f(b->dlt); f(b->mij); f(b->dp); f(b->AL); f(b->ml); f(b->uD); f(b->is_dir);
  f(b->Acn); f(b->dinv); f(b->work); f(b->insts); f(b->order); f(b->queue); f(b->stats_d);
  delete b;
}

}  // extern "C"
