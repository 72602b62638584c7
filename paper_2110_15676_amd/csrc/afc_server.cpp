// Request server: continuous batching of CDR requests (CN-FCT steps or a
// stationary MCL solve) on one GPU, over two lanes.
//
// Fused lane (N <= fuse_max_nodes): host setup threads build a request's
// operators and SELL layout (afc::serve_prepare) and upload them into one
// device block of its own.  The round thread keeps the set of active
// requests; each round is ONE launch (k_serve_round) in which every active
// request advances by one wall-clock quantum in a workgroup of its own, from
// the resumable state it left in device memory.  Requests that become ready
// while a round runs join the next round, finished ones leave it (result
// copied back, block returned to the pool), so the launches always carry the
// requests that are in flight at that moment.  Every reduction of a request
// runs in a fixed order inside its workgroup, so its result does not depend
// on the other requests, the quantum or the workgroup that ran it.
//
// Dedicated lane (larger requests, and the MU limiter): each slot owns a
// non-blocking stream and a worker thread that runs its request end to end on
// a handle of its own (afc_create, the CN steps or the stationary solve; the
// Krylov cycles replay captured HIP graphs), concurrently with the rounds.
//
// Admission: per lane in arrival order, while the device footprint of the
// admitted requests fits the HBM budget (fused: the exact block size;
// dedicated: afc_footprint_bytes) and, for the dedicated lane, a slot is free.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/afc.h"
#include "afc_batch_internal.h"
#include "afc_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

enum Lane { LANE_FUSED = 0, LANE_DEDICATED = 1 };

struct Request {
  int64_t id = 0;
  int32_t kind = AFC_REQ_CN;
  int32_t n = 0;
  int64_t nnz = 0;
  std::vector<int32_t> rp, col, dir_idx;
  std::vector<double> M, K, Kc, dir_val, u0, F, result;
  bool has_kc = false, has_u0 = false;
  double dt = 0.0;
  int32_t steps = 0;
  afc_options opt{};
  int lane = LANE_DEDICATED;
  int64_t footprint = 0;
  // fused lane
  afc::ServeImage img;
  void* block = nullptr;
  size_t block_cap = 0;
  int table = -1;
  Clock::time_point t_submit, t_start, t_done;
  afc_status status = AFC_OK;
  afc_stats stats{};
  std::string error;
  bool done = false;
  bool waited = false;
};

afc_problem problem_of(const Request& r) {
  afc_problem p{};
  p.n = r.n;
  p.nnz = r.nnz;
  p.mem_space = AFC_MEM_HOST;
  p.row_ptr = r.rp.data();
  p.col_idx = r.col.data();
  p.M = r.M.data();
  p.K = r.K.data();
  p.K_conv = r.has_kc ? r.Kc.data() : nullptr;
  p.ML = nullptr;
  p.n_dir = (int32_t)r.dir_idx.size();
  p.dir_idx = r.dir_idx.data();
  p.dir_val = r.dir_val.data();
  return p;
}

}  // namespace

struct afc_server_s {
  afc_server_config cfg{};
  int device = 0;
  int64_t in_use = 0;
  int64_t next_id = 1;
  bool stop = false;
  int waiters = 0;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_slot, cv_setup, cv_round, cv_quiet;
  std::deque<std::shared_ptr<Request>> fused_q, dedicated_q;  // submitted, not admitted
  std::deque<std::shared_ptr<Request>> setup_q;                // admitted to the fused lane, to prepare
  std::deque<std::shared_ptr<Request>> ready_q;                // prepared, to join the next round
  std::map<int64_t, std::shared_ptr<Request>> all;
  std::vector<std::shared_ptr<Request>> slot_req;  // dedicated lane: request of each slot (null = free)
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers, setup_threads;
  std::thread scheduler, rounds;
  std::string last_error;
  // fused lane, used by the round thread only (and create / destroy)
  hipStream_t loop_stream = nullptr;
  afc::SReq* reqs_d = nullptr;
  afc::SState* states_d = nullptr;
  afc::SState* states_h = nullptr;  // pinned
  int* list_d = nullptr;
  int* queue_d = nullptr;
  int64_t quantum_ticks = 0;
  int loop_grid = 0;
  std::vector<int> free_tables;
  std::vector<std::shared_ptr<Request>> active;
  // device block pool of the fused lane (guarded by mu)
  std::multimap<size_t, void*> pool;
  size_t pool_bytes = 0;
  std::vector<void*> all_blocks;
  int64_t rounds_run = 0;
  int64_t slices_run = 0;  // request-rounds: the requests carried by each round, summed
};

namespace {

double seconds(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

// ---------------------------------------------------------------------------
// dedicated lane
// ---------------------------------------------------------------------------

void run_dedicated(afc_server_s* s, int slot, Request& r) {
  (void)hipSetDevice(s->device);
  hipStream_t st = s->streams[slot];
  afc_options o = r.opt;
  o.stream = st;
  const afc_problem p = problem_of(r);
  afc_handle* h = nullptr;
  afc_status rc = afc_create(&p, &o, &h);
  if (rc != AFC_OK) {
    r.status = rc;
    r.error = afc_last_error(nullptr);
    return;
  }
  double *u = nullptr, *F = nullptr;
  const size_t bytes = (size_t)r.n * sizeof(double);
  if (hipMalloc(&u, bytes) != hipSuccess || hipMalloc(&F, bytes) != hipSuccess) {
    r.status = AFC_ENOMEM;
    r.error = "hipMalloc of request vectors failed";
  } else {
    (void)hipMemcpyAsync(F, r.F.data(), bytes, hipMemcpyHostToDevice, st);
    if (r.has_u0)
      (void)hipMemcpyAsync(u, r.u0.data(), bytes, hipMemcpyHostToDevice, st);
    else
      (void)hipMemsetAsync(u, 0, bytes, st);
    if (r.kind == AFC_REQ_CN) {
      afc_stats one{};
      for (int k = 0; k < r.steps; ++k) {
        rc = afc_step_cn(h, u, F, F, r.dt, &one);
        r.stats.fp_iters += one.fp_iters;
        r.stats.krylov_iters += one.krylov_iters;
        r.stats.inner_iters += one.inner_iters;
        r.stats.refine_sweeps += one.refine_sweeps;
        r.stats.res = one.res;
        if (k == 0) r.stats.res0 = one.res0;
        if (rc < 0) break;
        if (rc > 0) r.status = rc;
      }
      if (rc < 0) r.status = rc;
      r.stats.status = r.status;
    } else {
      rc = afc_solve_stationary(h, u, F, r.has_u0 ? 0 : 1, &r.stats);
      r.status = rc;
    }
    if (r.status < 0) r.error = afc_last_error(h);
    r.result.resize(r.n);
    (void)hipMemcpyAsync(r.result.data(), u, bytes, hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
  }
  if (u) (void)hipFree(u);
  if (F) (void)hipFree(F);
  afc_destroy(h);
}

void finish_locked(afc_server_s* s, Request& r) {
  r.t_done = Clock::now();
  r.done = true;
  s->in_use -= r.footprint;
  s->cv_done.notify_all();
  s->cv_sched.notify_all();
}

void worker_loop(afc_server_s* s, int slot) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_slot.wait(lk, [&] { return s->stop || s->slot_req[slot] != nullptr; });
    if (s->slot_req[slot] == nullptr && s->stop) return;
    std::shared_ptr<Request> r = s->slot_req[slot];
    lk.unlock();
    r->t_start = Clock::now();
    run_dedicated(s, slot, *r);
    lk.lock();
    s->slot_req[slot] = nullptr;
    finish_locked(s, *r);
  }
}

// ---------------------------------------------------------------------------
// fused lane: setup threads, block pool, rounds
// ---------------------------------------------------------------------------

// A device block of at least `bytes` from the pool (the smallest cached one
// of at most twice the size) or a new allocation.  Called with mu held.
void* pool_get(afc_server_s* s, size_t bytes, size_t* cap) {
  auto it = s->pool.lower_bound(bytes);
  if (it != s->pool.end() && it->first <= 2 * bytes) {
    void* p = it->second;
    *cap = it->first;
    s->pool_bytes -= it->first;
    s->pool.erase(it);
    return p;
  }
  return nullptr;
}

void setup_loop(afc_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_setup.wait(lk, [&] { return s->stop || !s->setup_q.empty(); });
    if (s->setup_q.empty()) return;  // stop
    std::shared_ptr<Request> r = s->setup_q.front();
    s->setup_q.pop_front();
    lk.unlock();
    r->t_start = Clock::now();
    const afc_problem p = problem_of(*r);
    std::string err;
    afc_status st = afc::serve_prepare(&p, r->kind, r->has_u0 ? r->u0.data() : nullptr, r->F.data(), r->img, &err);
    void* block = nullptr;
    size_t cap = 0;
    if (st == AFC_OK) {
      {
        std::lock_guard<std::mutex> g(s->mu);
        block = pool_get(s, r->img.block_bytes, &cap);
      }
      if (!block) {
        // keep the cached blocks and the admitted requests within the budget
        std::vector<void*> evict;
        {
          std::lock_guard<std::mutex> g(s->mu);
          while (!s->pool.empty() && s->in_use + (int64_t)s->pool_bytes > s->cfg.hbm_budget_bytes) {
            auto big = std::prev(s->pool.end());
            evict.push_back(big->second);
            s->pool_bytes -= big->first;
            s->pool.erase(big);
            s->all_blocks.erase(std::find(s->all_blocks.begin(), s->all_blocks.end(), evict.back()));
          }
        }
        for (void* e : evict) (void)hipFree(e);
        if (hipMalloc(&block, r->img.block_bytes) != hipSuccess) {
          block = nullptr;
          st = AFC_ENOMEM;
          err = "hipMalloc of a request block failed";
        } else {
          cap = r->img.block_bytes;
          std::lock_guard<std::mutex> g(s->mu);
          s->all_blocks.push_back(block);
        }
      }
    }
    if (st == AFC_OK && hipMemcpy(block, r->img.bytes.data(), r->img.upload_bytes, hipMemcpyHostToDevice) !=
                            hipSuccess) {
      st = AFC_EDEVICE;
      err = "upload of a request block failed";
    }
    r->img.bytes.clear();
    r->img.bytes.shrink_to_fit();
    lk.lock();
    if (st != AFC_OK) {
      if (block) {
        s->pool.emplace(cap, block);
        s->pool_bytes += cap;
      }
      r->status = st;
      r->stats.status = st;
      r->error = err;
      finish_locked(s, *r);
      continue;
    }
    r->block = block;
    r->block_cap = cap;
    s->ready_q.push_back(r);
    s->cv_round.notify_all();
  }
}

afc::SReq descriptor(const Request& r) {
  const afc::ServeImage& m = r.img;
  unsigned char* b = static_cast<unsigned char*>(r.block);
  const afc_options& o = r.opt;
  afc::SReq d{};
  d.kind = r.kind;
  d.N = m.N;
  d.nsl = m.nsl;
  d.steps = r.steps;
  d.init_low = (r.kind == AFC_REQ_STATIONARY && !r.has_u0) ? 1 : 0;
  d.dt = r.dt;
  d.o = afc::BatchOpts{o.alpha_mode, o.fp_tol_mode, o.fp_maxit, o.lin_maxit, o.dynamic_damping, o.fp_tol,
                       o.lin_atol, o.lin_rtol, o.prelimit, o.omega, o.lin_eta};
  d.slp = reinterpret_cast<const int*>(b + m.off_slp);
  d.dlt = reinterpret_cast<const int16_t*>(b + m.off_dlt);
  const bool cn = r.kind == AFC_REQ_CN;
  d.mij = cn ? reinterpret_cast<const double*>(b + m.off_mij) : nullptr;
  d.dp = cn ? reinterpret_cast<const double*>(b + m.off_dp) : nullptr;
  d.AL = cn ? reinterpret_cast<const double*>(b + m.off_AL) : nullptr;
  d.ml = cn ? reinterpret_cast<const double*>(b + m.off_ml) : nullptr;
  d.cc = cn ? nullptr : reinterpret_cast<const double*>(b + m.off_cc);
  d.ccT = cn ? nullptr : reinterpret_cast<const double*>(b + m.off_ccT);
  d.uD = reinterpret_cast<const double*>(b + m.off_uD);
  d.isd = reinterpret_cast<const uint8_t*>(b + m.off_isd);
  d.A = reinterpret_cast<double*>(b + m.off_A);
  d.dinv = reinterpret_cast<double*>(b + m.off_dinv);
  d.work = reinterpret_cast<double*>(b + m.off_work);
  d.u = reinterpret_cast<double*>(b + m.off_u);
  d.F = reinterpret_cast<const double*>(b + m.off_F);
  d.ldw = m.ldw;
  return d;
}

afc::SState fresh_state(const afc_options& o) {
  afc::SState st{};
  st.phase = -1;
  st.omega = o.omega;
  return st;
}

// One round at a time: admit the ready requests, launch one k_serve_round
// over the active set, read back the states, retire the finished requests.
void round_loop(afc_server_s* s) {
  (void)hipSetDevice(s->device);
  std::vector<int> list;
  std::vector<std::shared_ptr<Request>> retired;
  while (true) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_round.wait(lk, [&] { return s->stop || !s->ready_q.empty() || !s->active.empty(); });
      if (s->stop && s->ready_q.empty() && s->active.empty()) return;
      while (!s->ready_q.empty() && !s->free_tables.empty()) {
        std::shared_ptr<Request> r = s->ready_q.front();
        s->ready_q.pop_front();
        r->table = s->free_tables.back();
        s->free_tables.pop_back();
        s->active.push_back(r);
        const afc::SReq d = descriptor(*r);
        const afc::SState st0 = fresh_state(r->opt);
        (void)hipMemcpyAsync(s->reqs_d + r->table, &d, sizeof(d), hipMemcpyHostToDevice, s->loop_stream);
        (void)hipMemcpyAsync(s->states_d + r->table, &st0, sizeof(st0), hipMemcpyHostToDevice, s->loop_stream);
        // the host copies above are pageable: wait before d and st0 go out of scope
        (void)hipStreamSynchronize(s->loop_stream);
      }
    }
    list.clear();
    for (auto& r : s->active) list.push_back(r->table);
    const int count = (int)list.size();
    (void)hipMemcpyAsync(s->list_d, list.data(), sizeof(int) * count, hipMemcpyHostToDevice, s->loop_stream);
    (void)hipMemsetAsync(s->queue_d, 0, sizeof(int), s->loop_stream);
    afc::serve_round_launch(s->reqs_d, s->states_d, s->list_d, count, s->queue_d, s->quantum_ticks,
                            s->cfg.loop_threads, std::min(count, s->loop_grid), s->loop_stream);
    hipError_t e = hipGetLastError();
    (void)hipMemcpyAsync(s->states_h, s->states_d, sizeof(afc::SState) * s->cfg.max_active, hipMemcpyDeviceToHost,
                         s->loop_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->loop_stream);
    {
      std::lock_guard<std::mutex> g(s->mu);
      ++s->rounds_run;
      s->slices_run += count;
    }
    retired.clear();
    for (size_t k = 0; k < s->active.size();) {
      auto& r = s->active[k];
      const afc::SState& st = s->states_h[r->table];
      if (e != hipSuccess || st.done) {
        if (e == hipSuccess) {
          r->result.resize(r->n);
          (void)hipMemcpy(r->result.data(), static_cast<unsigned char*>(r->block) + r->img.off_u,
                          sizeof(double) * (size_t)r->n, hipMemcpyDeviceToHost);
          r->status = (afc_status)st.status;
          r->stats.status = st.status;
          r->stats.fp_iters = st.fp_total;
          r->stats.krylov_iters = st.kry;
          r->stats.res0 = st.res0;
          r->stats.res = st.res;
          r->stats.lin_res = st.lin_res;
          if (st.status < 0) r->error = std::string("served request: ") + afc_status_str(st.status);
        } else {
          r->status = AFC_EDEVICE;
          r->stats.status = AFC_EDEVICE;
          r->error = std::string("round launch failed: ") + hipGetErrorString(e);
        }
        retired.push_back(r);
        s->active.erase(s->active.begin() + (std::ptrdiff_t)k);
      } else {
        ++k;
      }
    }
    if (!retired.empty()) {
      std::lock_guard<std::mutex> g(s->mu);
      for (auto& r : retired) {
        s->free_tables.push_back(r->table);
        s->pool.emplace(r->block_cap, r->block);
        s->pool_bytes += r->block_cap;
        r->block = nullptr;
        finish_locked(s, *r);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// admission
// ---------------------------------------------------------------------------

void scheduler_loop(afc_server_s* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    bool moved = false;
    const auto fits = [&](const Request& r) { return s->in_use == 0 || s->in_use + r.footprint <= s->cfg.hbm_budget_bytes; };
    if (!s->fused_q.empty() && fits(*s->fused_q.front())) {
      auto r = s->fused_q.front();
      s->fused_q.pop_front();
      s->in_use += r->footprint;
      s->setup_q.push_back(r);
      s->cv_setup.notify_one();
      moved = true;
    }
    if (!s->dedicated_q.empty() && fits(*s->dedicated_q.front())) {
      for (int k = 0; k < s->cfg.slots; ++k) {
        if (!s->slot_req[k]) {
          auto r = s->dedicated_q.front();
          s->dedicated_q.pop_front();
          s->slot_req[k] = r;
          s->in_use += r->footprint;
          s->cv_slot.notify_all();
          moved = true;
          break;
        }
      }
    }
    if (moved) continue;
    if (s->stop) return;
    s->cv_sched.wait(lk);
  }
}

void cancel_locked(afc_server_s* s, std::deque<std::shared_ptr<Request>>& q) {
  for (auto& r : q) {
    r->status = AFC_ECANCELED;
    r->stats.status = AFC_ECANCELED;
    r->error = "dropped by afc_server_destroy";
    r->t_start = r->t_done = Clock::now();
    r->done = true;
  }
  q.clear();
}

}  // namespace

extern "C" {

int64_t afc_footprint_bytes(int32_t n, int64_t nnz, int32_t kind, const afc_options* opt) {
  afc_options o;
  afc_default_options(&o);
  if (opt) o = *opt;
  const int64_t N = n, Z = nnz;
  const int64_t ldv = (N + 63) / 64 * 64;
  // resident operators: col, 6 FP64 CSR value arrays and the CN values
  int64_t b = Z * 4 + Z * 8 * 6 + Z * 8;
  // SELL-64 system layout (slot map, offsets, A_low and CN values, c_ij and
  // c_ji in slot order, slot masks) and the FP32 Krylov layout without the
  // diagonal (slot map, offsets, two FP32 matrices); padding ~1 %
  b += (Z * (4 + 4 + 8 + 8 + 8 + 8) + N * 8) * 101 / 100;
  b += (Z * (4 + 4 + 4 + 4)) * 101 / 100;
  b += N * (4 + 8 * 4 + 1) + ldv * 8 * 18;  // row pointers, node vectors, work vectors
  const int64_t m = o.restart + 1;
  b += (o.precision == AFC_PREC_MIXED ? 4 : 8) * m * ldv;  // Krylov basis
  b += 8 * (int64_t)(afc::kMaxRed + afc::kBlkRows) * afc::kRedBlocks + 8 * (N / 256 + 1);  // reduction partials
  b += N * 8 * 2;                                          // request u and F
  b += 32 << 20;  // allocation granularity of ~60 device buffers, graphs and small state
  if (kind == AFC_REQ_CN) b += Z * 24 * 101 / 100;  // m_ij, d+_ij and A_low in slot order (CN passes)
  return b;
}

void afc_server_default_config(afc_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->slots = 4;
  c->hbm_budget_bytes = int64_t(64) << 30;
  c->fuse_max_nodes = 20000;
  c->loop_threads = 1024;
  c->loop_workgroups = 0;
  c->setup_threads = 4;
  c->max_active = 512;
  c->quantum_ms = 2.0;
}

afc_status afc_server_create_cfg(const afc_server_config* cfg, afc_server** out) {
  if (!out || !cfg) return AFC_EINVAL;
  *out = nullptr;
  const afc_server_config& c = *cfg;
  if (c.slots < 1 || c.slots > 64 || c.hbm_budget_bytes <= 0 || c.fuse_max_nodes < 0 ||
      (c.loop_threads != 256 && c.loop_threads != 512 && c.loop_threads != 1024) || c.loop_workgroups < 0 ||
      c.setup_threads < 1 || c.setup_threads > 32 || c.max_active < 1 || c.max_active > 65536 ||
      !(c.quantum_ms >= 0.0) || c.quantum_ms > 60000.0)
    return AFC_EINVAL;
  auto* s = new afc_server_s();
  s->cfg = c;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return AFC_EDEVICE;
  }
  int cus = 0, khz = 0;
  bool ok = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) == hipSuccess && khz > 0;
  s->loop_grid = c.loop_workgroups > 0 ? c.loop_workgroups : std::max(1, cus);
  s->quantum_ticks = (int64_t)(c.quantum_ms * (double)khz);
  s->slot_req.assign(c.slots, nullptr);
  s->streams.assign(c.slots, nullptr);
  for (int k = 0; ok && k < c.slots; ++k) ok = hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&s->loop_stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipMalloc(&s->reqs_d, sizeof(afc::SReq) * c.max_active) == hipSuccess;
  ok = ok && hipMalloc(&s->states_d, sizeof(afc::SState) * c.max_active) == hipSuccess;
  ok = ok && hipMalloc(&s->list_d, sizeof(int) * c.max_active) == hipSuccess;
  ok = ok && hipMalloc(&s->queue_d, sizeof(int)) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->states_h, sizeof(afc::SState) * c.max_active, hipHostMallocDefault) ==
                 hipSuccess;
  if (!ok) {
    for (auto st : s->streams)
      if (st) (void)hipStreamDestroy(st);
    if (s->loop_stream) (void)hipStreamDestroy(s->loop_stream);
    (void)hipFree(s->reqs_d);
    (void)hipFree(s->states_d);
    (void)hipFree(s->list_d);
    (void)hipFree(s->queue_d);
    if (s->states_h) (void)hipHostFree(s->states_h);
    delete s;
    return AFC_EDEVICE;
  }
  std::memset(s->states_h, 0, sizeof(afc::SState) * c.max_active);
  for (int k = c.max_active - 1; k >= 0; --k) s->free_tables.push_back(k);
  for (int k = 0; k < c.slots; ++k) s->workers.emplace_back(worker_loop, s, k);
  for (int k = 0; k < c.setup_threads; ++k) s->setup_threads.emplace_back(setup_loop, s);
  s->rounds = std::thread(round_loop, s);
  s->scheduler = std::thread(scheduler_loop, s);
  *out = s;
  return AFC_OK;
}

afc_status afc_server_create(int32_t slots, int64_t hbm_budget_bytes, afc_server** out) {
  afc_server_config c;
  afc_server_default_config(&c);
  c.slots = slots;
  c.hbm_budget_bytes = hbm_budget_bytes;
  return afc_server_create_cfg(&c, out);
}

afc_status afc_server_submit(afc_server* s, const afc_request* q, int64_t* id) {
  if (!s || !q || !id) return AFC_EINVAL;
  const afc_problem& p = q->problem;
  if (p.mem_space != AFC_MEM_HOST || p.n <= 0 || p.nnz <= 0 || !p.row_ptr || !p.col_idx || !p.M || !p.K || !q->F ||
      (p.n_dir > 0 && (!p.dir_idx || !p.dir_val)) || (q->kind != AFC_REQ_CN && q->kind != AFC_REQ_STATIONARY) ||
      (q->kind == AFC_REQ_CN && (!(q->dt > 0) || q->steps < 1 || !q->u0))) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->last_error = "invalid request";
    return AFC_EINVAL;
  }
  auto r = std::make_shared<Request>();
  r->kind = q->kind;
  r->n = p.n;
  r->nnz = p.nnz;
  r->rp.assign(p.row_ptr, p.row_ptr + p.n + 1);
  r->col.assign(p.col_idx, p.col_idx + p.nnz);
  r->M.assign(p.M, p.M + p.nnz);
  r->K.assign(p.K, p.K + p.nnz);
  if (p.K_conv) {
    r->Kc.assign(p.K_conv, p.K_conv + p.nnz);
    r->has_kc = true;
  }
  r->dir_idx.assign(p.dir_idx, p.dir_idx + p.n_dir);
  r->dir_val.assign(p.dir_val, p.dir_val + p.n_dir);
  r->F.assign(q->F, q->F + p.n);
  if (q->u0) {
    r->u0.assign(q->u0, q->u0 + p.n);
    r->has_u0 = true;
  }
  r->dt = q->dt;
  r->steps = q->steps;
  r->opt = q->opt;
  // the fused lane: small requests whose options it honours (MU stays dedicated)
  const bool fusable = p.n <= s->cfg.fuse_max_nodes &&
                       !(q->kind == AFC_REQ_STATIONARY && q->opt.limiter != AFC_LIMITER_MCL) &&
                       r->rp.front() == 0 && r->rp.back() == p.nnz;
  if (fusable) {
    // the fused layout stores column offsets j - i in 16 bits
    bool ok = true;
    for (int i = 0; i < p.n && ok; ++i) {
      ok = r->rp[i] <= r->rp[i + 1];
      for (int32_t k = r->rp[i]; ok && k < r->rp[i + 1]; ++k) ok = std::abs(r->col[k] - i) <= 32767;
    }
    r->lane = ok ? LANE_FUSED : LANE_DEDICATED;
  } else {
    r->lane = LANE_DEDICATED;
  }
  r->footprint = r->lane == LANE_FUSED ? (int64_t)afc::serve_block_bytes(p.n, r->rp.data(), q->kind)
                                        : afc_footprint_bytes(p.n, p.nnz, q->kind, &q->opt);
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    s->last_error = "server is stopping";
    return AFC_EINVAL;
  }
  r->id = s->next_id++;
  s->all[r->id] = r;
  (r->lane == LANE_FUSED ? s->fused_q : s->dedicated_q).push_back(r);
  *id = r->id;
  s->cv_sched.notify_all();
  return AFC_OK;
}

afc_status afc_server_wait(afc_server* s, int64_t id, double* u_out, afc_stats* stats, double* times) {
  if (!s) return AFC_EINVAL;
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end() || it->second->waited) return AFC_EINVAL;
    r = it->second;
    r->waited = true;
    ++s->waiters;
    s->cv_done.wait(lk, [&] { return r->done; });
    --s->waiters;
    auto again = s->all.find(id);
    if (again != s->all.end()) s->all.erase(again);
    if (r->status < 0) s->last_error = r->error;
    s->cv_quiet.notify_all();
  }
  if (u_out && !r->result.empty()) std::memcpy(u_out, r->result.data(), r->result.size() * sizeof(double));
  if (stats) *stats = r->stats;
  if (times) {
    times[0] = seconds(r->t_submit, r->t_start);  // queueing
    times[1] = seconds(r->t_start, r->t_done);    // setup and service
    times[2] = seconds(r->t_submit, r->t_done);   // latency
  }
  return r->status;
}

afc_status afc_server_poll(afc_server* s, int64_t id, int32_t* done) {
  if (!s || !done) return AFC_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end() || it->second->waited) return AFC_EINVAL;
  *done = it->second->done ? 1 : 0;
  return AFC_OK;
}

afc_status afc_server_info(const afc_server* s, int64_t* rounds, int64_t* request_rounds, int64_t* in_use_bytes) {
  if (!s) return AFC_EINVAL;
  auto* m = const_cast<afc_server*>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  if (rounds) *rounds = m->rounds_run;
  if (request_rounds) *request_rounds = m->slices_run;
  if (in_use_bytes) *in_use_bytes = m->in_use;
  return AFC_OK;
}

const char* afc_server_last_error(const afc_server* s) { return s ? s->last_error.c_str() : ""; }

void afc_server_destroy(afc_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->stop = true;
    cancel_locked(s, s->fused_q);
    cancel_locked(s, s->dedicated_q);
    s->cv_done.notify_all();
  }
  s->cv_sched.notify_all();
  s->cv_slot.notify_all();
  s->cv_setup.notify_all();
  s->cv_round.notify_all();
  // admitted requests finish; then the threads end
  if (s->scheduler.joinable()) s->scheduler.join();
  for (auto& t : s->setup_threads)
    if (t.joinable()) t.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_round.notify_all();
  }
  if (s->rounds.joinable()) s->rounds.join();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  {
    // every request is done now: let the threads blocked in afc_server_wait
    // return before the server's memory goes away
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.notify_all();
    s->cv_quiet.wait(lk, [&] { return s->waiters == 0; });
  }
  (void)hipSetDevice(s->device);
  for (void* b : s->all_blocks) (void)hipFree(b);
  (void)hipFree(s->reqs_d);
  (void)hipFree(s->states_d);
  (void)hipFree(s->list_d);
  (void)hipFree(s->queue_d);
  (void)hipHostFree(s->states_h);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  (void)hipStreamDestroy(s->loop_stream);
  delete s;
}

}  // extern "C"
