// Continuous-batching request server over the AFC entry points.
//
// Requests (a CDR instance + what to compute) are copied at submission and
// queued.  A scheduler thread admits them in arrival order whenever a slot is
// free and the modelled device footprint of the admitted set stays within the
// HBM budget.  Every slot owns one HIP stream and one worker thread that runs
// its request end to end (afc_create, the CN steps or the stationary solve,
// copy-back, afc_destroy); requests in different slots overlap on the device,
// and a finished request frees its slot and memory for the next arrival.  A
// request's result does not depend on what else runs: each one has its own
// handle, and every kernel of the library is deterministic.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/afc.h"
#include "afc_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

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
  int64_t footprint = 0;
  Clock::time_point t_submit, t_start, t_done;
  afc_status status = AFC_OK;
  afc_stats stats{};
  std::string error;
  bool done = false;
};

}  // namespace

struct afc_server_s {
  int slots = 0;
  int64_t budget = 0;
  int64_t in_use = 0;
  int device = 0;
  int64_t next_id = 1;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_slot;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<int64_t, std::shared_ptr<Request>> all;
  std::vector<std::shared_ptr<Request>> slot_req;  // request assigned to each slot (null = free)
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::thread scheduler;
  std::string last_error;
};

namespace {

double seconds(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

void run_request(afc_server_s* s, int slot, Request& r) {
  (void)hipSetDevice(s->device);
  hipStream_t st = s->streams[slot];
  afc_options o = r.opt;
  o.stream = st;
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

void worker_loop(afc_server_s* s, int slot) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_slot.wait(lk, [&] { return s->stop || s->slot_req[slot] != nullptr; });
    if (s->slot_req[slot] == nullptr && s->stop) return;
    std::shared_ptr<Request> r = s->slot_req[slot];
    lk.unlock();
    r->t_start = Clock::now();
    run_request(s, slot, *r);
    r->t_done = Clock::now();
    lk.lock();
    r->done = true;
    s->in_use -= r->footprint;
    s->slot_req[slot] = nullptr;
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
  }
}

void scheduler_loop(afc_server_s* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_sched.wait(lk, [&] {
      if (s->stop) return true;
      if (s->queue.empty()) return false;
      const auto& head = s->queue.front();
      const bool slot_free = std::any_of(s->slot_req.begin(), s->slot_req.end(), [](auto& p) { return !p; });
      const bool fits = s->in_use == 0 || s->in_use + head->footprint <= s->budget;
      return slot_free && fits;
    });
    if (s->stop) return;
    auto r = s->queue.front();
    s->queue.pop_front();
    for (int k = 0; k < s->slots; ++k) {
      if (!s->slot_req[k]) {
        s->slot_req[k] = r;
        s->in_use += r->footprint;
        break;
      }
    }
    s->cv_slot.notify_all();
  }
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

afc_status afc_server_create(int32_t slots, int64_t hbm_budget_bytes, afc_server** out) {
  if (!out || slots < 1 || slots > 64 || hbm_budget_bytes <= 0) return AFC_EINVAL;
  *out = nullptr;
  auto* s = new afc_server_s();
  s->slots = slots;
  s->budget = hbm_budget_bytes;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return AFC_EDEVICE;
  }
  s->slot_req.assign(slots, nullptr);
  s->streams.assign(slots, nullptr);
  for (int k = 0; k < slots; ++k) {
    if (hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking) != hipSuccess) {
      for (int q = 0; q < k; ++q) (void)hipStreamDestroy(s->streams[q]);
      delete s;
      return AFC_EDEVICE;
    }
  }
  for (int k = 0; k < slots; ++k) s->workers.emplace_back(worker_loop, s, k);
  s->scheduler = std::thread(scheduler_loop, s);
  *out = s;
  return AFC_OK;
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
  r->footprint = afc_footprint_bytes(p.n, p.nnz, q->kind, &q->opt);
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  s->all[r->id] = r;
  s->queue.push_back(r);
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
    if (it == s->all.end()) return AFC_EINVAL;
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->all.erase(it);
  }
  if (u_out && !r->result.empty()) std::memcpy(u_out, r->result.data(), r->result.size() * sizeof(double));
  if (stats) *stats = r->stats;
  if (times) {
    times[0] = seconds(r->t_submit, r->t_start);  // queueing
    times[1] = seconds(r->t_start, r->t_done);    // service
    times[2] = seconds(r->t_submit, r->t_done);   // latency
  }
  if (r->status < 0) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->last_error = r->error;
  }
  return r->status;
}

afc_status afc_server_poll(afc_server* s, int64_t id, int32_t* done) {
  if (!s || !done) return AFC_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return AFC_EINVAL;
  *done = it->second->done ? 1 : 0;
  return AFC_OK;
}

const char* afc_server_last_error(const afc_server* s) { return s ? s->last_error.c_str() : ""; }

void afc_server_destroy(afc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv_sched.notify_all();
  s->cv_slot.notify_all();
  if (s->scheduler.joinable()) s->scheduler.join();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  delete s;
}

}  // extern "C"
