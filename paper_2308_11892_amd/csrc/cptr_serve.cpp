// cptr_serve.cpp -- the solve server of cptr_serve.h: host-setup workers feed
// an admission queue; slot threads admit requests in arrival order when their
// exact device footprint fits the HBM arena and run them on their own streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cptr.h"
#include "cptr_serve.h"
#include "dev_arena.hpp"
#include "solver_internal.hpp"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  enum State { kQueued, kSetup, kReady, kRunning, kDone };
  int64_t id = 0;
  // inputs (copied at submission; A is dropped after the host setup)
  int32_t nb = 0;
  int64_t nnzb = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v, b;
  int32_t eidx[3] = {0, 1, 2};
  int32_t ne = 2;
  cptr_solve_opts so{};
  // progress
  State state = kQueued;
  cptr_solver h = nullptr;
  int64_t bytes = 0;  // device footprint: the handle plus b and x
  int placements = 0; // admissions that found no contiguous room in the arena
  int status = CPTR_OK;
  std::string err;
  std::vector<double> x;
  cptr_solve_info sinfo{};
  double t_submit = 0, t_setup0 = 0, t_setup1 = 0, t_admit = 0, t_dev = 0, t_done = 0;
};

}  // namespace

struct cptr_server_s {
  cptr_server_opts o{};
  void* arena_mem = nullptr;
  cptr::DevArena arena;
  std::mutex mu;
  std::condition_variable cv_setup;  // setup workers: queued requests or stop
  std::condition_variable cv_admit;  // slots: ready requests, freed memory or stop
  std::condition_variable cv_done;   // waiters: a request finished
  std::deque<Request*> setup_q, ready_q;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_id = 1;
  int64_t reserved = 0;     // footprints of admitted requests
  int inflight = 0;
  int64_t releases = 0;     // admitted requests that gave their memory back (done, failed or requeued)
  double t_created = 0;     // clock origin of cptr_serve_info's *_at_s times
  bool stop = false;        // no more submissions; setup workers drain and exit
  bool setups_done = false; // every setup worker has exited
  cptr_server_stats stats{};
  std::string last_err;
  std::vector<std::thread> setup_threads, slot_threads;
};

namespace {

// called with the lock held
void finish(cptr_server sv, Request* r, int status) {
  r->status = status;
  r->state = Request::kDone;
  r->t_done = now_s();
  if (status < 0) ++sv->stats.failed;
  else ++sv->stats.completed;
  sv->cv_done.notify_all();
}

void setup_worker(cptr_server sv) {
  (void)hipSetDevice(sv->o.device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_setup.wait(lk, [&] { return sv->stop || !sv->setup_q.empty(); });
      if (sv->setup_q.empty()) return;
      r = sv->setup_q.front();
      sv->setup_q.pop_front();
      r->state = Request::kSetup;
      r->t_setup0 = now_s();
    }
    const cptr_bsr A{r->nb, r->nnzb, r->rp.data(), r->ci.data(), r->v.data(), 0};
    cptr_setup_opts so = sv->o.setup;
    // automatic: most of a host setup is sequential, so small requests get one
    // thread and large ones up to four (one per 400k block rows)
    if (so.setup_threads <= 0) so.setup_threads = std::min(4, 1 + r->nb / 400000);
    cptr_solver h = nullptr;
    int rc = cptr::setup_host(&A, 3, r->eidx, r->ne, &so, &h);
    std::string err = rc ? cptr::last_error(nullptr) : "";
    int64_t bytes = 0;
    const int m = r->so.restart;
    if (!rc) {
      rc = cptr::measure_device(h, m, r->so.flexible != 0, &bytes);
      if (rc) err = cptr::last_error(h);
    }
    const int64_t vec = (int64_t)cptr::DevArena::round(sizeof(double) * 3 * (size_t)r->nb);
    bytes += 2 * vec;
    if (!rc && bytes > (int64_t)sv->arena.size()) {
      rc = CPTR_E_NOMEM;
      err = "request needs " + std::to_string(bytes) + " bytes of HBM; the budget is " +
            std::to_string(sv->arena.size());
    }
    // A's pattern is copied into the handle; its values are read in place
    // until the device half is built
    std::vector<int32_t>().swap(r->rp);
    std::vector<int32_t>().swap(r->ci);
    if (rc) std::vector<double>().swap(r->v);
    if (rc && h) {
      cptr_destroy(h);
      h = nullptr;
    }
    std::lock_guard<std::mutex> g(sv->mu);
    r->t_setup1 = now_s();
    if (rc) {
      r->err = err;
      finish(sv, r, rc);
    } else {
      r->h = h;
      r->bytes = bytes;
      r->state = Request::kReady;
      sv->ready_q.push_back(r);
      sv->cv_admit.notify_all();
    }
  }
}

// Runs an admitted request on `st`.  Returns false when the arena had no
// contiguous room (fragmentation) before any work was done: the request goes
// back to the head of the queue.
bool run_request(cptr_server sv, Request* r, hipStream_t st, int& rc) {
  const size_t n = 3 * (size_t)r->nb;
  rc = cptr::setup_device(r->h, &sv->arena, r->so.restart, r->so.flexible != 0, st);
  if (rc == CPTR_E_NOMEM) return false;  // retried later: A's values stay
  double* bd = nullptr;
  double* xd = nullptr;
  const int64_t vec = (int64_t)cptr::DevArena::round(sizeof(double) * n);
  if (!rc && cptr::device_bytes(r->h) + 2 * vec != r->bytes) {
    // the admitted footprint must be what the request holds
    rc = CPTR_E_STATE;
    r->err = "device footprint " + std::to_string(cptr::device_bytes(r->h) + 2 * vec) +
             " bytes differs from the measured " + std::to_string(r->bytes);
  }
  if (!rc) {
    bd = static_cast<double*>(sv->arena.alloc(sizeof(double) * n));
    xd = static_cast<double*>(sv->arena.alloc(sizeof(double) * n));
    if (!bd || !xd) {
      if (bd) sv->arena.release(bd);
      if (xd) sv->arena.release(xd);
      cptr::release_device(r->h);
      return false;
    }
  }
  // the device half stays: the handle no longer reads A's values
  cptr::drop_input(r->h);
  std::vector<double>().swap(r->v);
  r->t_dev = now_s();
  if (!rc) {
    hipError_t e = hipMemcpyAsync(bd, r->b.data(), sizeof(double) * n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
      rc = CPTR_E_HIP;
      r->err = std::string("uploading b: ") + hipGetErrorString(e);
    }
  }
  if (!rc) {
    cptr_solve_opts so = r->so;
    so.x0_is_zero = 1;
    rc = cptr_gmres_solve(r->h, bd, xd, &so, &r->sinfo, st);
    if (rc < 0) r->err = cptr::last_error(r->h);
  } else if (r->err.empty()) {
    r->err = cptr::last_error(r->h);
  }
  if (rc >= 0) {
    r->x.resize(n);
    hipError_t e = hipMemcpyAsync(r->x.data(), xd, sizeof(double) * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      rc = CPTR_E_HIP;
      r->err = std::string("downloading x: ") + hipGetErrorString(e);
    }
  }
  (void)hipStreamSynchronize(st);
  if (bd) sv->arena.release(bd);
  if (xd) sv->arena.release(xd);
  std::vector<double>().swap(r->b);
  return true;
}

void slot_worker(cptr_server sv) {
  (void)hipSetDevice(sv->o.device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    Request* r = nullptr;
    int64_t seen = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_admit.wait(lk, [&] {
        const bool fits = !sv->ready_q.empty() && sv->reserved + sv->ready_q.front()->bytes <=
                                                      (int64_t)sv->arena.size();
        return fits || (sv->setups_done && sv->ready_q.empty());
      });
      if (sv->ready_q.empty()) break;
      r = sv->ready_q.front();
      sv->ready_q.pop_front();
      sv->reserved += r->bytes;
      sv->inflight += 1;
      sv->stats.peak_inflight = std::max(sv->stats.peak_inflight, (int32_t)sv->inflight);
      sv->stats.peak_reserved_bytes = std::max(sv->stats.peak_reserved_bytes, sv->reserved);
      r->state = Request::kRunning;
      r->t_admit = now_s();
      seen = sv->releases;
    }
    int rc = CPTR_OK;
    bool ran = true;
    if (have_stream) {
      ran = run_request(sv, r, st, rc);
    } else {
      rc = CPTR_E_HIP;
      r->err = "creating the slot's stream failed";
    }
    if (ran) {
      cptr_destroy(r->h);  // returns the handle's pieces to the arena
      r->h = nullptr;
    }
    // the request's memory is back in the arena before its reservation ends
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->reserved -= r->bytes;
    sv->inflight -= 1;
    sv->releases += 1;
    sv->cv_admit.notify_all();
    if (ran) {
      finish(sv, r, rc);
      continue;
    }
    // The free memory was there but not in one piece.  An empty arena always
    // has room for a request whose footprint fits the budget (the footprint
    // counts every allocation of its build), so with nothing else in flight
    // the request is tried again at once; otherwise it waits at the head of
    // the queue until another request gives memory back.  A request that
    // keeps failing is reported instead of retried forever.
    r->placements += 1;
    if (r->placements > 64) {
      r->err = "HBM arena too fragmented for the request";
      cptr_destroy(r->h);
      r->h = nullptr;
      finish(sv, r, CPTR_E_NOMEM);
      continue;
    }
    r->state = Request::kReady;
    sv->ready_q.push_front(r);
    // `seen` counted releases before this admission; this request's own
    // release is one more
    if (sv->inflight > 0) sv->cv_admit.wait(lk, [&] { return sv->releases > seen + 1; });
  }
  if (have_stream) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

void cptr_server_opts_default(cptr_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_inflight = 4;
  o->setup_workers = 8;
  o->hbm_budget_bytes = (int64_t)16 << 30;
  o->device = 0;
  cptr_setup_opts_default(&o->setup);
  o->setup.precond_precision = CPTR_PRECISION_FP32;
  o->setup.setup_threads = 0;
}

cptr_status cptr_server_create(const cptr_server_opts* o_in, cptr_server* out) {
  if (!out) return CPTR_E_INVALID;
  *out = nullptr;
  cptr_server_opts o;
  cptr_server_opts_default(&o);
  if (o_in) o = *o_in;
  if (o.max_inflight < 1 || o.max_inflight > 64 || o.setup_workers < 1 || o.setup_workers > 64 ||
      o.hbm_budget_bytes < (int64_t)cptr::DevArena::kAlign || o.device < 0 || o.setup.host_only)
    return CPTR_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o.device >= ndev) return CPTR_E_HIP;
  if (hipSetDevice(o.device) != hipSuccess) return CPTR_E_HIP;
  std::unique_ptr<cptr_server_s> sv(new (std::nothrow) cptr_server_s());
  if (!sv) return CPTR_E_NOMEM;
  sv->o = o;
  sv->t_created = now_s();
  if (hipMalloc(&sv->arena_mem, (size_t)o.hbm_budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return CPTR_E_NOMEM;
  }
  sv->arena.init(sv->arena_mem, (size_t)o.hbm_budget_bytes);
  sv->stats.hbm_budget_bytes = (int64_t)sv->arena.size();
  cptr_server s = sv.get();
  for (int i = 0; i < o.setup_workers; ++i) sv->setup_threads.emplace_back(setup_worker, s);
  for (int i = 0; i < o.max_inflight; ++i) sv->slot_threads.emplace_back(slot_worker, s);
  *out = sv.release();
  return CPTR_OK;
}

cptr_status cptr_server_submit(cptr_server sv, const cptr_bsr* A, const int32_t* elliptic_idx,
                               int32_t n_elliptic, const double* b, const cptr_solve_opts* so,
                               int64_t* id) {
  if (!sv || !A || !b || !id || !elliptic_idx || A->on_device || !A->row_ptr || !A->col_idx ||
      !A->values || A->n_block_rows <= 0 || A->nnz_blocks <= 0 || n_elliptic < 1 || n_elliptic > 2)
    return CPTR_E_INVALID;
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return CPTR_E_NOMEM;
  try {
    r->nb = A->n_block_rows;
    r->nnzb = A->nnz_blocks;
    r->rp.assign(A->row_ptr, A->row_ptr + (size_t)r->nb + 1);
    r->ci.assign(A->col_idx, A->col_idx + (size_t)r->nnzb);
    r->v.assign(A->values, A->values + (size_t)r->nnzb * 9);
    r->b.assign(b, b + 3 * (size_t)r->nb);
  } catch (const std::bad_alloc&) {
    return CPTR_E_NOMEM;
  }
  r->ne = n_elliptic;
  for (int e = 0; e < n_elliptic; ++e) r->eidx[e] = elliptic_idx[e];
  cptr_solve_opts_default(&r->so);
  if (so) r->so = *so;
  if (r->so.restart < 1) return CPTR_E_INVALID;
  std::lock_guard<std::mutex> g(sv->mu);
  if (sv->stop) return CPTR_E_STATE;
  r->id = sv->next_id++;
  r->t_submit = now_s();
  *id = r->id;
  sv->setup_q.push_back(r.get());
  sv->reqs[r->id] = std::move(r);
  ++sv->stats.submitted;
  sv->cv_setup.notify_one();
  return CPTR_OK;
}

cptr_status cptr_server_wait(cptr_server sv, int64_t id, double* x, cptr_serve_info* info,
                             int32_t timeout_ms) {
  if (!sv) return CPTR_E_INVALID;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(id);
  if (it == sv->reqs.end()) return CPTR_E_INVALID;
  Request* r = it->second.get();
  auto done = [&] { return r->state == Request::kDone; };
  if (timeout_ms < 0) sv->cv_done.wait(lk, done);
  else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) return CPTR_E_STATE;
  if (x && !r->x.empty()) std::memcpy(x, r->x.data(), sizeof(double) * r->x.size());
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = r->status;
    info->iterations = r->sinfo.iterations;
    info->converged = r->sinfo.converged;
    info->rel_res_true = r->sinfo.rel_res_true;
    info->queue_s = r->t_setup0 > 0 ? r->t_setup0 - r->t_submit : 0.0;
    info->host_setup_s = r->t_setup1 > 0 ? r->t_setup1 - r->t_setup0 : 0.0;
    info->admit_wait_s = r->t_admit > 0 ? r->t_admit - r->t_setup1 : 0.0;
    info->device_setup_s = r->t_dev > 0 ? r->t_dev - r->t_admit : 0.0;
    info->solve_s = r->t_dev > 0 ? r->t_done - r->t_dev : 0.0;
    info->latency_s = r->t_done - r->t_submit;
    info->device_bytes = r->bytes;
    info->admitted_at_s = r->t_admit > 0 ? r->t_admit - sv->t_created : 0.0;
    info->done_at_s = r->t_done - sv->t_created;
  }
  const int status = r->status;
  if (status < 0) sv->last_err = r->err;
  sv->reqs.erase(it);
  return (cptr_status)status;
}

const char* cptr_server_last_error(cptr_server sv) { return sv ? sv->last_err.c_str() : ""; }

cptr_status cptr_server_get_stats(cptr_server sv, cptr_server_stats* st) {
  if (!sv || !st) return CPTR_E_INVALID;
  std::lock_guard<std::mutex> g(sv->mu);
  *st = sv->stats;
  return CPTR_OK;
}

cptr_status cptr_server_destroy(cptr_server sv) {
  if (!sv) return CPTR_E_INVALID;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv_setup.notify_all();
  for (auto& t : sv->setup_threads) t.join();
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->setups_done = true;
  }
  sv->cv_admit.notify_all();
  for (auto& t : sv->slot_threads) t.join();
  for (auto& kv : sv->reqs)
    if (kv.second->h) cptr_destroy(kv.second->h);
  (void)hipSetDevice(sv->o.device);
  if (sv->arena_mem) (void)hipFree(sv->arena_mem);
  delete sv;
  return CPTR_OK;
}

}  // extern "C"
