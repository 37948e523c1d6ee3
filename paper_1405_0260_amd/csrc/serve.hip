// Request loop with continuous batching over the batched ParO calls.
//
// Admission is by HBM footprint: every request needs one contiguous block
// of the caller's device arena (its workspace, nodal potential, orbitals
// and eigenvalues), handed out by a first-fit allocator with coalescing
// free lists.  Requests are admitted in arrival order while a slot is free
// and their block fits; each tick then advances all resident problems by
// one ParO step through the batched step, so new arrivals join the running
// batch at the next step boundary instead of waiting for it to drain.
//
// Uploading and assembling admitted requests (host copies, the stencil
// assembly, the shift read-back) runs on a worker thread of the server,
// on a stream of its own with the default priority, while the tick's
// thread drives the resident problems' step on the caller's stream; the
// first step of an admitted request waits for its admission round through
// an event.
#include <algorithm>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "paro_internal.h"

namespace {

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator over [0, bytes) with coalescing of free neighbours.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
    bytes_ = bytes;
    used_ = 0;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += n;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t bytes() const { return bytes_; }

 private:
  std::map<size_t, size_t> free_;  // offset -> size
  size_t bytes_ = 0, used_ = 0;
};

struct Request {
  int64_t id = 0;
  paro_box_t box{};
  paro_opts_t opts{};
  std::vector<double> V, U0;
  double* h_lambda = nullptr;
  double* h_U = nullptr;
  int64_t n = 0;
  int Nt = 0;
  size_t ws_bytes = 0;
  size_t need = 0;        // bytes of its arena block
  size_t block = 0, off = 0;  // the block while resident
  paro_problem* prob = nullptr;
  double* d_V = nullptr;
  double* d_U = nullptr;
  double* d_lam = nullptr;
  void* d_ws = nullptr;
  paro_report_t rep{};
  int admit_rc = PARO_OK;  // the admission worker's result
  bool done = false;
};

}  // namespace

struct paro_server {
  char* base = nullptr;
  Arena arena;
  void* batch_ws = nullptr;
  size_t batch_bytes = 0;
  int max_active = 0;
  hipStream_t stream = nullptr;   // steps (the caller's stream)
  hipStream_t astream = nullptr;  // admission copies and assembly
  hipEvent_t admitted = nullptr;  // end of the last admission round
  int64_t next_id = 1, ticks = 0, retired = 0;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::vector<Request*> ready;     // assembled, waiting for Step 1
  std::deque<int64_t> unreported;  // retired, id not yet returned
  std::unordered_map<int64_t, Request*> all;
  // Admission worker: `job` (arena blocks already taken) is handed over
  // with pending = true and handed back with pending = false, done = true.
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;
  std::vector<Request*> job;
  bool pending = false, done = false, stop = false;
};

namespace {

#define SRV_HIP(expr)                                                    \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess) {                                              \
      std::string m_ = std::string(#expr) + ": " + hipGetErrorString(e_); \
      return paro::set_error(PARO_EDEVICE, m_.c_str());                  \
    }                                                                    \
  } while (0)

void release(paro_server* s, Request* r) {
  if (r->prob) paro_destroy(r->prob);
  r->prob = nullptr;
  if (r->block) s->arena.release(r->off, r->block);
  r->block = 0;
}

// Copy the inputs of r into its arena block and assemble it (admission
// worker, admission stream).
int admit_one(paro_server* s, Request* r) {
  char* blk = s->base + r->off;
  size_t o = 0;
  r->d_ws = blk + o;
  o += up256(r->ws_bytes);
  r->d_V = reinterpret_cast<double*>(blk + o);
  o += up256(sizeof(double) * r->V.size());
  r->d_U = reinterpret_cast<double*>(blk + o);
  o += up256(sizeof(double) * r->U0.size());
  r->d_lam = reinterpret_cast<double*>(blk + o);
  SRV_HIP(hipMemcpyAsync(r->d_V, r->V.data(), sizeof(double) * r->V.size(),
                         hipMemcpyHostToDevice, s->astream));
  SRV_HIP(hipMemcpyAsync(r->d_U, r->U0.data(),
                         sizeof(double) * r->U0.size(),
                         hipMemcpyHostToDevice, s->astream));
  const int rc = paro_assemble(&r->box, r->d_V, &r->opts, r->d_ws,
                               r->ws_bytes, s->astream, &r->prob);
  // Host copies are no longer needed once on the device.
  SRV_HIP(hipStreamSynchronize(s->astream));
  std::vector<double>().swap(r->V);
  std::vector<double>().swap(r->U0);
  return rc;
}

void worker_main(paro_server* s, int device) {
  const bool on_device = hipSetDevice(device) == hipSuccess;
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv.wait(lk, [s] { return s->stop || s->pending; });
    if (s->stop) return;
    const std::vector<Request*> job = s->job;
    lk.unlock();
    for (Request* r : job) {
      try {
        r->admit_rc = on_device ? admit_one(s, r) : PARO_EDEVICE;
      } catch (...) {
        r->admit_rc = PARO_EDEVICE;
      }
    }
    const hipError_t e = hipEventRecord(s->admitted, s->astream);
    if (e != hipSuccess)
      for (Request* r : job)
        if (r->admit_rc == PARO_OK) r->admit_rc = PARO_EDEVICE;
    lk.lock();
    s->pending = false;
    s->done = true;
    s->cv.notify_all();
  }
}

// The admission stream, event and worker, made on the first admission
// (creating a server touches no device).
int start_admission(paro_server* s) {
  if (s->worker.joinable()) return PARO_OK;
  int device = 0;
  SRV_HIP(hipGetDevice(&device));  // the worker uses the caller's device
  if (!s->astream)
    SRV_HIP(hipStreamCreateWithFlags(&s->astream, hipStreamNonBlocking));
  if (!s->admitted)
    SRV_HIP(hipEventCreateWithFlags(&s->admitted, hipEventDisableTiming));
  try {
    s->worker = std::thread(worker_main, s, device);
  } catch (...) {
    return paro::set_error(PARO_EDEVICE, "admission thread");
  }
  return PARO_OK;
}

// Hand the finished admission round back: assembled requests wait for
// Step 1, the others retire with their error.  wait: block until the
// round in flight (if any) is over.
void collect(paro_server* s, bool wait, std::vector<Request*>& finished) {
  std::unique_lock<std::mutex> lk(s->mu);
  if (wait) s->cv.wait(lk, [s] { return !s->pending; });
  if (!s->done) return;
  for (Request* r : s->job) {
    if (r->admit_rc == PARO_OK) {
      s->ready.push_back(r);
    } else {
      r->rep.status = r->admit_rc;
      finished.push_back(r);
    }
  }
  s->job.clear();
  s->done = false;
}

// Fail every request of `rs` with `code` (a device error of a batched
// call): they leave the device and are reported like any retired request
// (one that had already failed on its own keeps its status).
void fail_all(paro_server* s, std::vector<Request*>& rs, int code) {
  for (Request* r : rs) {
    if (r->rep.status == PARO_OK || r->rep.status == PARO_ENOCONV)
      r->rep.status = code;
    release(s, r);
    r->done = true;
    s->retired += 1;
    s->unreported.push_back(r->id);
  }
  rs.clear();
}

int retire(paro_server* s, Request* r) {
  if (r->prob) {
    SRV_HIP(hipMemcpyAsync(r->h_lambda, r->d_lam, sizeof(double) * r->Nt,
                           hipMemcpyDeviceToHost, s->stream));
    SRV_HIP(hipMemcpyAsync(r->h_U, r->d_U, sizeof(double) * r->n * r->Nt,
                           hipMemcpyDeviceToHost, s->stream));
    SRV_HIP(hipStreamSynchronize(s->stream));
  }
  release(s, r);
  r->done = true;
  s->retired += 1;
  return PARO_OK;
}

}  // namespace

extern "C" {

int paro_server_create(void* d_arena, size_t arena_bytes, int32_t max_active,
                       void* stream, paro_server** out) {
  if (!out) return paro::set_error(PARO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_arena || ((uintptr_t)d_arena & 255))
    return paro::set_error(PARO_EINVAL, "arena must be 256-byte aligned");
  if (max_active < 1 || max_active > PARO_BATCH_MAX)
    return paro::set_error(PARO_EINVAL, "max_active out of range");
  const size_t bb = up256(paro_batch_workspace_bytes(max_active));
  if (arena_bytes <= bb)
    return paro::set_error(PARO_ENOMEM, "arena smaller than the batch table");
  paro_server* s = new (std::nothrow) paro_server();
  if (!s) return paro::set_error(PARO_EDEVICE, "host allocation failed");
  s->base = static_cast<char*>(d_arena) + bb;
  s->batch_ws = d_arena;
  s->batch_bytes = bb;
  s->arena.reset((arena_bytes - bb) & ~size_t(255));
  s->max_active = max_active;
  s->stream = static_cast<hipStream_t>(stream);
  *out = s;
  return PARO_OK;
}

int paro_server_submit(paro_server* s, const paro_box_t* box,
                       const double* h_V, const paro_opts_t* opts,
                       const double* h_U0, double* h_lambda, double* h_U,
                       int64_t* id) {
  try {
    if (!s || !box || !h_V || !opts || !h_U0 || !h_lambda || !h_U || !id)
      return paro::set_error(PARO_EINVAL, "NULL argument to submit");
    int64_t n = 0, z = 0;
    size_t ws = 0;
    int rc = paro_query(box, opts, &n, &z, &ws);
    if (rc) return rc;
    Request* r = new Request();
    r->box = *box;
    r->opts = *opts;
    r->n = n;
    r->Nt = opts->N + opts->m;
    r->ws_bytes = ws;
    const size_t nv = (size_t)(box->nx + 1) * (box->ny + 1) * (box->nz + 1);
    r->V.assign(h_V, h_V + nv);
    r->U0.assign(h_U0, h_U0 + (size_t)n * r->Nt);
    r->h_lambda = h_lambda;
    r->h_U = h_U;
    r->need = up256(ws) + up256(sizeof(double) * nv) +
              up256(sizeof(double) * (size_t)n * r->Nt) +
              up256(sizeof(double) * r->Nt);
    if (r->need > s->arena.bytes()) {
      delete r;
      return paro::set_error(PARO_ENOMEM, "request exceeds the whole arena");
    }
    r->id = s->next_id++;
    s->queue.push_back(r);
    s->all[r->id] = r;
    *id = r->id;
    return PARO_OK;
  } catch (...) {
    return paro::set_error(PARO_EDEVICE, "unexpected exception in submit");
  }
}

int paro_server_tick(paro_server* s, int64_t* done_ids, int32_t max_done,
                     int32_t* n_done, paro_server_stats_t* stats) {
  try {
    if (!s) return paro::set_error(PARO_EINVAL, "NULL server");
    if (n_done) *n_done = 0;
    std::vector<Request*> finished;
    // 1. Hand back a finished admission round; start the next one (in
    // arrival order, while a slot is free and the block fits).  With no
    // problem to step meanwhile, wait for the round.
    if (!s->queue.empty()) {
      const int rc = start_admission(s);
      if (rc != PARO_OK) return rc;
    }
    collect(s, false, finished);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (!s->pending && !s->done) {
        while (!s->queue.empty() &&
               (int)(s->active.size() + s->ready.size() + s->job.size()) <
                   s->max_active) {
          Request* r = s->queue.front();
          size_t off = 0;
          if (!s->arena.alloc(r->need, &off)) break;
          s->queue.pop_front();
          r->off = off;
          r->block = r->need;
          s->job.push_back(r);
        }
        if (!s->job.empty()) {
          s->pending = true;
          s->cv.notify_all();
        }
      }
    }
    if (s->active.empty() && s->ready.empty()) collect(s, true, finished);
    // 2. Step 1 for the assembled arrivals (one batched call), in place on
    // d_U, after their admission round.
    if (!s->ready.empty()) {
      std::vector<paro_problem*> ps;
      std::vector<const double*> u0;
      std::vector<double*> ls, us;
      for (Request* r : s->ready) {
        ps.push_back(r->prob);
        u0.push_back(r->d_U);
        ls.push_back(r->d_lam);
        us.push_back(r->d_U);
      }
      int rc = hipStreamWaitEvent(s->stream, s->admitted, 0) == hipSuccess
                   ? PARO_OK
                   : paro::set_error(PARO_EDEVICE, "admission event wait");
      std::vector<int> st;
      if (rc == PARO_OK)
        rc = paro::batch_init_impl(ps.data(), (int)ps.size(), u0.data(),
                                   ls.data(), us.data(), s->batch_ws,
                                   s->batch_bytes, s->stream, &st);
      if (rc != PARO_OK) {
        fail_all(s, s->ready, rc);
        fail_all(s, s->active, rc);
        fail_all(s, finished, rc);
        return rc;
      }
      for (size_t k = 0; k < s->ready.size(); ++k) {
        Request* r = s->ready[k];
        r->rep.n_dof = r->n;
        r->rep.reorth = (st[k] & paro::kStReorth) ? 1 : 0;
        if (st[k] & ~paro::kStReorth) {  // dependent even after the retry
          r->rep.status = paro::status_code(st[k] & ~paro::kStReorth);
          finished.push_back(r);
        } else {
          s->active.push_back(r);
        }
      }
      s->ready.clear();
    }
    // 3. One ParO step for every resident problem.
    if (!s->active.empty()) {
      std::vector<paro_problem*> ps;
      std::vector<double*> ls, us;
      for (Request* r : s->active) {
        ps.push_back(r->prob);
        ls.push_back(r->d_lam);
        us.push_back(r->d_U);
      }
      std::vector<paro_report_t> reps(ps.size());
      // The served problems' U and lambda come from their last rotation.
      const int rc = paro::batch_step_impl(
          ps.data(), (int)ps.size(), ls.data(), us.data(), s->batch_ws,
          s->batch_bytes, s->stream, reps.data(), true);
      if (rc != PARO_OK) {
        fail_all(s, s->active, rc);
        fail_all(s, finished, rc);
        return rc;
      }
      std::vector<Request*> still;
      for (size_t k = 0; k < s->active.size(); ++k) {
        Request* r = s->active[k];
        const paro_report_t& x = reps[k];
        paro_report_t& a = r->rep;
        a.steps += 1;
        a.pcg_iters += x.pcg_iters;
        a.refinements += x.refinements;
        a.reorth += x.reorth;
        a.n_dof = x.n_dof;
        a.nnz = x.nnz;
        a.sigma = x.sigma;
        a.max_dlambda = x.max_dlambda;
        a.max_resid = x.max_resid;
        a.seconds += x.seconds;
        bool done = false;
        if (x.status != PARO_OK && x.status != PARO_ENOCONV) {
          a.status = x.status;
          done = true;
        } else if (r->opts.lambda_tol > 0.0 &&
                   x.max_dlambda <= r->opts.lambda_tol &&
                   x.max_resid <= r->opts.resid_tol) {
          a.status = PARO_OK;
          done = true;
        } else if (a.steps >= r->opts.max_steps) {
          a.status = PARO_ENOCONV;
          done = true;
        }
        if (done)
          finished.push_back(r);
        else
          still.push_back(r);
      }
      s->active.swap(still);
    }
    // 4. Retire: results to the host, arena space back.
    for (size_t k = 0; k < finished.size(); ++k) {
      Request* r = finished[k];
      const int rc = retire(s, r);
      if (rc != PARO_OK) {
        std::vector<Request*> rest(finished.begin() + k, finished.end());
        fail_all(s, rest, rc);
        fail_all(s, s->active, rc);
        return rc;
      }
      s->unreported.push_back(r->id);
    }
    int32_t nd = 0;
    while (done_ids && nd < max_done && !s->unreported.empty()) {
      done_ids[nd++] = s->unreported.front();
      s->unreported.pop_front();
    }
    if (n_done) *n_done = nd;
    s->ticks += 1;
    if (stats) {
      std::lock_guard<std::mutex> lk(s->mu);
      stats->queued = (int32_t)(s->queue.size() + s->job.size() +
                                s->ready.size());
      stats->active = (int32_t)s->active.size();
      stats->done = s->retired;
      stats->arena_used = s->arena.used();
      stats->arena_bytes = s->arena.bytes();
      stats->ticks = s->ticks;
    }
    return PARO_OK;
  } catch (...) {
    return paro::set_error(PARO_EDEVICE, "unexpected exception in tick");
  }
}

int paro_server_report(paro_server* s, int64_t id, paro_report_t* report) {
  if (!s || !report) return paro::set_error(PARO_EINVAL, "NULL argument");
  auto it = s->all.find(id);
  if (it == s->all.end()) return paro::set_error(PARO_EINVAL, "unknown id");
  if (!it->second->done)
    return paro::set_error(PARO_EINVAL, "request has not retired yet");
  *report = it->second->rep;
  return PARO_OK;
}

void paro_server_destroy(paro_server* s) {
  if (!s) return;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();  // after the round in flight, if any
  }
  for (auto& kv : s->all) {
    if (kv.second->prob) paro_destroy(kv.second->prob);
    delete kv.second;
  }
  if (s->admitted) (void)hipEventDestroy(s->admitted);
  if (s->astream) (void)hipStreamDestroy(s->astream);
  delete s;
}

}  // extern "C"
