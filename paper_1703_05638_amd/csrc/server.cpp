// Serving loop: posterior requests (eigenpairs of the prior-preconditioned
// misfit Hessian and the posterior variance, Sec. 2 and Sec. 6) of uneven
// mesh and time sizes, admitted against a device-memory budget and run
// concurrently.
//
// Each worker thread owns a HIP stream (non-blocking, default priority) and
// keeps one resident problem: that of the last size class it served (mesh,
// time steps, horizon, tolerance, rank cap, precision), with its multigrid
// hierarchy, device memory pool and stencil weights.  A worker takes, among
// the first pending requests whose memory estimate fits in what is left of
// the budget, one of its resident size class if there is one (requests of a
// class are thereby served back to back on the problem that stays on the
// device, re-targeted to each request's prior, noise and box), else the
// oldest.  Requests that arrive while others run are admitted as soon as a
// worker and memory free up, and their kernels overlap on the device with
// the running ones.  A resident problem's memory stays counted against the
// budget while it is parked.  Every request runs through the public entry
// points on the worker's stream, and a re-targeted problem computes exactly
// what a new one would, so a result does not depend on what else is running
// or ran before.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "lrpost.h"

namespace lrp {
void set_last_error(const std::string& msg);
}

namespace {

using clk = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  lrpost_problem_desc desc{};
  int k = 0;
  int want_diag = 1;
  size_t est_bytes = 0;
  clk::time_point t_submit;
  // results
  bool done = false;
  int status = 0;
  std::string error;
  std::vector<double> lambda, diag;
  double latency_s = 0.0;
  size_t peak_bytes = 0;
};

// Device-memory estimate of one request, in bytes: the rational Krylov pole
// solutions and bases of a block of four applies with their multigrid work
// (rank cap x poles x about ten nodal vectors), the shared Lanczos basis and
// the posterior variance.
size_t estimate_bytes(const lrpost_problem_desc& d, int k) {
  const double nx = (double)(d.N - 1) * (d.N - 1);
  const double lt = -std::log10(d.trunc_tol);
  const double poles = std::max(4.0, std::min(24.0, std::round(1.5 * lt) + 1.0));
  const double cols = d.rank_cap * poles * 10.0 + 16.0 * (4.0 * k + 16.0) + 1024.0 + (double)d.nt;
  return (size_t)(8.0 * nx * cols * 2.0);
}

// Requests of one size class can share a problem (lrpost_retarget).
bool same_class(const lrpost_problem_desc& a, const lrpost_problem_desc& b) {
  return a.N == b.N && a.nt == b.nt && a.T == b.T && a.trunc_tol == b.trunc_tol && a.rank_cap == b.rank_cap &&
         a.precision == b.precision && a.mg_levels == b.mg_levels;
}

// how far down the pending queue a worker looks for a request of its class
constexpr int kClassLookahead = 8;

}  // namespace

namespace {
struct Resident {
  lrpost_problem* p = nullptr;
  lrpost_problem_desc desc{};
  size_t bytes = 0;  // memory estimate kept reserved while parked
};
}  // namespace

struct lrpost_server {
  size_t budget = 0, in_use = 0, peak_in_use = 0;
  int64_t resident_hits = 0, served = 0;
  int device = 0;
  int running = 0, peak_running = 0;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> pending;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<std::thread> workers;

  void worker_loop() {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    Resident res;
    for (;;) {
      std::shared_ptr<Request> rq;
      bool reuse = false;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stop) break;
          // a request of the resident class among the first few that fit,
          // else the oldest that fits (the resident problem's reservation is
          // released for a request of another class); with nothing running,
          // the oldest always runs
          auto fits = [&](const Request& r) {
            const bool same = res.p && same_class(res.desc, r.desc);
            const size_t need = r.est_bytes > (same ? res.bytes : 0) ? r.est_bytes - (same ? res.bytes : 0) : 0;
            const size_t freed = same ? 0 : res.bytes;
            return running == 0 || in_use - freed + need <= budget;
          };
          auto pick = pending.end();
          int looked = 0;
          for (auto it = pending.begin(); it != pending.end() && looked < kClassLookahead; ++it, ++looked)
            if (res.p && same_class(res.desc, (*it)->desc) && fits(**it)) {
              pick = it;
              break;
            }
          if (pick == pending.end())
            for (auto it = pending.begin(); it != pending.end(); ++it)
              if (fits(**it)) {
                pick = it;
                break;
              }
          if (pick != pending.end()) {
            rq = *pick;
            pending.erase(pick);
            break;
          }
          cv_work.wait(lk);
        }
        if (!rq) break;
        reuse = res.p && same_class(res.desc, rq->desc);
        // the request's reservation replaces the parked one
        in_use = in_use - res.bytes + rq->est_bytes;
        peak_in_use = std::max(peak_in_use, in_use);
        ++running;
        peak_running = std::max(peak_running, running);
        ++served;
        if (reuse) ++resident_hits;
      }
      if (!reuse && res.p) {
        lrpost_destroy(res.p);
        res.p = nullptr;
      }
      run(rq.get(), st, res);
      {
        std::lock_guard<std::mutex> lk(mu);
        // the problem stays resident (and reserved) when the request ran
        if (!res.p) in_use -= rq->est_bytes;
        else res.bytes = rq->est_bytes;
        --running;
        rq->done = true;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (res.p) {
      lrpost_destroy(res.p);
      std::lock_guard<std::mutex> lk(mu);
      in_use -= res.bytes;
    }
    if (st) (void)hipStreamDestroy(st);
  }

  // Runs one request on the worker's resident problem (re-targeted when it is
  // of the request's class, else created).  On failure the problem is dropped.
  static void run(Request* rq, hipStream_t st, Resident& res) {
    lrpost_problem_desc d = rq->desc;
    d.hip_stream = st;
    lrpost_problem* p = res.p;
    lrpost_eigs* e = nullptr;
    int rc = LRPOST_OK;
    if (p) {
      rc = lrpost_retarget(p, d.alpha, d.sigma, d.box, d.seed);
    } else {
      rc = lrpost_create(&d, &p);
      // V-cycles launched kernel by kernel: a graph capture on one worker's
      // stream while another worker issues its ordered dense-library calls was
      // reported by the runtime as a stream-capture isolation error
      if (rc == LRPOST_OK) rc = lrpost_set_graphs(p, 0);
    }
    if (rc == LRPOST_OK) rc = lrpost_eigensolve(p, rq->k, LRPOST_BLOCK_LANCZOS, 0, &e);
    // the request's host buffers may fail to allocate: that request fails,
    // the worker goes on
    bool host_oom = false;
    try {
      if (rc == LRPOST_OK) {
        const int kk = lrpost_eig_count(e);
        rq->lambda.assign(kk, 0.0);
        rc = lrpost_eig_values(e, rq->lambda.data());
      }
      if (rc == LRPOST_OK && rq->want_diag) {
        rq->diag.assign((size_t)(d.N - 1) * (d.N - 1) * d.nt, 0.0);
        rc = lrpost_post_variance(p, e, rq->diag.data(), 0);
      }
      if (rc != LRPOST_OK) rq->error = lrpost_last_error();
    } catch (const std::bad_alloc&) {
      host_oom = true;
    }
    if (host_oom) {
      rc = LRPOST_ENOMEM;
      std::vector<double>().swap(rq->lambda);
      std::vector<double>().swap(rq->diag);
      rq->error = "host memory";  // (short enough to need no allocation)
    }
    rq->status = rc;
    if (e) lrpost_eigs_free(e);
    if (rc == LRPOST_OK) {
      res.p = p;
      res.desc = rq->desc;
    } else {
      if (p) lrpost_destroy(p);
      res.p = nullptr;
    }
    rq->latency_s = std::chrono::duration<double>(clk::now() - rq->t_submit).count();
  }
};

extern "C" {

int lrpost_server_create(size_t hbm_budget_bytes, int workers, lrpost_server** out) {
  if (!out || workers < 1 || workers > 16 || hbm_budget_bytes == 0) return LRPOST_EINVAL;
  auto s = new lrpost_server();
  s->budget = hbm_budget_bytes;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return LRPOST_EHIP;
  }
  for (int i = 0; i < workers; ++i) s->workers.emplace_back([s] { s->worker_loop(); });
  *out = s;
  return LRPOST_OK;
}

int lrpost_server_submit(lrpost_server* s, const lrpost_problem_desc* d, int k, int want_diag, uint64_t* ticket) {
  if (!s || !d || !ticket || k < 1) return LRPOST_EINVAL;
  auto rq = std::make_shared<Request>();
  rq->desc = *d;
  rq->k = k;
  rq->want_diag = want_diag;
  rq->est_bytes = estimate_bytes(*d, k);
  rq->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return LRPOST_EINVAL;
    rq->ticket = s->next_ticket++;
    s->pending.push_back(rq);
    s->all[rq->ticket] = rq;
    *ticket = rq->ticket;
  }
  s->cv_work.notify_all();
  return LRPOST_OK;
}

int lrpost_server_wait(lrpost_server* s, uint64_t ticket, double* lambda, int k, double* diag, double* latency_s) {
  if (!s) return LRPOST_EINVAL;
  std::shared_ptr<Request> rq;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return LRPOST_EINVAL;
    rq = it->second;
    s->cv_done.wait(lk, [&] { return rq->done; });
    s->all.erase(ticket);
  }
  if (latency_s) *latency_s = rq->latency_s;
  if (rq->status != LRPOST_OK) {
    lrp::set_last_error(rq->error);
    return rq->status;
  }
  if (lambda)
    for (int i = 0; i < k; ++i) lambda[i] = i < (int)rq->lambda.size() ? rq->lambda[i] : 0.0;
  if (diag && !rq->diag.empty()) std::memcpy(diag, rq->diag.data(), sizeof(double) * rq->diag.size());
  return LRPOST_OK;
}

int lrpost_server_info(lrpost_server* s, int* peak_running, size_t* peak_admitted_bytes) {
  if (!s) return LRPOST_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (peak_running) *peak_running = s->peak_running;
  if (peak_admitted_bytes) *peak_admitted_bytes = s->peak_in_use;
  return LRPOST_OK;
}

int lrpost_server_class_stats(lrpost_server* s, int64_t* served, int64_t* resident_hits) {
  if (!s) return LRPOST_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (served) *served = s->served;
  if (resident_hits) *resident_hits = s->resident_hits;
  return LRPOST_OK;
}

int lrpost_server_destroy(lrpost_server* s) {
  if (!s) return LRPOST_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto& rq : s->pending) {
      rq->status = LRPOST_EINVAL;
      rq->error = "server destroyed before the request ran";
      rq->done = true;
    }
    s->pending.clear();
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  for (auto& t : s->workers) t.join();
  delete s;
  return LRPOST_OK;
}

}  // extern "C"
