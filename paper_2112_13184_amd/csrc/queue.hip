// Serving queue: independent CTMRG solves (a Hamiltonian parameter scan, say)
// admitted by HBM footprint and run concurrently on one GPU.
//
// Admission: a pending request starts as soon as a worker slot is free and the
// summed footprints of the running solves plus its own stay within the budget
// (first fit in arrival order, so a large request does not hold back small
// ones; a request skipped by 8 later admissions blocks further skipping, so
// it cannot starve).  Every running solve owns a context with its own HIP
// stream (default priority), so the kernels of different solves overlap on the
// device while each worker thread waits for its own stream.  A solve runs
// sweeps until the corner-spectrum change drops below its tolerance, its sweep
// cap, or a cancellation (checked between sweeps), then evaluates the energy
// per site and one-site magnetisations, frees its context and publishes the
// result.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "context.hpp"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Job {
  uint64_t ticket = 0;
  ctm_request req{};
  std::vector<double> tensors, bond, onsite;
  size_t footprint = 0;
  int skipped = 0;
  std::atomic<bool> cancel{false};
  enum { PENDING, ACTIVE, DONE } state = PENDING;
  ctm_result res{};
};

size_t site_elems(const ctm_config& c) {
  const long D = c.D, d = (c.layers == 2) ? c.d : 1;
  return (size_t)c.Lx * c.Ly * D * D * D * D * d;
}

}  // namespace

struct ctm_queue {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Job>> pending;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
  size_t budget = 0, used = 0;
  int max_active = 1, active = 0, device = 0;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::vector<std::thread> workers;
};

namespace {

// Index in q->pending of the next request to admit, or -1.
long pick(ctm_queue* q) {
  if (q->active >= q->max_active) return -1;
  for (size_t i = 0; i < q->pending.size(); ++i) {
    const auto& j = q->pending[i];
    if (q->used + j->footprint <= q->budget) {
      for (size_t s = 0; s < i; ++s) q->pending[s]->skipped += 1;
      return (long)i;
    }
    if (j->skipped >= 8) return -1;   // oldest request has waited long enough
  }
  return -1;
}

void run_job(ctm_queue* q, Job& j) {
  ctm_result& r = j.res;
  ctm_config cfg = j.req.cfg;
  cfg.stream = nullptr;   // the context creates its own stream
  ctm_ctx* ctx = nullptr;
  ctm_status st = ctm_init(&cfg, j.tensors.data(), 0, nullptr, &ctx);
  if (st != CTM_OK) {
    r.status = st;
    return;
  }
  const int N = cfg.Lx * cfg.Ly;
  const int d = (cfg.layers == 2) ? cfg.d : 1;
  int sweeps = 0, conv = 0;
  double delta = INFINITY;
  ctm::Context& c = ctm::context_of(ctx);
  try {
    ctm::do_sweeps(c, j.req.max_sweeps, j.req.tol, &sweeps, &delta, &conv, &j.cancel);
    if (j.cancel.load()) {
      st = CTM_ECANCELED;
    } else {
      double e = 0.0, v = 0.0;
      for (int s = 0; s < N && st == CTM_OK; ++s) {
        for (int dir = 0; dir < 2 && st == CTM_OK; ++dir) {
          st = ctm_expect_2site(ctx, s, dir, j.bond.data(), &v);
          e += v;
        }
        if (st == CTM_OK && !j.onsite.empty()) {
          st = ctm_expect_1site(ctx, s, j.onsite.data(), &v);
          e += v;
        }
      }
      r.energy_per_site = e / N;
      if (st == CTM_OK && d == 2 && cfg.layers == 2) {
        const double sz[4] = {1.0, 0.0, 0.0, -1.0};
        for (int s = 0; s < std::min(N, 4) && st == CTM_OK; ++s) st = ctm_expect_1site(ctx, s, sz, &r.mz[s]);
      }
    }
  } catch (const ctm::Error& e) {
    st = (ctm_status)e.status;
  } catch (const std::exception&) {
    st = CTM_EDEVICE;
  }
  r.status = st;
  r.sweeps = sweeps;
  r.converged = conv;
  r.delta = delta;
  ctm_free(ctx);
}

void worker(ctm_queue* q) {
  (void)hipSetDevice(q->device);
  std::unique_lock<std::mutex> lk(q->mu);
  for (;;) {
    long i = -1;
    q->cv_work.wait(lk, [&] { return q->stop || (i = pick(q)) >= 0; });
    if (i < 0) return;   // stopping and nothing admissible
    std::shared_ptr<Job> j = q->pending[i];
    q->pending.erase(q->pending.begin() + i);
    q->used += j->footprint;
    q->active += 1;
    j->state = Job::ACTIVE;
    j->res.t_admit_ns = now_ns();
    lk.unlock();
    run_job(q, *j);
    lk.lock();
    q->used -= j->footprint;
    q->active -= 1;
    j->res.t_done_ns = now_ns();
    j->state = Job::DONE;
    q->cv_done.notify_all();
    q->cv_work.notify_all();
  }
}

bool fill(ctm_queue* q, uint64_t ticket, ctm_result* res, ctm_status* st) {
  auto it = q->jobs.find(ticket);
  if (it == q->jobs.end()) {
    *st = CTM_EINVAL;
    return true;
  }
  if (it->second->state != Job::DONE) return false;
  if (res) *res = it->second->res;
  *st = it->second->res.status;
  return true;
}

}  // namespace

extern "C" {

ctm_status ctm_queue_create(size_t hbm_budget_bytes, int max_active, ctm_queue** out) {
  if (!out || hbm_budget_bytes == 0 || max_active < 1 || max_active > 64) return CTM_EINVAL;
  *out = nullptr;
  ctm_queue* q = new (std::nothrow) ctm_queue();
  if (!q) return CTM_ENOMEM;
  q->budget = hbm_budget_bytes;
  q->max_active = max_active;
  if (hipGetDevice(&q->device) != hipSuccess) {
    delete q;
    return CTM_EDEVICE;
  }
  try {
    for (int i = 0; i < max_active; ++i) q->workers.emplace_back(worker, q);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(q->mu);
      q->stop = true;
    }
    q->cv_work.notify_all();
    for (auto& t : q->workers) t.join();
    delete q;
    return CTM_ENOMEM;
  }
  *out = q;
  return CTM_OK;
}

ctm_status ctm_queue_submit(ctm_queue* q, const ctm_request* req, uint64_t* ticket) {
  if (!q || !req || !ticket || !req->tensors || !req->bond_op || req->max_sweeps < 0) return CTM_EINVAL;
  const size_t fp = ctm_footprint_bytes(&req->cfg);
  if (fp == 0) return CTM_EINVAL;
  if (fp > q->budget) return CTM_ETOOBIG;
  auto j = std::make_shared<Job>();
  const ctm_config& c = req->cfg;
  const int d = (c.layers == 2) ? c.d : 1;
  j->req = *req;
  j->tensors.assign(req->tensors, req->tensors + site_elems(c));
  j->bond.assign(req->bond_op, req->bond_op + (size_t)d * d * d * d);
  if (req->onsite_op) j->onsite.assign(req->onsite_op, req->onsite_op + (size_t)d * d);
  j->footprint = fp;
  j->res.tag = req->tag;
  j->res.t_submit_ns = now_ns();
  j->res.status = CTM_EAGAIN;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    if (q->stop) return CTM_ECANCELED;
    j->ticket = q->next_ticket++;
    q->jobs[j->ticket] = j;
    q->pending.push_back(j);
    *ticket = j->ticket;
  }
  q->cv_work.notify_one();
  return CTM_OK;
}

ctm_status ctm_queue_poll(ctm_queue* q, uint64_t ticket, ctm_result* res) {
  if (!q) return CTM_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  ctm_status st;
  return fill(q, ticket, res, &st) ? st : CTM_EAGAIN;
}

ctm_status ctm_queue_wait(ctm_queue* q, uint64_t ticket, int timeout_ms, ctm_result* res) {
  if (!q) return CTM_EINVAL;
  std::unique_lock<std::mutex> lk(q->mu);
  ctm_status st = CTM_EAGAIN;
  auto ready = [&] { return fill(q, ticket, res, &st); };
  if (timeout_ms < 0) {
    q->cv_done.wait(lk, ready);
  } else if (!q->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return CTM_EAGAIN;
  }
  return st;
}

ctm_status ctm_queue_cancel(ctm_queue* q, uint64_t ticket) {
  if (!q) return CTM_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->jobs.find(ticket);
  if (it == q->jobs.end()) return CTM_EINVAL;
  Job& j = *it->second;
  j.cancel.store(true);
  if (j.state == Job::PENDING) {
    for (auto p = q->pending.begin(); p != q->pending.end(); ++p)
      if ((*p)->ticket == ticket) {
        q->pending.erase(p);
        break;
      }
    j.state = Job::DONE;
    j.res.status = CTM_ECANCELED;
    j.res.t_done_ns = now_ns();
    q->cv_done.notify_all();
  }
  return CTM_OK;
}

void ctm_queue_destroy(ctm_queue* q) {
  if (!q) return;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->stop = true;
    for (auto& j : q->pending) {
      j->cancel.store(true);
      j->state = Job::DONE;
      j->res.status = CTM_ECANCELED;
      j->res.t_done_ns = now_ns();
    }
    q->pending.clear();
  }
  q->cv_work.notify_all();
  q->cv_done.notify_all();
  for (auto& t : q->workers) t.join();
  delete q;
}

}  // extern "C"
