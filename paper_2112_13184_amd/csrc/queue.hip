// Serving queue: independent CTMRG solves (a Hamiltonian parameter scan, say)
// admitted by HBM footprint and run concurrently on one GPU.
//
// Admission: a pending request starts as soon as a worker slot is free and the
// summed footprints of the running groups plus its own stay within the budget
// (first fit in arrival order, so a large request does not hold back small
// ones; a request skipped by 8 later admissions blocks further skipping, so
// it cannot starve).  Pending requests of the same shape (unit cell, D, d,
// chi, precision, sketch sizes, projector path) are admitted together as one
// group, up to 8, while the group's footprint fits: the group shares one
// context, and the cuts of all its live solves are batched into the same
// launches (enlarged-corner products, sketch GEMMs, Cholesky QR, Jacobi SVD).
// Every group owns its HIP stream (default priority), so different groups
// overlap on the device while each worker thread waits for its own stream.
//
// A group is driven sweep by sweep.  A solve stops when the corner-spectrum
// change drops below its tolerance, at its sweep cap, when cancelled (checked
// between sweeps) or when its own numbers fail (NaN / Inf or a cut without
// singular values; the context isolates replicas, so the others go on).  Its
// observables are evaluated and its result published at once, and its slot
// is free: at the next sweep boundary the oldest pending request of the same
// shape is started in that slot (fresh site tensors and environment, its own
// move count and seed), without new memory.  The group's footprint returns to
// the budget when its last solve is published.
#include <atomic>
#include <chrono>
#include <cmath>
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
  std::vector<double> tensors, bond, onsite, obs, obs2;
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

constexpr int kMaxGroup = 8;

bool same_shape(const ctm_config& a, const ctm_config& b) {
  return a.Lx == b.Lx && a.Ly == b.Ly && a.d == b.d && a.D == b.D && a.chi == b.chi && a.layers == b.layers &&
         a.prec == b.prec && a.svd_rel_cutoff == b.svd_rel_cutoff && a.rsvd_oversample == b.rsvd_oversample &&
         a.rsvd_power_iters == b.rsvd_power_iters && a.projector_path == b.projector_path;
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
  hipStream_t stream = nullptr;   // caller's stream for device-side request tensors
  std::vector<std::thread> workers;
};

namespace {

// The next group to admit: indices into q->pending (ascending), and its
// footprint; empty if nothing fits now.
std::vector<size_t> pick(ctm_queue* q, size_t* footprint) {
  std::vector<size_t> g;
  if (q->active >= q->max_active) return g;
  for (size_t i = 0; i < q->pending.size(); ++i) {
    const auto& j = q->pending[i];
    if (q->used + j->footprint <= q->budget) {
      for (size_t s = 0; s < i; ++s) q->pending[s]->skipped += 1;
      g.push_back(i);
      *footprint = j->footprint;
      // later requests of the same shape join while the group fits
      const int cap = std::min(kMaxGroup, 64 / std::max(j->req.cfg.Lx, j->req.cfg.Ly));
      for (size_t k = i + 1; k < q->pending.size() && (int)g.size() < cap; ++k) {
        if (!same_shape(q->pending[k]->req.cfg, j->req.cfg)) continue;
        const size_t fp = ctm::context_footprint_group(j->req.cfg, (int)g.size() + 1);
        if (q->used + fp > q->budget) break;
        g.push_back(k);
        *footprint = fp;
      }
      return g;
    }
    if (j->skipped >= 8) return g;   // oldest request has waited long enough
  }
  return g;
}

// Energy and observables of replica r (one finished solve).
void measure(ctm::Context& c, int r, const Job& j, ctm_result& res) {
  const int N = c.N, d = c.d;
  double e = 0.0;
  for (int s = 0; s < N; ++s) {
    for (int dir = 0; dir < 2; ++dir) e += ctm::expect_2site(c, s, dir, j.bond.data(), r);
    if (!j.onsite.empty()) e += ctm::expect_1site(c, s, j.onsite.data(), r);
  }
  res.energy_per_site = e / N;
  for (int k = 0; k < j.req.n_obs; ++k)
    for (int s = 0; s < N; ++s) res.obs[k][s] = ctm::expect_1site(c, s, j.obs.data() + (size_t)k * d * d, r);
  for (int k = 0; k < j.req.n_obs2; ++k)
    for (int s = 0; s < N; ++s)
      for (int dir = 0; dir < 2; ++dir)
        res.obs2[k][s][dir] = ctm::expect_2site(c, s, dir, j.obs2.data() + (size_t)k * d * d * d * d, r);
}

void publish(ctm_queue* q, const std::shared_ptr<Job>& j) {
  std::lock_guard<std::mutex> lk(q->mu);
  j->res.t_done_ns = now_ns();
  j->state = Job::DONE;
  q->cv_done.notify_all();
}

// Runs a group to its end: the admitted jobs in slots 0..R-1, later
// same-shape requests in the slots that free up.
void run_group(ctm_queue* q, std::vector<std::shared_ptr<Job>> jobs) {
  const int R = (int)jobs.size();
  ctm_config cfg = jobs[0]->req.cfg;
  cfg.stream = nullptr;   // the context creates its own stream
  std::vector<double> tensors;
  std::vector<uint64_t> seeds(R);
  for (int r = 0; r < R; ++r) {
    tensors.insert(tensors.end(), jobs[r]->tensors.begin(), jobs[r]->tensors.end());
    seeds[r] = jobs[r]->req.cfg.seed;
  }
  ctm_status st = CTM_OK;
  ctm_ctx* ctx = ctm::create_group(cfg, tensors.data(), R, seeds.data(), &st);
  if (!ctx) {
    for (auto& j : jobs) {
      j->res.status = st;
      publish(q, j);
    }
    return;
  }
  ctm::Context& c = ctm::context_of(ctx);
  c.isolate = true;
  std::vector<std::shared_ptr<Job>> slot = jobs;   // null: free slot
  std::vector<int> done(R, 0);
  std::vector<double> delta(R, INFINITY);
  auto finish = [&](int r, ctm_status status, bool converged) {
    Job& j = *slot[r];
    j.res.status = status;
    j.res.sweeps = done[r];
    j.res.delta = delta[r];
    j.res.converged = converged ? 1 : 0;
    c.frozen[r] = 1;
    if (status == CTM_OK) {
      try {
        measure(c, r, j, j.res);
      } catch (const ctm::Error& e) {
        j.res.status = (ctm_status)e.status;
      } catch (...) {
        j.res.status = CTM_EDEVICE;
      }
    }
    std::shared_ptr<Job> held = slot[r];
    publish(q, held);
    slot[r] = nullptr;
    // a solve that failed on its own leaves NaN / Inf or zeros in its slot:
    // restart the slot from its (finite) tensors so that the launches over
    // every corner of the context (the stop rule's spectra) only see finite
    // data.  (After a device error the whole group ends instead.)
    if (c.failed[r]) {
      try {
        ctm::replica_reset(c, r, held->tensors.data(), held->req.cfg.seed);
        c.frozen[r] = 1;
      } catch (...) {
      }
    }
  };
  // a free slot takes the oldest pending request of this shape
  auto refill = [&]() {
    for (int r = 0; r < R; ++r) {
      if (slot[r]) continue;
      std::shared_ptr<Job> j;
      {
        std::lock_guard<std::mutex> lk(q->mu);
        for (auto it = q->pending.begin(); it != q->pending.end(); ++it)
          if (same_shape((*it)->req.cfg, cfg)) {
            j = *it;
            q->pending.erase(it);
            j->state = Job::ACTIVE;
            j->res.t_admit_ns = now_ns();
            break;
          }
      }
      if (!j) return;
      slot[r] = j;
      done[r] = 0;
      delta[r] = INFINITY;
      ctm::replica_reset(c, r, j->tensors.data(), j->req.cfg.seed);
    }
  };
  try {
    ctm::group_start(c);
    std::vector<double> h(R);
    for (;;) {
      for (int r = 0; r < R; ++r) {
        if (!slot[r]) continue;
        if (slot[r]->cancel.load()) finish(r, CTM_ECANCELED, false);
        else if (done[r] >= slot[r]->req.max_sweeps) finish(r, CTM_OK, false);
      }
      refill();
      for (int r = 0; r < R; ++r)   // a new solve with max_sweeps = 0 ends at once
        if (slot[r] && done[r] >= slot[r]->req.max_sweeps) finish(r, CTM_OK, false);
      bool live = false;
      for (int r = 0; r < R; ++r) {
        c.frozen[r] = slot[r] ? 0 : 1;
        live |= slot[r] != nullptr;
      }
      if (!live) break;
      ctm::group_sweep(c, h.data());
      for (int r = 0; r < R; ++r) {
        if (!slot[r]) continue;
        if (c.failed[r]) {
          finish(r, CTM_ENUMERIC, false);
          continue;
        }
        done[r] += 1;
        delta[r] = h[r];
        if (delta[r] < slot[r]->req.tol) finish(r, CTM_OK, true);
      }
    }
  } catch (const ctm::Error& e) {
    for (int r = 0; r < R; ++r)
      if (slot[r]) finish(r, (ctm_status)e.status, false);
  } catch (const std::exception&) {
    for (int r = 0; r < R; ++r)
      if (slot[r]) finish(r, CTM_EDEVICE, false);
  }
  ctm_free(ctx);
}

void worker(ctm_queue* q) {
  (void)hipSetDevice(q->device);
  std::unique_lock<std::mutex> lk(q->mu);
  for (;;) {
    std::vector<size_t> idx;
    size_t fp = 0;
    q->cv_work.wait(lk, [&] { return q->stop || !(idx = pick(q, &fp)).empty(); });
    if (idx.empty()) return;   // stopping and nothing admissible
    std::vector<std::shared_ptr<Job>> jobs;
    for (size_t i : idx) jobs.push_back(q->pending[i]);
    for (size_t k = idx.size(); k-- > 0;) q->pending.erase(q->pending.begin() + idx[k]);
    q->used += fp;
    q->active += 1;
    const int64_t t = now_ns();
    for (auto& j : jobs) {
      j->state = Job::ACTIVE;
      j->res.t_admit_ns = t;
    }
    lk.unlock();
    run_group(q, std::move(jobs));
    lk.lock();
    q->used -= fp;
    q->active -= 1;
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

ctm_status ctm_queue_create(size_t hbm_budget_bytes, int max_active, void* stream, ctm_queue** out) {
  if (!out || hbm_budget_bytes == 0 || max_active < 1 || max_active > 64) return CTM_EINVAL;
  *out = nullptr;
  ctm_queue* q = new (std::nothrow) ctm_queue();
  if (!q) return CTM_ENOMEM;
  q->budget = hbm_budget_bytes;
  q->max_active = max_active;
  q->stream = (hipStream_t)stream;
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
  if (req->n_obs < 0 || req->n_obs > CTM_MAX_OBS || req->n_obs2 < 0 || req->n_obs2 > CTM_MAX_OBS ||
      (req->n_obs > 0 && !req->obs_ops) || (req->n_obs2 > 0 && !req->obs2_ops))
    return CTM_EINVAL;
  const size_t fp = ctm_footprint_bytes(&req->cfg);
  if (fp == 0) return CTM_EINVAL;
  if (fp > q->budget) return CTM_ETOOBIG;
  auto j = std::make_shared<Job>();
  const ctm_config& c = req->cfg;
  const int d = (c.layers == 2) ? c.d : 1;
  j->req = *req;
  j->tensors.resize(site_elems(c));
  if (req->tensors_on_device) {
    if (hipMemcpyAsync(j->tensors.data(), req->tensors, sizeof(double) * j->tensors.size(), hipMemcpyDeviceToHost,
                       q->stream) != hipSuccess ||
        hipStreamSynchronize(q->stream) != hipSuccess)
      return CTM_EDEVICE;
  } else {
    std::memcpy(j->tensors.data(), req->tensors, sizeof(double) * j->tensors.size());
  }
  for (double v : j->tensors)
    if (!std::isfinite(v)) return CTM_ENUMERIC;
  j->bond.assign(req->bond_op, req->bond_op + (size_t)d * d * d * d);
  if (req->onsite_op) j->onsite.assign(req->onsite_op, req->onsite_op + (size_t)d * d);
  if (req->n_obs > 0) j->obs.assign(req->obs_ops, req->obs_ops + (size_t)req->n_obs * d * d);
  if (req->n_obs2 > 0) j->obs2.assign(req->obs2_ops, req->obs2_ops + (size_t)req->n_obs2 * d * d * d * d);
  // the request no longer refers to caller memory
  j->req.tensors = nullptr;
  j->req.bond_op = j->req.onsite_op = j->req.obs_ops = j->req.obs2_ops = nullptr;
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
