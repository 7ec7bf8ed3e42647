// Dose-serving loop: continuous batching of run-to-sigma requests over the
// batched transport engine on one GPU.
//
// A host thread owns a private context.  Requests queue in arrival order and
// are admitted while their device footprint (tallies, plus the phantom when
// it is not already resident) fits the budget; loaded phantoms stay resident
// and are evicted least-recently-used when an admission needs the room.
// Every round gives each admitted request one batch of the configured size in
// a single launch of the multi-case kernel, so requests that arrive while a
// round runs join the next one.  A request follows exactly the batch schedule
// of ctd_run_to_sigma (pilot of n_batches, then the shared sigma plan), and
// tallies depend only on a case's own batches, so each result is identical
// whether the request runs alone or among others.  On completion the exact
// sums are copied to host memory and the request's device memory is freed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "ctd_api_internal.h"

using namespace ctd;

namespace {

struct PhantomEntry {
  ctd_grid g{};
  std::vector<uint8_t> mat;
  std::vector<float> rho;
  ctd_phantom *dev = nullptr;  // resident copy, or null
  uint64_t dev_bytes = 0;
  int users = 0;               // admitted requests using the resident copy
  uint64_t last_use = 0;
};

struct Request {
  uint64_t ticket = 0, phantom_key = 0;
  ctd_matset *ms = nullptr;
  ctd_spectrum *sp = nullptr;
  ctd_geometry *geo = nullptr;
  ctd_params p{};
  double target = 0.0;
  bool held = false;  // holds a reference on ms, sp and geo until finished
  int state = 0;   // 0 queued, 1 running, 2 done, 3 cancelled, 4 failed
  int status = CTD_OK;
  bool cancel = false;
  double sigma = NAN;
  double t_submit = 0, t_admit = 0, t_done = 0;
  ctd_case *cs = nullptr;
  uint64_t planned = 0;      // batches the current plan runs to
  uint64_t footprint = 0;    // device bytes of the case
  // progress, updated by the server thread under the lock (poll reads these,
  // never the case, which the thread updates unlocked during a round)
  uint64_t histories = 0;
  uint32_t batches = 0;
  // results kept on the host after completion
  std::vector<int64_t> s1;
  std::vector<uint64_t> s2_hi, s2_lo;
};

}  // namespace

struct ctd_server {
  ctd_ctx *ctx = nullptr;
  ctd_server_config cfg{};
  std::thread th;
  mutable std::mutex mu;   // guards everything below, err included
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::vector<Request *> active;
  std::map<uint64_t, std::unique_ptr<Request>> all;
  std::map<uint64_t, PhantomEntry> phantoms;
  uint64_t used_bytes = 0, next_ticket = 1, use_clock = 0;
  bool stop = false;
  std::string err;
  std::chrono::steady_clock::time_point t0;
  ctd_server_stats stats{};
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

// Record the message of a failing call.  Lock held.
static int sv_err(ctd_server *sv, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  sv->err = buf;
  return code;
}

// ---------------------------------------------------------- server thread

// Evict unused resident phantoms (least recently used first) until `need`
// more bytes fit; `keep`, the phantom of the request being admitted, is never
// evicted (its size is not part of `need` when it is resident).  Called with
// the lock held.
static bool make_room(ctd_server *sv, uint64_t need, const PhantomEntry *keep) {
  while (sv->used_bytes + need > sv->cfg.hbm_budget_bytes) {
    PhantomEntry *victim = nullptr;
    for (auto &kv : sv->phantoms) {
      PhantomEntry &e = kv.second;
      if (&e != keep && e.dev && e.users == 0 && (!victim || e.last_use < victim->last_use))
        victim = &e;
    }
    if (!victim) return false;
    ctd_phantom_release(sv->ctx, victim->dev);
    victim->dev = nullptr;
    sv->used_bytes -= victim->dev_bytes;
    sv->stats.evictions++;
  }
  return true;
}

static void finish(ctd_server *sv, Request *r, int state, int status) {
  r->state = state;
  r->status = status;
  r->t_done = sv->now();
  if (r->cs) {
    if (state == 2) {
      const int64_t V = r->cs->ph->V;
      r->s1.resize((size_t)V);
      r->s2_hi.resize((size_t)V);
      r->s2_lo.resize((size_t)V);
      uint32_t nb = 0;
      int rc = ctd_read_tally(sv->ctx, r->cs, r->s1.data(), r->s2_hi.data(), r->s2_lo.data(),
                              &nb);
      if (rc != CTD_OK) {
        r->state = 4;
        r->status = rc;
      }
    }
    r->histories = r->cs->h_next;
    r->batches = r->cs->batches;
    ctd_case_destroy(sv->ctx, r->cs);
    r->cs = nullptr;
    sv->used_bytes -= r->footprint;
    auto it = sv->phantoms.find(r->phantom_key);
    if (it != sv->phantoms.end()) it->second.users--;
  }
  if (r->held) {
    r->ms->refs--;
    r->sp->refs--;
    r->geo->refs--;
    r->held = false;
  }
  if (r->state == 2) sv->stats.completed++;
}

// Admit queued requests in arrival order while they fit.  Lock held.
static void admit(ctd_server *sv) {
  while (!sv->queue.empty() && (int)sv->active.size() < sv->cfg.max_active) {
    Request *r = sv->queue.front();
    if (r->cancel) {
      sv->queue.pop_front();
      finish(sv, r, 3, CTD_ECANCELLED);
      continue;
    }
    auto it = sv->phantoms.find(r->phantom_key);
    PhantomEntry &e = it->second;
    const int64_t V = (int64_t)e.g.nx * e.g.ny * e.g.nz;
    const int copies = sv->cfg.tuning.block && sv->cfg.tuning.tally_mode != 0 ? kTallyCopies : 1;
    const uint64_t case_bytes = case_footprint(e.g, r->geo, r->p, r->ms->eg.ne, copies,
                                               sv->cfg.batch_histories);
    // records, plus a palette index or the bound grids (1, 2, 4-voxel blocks)
    const uint64_t ph_bytes =
        e.dev ? 0 : (uint64_t)V * 9 + (uint64_t)V / 8 + (uint64_t)V / 64 + 8192;
    const uint64_t need = case_bytes + ph_bytes;
    if (need > sv->cfg.hbm_budget_bytes) {  // can never fit
      sv->queue.pop_front();
      finish(sv, r, 4, CTD_ENOMEM);
      continue;
    }
    if (!make_room(sv, need, &e)) break;  // wait for running requests to finish
    int rc = CTD_OK;
    if (!e.dev) {
      rc = ctd_phantom_load(sv->ctx, &e.g, e.mat.data(), e.rho.data(), CTD_MEM_HOST, &e.dev);
      if (rc == CTD_OK) {
        e.dev_bytes = ph_bytes;
        sv->used_bytes += ph_bytes;
        sv->stats.phantom_loads++;
      }
    } else {
      sv->stats.phantom_hits++;
    }
    sv->queue.pop_front();
    if (rc == CTD_OK) rc = ctd_case_create(sv->ctx, e.dev, r->ms, r->sp, r->geo, &r->p, &r->cs);
    if (rc == CTD_OK && sv->cfg.tuning.block)
      rc = ctd_set_tuning(sv->ctx, r->cs, &sv->cfg.tuning);
    if (rc != CTD_OK) {
      if (r->cs) {
        ctd_case_destroy(sv->ctx, r->cs);
        r->cs = nullptr;
      }
      sv->err = ctd_last_error(sv->ctx);
      finish(sv, r, 4, rc);
      continue;
    }
    e.users++;
    e.last_use = ++sv->use_clock;
    r->footprint = case_bytes;
    sv->used_bytes += case_bytes;
    r->planned = std::min<uint64_t>((uint64_t)r->p.n_batches,
                                    std::max<uint64_t>(sv->cfg.max_histories /
                                                       sv->cfg.batch_histories, 2));
    r->state = 1;
    r->t_admit = sv->now();
    sv->active.push_back(r);
  }
}

static void server_loop(ctd_server *sv) {
  (void)hipSetDevice(sv->ctx->device);
  const uint64_t bh = sv->cfg.batch_histories;
  const uint64_t max_b = std::max<uint64_t>(sv->cfg.max_histories / bh, 2);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // cancelled running requests leave between rounds
    for (size_t i = 0; i < sv->active.size();) {
      Request *r = sv->active[i];
      if (r->cancel) {
        finish(sv, r, 3, CTD_ECANCELLED);
        sv->active.erase(sv->active.begin() + (long)i);
      } else {
        ++i;
      }
    }
    admit(sv);
    if (sv->active.empty()) {
      sv->cv_done.notify_all();
      if (sv->stop) break;
      sv->cv_work.wait(lk);
      continue;
    }
    if (sv->stop) {
      for (Request *r : sv->active) finish(sv, r, 3, CTD_ECANCELLED);
      sv->active.clear();
      continue;
    }
    // one round: every admitted request with planned batches left runs one
    std::vector<ctd_case *> cases;
    std::vector<Request *> reqs;
    for (Request *r : sv->active) {
      if (r->cs->batches < r->planned) {
        cases.push_back(r->cs);
        reqs.push_back(r);
      }
    }
    lk.unlock();
    int rc = CTD_OK;
    if (!cases.empty()) {
      const ctd_tuning t = sv->cfg.tuning.block ? sv->cfg.tuning : cases[0]->tune;
      rc = run_round(sv->ctx, cases, std::vector<uint64_t>(cases.size(), bh), t);
      if (rc == CTD_OK && hipStreamSynchronize(sv->ctx->stream) != hipSuccess)
        rc = CTD_EDEVICE;
    }
    // requests whose plan is complete: sigma-bar, then stop or plan more
    std::vector<std::pair<Request *, double>> checked;
    if (rc == CTD_OK) {
      for (Request *r : sv->active) {
        if (r->cs->batches < r->planned) continue;
        double sig = INFINITY;
        int rs = sigma_now(sv->ctx, r->cs, sv->cfg.sigma_kind, sv->cfg.dose_frac, &sig);
        checked.push_back({r, rs == CTD_OK ? sig : NAN});
      }
    }
    lk.lock();
    for (Request *r : reqs) {
      r->histories = r->cs->h_next;
      r->batches = r->cs->batches;
    }
    sv->stats.rounds++;
    sv->stats.histories += (uint64_t)cases.size() * bh;
    if (rc != CTD_OK) {
      sv->err = ctd_last_error(sv->ctx);
      for (Request *r : reqs) {
        sv->active.erase(std::find(sv->active.begin(), sv->active.end(), r));
        finish(sv, r, 4, rc);
      }
      sv->cv_done.notify_all();
      continue;
    }
    for (auto &c : checked) {
      Request *r = c.first;
      r->sigma = c.second;
      r->histories = r->cs->h_next;
      r->batches = r->cs->batches;
      const uint64_t more = std::isnan(c.second) ? 0 : sigma_plan(r->cs->batches, c.second,
                                                                   r->target, max_b);
      if (more == 0) {
        sv->active.erase(std::find(sv->active.begin(), sv->active.end(), r));
        finish(sv, r, std::isnan(c.second) ? 4 : 2, std::isnan(c.second) ? CTD_EDEVICE : CTD_OK);
      } else {
        r->planned = r->cs->batches + more;
      }
    }
    sv->cv_done.notify_all();
  }
}

// ------------------------------------------------------------------- C ABI

extern "C" int32_t ctd_server_start(int32_t device, const ctd_server_config *cfg,
                                    ctd_server **out) {
  if (!cfg || !out) return CTD_EINVAL;
  *out = nullptr;
  if (cfg->batch_histories == 0 || cfg->hbm_budget_bytes == 0 || cfg->max_active < 1 ||
      !(cfg->dose_frac >= 0.0 && cfg->dose_frac < 1.0) ||
      (cfg->sigma_kind != CTD_SIGMA_LOCAL && cfg->sigma_kind != CTD_SIGMA_PAPER))
    return CTD_EINVAL;
  ctd_server *sv = new (std::nothrow) ctd_server();
  if (!sv) return CTD_ENOMEM;
  int rc = ctd_create(&sv->ctx, device);
  if (rc != CTD_OK) {
    delete sv;
    return rc;
  }
  sv->cfg = *cfg;
  sv->t0 = std::chrono::steady_clock::now();
  try {
    sv->th = std::thread(server_loop, sv);
  } catch (...) {
    ctd_destroy(sv->ctx);
    delete sv;
    return CTD_ENOMEM;
  }
  *out = sv;
  return CTD_OK;
}

// The message is copied under the lock into a per-thread buffer, so the
// pointer stays valid on the calling thread until its next call here.
extern "C" const char *ctd_server_last_error(const ctd_server *sv) {
  thread_local std::string copy;
  if (!sv) return "null server";
  std::lock_guard<std::mutex> lk(sv->mu);
  copy = sv->err;
  return copy.c_str();
}

extern "C" double ctd_server_now(const ctd_server *sv) { return sv ? sv->now() : 0.0; }

extern "C" int32_t ctd_server_add_phantom(ctd_server *sv, uint64_t key, const ctd_grid *g,
                                          const uint8_t *mat, const float *rho) {
  if (!sv || !g || !mat || !rho) return CTD_EINVAL;
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || !(g->dx > 0 && g->dy > 0 && g->dz > 0)) {
    std::lock_guard<std::mutex> lk(sv->mu);
    return sv_err(sv, CTD_EINVAL, "bad grid");
  }
  const int64_t V = (int64_t)g->nx * g->ny * g->nz;
  PhantomEntry e;
  e.g = *g;
  e.mat.assign(mat, mat + V);
  e.rho.assign(rho, rho + V);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->phantoms.count(key)) return sv_err(sv, CTD_EBUSY, "phantom key already registered");
  sv->phantoms.emplace(key, std::move(e));
  return CTD_OK;
}

extern "C" int32_t ctd_server_submit(ctd_server *sv, uint64_t phantom_key, ctd_matset *ms,
                                     ctd_spectrum *sp, ctd_geometry *geo, const ctd_params *p,
                                     double sigma_target, uint64_t *ticket) {
  if (!sv || !ms || !sp || !geo || !p || !ticket) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (!(sigma_target > 0.0)) return sv_err(sv, CTD_EINVAL, "sigma target must be positive");
  if (p->n_batches < 2) return sv_err(sv, CTD_EINVAL, "n_batches must be >= 2");
  if (sv->stop) return sv_err(sv, CTD_EBUSY, "server is stopping");
  if (!sv->phantoms.count(phantom_key)) return sv_err(sv, CTD_ENOTFOUND, "unknown phantom key");
  auto r = std::make_unique<Request>();
  r->ticket = sv->next_ticket++;
  r->phantom_key = phantom_key;
  r->ms = ms;
  r->sp = sp;
  r->geo = geo;
  r->p = *p;
  r->target = sigma_target;
  r->t_submit = sv->now();
  ms->refs++;
  sp->refs++;
  geo->refs++;
  r->held = true;
  *ticket = r->ticket;
  sv->queue.push_back(r.get());
  sv->all.emplace(r->ticket, std::move(r));
  sv->stats.submitted++;
  sv->cv_work.notify_all();
  return CTD_OK;
}

static void fill_info(const Request *r, ctd_request_info *info) {
  info->state = r->state;
  info->status = r->status;
  info->sigma = r->sigma;
  info->histories = r->histories;
  info->batches = r->batches;
  info->reserved = 0;
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_done = r->t_done;
}

extern "C" int32_t ctd_server_poll(ctd_server *sv, uint64_t ticket, ctd_request_info *info) {
  if (!sv || !info) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return CTD_ENOTFOUND;
  fill_info(it->second.get(), info);
  return CTD_OK;
}

extern "C" int32_t ctd_server_wait(ctd_server *sv, uint64_t ticket, ctd_request_info *info) {
  if (!sv) return CTD_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return CTD_ENOTFOUND;
  // look the ticket up again on every wake-up: another thread may release it
  Request *r = nullptr;
  sv->cv_done.wait(lk, [&] {
    it = sv->all.find(ticket);
    r = it == sv->all.end() ? nullptr : it->second.get();
    return !r || r->state >= 2;
  });
  if (!r) return CTD_ENOTFOUND;
  if (info) fill_info(r, info);
  return r->state == 2 ? CTD_OK : r->status;
}

extern "C" int32_t ctd_server_cancel(ctd_server *sv, uint64_t ticket) {
  if (!sv) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return CTD_ENOTFOUND;
  it->second->cancel = true;
  sv->cv_work.notify_all();
  return CTD_OK;
}

extern "C" int32_t ctd_server_read_tally(ctd_server *sv, uint64_t ticket, uint64_t n_voxels,
                                         int64_t *s1, uint64_t *s2_hi, uint64_t *s2_lo,
                                         uint32_t *n_batches) {
  if (!sv) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return CTD_ENOTFOUND;
  const Request *r = it->second.get();
  if (r->state != 2) return sv_err(sv, CTD_EBUSY, "request not done");
  const size_t V = r->s1.size();
  if (n_voxels != (uint64_t)V)
    return sv_err(sv, CTD_EINVAL, "arrays of %llu entries for a %llu-voxel phantom",
                  (unsigned long long)n_voxels, (unsigned long long)V);
  if (s1) std::memcpy(s1, r->s1.data(), 8 * V);
  if (s2_hi) std::memcpy(s2_hi, r->s2_hi.data(), 8 * V);
  if (s2_lo) std::memcpy(s2_lo, r->s2_lo.data(), 8 * V);
  if (n_batches) *n_batches = r->batches;
  return CTD_OK;
}

extern "C" int32_t ctd_server_release(ctd_server *sv, uint64_t ticket) {
  if (!sv) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return CTD_ENOTFOUND;
  if (it->second->state < 2) return sv_err(sv, CTD_EBUSY, "request still queued or running");
  sv->all.erase(it);
  sv->cv_done.notify_all();  // waiters on this ticket return CTD_ENOTFOUND
  return CTD_OK;
}

extern "C" int32_t ctd_server_read_stats(ctd_server *sv, ctd_server_stats *out) {
  if (!sv || !out) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->stats;
  out->queued = (uint32_t)sv->queue.size();
  out->active = (uint32_t)sv->active.size();
  out->resident_bytes = sv->used_bytes;
  return CTD_OK;
}

extern "C" int32_t ctd_server_stop(ctd_server *sv) {
  if (!sv) return CTD_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (Request *r : sv->queue) r->cancel = true;
    sv->cv_work.notify_all();
  }
  if (sv->th.joinable()) sv->th.join();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (Request *r : sv->queue) finish(sv, r, 3, CTD_ECANCELLED);
    sv->queue.clear();
    for (auto &kv : sv->phantoms)
      if (kv.second.dev) ctd_phantom_release(sv->ctx, kv.second.dev);
    sv->cv_done.notify_all();
  }
  ctd_destroy(sv->ctx);
  delete sv;
  return CTD_OK;
}
