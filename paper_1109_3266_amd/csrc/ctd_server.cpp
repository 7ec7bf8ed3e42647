// Dose-serving loop: continuous batching of run-to-sigma requests over the
// batched transport engine on one GPU.
//
// Two host threads, each with a private context on the device:
//
//  * the runner owns the transport stream.  Each iteration enqueues several
//    rounds back to back (up to kIterationHistories histories, kIterationRounds
//    rounds); a round gives every admitted request with planned batches left
//    one batch of the configured size in a single launch of the multi-case
//    kernel.  A request whose plan completes in a round gets its sigma-bar
//    reduction enqueued right behind that round, with the three results
//    copied to a pinned host slot, so the host waits once per iteration.
//    Then it stops the request or plans more batches, exactly as
//    ctd_run_to_sigma does alone.
//  * the host worker does the rest on a second stream while the rounds run:
//    admissions (phantom upload through pinned and device staging, packing,
//    case set-up) and the copy of finished requests' exact sums to host
//    memory.
//
// Freeing device memory waits for the whole device, so the runner frees the
// cases of finished requests once per iteration, after enqueueing the next
// one; nothing else is freed while rounds run except evicted phantoms and
// the staging buffers when a larger phantom first needs them.
//
// Requests queue in arrival order and are admitted while their device
// footprint (tallies, plus the phantom when it is not already resident) fits
// the budget; loaded phantoms stay resident and are evicted least-recently-
// used when an admission needs the room.  A request follows exactly the batch
// schedule of ctd_run_to_sigma (pilot of n_batches, then the shared sigma
// plan), and tallies depend only on a case's own batches, so each result is
// identical whether the request runs alone or among others.
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

// Work the runner enqueues between two host waits: about 20-40 ms of
// transport on MI355X, long next to the wait and the re-planning between
// iterations and short next to a request's seconds of service.  The round
// cap keeps an iteration within a context's 64 launch-table slots (up to
// three launches per round, one per step kind, when the requests mix them),
// so no launch of an iteration waits for an earlier one to free its slot.
constexpr uint64_t kIterationHistories = 200000000ull;
constexpr int kIterationRounds = 21;

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
  uint64_t planned = 0;      // batches the current plan runs to (runner)
  uint64_t footprint = 0;    // device bytes of the case
  int end_state = 0, end_status = CTD_OK;  // taken once the case is freed
  // progress, updated by the runner under the lock (poll reads these, never
  // the case, which the runner updates unlocked during an iteration)
  uint64_t histories = 0;
  uint32_t batches = 0;
  // results kept on the host after completion
  std::vector<int64_t> s1;
  std::vector<uint64_t> s2_hi, s2_lo;
};

// A pinned host or device buffer that only grows: freeing waits for the
// whole device, so it is replaced only when a larger size is first needed.
struct GrowBuf {
  void *p = nullptr;
  size_t cap = 0;
  bool host = false;
  hipError_t reserve(size_t bytes) {
    if (cap >= bytes) return hipSuccess;
    release();
    hipError_t e = host ? hipHostMalloc(&p, bytes, hipHostMallocDefault) : hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = bytes;
    return hipSuccess;
  }
  void release() {
    if (p) (void)(host ? hipHostFree(p) : hipFree(p));
    p = nullptr;
    cap = 0;
  }
};

}  // namespace

struct ctd_server {
  ctd_ctx *ctx = nullptr;   // the runner's: rounds, folds, sigma-bar checks
  ctd_ctx *aux = nullptr;   // the host worker's: admissions, result copies
  ctd_server_config cfg{};
  std::thread runner, worker;
  mutable std::mutex mu;   // guards everything below, err included
  std::condition_variable cv_run, cv_host, cv_done;
  std::deque<Request *> queue;     // submitted, not admitted
  std::vector<Request *> ready;    // admitted, joining the next iteration
  std::vector<Request *> active;   // in the rounds
  std::deque<Request *> readback;  // plan done at sigma-bar: sums to copy out
  std::vector<Request *> retire;   // cases to free before the final state
  std::map<uint64_t, std::unique_ptr<Request>> all;
  std::map<uint64_t, PhantomEntry> phantoms;
  uint64_t used_bytes = 0, next_ticket = 1, use_clock = 0;
  uint64_t free_epoch = 0;   // counts device frees: admissions waiting for room retry
  int64_t max_voxels = 0;    // largest registered phantom (sizes the staging)
  bool stop = false, runner_quiet = false, worker_done = false;
  std::string err;
  std::chrono::steady_clock::time_point t0;
  ctd_server_stats stats{};
  // runner only
  GrowBuf sig_host{nullptr, 0, true};
  // host worker only
  GrowBuf up_host{nullptr, 0, true}, up_dev{nullptr, 0, false}, rb_host{nullptr, 0, true};
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void wake() {
    cv_run.notify_all();
    cv_host.notify_all();
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

// ------------------------------------------------------------ both threads

// Final state of a request that holds no case.  Lock held.
static void complete(ctd_server *sv, Request *r, int state, int status) {
  r->state = state;
  r->status = status;
  r->t_done = sv->now();
  if (r->held) {
    r->ms->refs--;
    r->sp->refs--;
    r->geo->refs--;
    r->held = false;
  }
  if (state == 2) sv->stats.completed++;
  sv->cv_done.notify_all();
}

// Hand a request with a case to the runner, which frees the case and then
// gives the request its final state.  Lock held.
static void retire_later(ctd_server *sv, Request *r, int state, int status) {
  r->end_state = state;
  r->end_status = status;
  sv->retire.push_back(r);
  sv->cv_run.notify_all();
}

// ------------------------------------------------------------------ runner

// Free the cases of retiring requests (no lock: each free waits for the
// device).
static void free_cases(ctd_server *sv, const std::vector<Request *> &dead) {
  for (Request *r : dead) {
    if (!r->cs) continue;
    ctd_case_destroy(sv->ctx, r->cs);
    r->cs = nullptr;
  }
}

// Their final states, once the memory is back.  Lock held.
static void complete_retired(ctd_server *sv, const std::vector<Request *> &dead) {
  for (Request *r : dead) {
    sv->used_bytes -= r->footprint;
    r->footprint = 0;
    auto it = sv->phantoms.find(r->phantom_key);
    if (it != sv->phantoms.end()) it->second.users--;
    complete(sv, r, r->end_state, r->end_status);
  }
  if (!dead.empty()) {
    sv->free_epoch++;
    sv->cv_host.notify_all();   // an admission may fit now
  }
}

static void runner_loop(ctd_server *sv) {
  (void)hipSetDevice(sv->ctx->device);
  const uint64_t bh = sv->cfg.batch_histories;
  const uint64_t max_b = std::max<uint64_t>(sv->cfg.max_histories / bh, 2);
  std::vector<Request *> dead, act, checked;
  std::vector<int> check_rc;
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // admitted requests join; cancelled ones, and all of them on stop, leave
    for (Request *r : sv->ready) sv->active.push_back(r);
    sv->ready.clear();
    for (size_t i = 0; i < sv->active.size();) {
      Request *r = sv->active[i];
      if (r->cancel || sv->stop) {
        retire_later(sv, r, 3, CTD_ECANCELLED);
        sv->active.erase(sv->active.begin() + (long)i);
      } else {
        ++i;
      }
    }
    if (sv->stop && !sv->runner_quiet) {
      sv->runner_quiet = true;   // no more requests will reach the read-back list
      sv->cv_host.notify_all();
    }
    dead.clear();
    dead.swap(sv->retire);
    if (sv->active.empty()) {
      if (!dead.empty()) {
        lk.unlock();
        free_cases(sv, dead);
        lk.lock();
        complete_retired(sv, dead);
        continue;
      }
      if (sv->stop && sv->worker_done) break;
      sv->cv_run.wait(lk);
      continue;
    }
    act = sv->active;
    if (sv->sig_host.reserve(sizeof(double) * 4 * act.size()) != hipSuccess) {
      sv_err(sv, CTD_ENOMEM, "pinned sigma-bar slots");
      for (Request *r : act) retire_later(sv, r, 4, CTD_ENOMEM);
      sv->active.clear();
      sv->retire.insert(sv->retire.end(), dead.begin(), dead.end());
      continue;
    }
    double *slot = (double *)sv->sig_host.p;
    lk.unlock();

    // one iteration: rounds back to back, sigma-bar behind each completed plan
    int rc = CTD_OK;
    uint64_t hist = 0;
    int rounds = 0;
    checked.clear();
    check_rc.clear();
    std::vector<ctd_case *> cases;
    std::vector<Request *> reqs;
    while (rc == CTD_OK && rounds < kIterationRounds && hist < kIterationHistories) {
      cases.clear();
      reqs.clear();
      for (Request *r : act) {
        if (r->cs->batches < r->planned) {
          cases.push_back(r->cs);
          reqs.push_back(r);
        }
      }
      if (cases.empty()) break;
      const ctd_tuning t = sv->cfg.tuning.block ? sv->cfg.tuning : cases[0]->tune;
      rc = run_round(sv->ctx, cases, std::vector<uint64_t>(cases.size(), bh), t);
      if (rc != CTD_OK) break;
      ++rounds;
      hist += (uint64_t)cases.size() * bh;
      for (Request *r : reqs) {
        if (r->cs->batches < r->planned) continue;
        check_rc.push_back(sigma_async(sv->ctx, r->cs, sv->cfg.sigma_kind, sv->cfg.dose_frac,
                                       slot + 4 * checked.size()));
        checked.push_back(r);
      }
    }
    // retiring cases are freed while the iteration runs
    free_cases(sv, dead);
    if (hipStreamSynchronize(sv->ctx->stream) != hipSuccess && rc == CTD_OK) rc = CTD_EDEVICE;

    lk.lock();
    complete_retired(sv, dead);
    for (Request *r : act) {
      r->histories = r->cs->h_next;
      r->batches = r->cs->batches;
    }
    sv->stats.rounds += (uint64_t)rounds;
    sv->stats.histories += hist;
    if (rc != CTD_OK) {
      sv->err = ctd_last_error(sv->ctx);
      for (Request *r : act) retire_later(sv, r, 4, rc);
      sv->active.clear();
      continue;
    }
    for (size_t i = 0; i < checked.size(); ++i) {
      Request *r = checked[i];
      const double sig = check_rc[i] == CTD_OK ? slot[4 * i] : NAN;
      r->sigma = sig;
      const uint64_t more = std::isnan(sig) ? 0 : sigma_plan(r->cs->batches, sig, r->target, max_b);
      if (more > 0) {
        r->planned = r->cs->batches + more;
        continue;
      }
      sv->active.erase(std::find(sv->active.begin(), sv->active.end(), r));
      if (std::isnan(sig)) {
        if (check_rc[i] != CTD_OK) sv->err = ctd_last_error(sv->ctx);
        retire_later(sv, r, 4, check_rc[i] != CTD_OK ? check_rc[i] : CTD_EDEVICE);
      } else {
        sv->readback.push_back(r);
        sv->cv_host.notify_all();
      }
    }
    sv->cv_done.notify_all();   // progress
  }
}

// ------------------------------------------------------------- host worker

// Copy a finished request's exact sums to its host arrays through the pinned
// staging buffer, on the worker's stream.  No lock.
static int read_back(ctd_server *sv, Request *r, int64_t max_voxels) {
  ctd_ctx *aux = sv->aux;
  const ctd_case *cs = r->cs;
  const size_t V = (size_t)cs->ph->V;
  hipError_t e = sv->rb_host.reserve(24 * std::max<size_t>(V, (size_t)max_voxels));
  if (e != hipSuccess) return hip_err(aux, e, "pinned read-back buffer");
  char *h = (char *)sv->rb_host.p;
  if ((e = hipMemcpyAsync(h, cs->d_s1, 8 * V, hipMemcpyDeviceToHost, aux->stream)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(h + 8 * V, cs->d_s2, 16 * V, hipMemcpyDeviceToHost, aux->stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(aux->stream)) != hipSuccess)
    return hip_err(aux, e, "result read-back");
  const int64_t *s1 = (const int64_t *)h;
  const uint64_t *s2 = (const uint64_t *)(h + 8 * V);
  r->s1.assign(s1, s1 + V);
  r->s2_hi.resize(V);
  r->s2_lo.resize(V);
  for (size_t v = 0; v < V; ++v) {
    r->s2_lo[v] = s2[2 * v];
    r->s2_hi[v] = s2[2 * v + 1];
  }
  return CTD_OK;
}

// Upload a registered phantom through the pinned and device staging buffers
// (mat at 0, rho at the next 256-byte boundary) and pack it.  No lock.
static int load_phantom(ctd_server *sv, const PhantomEntry &e, int64_t max_voxels,
                        ctd_phantom **out) {
  ctd_ctx *aux = sv->aux;
  const size_t V = e.mat.size();
  const size_t Vm = std::max<size_t>(V, (size_t)max_voxels);
  const size_t off = (V + 255) & ~(size_t)255;
  const size_t bytes = off + 4 * V;
  hipError_t err = sv->up_host.reserve(((Vm + 255) & ~(size_t)255) + 4 * Vm);
  if (err == hipSuccess) err = sv->up_dev.reserve(((Vm + 255) & ~(size_t)255) + 4 * Vm);
  if (err != hipSuccess) return hip_err(aux, err, "phantom staging");
  char *h = (char *)sv->up_host.p;
  char *d = (char *)sv->up_dev.p;
  std::memcpy(h, e.mat.data(), V);
  std::memcpy(h + off, e.rho.data(), 4 * V);
  if ((err = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, aux->stream)) != hipSuccess)
    return hip_err(aux, err, "phantom upload");
  // packing runs behind the copy on the same stream and is waited for
  return ctd_phantom_load(aux, &e.g, (const uint8_t *)d, (const float *)(d + off),
                          CTD_MEM_DEVICE, out);
}

// Admit the request at the head of the queue if it fits (evicting unused
// resident phantoms, least recently used first, never its own).  Entered and
// left with the lock held; the device work runs unlocked.  Returns false
// when the request must wait for memory.
static bool admit_one(ctd_server *sv, std::unique_lock<std::mutex> &lk) {
  Request *r = sv->queue.front();
  PhantomEntry &e = sv->phantoms.find(r->phantom_key)->second;
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
    complete(sv, r, 4, CTD_ENOMEM);
    return true;
  }
  std::vector<ctd_phantom *> evict;
  uint64_t evict_bytes = 0;
  for (;;) {
    if (sv->used_bytes - evict_bytes + need <= sv->cfg.hbm_budget_bytes) break;
    PhantomEntry *victim = nullptr;
    for (auto &kv : sv->phantoms) {
      PhantomEntry &x = kv.second;
      if (&x != &e && x.dev && x.users == 0 &&
          std::find(evict.begin(), evict.end(), x.dev) == evict.end() &&
          (!victim || x.last_use < victim->last_use))
        victim = &x;
    }
    if (!victim) return false;   // wait for running requests to finish
    evict.push_back(victim->dev);
    evict_bytes += victim->dev_bytes;
  }
  for (auto &kv : sv->phantoms) {
    PhantomEntry &x = kv.second;
    if (x.dev && std::find(evict.begin(), evict.end(), x.dev) != evict.end()) {
      x.dev = nullptr;
      x.dev_bytes = 0;
      sv->stats.evictions++;
    }
  }
  sv->used_bytes = sv->used_bytes - evict_bytes + need;   // reserved while unlocked
  sv->queue.pop_front();
  ctd_phantom *ph = e.dev;
  const bool load = ph == nullptr;
  const int64_t max_voxels = sv->max_voxels;
  lk.unlock();

  for (ctd_phantom *x : evict) ctd_phantom_release(sv->aux, x);
  int rc = CTD_OK;
  if (load) rc = load_phantom(sv, e, max_voxels, &ph);
  ctd_case *cs = nullptr;
  if (rc == CTD_OK) rc = ctd_case_create(sv->aux, ph, r->ms, r->sp, r->geo, &r->p, &cs);
  if (rc == CTD_OK && sv->cfg.tuning.block) rc = ctd_set_tuning(sv->aux, cs, &sv->cfg.tuning);
  if (rc == CTD_OK && cs->d_mh_state) rc = ensure_mh_buffer(sv->aux, cs, sv->cfg.batch_histories);
  if (rc != CTD_OK && cs) {
    ctd_case_destroy(sv->aux, cs);
    cs = nullptr;
  }
  std::string msg = rc != CTD_OK ? ctd_last_error(sv->aux) : std::string();

  lk.lock();
  if (load) {
    if (ph) {   // loaded (the case may still have failed)
      e.dev = ph;
      e.dev_bytes = ph_bytes;
      sv->stats.phantom_loads++;
    } else {
      sv->used_bytes -= ph_bytes;
    }
  } else {
    sv->stats.phantom_hits++;
  }
  sv->free_epoch++;   // the evictions
  if (rc != CTD_OK) {
    sv->used_bytes -= case_bytes;
    sv->err = msg;
    complete(sv, r, 4, rc);
    return true;
  }
  e.users++;
  e.last_use = ++sv->use_clock;
  r->cs = cs;
  r->footprint = case_bytes;
  r->planned = std::min<uint64_t>((uint64_t)r->p.n_batches,
                                  std::max<uint64_t>(sv->cfg.max_histories /
                                                     sv->cfg.batch_histories, 2));
  r->state = 1;
  r->t_admit = sv->now();
  sv->ready.push_back(r);
  sv->cv_run.notify_all();
  return true;
}

static void worker_loop(ctd_server *sv) {
  (void)hipSetDevice(sv->aux->device);
  uint64_t blocked_at = ~0ull;   // free_epoch when the head request last did not fit
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    if (!sv->readback.empty()) {
      Request *r = sv->readback.front();
      sv->readback.pop_front();
      const int64_t max_voxels = sv->max_voxels;
      lk.unlock();
      const int rc = read_back(sv, r, max_voxels);
      std::string msg = rc != CTD_OK ? ctd_last_error(sv->aux) : std::string();
      lk.lock();
      if (rc != CTD_OK) sv->err = msg;
      retire_later(sv, r, rc == CTD_OK ? 2 : 4, rc);
      continue;
    }
    for (size_t i = 0; i < sv->queue.size();) {   // cancelled while queued
      Request *r = sv->queue[i];
      if (r->cancel) {
        sv->queue.erase(sv->queue.begin() + (long)i);
        complete(sv, r, 3, CTD_ECANCELLED);
      } else {
        ++i;
      }
    }
    if (sv->stop) {
      if (sv->runner_quiet) break;
      sv->cv_host.wait(lk);
      continue;
    }
    const bool slot_free =
        (int)(sv->ready.size() + sv->active.size()) < sv->cfg.max_active;
    if (sv->queue.empty() || !slot_free || blocked_at == sv->free_epoch) {
      sv->cv_host.wait(lk);
      continue;
    }
    if (!admit_one(sv, lk)) blocked_at = sv->free_epoch;
  }
  sv->worker_done = true;
  sv->cv_run.notify_all();
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
  if (rc == CTD_OK) rc = ctd_create(&sv->aux, device);
  if (rc != CTD_OK) {
    if (sv->ctx) ctd_destroy(sv->ctx);
    delete sv;
    return rc;
  }
  sv->cfg = *cfg;
  sv->t0 = std::chrono::steady_clock::now();
  try {
    sv->worker = std::thread(worker_loop, sv);
    sv->runner = std::thread(runner_loop, sv);
  } catch (...) {
    if (sv->worker.joinable()) {
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->runner_quiet = true;   // no runner: nothing will reach the read-back list
        sv->wake();
      }
      sv->worker.join();
    }
    ctd_destroy(sv->aux);
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
  sv->max_voxels = std::max(sv->max_voxels, V);
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
  sv->cv_host.notify_all();
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
  sv->wake();
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
  // admitted and not yet finished: joining, in the rounds, being read back or freed
  out->active = (uint32_t)(sv->ready.size() + sv->active.size() + sv->readback.size() +
                           sv->retire.size());
  out->resident_bytes = sv->used_bytes;
  return CTD_OK;
}

extern "C" int32_t ctd_server_stop(ctd_server *sv) {
  if (!sv) return CTD_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (Request *r : sv->queue) r->cancel = true;
    sv->wake();
  }
  // the runner finishes its iteration and cancels the admitted requests; the
  // worker copies out what had already reached its sigma-bar target
  if (sv->worker.joinable()) sv->worker.join();
  if (sv->runner.joinable()) sv->runner.join();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (Request *r : sv->queue) complete(sv, r, 3, CTD_ECANCELLED);
    sv->queue.clear();
    for (auto &kv : sv->phantoms)
      if (kv.second.dev) ctd_phantom_release(sv->aux, kv.second.dev);
    sv->cv_done.notify_all();
  }
  sv->sig_host.release();
  sv->up_host.release();
  sv->up_dev.release();
  sv->rb_host.release();
  ctd_destroy(sv->aux);
  ctd_destroy(sv->ctx);
  delete sv;
  return CTD_OK;
}
