// Serving loop: continuous batching of independent SPH events.
//
// Events of uneven particle count are submitted as they arrive.  A host
// worker thread admits them, first come first served, when a slot of the
// event table is free, a contiguous particle range and a contiguous cell
// range are free in the device arena, and their footprint fits the byte
// budget.  Every iteration advances all resident events by one Heun step with
// the same batched launches a single simulation uses; an event leaves when it
// reaches its end time, its state is copied to the host, its ranges are
// freed and newcomers are admitted at the next step boundary.  Events never
// interact: each has its own cell grid, sorted order and counters, so a
// result is bit-identical alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "ccake.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

using namespace ccake;

namespace {

// first-fit allocator over [0, cap)
struct RangeAlloc {
  int64_t cap = 0;
  std::vector<std::pair<int64_t, int64_t>> free_;  // (start, length), sorted by start
  void init(int64_t c) {
    cap = c;
    free_.assign(1, {0, c});
  }
  int64_t take(int64_t len) {
    for (size_t i = 0; i < free_.size(); ++i)
      if (free_[i].second >= len) {
        int64_t at = free_[i].first;
        free_[i].first += len;
        free_[i].second -= len;
        if (free_[i].second == 0) free_.erase(free_.begin() + i);
        return at;
      }
    return -1;
  }
  void give(int64_t at, int64_t len) {
    free_.push_back({at, len});
    std::sort(free_.begin(), free_.end());
    std::vector<std::pair<int64_t, int64_t>> m;
    for (auto& r : free_) {
      if (!m.empty() && m.back().first + m.back().second == r.first)
        m.back().second += r.second;
      else
        m.push_back(r);
    }
    free_ = m;
  }
  int64_t high_water() const {
    // end of the highest allocated range
    int64_t hw = cap;
    if (!free_.empty() && free_.back().first + free_.back().second == cap) hw = free_.back().first;
    return hw;
  }
};

struct Pending {
  int64_t ticket, tag, n;
  double t0, t_end, t_submit;
  int32_t dens_kind;
  std::vector<double> xi, u, dens;
};

struct Resident {
  bool used = false;
  int64_t ticket = 0, tag = 0, n = 0;
  int64_t p_base = 0, c_base = 0, c_cap = 0;
  size_t bytes = 0;
  int steps_total = 0, steps_done = 0;
  double t_submit = 0, t_admit = 0;
};

}  // namespace

struct ccake_server : Handle {
  ccake_config cfg;
  Params prm;
  EosDev eos;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  size_t budget = 0, used_bytes = 0, per_particle_bytes = 0;
  int64_t max_particles = 0, ccap = 0;
  int max_events = 0;
  double dt = 0;
  char* arena = nullptr;
  bool own_arena = false;  // allocated by the server (no caller workspace)
  Layout L;
  BatchDev b;
  double* h_stage = nullptr;  // pinned staging for uploads / downloads
  size_t h_stage_doubles = 0;
  RangeAlloc palloc, calloc_;
  std::vector<Resident> slots;
  std::deque<Pending> queue;
  std::vector<ccake_event_result> done;
  int64_t next_ticket = 1;
  int64_t outstanding = 0;
  int64_t steps = 0, particle_steps = 0;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::thread worker;
  bool stop = false;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

static size_t event_bytes(const ccake_server* s, int64_t n) {
  return s->per_particle_bytes * (size_t)n + 2 * sizeof(int32_t) * (size_t)(cell_capacity(s->cfg, n) + 1);
}

static ccake_status srv_hip(ccake_server* s, hipError_t e, const char* what) {
  if (e == hipSuccess) return CCAKE_OK;
  return fail(s, CCAKE_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Upload and initialise newly admitted events (all resident events are
// re-binned, which leaves their state unchanged).
static ccake_status admit_and_init(ccake_server* s, std::vector<std::pair<int, Pending>>& fresh) {
  if (fresh.empty()) return CCAKE_OK;
  const int D = s->prm.dim;
  for (auto& fp : fresh) {
    const int e = fp.first;
    Pending& p = fp.second;
    Resident& r = s->slots[e];
    const int64_t n = p.n;
    // rows x, u into the stage buffer (Y1 region), densities into rec region
    std::vector<double> up((size_t)NROW * n, 0.0);
    for (int d = 0; d < D; ++d) {
      memcpy(&up[(size_t)(R_X1 + d) * n], &p.xi[(size_t)d * n], n * sizeof(double));
      memcpy(&up[(size_t)(R_U1 + d) * n], &p.u[(size_t)d * n], n * sizeof(double));
    }
    ccake_status st;
    if ((st = srv_hip(s, hipMemcpyAsync(s->b.Y1, up.data(), up.size() * sizeof(double), hipMemcpyHostToDevice,
                                        s->stream), "upload")))
      return st;
    if ((st = srv_hip(s, hipMemcpyAsync(s->b.rec, p.dens.data(), p.dens.size() * sizeof(double),
                                        hipMemcpyHostToDevice, s->stream), "upload dens")))
      return st;
    EventDev E;
    memset(&E, 0, sizeof E);
    E.p_base = r.p_base;
    E.c_base = r.c_base;
    E.n = (int32_t)n;
    E.c_cap = (int32_t)r.c_cap;
    E.active = 1;
    E.t = p.t0;
    E.dt = s->dt;
    E.first_bad = INT32_MAX;
    E.edge = s->prm.cell_edge;
    E.rebin = 1;
    E.need_bin = 1;  // its first step bins, as a single simulation's does
    E.disp = 0.0;
    for (int k = 0; k < 3; ++k) {
      E.bb_min[k] = BB_EMPTY_MIN;
      E.bb_max[k] = BB_EMPTY_MAX;
    }
    if ((st = srv_hip(s, hipMemcpyAsync(s->b.evt + e, &E, sizeof E, hipMemcpyHostToDevice, s->stream), "event")))
      return st;
    std::vector<int32_t> ev((size_t)n, e);
    if ((st = srv_hip(s, hipMemcpyAsync(s->b.ev + r.p_base, ev.data(), n * sizeof(int32_t), hipMemcpyHostToDevice,
                                        s->stream), "slot map")))
      return st;
    if ((st = srv_hip(s, launch_upload(s->b, e, n, s->b.Y1, NROW, s->stream), "k_upload"))) return st;
    // the pageable sources must stay alive until the copies are done
    if ((st = srv_hip(s, hipStreamSynchronize(s->stream), "sync"))) return st;
    // initialise this event alone: bin it (the others keep their cells and
    // order), k_init restricted to it
    const int64_t nslots = s->palloc.high_water();
    if ((st = srv_hip(s, launch_bin_only(s->b, e, s->stream), "bin only"))) return st;
    if ((st = srv_hip(s, launch_bin(s->b, s->prm, s->max_events, nslots, n, 0x1FFFFu, s->stream), "bin"))) return st;
    if ((st = srv_hip(s, launch_init(s->b, s->prm, s->eos, p.dens_kind, s->b.rec, nslots, s->stream, e), "init")))
      return st;
    if ((st = srv_hip(s, launch_commit(s->b, nslots, 0x1FFFFu, s->stream), "commit"))) return st;
  }
  return CCAKE_OK;
}

static void finish_event(ccake_server* s, int e, ccake_status status) {
  Resident& r = s->slots[e];
  ccake_event_result res;
  memset(&res, 0, sizeof res);
  res.ticket = r.ticket;
  res.user_tag = r.tag;
  res.n = r.n;
  res.status = status;
  res.steps = r.steps_done;
  res.t_submit = r.t_submit;
  res.t_admit = r.t_admit;
  res.state = new double[(size_t)NROW * r.n];
  // state in the caller's order
  hipError_t he = launch_unsort(s->b, e, r.n, live_rows(s->prm), s->b.Y1, s->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(res.state, s->b.Y1, sizeof(double) * NROW * r.n, hipMemcpyDeviceToHost, s->stream);
  EventDev E;
  if (he == hipSuccess) he = hipMemcpyAsync(&E, s->b.evt + e, sizeof E, hipMemcpyDeviceToHost, s->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(s->stream);
  if (he != hipSuccess) res.status = CCAKE_E_HIP;
  else if (res.status == CCAKE_OK && E.nonfinite) res.status = CCAKE_E_NONFINITE;
  else if (res.status == CCAKE_OK && E.noconv) res.status = CCAKE_E_EOS_NOCONV;
  // a grid that no longer covers the event (coarsened to one cell, or no
  // finite coordinate) drops candidates: the result is not to be used
  else if (res.status == CCAKE_OK && E.capacity_err) res.status = CCAKE_E_CAPACITY;
  for (int64_t i = 0; i < r.n; ++i) {
    res.totals[0] += res.state[(size_t)R_S * r.n + i];
    for (int q = 0; q < 3; ++q) res.totals[1 + q] += res.state[(size_t)(R_NB + q) * r.n + i];
  }
  for (int k = 4; k < 8; ++k) res.totals[k] = NAN;
  // release the slot
  E.active = 0;
  (void)hipMemcpyAsync(s->b.evt + e, &E, sizeof E, hipMemcpyHostToDevice, s->stream);
  (void)hipMemsetAsync(s->b.ev + r.p_base, 0xFF, sizeof(int32_t) * r.n, s->stream);
  (void)hipStreamSynchronize(s->stream);
  res.t_finish = s->now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->palloc.give(r.p_base, r.n);
    s->calloc_.give(r.c_base, r.c_cap + 1);
    s->used_bytes -= r.bytes;
    s->done.push_back(res);
    s->outstanding -= 1;
    r = Resident();
  }
  s->cv_done.notify_all();
}

static void worker_loop(ccake_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    std::vector<std::pair<int, Pending>> fresh;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop) return;
      bool any_resident = false;
      for (auto& r : s->slots) any_resident = any_resident || r.used;
      if (!any_resident && s->queue.empty()) s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->stop) return;
      // first come, first served admission
      while (!s->queue.empty()) {
        Pending& p = s->queue.front();
        const size_t bytes = event_bytes(s, p.n);
        int e = -1;
        for (int k = 0; k < s->max_events; ++k)
          if (!s->slots[k].used) {
            e = k;
            break;
          }
        if (e < 0 || s->used_bytes + bytes > s->budget) break;
        const int64_t ccap = cell_capacity(s->cfg, p.n);
        const int64_t pb = s->palloc.take(p.n);
        if (pb < 0) break;
        const int64_t cb = s->calloc_.take(ccap + 1);
        if (cb < 0) {
          s->palloc.give(pb, p.n);
          break;
        }
        Resident& r = s->slots[e];
        r.used = true;
        r.ticket = p.ticket;
        r.tag = p.tag;
        r.n = p.n;
        r.p_base = pb;
        r.c_base = cb;
        r.c_cap = ccap;
        r.bytes = bytes;
        r.steps_total = (int)std::llround((p.t_end - p.t0) / s->dt);
        r.steps_done = 0;
        r.t_submit = p.t_submit;
        r.t_admit = s->now();
        s->used_bytes += bytes;
        fresh.emplace_back(e, std::move(p));
        s->queue.pop_front();
      }
    }
    ccake_status st = admit_and_init(s, fresh);
    if (st) {
      for (auto& fp : fresh) finish_event(s, fp.first, st);
      continue;
    }
    for (auto& fp : fresh)
      if (s->slots[fp.first].steps_total <= 0) finish_event(s, fp.first, CCAKE_OK);
    // one batched Heun step over every resident event
    int64_t resident_particles = 0, largest = 0;
    bool any = false;
    for (auto& r : s->slots)
      if (r.used) {
        any = true;
        resident_particles += r.n;
        largest = std::max<int64_t>(largest, r.n);
      }
    if (!any) continue;
    const int64_t nslots = s->palloc.high_water();
    hipError_t he = launch_schedule(s->b, s->cfg.skin, s->prm.hyperbolic && s->prm.dim == 3, s->stream);
    if (he == hipSuccess) he = launch_bin(s->b, s->prm, s->max_events, nslots, largest, live_rows(s->prm), s->stream);
    if (he == hipSuccess) he = launch_passes(s->b, s->prm, s->eos, nslots, 0, nullptr, nullptr, s->stream);
    if (he == hipSuccess) he = launch_advance(s->b, s->stream);
    s->steps += 1;
    s->particle_steps += resident_particles;
    for (int e = 0; e < s->max_events; ++e) {
      Resident& r = s->slots[e];
      if (!r.used) continue;
      r.steps_done += 1;
      if (he != hipSuccess)
        finish_event(s, e, CCAKE_E_HIP);
      else if (r.steps_done >= r.steps_total)
        finish_event(s, e, CCAKE_OK);
    }
  }
}

static int64_t server_cell_capacity(int64_t max_particles, int32_t max_events) {
  return 4 * max_particles + (int64_t)max_events * 8200;
}

extern "C" ccake_status ccake_server_workspace_bytes(const ccake_config* cfg, int64_t max_particles,
                                                     int32_t max_events, size_t* bytes) {
  std::string why;
  if (!bytes || !validate_config(cfg, &why) || max_particles <= 0 || max_events <= 0) return CCAKE_E_ARG;
  *bytes = make_layout(max_particles, server_cell_capacity(max_particles, max_events), max_events, cfg->dim).total;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_server_create(ccake_server** out, const ccake_config* cfg, const ccake_eos* eos,
                                            size_t budget_bytes, int64_t max_particles, int32_t max_events,
                                            double dt, void* stream, void* workspace, size_t ws_bytes) {
  std::string why;
  if (!out || !eos || !validate_config(cfg, &why) || max_particles <= 0 || max_events <= 0 || !(dt > 0.0))
    return CCAKE_E_ARG;
  if (workspace && (((uintptr_t)workspace & 255u) != 0 ||
                    ws_bytes < make_layout(max_particles, server_cell_capacity(max_particles, max_events),
                                           max_events, cfg->dim).total))
    return CCAKE_E_ARG;
  if (eos->dev.kind == EOS_CONFORMAL && cfg->ncharge != 0) return CCAKE_E_ARG;
  if (eos->dev.inv.val && eos->dev.inv.ncharge != cfg->ncharge) return CCAKE_E_ARG;
  if (2.0 * dt * (cfg->dim == 3 && cfg->coords == CCAKE_HYPERBOLIC ? 2.0 : 1.0) > cfg->skin) return CCAKE_E_ARG;
  ccake_server* s = new ccake_server();
  s->magic = HANDLE_SERVER;
  s->cfg = *cfg;
  s->prm = to_params(*cfg);
  s->eos = eos->dev;
  s->dt = dt;
  s->max_particles = max_particles;
  s->max_events = max_events;
  s->ccap = server_cell_capacity(max_particles, max_events);
  s->L = make_layout(max_particles, s->ccap, max_events, cfg->dim);
  // bytes per resident particle of the arena (everything but the cells)
  s->per_particle_bytes = (s->L.cs) / (size_t)max_particles + 1;
  s->budget = budget_bytes;
  (void)hipGetDevice(&s->device);
  if (stream) {
    s->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return CCAKE_E_HIP;
    }
    s->own_stream = true;
  }
  if (workspace) {
    s->arena = (char*)workspace;
  } else if (hipMalloc((void**)&s->arena, s->L.total) == hipSuccess) {
    s->own_arena = true;
  } else {
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return CCAKE_E_NOMEM;
  }
  s->b = bind_batch(s->arena, s->L, max_particles, s->ccap, max_events, cfg->dim);
  (void)hipMemset(s->b.ev, 0xFF, sizeof(int32_t) * max_particles);
  (void)hipMemset(s->b.evt, 0, sizeof(EventDev) * max_events);
  (void)hipMemset(s->b.cell_fill, 0, sizeof(int32_t) * (s->ccap + 1));
  (void)hipMemset(s->b.fo_mark, 0xFF, sizeof(int32_t) * max_particles);
  (void)hipMemset(s->b.fo_ctr, 0, 2 * sizeof(uint32_t));
  (void)hipDeviceSynchronize();
  s->palloc.init(max_particles);
  s->calloc_.init(s->ccap + max_events);
  s->slots.assign(max_events, Resident());
  s->t0 = std::chrono::steady_clock::now();
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_server_submit(ccake_server* s, const ccake_event_desc* ev, int64_t* ticket) {
  if (!s) return CCAKE_E_ARG;
  if (!ev || !ticket || ev->n <= 0 || !ev->xi || !ev->u || !ev->dens || !(ev->t_end >= ev->t0) ||
      (ev->dens_kind != 0 && ev->dens_kind != 1) || (s->prm.hyperbolic && !(ev->t0 > 0.0)))
    return fail(s, CCAKE_E_ARG, "ccake_server_submit: bad event");
  if (s->prm.hyperbolic && s->prm.dim == 3 && 2.0 * s->dt * std::fmax(1.0, 1.0 / ev->t0) > s->cfg.skin)
    return fail(s, CCAKE_E_ARG, "ccake_server_submit: skin below 2 dt / tau0 for this event");
  if (ev->n > s->max_particles || event_bytes(s, ev->n) > s->budget)
    return fail(s, CCAKE_E_CAPACITY, "event of %lld particles can never fit", (long long)ev->n);
  const int D = s->prm.dim;
  Pending p;
  p.n = ev->n;
  p.t0 = ev->t0;
  p.t_end = ev->t_end;
  p.tag = ev->user_tag;
  p.dens_kind = ev->dens_kind;
  p.xi.assign(ev->xi, ev->xi + (size_t)D * ev->n);
  p.u.assign(ev->u, ev->u + (size_t)D * ev->n);
  p.dens.assign(ev->dens, ev->dens + (size_t)4 * ev->n);
  for (double v : p.xi)
    if (!std::isfinite(v)) return fail(s, CCAKE_E_ARG, "non-finite position");
  for (double v : p.u)
    if (!std::isfinite(v)) return fail(s, CCAKE_E_ARG, "non-finite flow");
  for (int64_t i = 0; i < 4 * ev->n; ++i)
    if (!std::isfinite(p.dens[i]) || (i < ev->n && !(p.dens[i] > 0.0)))
      return fail(s, CCAKE_E_ARG, "bad density of particle %lld", (long long)(i % ev->n));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    p.ticket = s->next_ticket++;
    p.t_submit = s->now();
    *ticket = p.ticket;
    s->queue.push_back(std::move(p));
    s->outstanding += 1;
  }
  s->cv.notify_all();
  return CCAKE_OK;
}

extern "C" ccake_status ccake_server_poll(ccake_server* s, ccake_event_result* res, int32_t cap, int32_t* count) {
  if (!s || !count || (cap > 0 && !res)) return CCAKE_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t k = 0;
  while (k < cap && !s->done.empty()) {
    res[k++] = s->done.front();
    s->done.erase(s->done.begin());
  }
  *count = k;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_server_drain(ccake_server* s) {
  if (!s) return CCAKE_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
  return CCAKE_OK;
}

extern "C" ccake_status ccake_server_release(ccake_server* s, ccake_event_result* res) {
  if (!s || !res) return CCAKE_E_ARG;
  delete[] res->state;
  res->state = nullptr;
  return CCAKE_OK;
}

extern "C" ccake_status ccake_server_stats(ccake_server* s, double* now, int64_t* steps, int64_t* particle_steps,
                                           int32_t* resident) {
  if (!s) return CCAKE_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (now) *now = s->now();
  if (steps) *steps = s->steps;
  if (particle_steps) *particle_steps = s->particle_steps;
  if (resident) {
    int32_t r = 0;
    for (auto& x : s->slots) r += x.used ? 1 : 0;
    *resident = r;
  }
  return CCAKE_OK;
}

extern "C" ccake_status ccake_server_destroy(ccake_server* s) {
  if (!s) return CCAKE_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipStreamSynchronize(s->stream);
  for (auto& r : s->done) delete[] r.state;
  if (s->arena && s->own_arena) (void)hipFree(s->arena);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return CCAKE_OK;
}
