// vopp_server.hip -- serving planning steps of many episodes with continuous
// batching.
//
// An episode keeps its planner workspace and its belief particles resident in
// HBM for its whole life.  Request t of an episode is one phase program:
//   t > 0:  execute the previous action in the simulated true environment,
//           then the SIR belief update (weight, scan, resample);
//   always: the planning step (set-up ... select) on the updated particles.
// Every tick issues up to phases_per_tick k_batch launches back to back, each
// advancing every active request by one phase.  Requests that arrive while others run simply join
// the next tick: new episodes are admitted as soon as a slot and HBM (the
// configured budget, counted over the resident footprints) are free, and an
// episode's next request is issued as soon as the server has seen the result
// of its previous one.  Results are read back per tick through a small ring
// of pinned buffers, so the host runs a few launches ahead of the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <vector>

#include "../../include/vopp.h"
#include "vopp_device.hpp"
#include "vopp_internal.hpp"
#include "vopp_launch.hpp"

using namespace vopp;

namespace {

constexpr int kMaxInflight = 8;
constexpr int kMaxPhasesPerTick = 64;

// Device resources of one resident episode (reused through a pool).
struct Resources {
  vopp_workspace* ws = nullptr;
  void* fbuf = nullptr;       // particles | moved particles | weights | env words
  size_t fbytes = 0;
};

struct Episode {
  vopp_episode_desc d{};
  char* init = nullptr;       // pinned copy of the initial particles
  size_t init_bytes = 0;
  int init_state[2] = {0, 0};
  int state_words = 1;
  int slot = -1;
  Resources res;
  size_t footprint = 0;
  int step = 0;               // current request
  std::vector<Phase> phases;  // its program
  size_t next = 0;            // next phase to issue
  bool waiting = false;       // select issued, result not seen yet
  bool new_view = false;      // view of the current request not uploaded yet
  double arrival = 0.0;
  bool admitted = false, finished = false;
  int* final_env = nullptr;   // pinned env words: initial state in, final state out
};

struct TickRec {
  hipEvent_t ev = nullptr;
  int ring = 0;               // ring slot of its item and result buffers
  std::vector<int> selects;   // episode ids whose select ran in this tick
};

}  // namespace

struct vopp_server {
  vopp_server_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  PlanView* views_dev = nullptr;
  PlanView* views_host = nullptr;       // pinned staging
  double* out_dev = nullptr;
  BatchItem* items_dev[kMaxInflight + 1] = {};
  BatchItem* items_host[kMaxInflight + 1] = {};
  double* out_host[kMaxInflight + 1] = {};
  hipEvent_t ev[kMaxInflight + 1] = {};
  int ring = 0;
  std::vector<Episode> eps;
  std::deque<int> queue;
  std::vector<int> slot_ep;
  size_t used = 0;
  std::deque<TickRec> inflight;
  std::vector<vopp_served> done;
  std::vector<Resources> pool;
  std::chrono::steady_clock::time_point t0;
};

namespace {

double now_s(const vopp_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

size_t filter_bytes(const Episode& e) {
  const size_t M = (size_t)e.d.n_particles;
  return 2 * M * 4 * e.state_words + M * 8 + 256 + 1024;
}

void free_resources(Resources& r) {
  if (r.ws) vopp_workspace_free(r.ws);
  if (r.fbuf) (void)hipFree(r.fbuf);
  r = Resources{};
}

// Take pooled resources that fit, else allocate.
vopp_status acquire(vopp_server* s, Episode& e) {
  const WsSizes need = sizes_for(e.d.pomdp, e.d.params.n_particles, e.d.budget, e.d.depth,
                                 e.d.params.schedule);
  const size_t fb = filter_bytes(e);
  for (size_t i = 0; i < s->pool.size(); ++i) {
    Resources& r = s->pool[i];
    if (fits(r.ws->z, need) && r.fbytes >= fb) {
      e.res = r;
      s->pool.erase(s->pool.begin() + i);
      return VOPP_OK;
    }
  }
  vopp_status st = vopp_workspace_create(e.d.pomdp, &e.d.params, e.d.budget, e.d.depth,
                                         &e.res.ws);
  if (st != VOPP_OK) return st;
  hipError_t err = hipMalloc(&e.res.fbuf, fb);
  if (err != hipSuccess) {
    free_resources(e.res);
    return fail(VOPP_E_NOMEM, "hipMalloc(particle buffers): %s", hipGetErrorString(err));
  }
  e.res.fbytes = fb;
  return VOPP_OK;
}

void release(vopp_server* s, Episode& e) {
  s->pool.push_back(e.res);
  e.res = Resources{};
  while (s->pool.size() > 64) {
    free_resources(s->pool.front());
    s->pool.erase(s->pool.begin());
  }
}

// Buffers inside fbuf.
void carve(const Episode& e, void** part, void** prop, unsigned long long** w, int** env) {
  const size_t M = (size_t)e.d.n_particles;
  char* b = (char*)e.res.fbuf;
  *env = (int*)b;
  *w = (unsigned long long*)(b + 256);
  *part = (void*)(b + 256 + M * 8);
  *prop = (void*)(b + 256 + M * 8 + M * 4 * e.state_words);
}

// The view and phase program of request e.step.
void start_request(vopp_server* s, Episode& e, double arrival) {
  vopp_params prm = e.d.params;
  prm.step = (uint32_t)e.step;
  void *part, *prop;
  unsigned long long* w;
  int* env;
  carve(e, &part, &prop, &w, &env);
  PlanView P = make_view(e.d.pomdp, e.res.ws, part, e.d.n_particles, e.d.budget, e.d.depth,
                         &prm);
  P.out = s->out_dev + (size_t)e.slot * kOutStride;
  P.f.part = part;
  P.f.prop = prop;
  P.f.w = w;
  P.f.M = e.d.n_particles;
  P.f.env = env;
  P.f.env_seed_lo = (uint32_t)e.d.env_seed;
  P.f.env_seed_hi = (uint32_t)(e.d.env_seed >> 32);
  s->views_host[e.slot] = P;
  e.phases.clear();
  if (e.step > 0) {
    const int t = e.step - 1;
    const int pb = (e.d.n_particles + kBlock - 1) / kBlock;
    e.phases.push_back({kPhaseEnv, t, 0, 1});
    e.phases.push_back({kPhasePFWeight, t, 0, pb});
    e.phases.push_back({kPhasePFScan, 0, 0, 1});
    e.phases.push_back({kPhasePFResample, t, 0, pb});
  }
  std::vector<Phase> plan = plan_phases(e.d.pomdp, P, kAccumCap, kBackupCap);
  e.phases.insert(e.phases.end(), plan.begin(), plan.end());
  e.next = 0;
  e.waiting = false;
  e.new_view = true;
  e.arrival = arrival;
}

vopp_status admit(vopp_server* s, int id) {
  Episode& e = s->eps[id];
  vopp_status st = acquire(s, e);
  if (st != VOPP_OK) return st;
  int slot = -1;
  for (int i = 0; i < (int)s->slot_ep.size(); ++i)
    if (s->slot_ep[i] < 0) { slot = i; break; }
  e.slot = slot;
  s->slot_ep[slot] = id;
  s->used += e.footprint;
  e.admitted = true;
  // Upload the iteration schedule, the initial particles and the true state.
  int* sb = e.res.ws->step_host;
  sb[0] = 0;
  for (int k = 1; k <= e.d.budget; ++k)
    sb[k] = sb[k - 1] + (e.d.params.schedule == VOPP_SCHEDULE_FIXED ? e.d.depth
                                                                    : std::min(k, e.d.depth));
  void *part, *prop;
  unsigned long long* w;
  int* env;
  carve(e, &part, &prop, &w, &env);
  // All sources are pinned and owned by this episode or its workspace, so the
  // copies can stay queued behind the launches in flight.
  int* env_init = e.final_env;
  env_init[0] = e.init_state[0];
  env_init[1] = e.init_state[1];
  for (int i = 2; i < 8; ++i) env_init[i] = 0;
  hipError_t err = hipMemcpyAsync(e.res.ws->step_base_dev, sb, (e.d.budget + 1) * sizeof(int),
                                  hipMemcpyHostToDevice, s->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(part, e.init, e.init_bytes, hipMemcpyHostToDevice, s->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(env, env_init, 8 * sizeof(int), hipMemcpyHostToDevice, s->stream);
  if (err != hipSuccess) return hip_fail(err, "episode admission");
  start_request(s, e, e.arrival);
  return VOPP_OK;
}

// Fold the oldest in-flight launch: read its results, issue next requests.
vopp_status harvest_one(vopp_server* s, bool wait) {
  if (s->inflight.empty()) return VOPP_OK;
  TickRec& tk = s->inflight.front();
  hipError_t err = wait ? hipEventSynchronize(tk.ev) : hipEventQuery(tk.ev);
  if (err == hipErrorNotReady) return VOPP_E_BUSY;
  if (err != hipSuccess) return hip_fail(err, "server launch");
  const double t = now_s(s);
  const double* outs = s->out_host[tk.ring];
  for (int id : tk.selects) {
    Episode& e = s->eps[id];
    const double* o = outs + (size_t)e.slot * kOutStride;
    const int A = e.d.pomdp->nA;
    vopp_served v;
    v.episode = id;
    v.step = e.step;
    v.action = (int32_t)o[0];
    const int flags = (int)o[A + 5];
    v.status = (flags & 2) ? VOPP_E_INTERNAL : (flags & 1) ? VOPP_E_INVALID : VOPP_OK;
    v.v_root = o[A + 1];
    v.particle_steps = (int64_t)o[A + 2];
    v.arrival_s = e.arrival;
    v.done_s = t;
    s->done.push_back(v);
    e.step += 1;
    if (e.step >= e.d.n_steps) {
      // Episode over: keep its final true state, free its slot and memory.
      void *part, *prop;
      unsigned long long* w;
      int* env;
      carve(e, &part, &prop, &w, &env);
      (void)hipMemcpyAsync(e.final_env, env, 8 * sizeof(int), hipMemcpyDeviceToHost, s->stream);
      s->slot_ep[e.slot] = -1;
      s->used -= e.footprint;
      e.slot = -1;
      e.finished = true;
      release(s, e);
    } else {
      start_request(s, e, t);
    }
  }
  s->inflight.pop_front();
  return VOPP_OK;
}

}  // namespace

extern "C" vopp_status vopp_server_create(const vopp_server_config* cfg, vopp_server** out) {
  clear_error();
  if (!cfg || !out) return fail(VOPP_E_INVALID, "null argument");
  *out = nullptr;
  if (cfg->max_active < 1 || cfg->max_active > 4096)
    return fail(VOPP_E_INVALID, "max_active must be in [1, 4096]");
  if (cfg->max_inflight < 1 || cfg->max_inflight > kMaxInflight)
    return fail(VOPP_E_INVALID, "max_inflight must be in [1, %d]", kMaxInflight);
  if (cfg->phases_per_tick < 0 || cfg->phases_per_tick > kMaxPhasesPerTick)
    return fail(VOPP_E_INVALID, "phases_per_tick must be in [0, %d]", kMaxPhasesPerTick);
  vopp_server* s = new vopp_server();
  s->cfg = *cfg;
  (void)hipGetDevice(&s->device);
  s->slot_ep.assign(cfg->max_active, -1);
  s->t0 = std::chrono::steady_clock::now();
  const size_t na = (size_t)cfg->max_active;
  hipError_t e = hipStreamCreate(&s->stream);                 // default priority
  if (e == hipSuccess) e = hipMalloc(&s->views_dev, na * sizeof(PlanView));
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&s->views_host, na * sizeof(PlanView), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&s->out_dev, na * kOutStride * sizeof(double));
  const size_t per_tick = (size_t)std::max(1, cfg->phases_per_tick);
  for (int k = 0; k <= cfg->max_inflight && e == hipSuccess; ++k) {
    e = hipMalloc(&s->items_dev[k], na * per_tick * sizeof(BatchItem));
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&s->items_host[k], na * per_tick * sizeof(BatchItem),
                        hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&s->out_host[k], na * kOutStride * sizeof(double),
                        hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    vopp_server_free(s);
    return hip_fail(e, "server set-up");
  }
  *out = s;
  return VOPP_OK;
}

extern "C" void vopp_server_free(vopp_server* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (Episode& e : s->eps) {
    if (!e.finished && e.admitted) free_resources(e.res);
    if (e.final_env) (void)hipHostFree(e.final_env);
    if (e.init) (void)hipHostFree(e.init);
  }
  for (Resources& r : s->pool) free_resources(r);
  for (int k = 0; k <= kMaxInflight; ++k) {
    if (s->items_dev[k]) (void)hipFree(s->items_dev[k]);
    if (s->items_host[k]) (void)hipHostFree(s->items_host[k]);
    if (s->out_host[k]) (void)hipHostFree(s->out_host[k]);
    if (s->ev[k]) (void)hipEventDestroy(s->ev[k]);
  }
  if (s->views_dev) (void)hipFree(s->views_dev);
  if (s->views_host) (void)hipHostFree(s->views_host);
  if (s->out_dev) (void)hipFree(s->out_dev);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

extern "C" vopp_status vopp_server_submit(vopp_server* s, const vopp_episode_desc* d,
                                          int32_t* episode) {
  clear_error();
  if (!s || !d || !episode) return fail(VOPP_E_INVALID, "null argument");
  vopp_status st = check_params(d->pomdp, &d->params, d->budget, d->depth);
  if (st != VOPP_OK) return st;
  if (!d->init_particles || d->n_particles < 1 || d->n_particles > (1 << 24))
    return fail(VOPP_E_INVALID, "bad initial particles");
  if (!d->true_state || d->n_steps < 1) return fail(VOPP_E_INVALID, "bad episode");
  if (d->pomdp->view.Apad > 16) return fail(VOPP_E_INVALID, "served models need |A| <= 16");
  if (d->pomdp->device != s->device) return fail(VOPP_E_INVALID, "model on another device");
  Episode e;
  e.d = *d;
  e.state_words = d->pomdp->kind == kTabular ? 1 : 2;
  const size_t bytes = (size_t)d->n_particles * 4 * e.state_words;
  std::memcpy(e.init_state, d->true_state, 4 * e.state_words);
  if (e.state_words == 1 && (e.init_state[0] < 0 || e.init_state[0] >= d->pomdp->view.nS))
    return fail(VOPP_E_INVALID, "true state outside [0, nS)");
  if (e.state_words == 1)
    for (int i = 0; i < d->n_particles; ++i) {
      const int v = ((const int*)d->init_particles)[i];
      if (v < 0 || v >= d->pomdp->view.nS)
        return fail(VOPP_E_INVALID, "initial particle outside [0, nS)");
    }
  e.footprint = vopp_plan_footprint(d->pomdp, &d->params, d->budget, d->depth) + filter_bytes(e);
  if (e.footprint > s->cfg.hbm_budget_bytes)
    return fail(VOPP_E_NOMEM, "episode footprint %zu exceeds the HBM budget", e.footprint);
  hipError_t err = hipHostMalloc((void**)&e.final_env, 8 * sizeof(int), hipHostMallocDefault);
  if (err == hipSuccess) err = hipHostMalloc((void**)&e.init, bytes, hipHostMallocDefault);
  if (err != hipSuccess) {
    if (e.final_env) (void)hipHostFree(e.final_env);
    return hip_fail(err, "hipHostMalloc");
  }
  std::memcpy(e.init, d->init_particles, bytes);
  e.init_bytes = bytes;
  std::memset(e.final_env, 0, 8 * sizeof(int));
  e.arrival = now_s(s);
  e.d.init_particles = nullptr;
  e.d.true_state = nullptr;
  s->eps.push_back(std::move(e));
  *episode = (int32_t)(s->eps.size() - 1);
  s->queue.push_back(*episode);
  return VOPP_OK;
}

extern "C" vopp_status vopp_server_tick(vopp_server* s, int32_t* pending) {
  clear_error();
  if (!s) return fail(VOPP_E_INVALID, "null server");
  // 1. Results of finished launches (wait only when the ring is full).
  while (!s->inflight.empty()) {
    const bool full = (int)s->inflight.size() >= s->cfg.max_inflight;
    vopp_status st = harvest_one(s, full);
    if (st == VOPP_E_BUSY) break;
    if (st != VOPP_OK) return st;
  }
  // 2. Admission by free slot and HBM budget, first come first served.
  int active = 0;
  for (int id : s->slot_ep) active += id >= 0 ? 1 : 0;
  while (!s->queue.empty() && active < s->cfg.max_active) {
    Episode& e = s->eps[s->queue.front()];
    if (s->used + e.footprint > s->cfg.hbm_budget_bytes) break;
    const int id = s->queue.front();
    s->queue.pop_front();
    vopp_status st = admit(s, id);
    if (st != VOPP_OK) return st;
    ++active;
  }
  // 3. Up to phases_per_tick launches, queued back to back: launch g runs the
  // next phase of every active request that has one and has not reached its
  // select in an earlier launch of this tick.
  const int k = s->ring;
  const int per_tick = std::max(1, s->cfg.phases_per_tick);
  const size_t na = s->slot_ep.size();
  BatchItem* items = s->items_host[k];
  TickRec tk;
  std::vector<int> lo, cnt, nblocks;
  int total = 0, amax = 4;
  hipError_t err = hipSuccess;
  // One request with phases to run: its phases go to the single-plan kernels
  // (no batch dispatch), as many as a tick takes.
  int pending_slot = -1, n_pending = 0;
  for (int slot = 0; slot < (int)na; ++slot) {
    const int id = s->slot_ep[slot];
    if (id < 0) continue;
    const Episode& e = s->eps[id];
    if (!e.waiting && e.next < e.phases.size()) {
      ++n_pending;
      pending_slot = slot;
    }
  }
  if (n_pending == 1) {
    const int id = s->slot_ep[pending_slot];
    Episode& e = s->eps[id];
    if (e.new_view) {
      err = hipMemcpyAsync(s->views_dev + pending_slot, s->views_host + pending_slot,
                           sizeof(PlanView), hipMemcpyHostToDevice, s->stream);
      if (err != hipSuccess) return hip_fail(err, "view upload");
      e.new_view = false;
    }
    const PlanView& P = s->views_host[pending_slot];
    for (int g = 0; g < per_tick && !e.waiting && e.next < e.phases.size() && err == hipSuccess;
         ++g) {
      const Phase& f = e.phases[e.next++];
      switch (f.kind) {
        case kPhaseSetup: err = launch_setup(P, s->stream); break;
        case kPhaseForward: err = launch_forward(P, f.a0, f.a1, s->stream); break;
        case kPhaseAccum: err = launch_accum(P, f.a0, f.nblk, s->stream); break;
        case kPhaseLeaf: err = launch_backup_leaf(P, f.a0, f.a1, f.nblk, s->stream); break;
        case kPhaseLevel: err = launch_backup_level(P, f.a0, f.a1, f.nblk, s->stream); break;
        case kPhaseRoot: err = launch_backup_root(P, f.a0, s->stream); break;
        case kPhaseEnv: err = launch_env(P, f.a0, s->stream); break;
        case kPhasePFWeight: err = launch_pf_part(P, 0, f.a0, s->stream); break;
        case kPhasePFScan: err = launch_pf_part(P, 1, f.a0, s->stream); break;
        case kPhasePFResample: err = launch_pf_part(P, 2, f.a0, s->stream); break;
        case kPhaseSelect:
          err = launch_select(P, s->stream);
          e.waiting = true;
          tk.selects.push_back(id);
          break;
        default: break;
      }
    }
    if (err == hipSuccess && !tk.selects.empty())
      err = hipMemcpyAsync(s->out_host[k], s->out_dev,
                           s->slot_ep.size() * kOutStride * sizeof(double),
                           hipMemcpyDeviceToHost, s->stream);
    if (err == hipSuccess) err = hipEventRecord(s->ev[k], s->stream);
    if (err != hipSuccess) return hip_fail(err, "server launch");
    tk.ev = s->ev[k];
    tk.ring = k;
    s->inflight.push_back(tk);
    s->ring = (s->ring + 1) % (s->cfg.max_inflight + 1);
    n_pending = -1;                         // issued
  }
  for (int g = 0; g < per_tick && n_pending >= 0; ++g) {
    int n = 0, blocks = 0;
    BatchItem* it = items + (size_t)g * na;
    for (int slot = 0; slot < (int)na; ++slot) {
      const int id = s->slot_ep[slot];
      if (id < 0) continue;
      Episode& e = s->eps[id];
      if (e.waiting || e.next >= e.phases.size()) continue;
      if (e.new_view) {
        err = hipMemcpyAsync(s->views_dev + slot, s->views_host + slot, sizeof(PlanView),
                             hipMemcpyHostToDevice, s->stream);
        if (err != hipSuccess) return hip_fail(err, "view upload");
        e.new_view = false;
      }
      const Phase& f = e.phases[e.next++];
      it[n] = BatchItem{slot, f.kind, f.a0, f.a1, blocks, f.nblk};
      blocks += f.nblk;
      ++n;
      amax = std::max(amax, e.d.pomdp->view.Apad);
      if (f.kind == kPhaseSelect) {
        e.waiting = true;
        tk.selects.push_back(id);
      }
    }
    if (n == 0) break;
    lo.push_back(g);
    cnt.push_back(n);
    nblocks.push_back(blocks);
    total = g + 1;
  }
  if (n_pending < 0) {
    // issued above
  } else if (total > 0) {
    err = hipMemcpyAsync(s->items_dev[k], items, (size_t)total * na * sizeof(BatchItem),
                         hipMemcpyHostToDevice, s->stream);
    for (size_t g = 0; g < lo.size() && err == hipSuccess; ++g)
      err = launch_batch(s->views_dev, s->items_dev[k] + (size_t)lo[g] * na, cnt[g],
                         nblocks[g], amax, s->stream);
    if (err == hipSuccess && !tk.selects.empty())
      err = hipMemcpyAsync(s->out_host[k], s->out_dev,
                           s->slot_ep.size() * kOutStride * sizeof(double),
                           hipMemcpyDeviceToHost, s->stream);
    if (err == hipSuccess) err = hipEventRecord(s->ev[k], s->stream);
    if (err != hipSuccess) return hip_fail(err, "server launch");
    tk.ev = s->ev[k];
    tk.ring = k;
    s->inflight.push_back(tk);
    s->ring = (s->ring + 1) % (s->cfg.max_inflight + 1);
  } else if (!s->inflight.empty()) {
    // Nothing to issue until a result arrives.
    vopp_status st = harvest_one(s, true);
    if (st != VOPP_OK) return st;
  }
  if (pending) {
    int p = (int)s->queue.size();
    for (int id : s->slot_ep) p += id >= 0 ? 1 : 0;
    *pending = p;
  }
  return VOPP_OK;
}

extern "C" int32_t vopp_server_poll(vopp_server* s, vopp_served* out, int32_t max) {
  if (!s || !out || max <= 0) return 0;
  const int n = std::min((int)s->done.size(), (int)max);
  std::copy(s->done.begin(), s->done.begin() + n, out);
  s->done.erase(s->done.begin(), s->done.begin() + n);
  return n;
}

extern "C" vopp_status vopp_server_episode_state(vopp_server* s, int32_t id, void* true_state,
                                                 int32_t* steps_done) {
  clear_error();
  if (!s || id < 0 || id >= (int)s->eps.size()) return fail(VOPP_E_INVALID, "bad episode");
  Episode& e = s->eps[id];
  hipError_t err = hipStreamSynchronize(s->stream);
  if (err != hipSuccess) return hip_fail(err, "episode state");
  int words[8] = {e.init_state[0], e.init_state[1], 0, 0, 0, 0, 0, 0};
  if (e.finished) {
    std::memcpy(words, e.final_env, sizeof(words));
  } else if (e.admitted) {
    void *part, *prop;
    unsigned long long* w;
    int* env;
    carve(e, &part, &prop, &w, &env);
    err = hipMemcpy(words, env, sizeof(words), hipMemcpyDeviceToHost);
    if (err != hipSuccess) return hip_fail(err, "episode state");
  }
  if (true_state) std::memcpy(true_state, words, 4 * e.state_words);
  if (steps_done) *steps_done = e.step;
  return VOPP_OK;
}
