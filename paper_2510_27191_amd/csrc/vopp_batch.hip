// vopp_batch.hip -- batched planning: many independent instances advanced
// together.
//
// Each instance's plan is a fixed list of phases (set-up; per iteration the
// forward search, the accumulate sweep, the leaf sweep, one sweep per depth,
// the root; finally select), each split into tiles (one block's share).
//   - Persistent launch: one kernel whose blocks take tiles
//     from a device queue; every instance moves through its own phases as
//     soon as its previous phase's tiles are done, so short and long
//     instances do not wait for each other.  Captured with the queue reset in
//     one hipGraph.
//   - Per-phase launches: launch g runs the g-th phase of every instance
//     that still has one; the sequence is captured in a hipGraph or issued
//     eagerly.
// The autotuner times both (the persistent launch over its tile sizes, the
// per-phase graph over its block caps) and VOPP_BATCH_AUTO then runs the
// faster; before any autotuning it runs the persistent launch.
// Instances share no state, so each result is the same as that of a plain
// vopp_plan call with the same inputs, in every mode and for every tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/vopp.h"
#include "vopp_device.hpp"
#include "vopp_internal.hpp"
#include "vopp_launch.hpp"

using namespace vopp;

struct vopp_batch {
  int n = 0;
  int device = 0;
  std::vector<vopp_request> reqs;
  std::vector<vopp_workspace*> ws;
  std::vector<PlanView> views;
  PlanView* views_dev = nullptr;
  std::vector<BatchItem> items;          // all launches, concatenated
  std::vector<int> launch_off, launch_items, launch_blocks;
  BatchItem* items_dev = nullptr;
  double* out_dev = nullptr;
  double* out_host = nullptr;            // pinned
  int amax = 4;
  vopp_tuning tuning{kAccumCap, kBackupCap, 0, 1, 4};
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_in = nullptr;
  hipGraph_t graph = nullptr;             // the per-phase launch sequence
  hipGraphExec_t exec = nullptr;
  // The persistent launch: every instance's phases, its queue state, and the
  // graph of (queue reset, persistent kernel).
  BatchItem* ph_dev = nullptr;
  int* ph_off_dev = nullptr;
  unsigned long long* word_dev = nullptr;
  unsigned int* done_dev = nullptr;       // [n] then the finished counter
  int n_cu = 0;
  int persist_blocks = 0;
  int auto_mode = VOPP_BATCH_PERSISTENT;  // what VOPP_BATCH_AUTO runs
  hipGraph_t pgraph = nullptr;
  hipGraphExec_t pexec = nullptr;
};

namespace vopp {

std::vector<Phase> plan_phases(const vopp_pomdp* p, const PlanView& P, int accum_cap,
                               int backup_cap) {
  std::vector<Phase> ph;
  const int K = P.K;
  std::vector<int> D(K + 1, 0);
  for (int k = 1; k <= K; ++k)
    D[k] = P.schedule == VOPP_SCHEDULE_FIXED ? P.depth : std::min(k, P.depth);
  ph.push_back({kPhaseSetup, 0, 0, setup_blocks(P)});
  int t = 0;
  for (int k = 1; k <= K; ++k) {
    ph.push_back({kPhaseForward, k, D[k], forward_blocks(P)});
    ph.push_back({kPhaseAccum, D[k], 0, accum_blocks(P, D[k], accum_cap)});
    t += D[k];
    ph.push_back({kPhaseLeaf, D[k], k, backup_grid(p, P.n_p, D.data(), D[k], k, backup_cap)});
    for (int dep = D[k]; dep >= 2; --dep)
      ph.push_back({kPhaseLevel, dep, k, backup_grid(p, P.n_p, D.data(), dep - 1, k, backup_cap)});
    ph.push_back({kPhaseRoot, k, 0, 1});
  }
  ph.push_back({kPhaseSelect, 0, 0, 1});
  return ph;
}

}  // namespace vopp

namespace {

void release_graph(vopp_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->pexec) (void)hipGraphExecDestroy(b->pexec);
  if (b->pgraph) (void)hipGraphDestroy(b->pgraph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->pexec = nullptr;
  b->pgraph = nullptr;
}

PersistView persist_view(const vopp_batch* b) {
  PersistView V;
  V.word = b->word_dev;
  V.done = b->done_dev;
  V.finished = b->done_dev + b->n;
  V.phases = b->ph_dev;
  V.ph_off = b->ph_off_dev;
  V.n = b->n;
  return V;
}

// Build views and the launch schedule for the current tuning; upload them.
vopp_status build_schedule(vopp_batch* b) {
  const int n = b->n;
  b->views.assign(n, PlanView{});
  std::vector<std::vector<Phase>> phases(n);
  size_t longest = 0;
  for (int i = 0; i < n; ++i) {
    const vopp_request& r = b->reqs[i];
    PlanView P = make_view(r.pomdp, b->ws[i], r.belief_particles, r.n_belief, r.budget,
                           r.depth, &r.params);
    P.out = b->out_dev + (size_t)i * kOutStride;
    b->views[i] = P;
    phases[i] = plan_phases(r.pomdp, P, b->tuning.accum_cap, b->tuning.backup_cap);
    longest = std::max(longest, phases[i].size());
  }
  b->items.clear();
  b->launch_off.clear();
  b->launch_items.clear();
  b->launch_blocks.clear();
  for (size_t g = 0; g < longest; ++g) {
    int blocks = 0, cnt = 0;
    b->launch_off.push_back((int)b->items.size());
    for (int i = 0; i < n; ++i) {
      if (g >= phases[i].size()) continue;
      const Phase& f = phases[i][g];
      BatchItem it;
      it.inst = i;
      it.kind = f.kind;
      it.a0 = f.a0;
      it.a1 = f.a1;
      it.blk0 = blocks;
      it.nblk = f.nblk;
      blocks += f.nblk;
      b->items.push_back(it);
      ++cnt;
    }
    b->launch_items.push_back(cnt);
    b->launch_blocks.push_back(blocks);
  }
  // The persistent launch's queue: each instance's phases in order, with
  // tiles sized by work: a sweep tile covers sweep_group chunks of record
  // positions (or trace items), a forward tile forward_group blocks of
  // episodes, so the phases of large instances get many tiles and those of
  // small ones few.
  std::vector<BatchItem> ph;
  std::vector<int> ph_off(1, 0);
  const int big = 1 << 30;
  for (int i = 0; i < n; ++i) {
    const vopp_request& r = b->reqs[i];
    for (const Phase& f0 : plan_phases(r.pomdp, b->views[i], big, big)) {
      Phase f = f0;
      if (f.kind == kPhaseAccum || f.kind == kPhaseLeaf || f.kind == kPhaseLevel) {
        const int g = std::max(1, b->tuning.sweep_group);
        f.nblk = (f.nblk + g - 1) / g;
      }
      BatchItem it;
      it.inst = i;
      it.kind = f.kind;
      it.a0 = f.a0;
      it.a1 = f.a1;
      it.blk0 = 0;
      it.nblk = f.nblk;
      if (f.kind == kPhaseForward) {        // fewer, larger forward tiles
        const int g = std::max(1, b->tuning.forward_group);
        it.blk0 = f.nblk;
        it.nblk = (f.nblk + g - 1) / g;
      } else if (f.kind == kPhaseSetup) {   // set-up strides over its table fill
        const int g = std::max(1, b->tuning.sweep_group);
        it.nblk = (f.nblk + g - 1) / g;
      }
      ph.push_back(it);
    }
    ph_off.push_back((int)ph.size());
  }
  const int per_cu = persistent_blocks_per_cu(b->amax);
  const int want = b->tuning.blocks_per_cu > 0 ? std::min(b->tuning.blocks_per_cu, per_cu) : per_cu;
  b->persist_blocks = std::max(1, want * b->n_cu);
  hipError_t e = hipSuccess;
  if (b->ph_dev) (void)hipFree(b->ph_dev);
  b->ph_dev = nullptr;
  e = hipMalloc(&b->ph_dev, ph.size() * sizeof(BatchItem));
  if (e == hipSuccess)
    e = hipMemcpy(b->ph_dev, ph.data(), ph.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->ph_off_dev, ph_off.data(), ph_off.size() * sizeof(int),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch queue upload");
  if (b->items_dev) (void)hipFree(b->items_dev);
  b->items_dev = nullptr;
  e = hipMalloc(&b->items_dev, b->items.size() * sizeof(BatchItem));
  if (e == hipSuccess)
    e = hipMemcpy(b->items_dev, b->items.data(), b->items.size() * sizeof(BatchItem),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->views_dev, b->views.data(), n * sizeof(PlanView), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch schedule upload");
  return VOPP_OK;
}

hipError_t enqueue_launches(vopp_batch* b, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (size_t g = 0; g < b->launch_items.size() && e == hipSuccess; ++g)
    e = launch_batch(b->views_dev, b->items_dev + b->launch_off[g], b->launch_items[g],
                     b->launch_blocks[g], b->amax, s);
  return e;
}

vopp_status capture(vopp_batch* b) {
  release_graph(b);
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  hipError_t e2 = enqueue_launches(b, b->stream);
  e = hipStreamEndCapture(b->stream, &b->graph);
  if (e2 != hipSuccess) return hip_fail(e2, "batched launch during capture");
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  // The persistent launch: the queue reset (a kernel, not a memset node) and
  // the persistent kernel, one graph.
  e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  e2 = launch_persistent(b->views_dev, persist_view(b), b->persist_blocks, b->amax, b->stream);
  e = hipStreamEndCapture(b->stream, &b->pgraph);
  if (e2 != hipSuccess) return hip_fail(e2, "persistent launch during capture");
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->pexec, b->pgraph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return VOPP_OK;
}

void parse_results(const vopp_batch* b, vopp_result* res) {
  for (int i = 0; i < b->n; ++i) {
    const double* o = b->out_host + (size_t)i * kOutStride;
    const int A = b->reqs[i].pomdp->nA;
    vopp_result& r = res[i];
    std::memset(&r, 0, sizeof(r));
    r.action = (int32_t)o[0];
    for (int j = 0; j < A; ++j) r.values[j] = o[1 + j];
    r.v_root = o[A + 1];
    r.particle_steps = (int64_t)o[A + 2];
    r.n_beliefs = (int64_t)o[A + 3];
    r.n_actions = (int64_t)o[A + 4];
    const int flags = (int)o[A + 5];
    r.status = (flags & 2) ? VOPP_E_INTERNAL : (flags & 1) ? VOPP_E_INVALID : VOPP_OK;
  }
}

}  // namespace

extern "C" size_t vopp_batch_footprint(const vopp_request* reqs, int32_t n) {
  if (!reqs || n < 1) return 0;
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    const size_t f = vopp_plan_footprint(reqs[i].pomdp, &reqs[i].params, reqs[i].budget,
                                         reqs[i].depth);
    if (f == 0) return 0;
    total += f;
  }
  return total;
}

extern "C" void vopp_batch_free(vopp_batch* b) {
  if (!b) return;
  release_graph(b);
  for (vopp_workspace* w : b->ws) vopp_workspace_free(w);
  if (b->views_dev) (void)hipFree(b->views_dev);
  if (b->items_dev) (void)hipFree(b->items_dev);
  if (b->ph_dev) (void)hipFree(b->ph_dev);
  if (b->ph_off_dev) (void)hipFree(b->ph_off_dev);
  if (b->word_dev) (void)hipFree(b->word_dev);
  if (b->done_dev) (void)hipFree(b->done_dev);
  if (b->out_dev) (void)hipFree(b->out_dev);
  if (b->out_host) (void)hipHostFree(b->out_host);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

extern "C" vopp_status vopp_batch_create(const vopp_request* reqs, int32_t n,
                                         const vopp_tuning* tuning, vopp_batch** out) {
  clear_error();
  if (!out) return fail(VOPP_E_INVALID, "null out");
  *out = nullptr;
  if (!reqs || n < 1) return fail(VOPP_E_INVALID, "empty batch");
  int dev = 0;
  (void)hipGetDevice(&dev);
  int amax = 4;
  for (int i = 0; i < n; ++i) {
    const vopp_request& r = reqs[i];
    vopp_status st = check_params(r.pomdp, &r.params, r.budget, r.depth);
    if (st != VOPP_OK) return fail(st, "request %d: %s", i, vopp_last_error());
    if (!r.belief_particles || r.n_belief < 1)
      return fail(VOPP_E_INVALID, "request %d: empty belief", i);
    if (r.pomdp->device != dev)
      return fail(VOPP_E_INVALID, "request %d: model lives on another device", i);
    if (r.pomdp->view.Apad > 16)
      return fail(VOPP_E_INVALID, "request %d: batched plans support |A| <= 16", i);
    amax = std::max(amax, r.pomdp->view.Apad);
  }
  if (tuning && (tuning->accum_cap < 1 || tuning->backup_cap < 1 ||
                 tuning->blocks_per_cu < 0 || tuning->forward_group < 1 ||
                 tuning->sweep_group < 1))
    return fail(VOPP_E_INVALID, "bad tuning");
  vopp_batch* b = new vopp_batch();
  b->n = n;
  b->device = dev;
  b->amax = amax;
  b->reqs.assign(reqs, reqs + n);
  if (tuning) b->tuning = *tuning;
  b->ws.assign(n, nullptr);
  for (int i = 0; i < n; ++i) {
    vopp_status st = vopp_workspace_create(reqs[i].pomdp, &reqs[i].params, reqs[i].budget,
                                           reqs[i].depth, &b->ws[i]);
    if (st != VOPP_OK) {
      vopp_batch_free(b);
      return st;
    }
    // Upload the instance's iteration schedule once.
    int* sb = b->ws[i]->step_host;
    sb[0] = 0;
    for (int k = 1; k <= reqs[i].budget; ++k)
      sb[k] = sb[k - 1] + (reqs[i].params.schedule == VOPP_SCHEDULE_FIXED
                               ? reqs[i].depth
                               : std::min(k, reqs[i].depth));
    hipError_t e = hipMemcpy(b->ws[i]->step_base_dev, sb, (reqs[i].budget + 1) * sizeof(int),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      vopp_batch_free(b);
      return hip_fail(e, "batch schedule");
    }
  }
  hipError_t e = hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess && b->n_cu < 1) b->n_cu = 1;
  if (e == hipSuccess) e = hipMalloc(&b->views_dev, n * sizeof(PlanView));
  if (e == hipSuccess) e = hipMalloc(&b->ph_off_dev, (size_t)(n + 1) * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&b->word_dev, (size_t)n * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&b->done_dev, (size_t)(n + 1) * sizeof(unsigned int));
  if (e == hipSuccess) e = hipMalloc(&b->out_dev, (size_t)n * kOutStride * sizeof(double));
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&b->out_host, (size_t)n * kOutStride * sizeof(double),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreate(&b->stream);   // default priority
  if (e == hipSuccess) e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e == hipSuccess) e = hipEventCreate(&b->ev_in);
  if (e != hipSuccess) {
    vopp_batch_free(b);
    return hip_fail(e, "batch set-up");
  }
  vopp_status st = build_schedule(b);
  if (st == VOPP_OK) st = capture(b);
  if (st != VOPP_OK) {
    vopp_batch_free(b);
    return st;
  }
  *out = b;
  return VOPP_OK;
}

extern "C" vopp_status vopp_batch_set_request(vopp_batch* b, int32_t i, const void* belief,
                                              int32_t n_belief, uint64_t seed, uint32_t step) {
  clear_error();
  if (!b || i < 0 || i >= b->n) return fail(VOPP_E_INVALID, "bad batch index");
  if (!belief || n_belief < 1) return fail(VOPP_E_INVALID, "empty belief");
  vopp_request& r = b->reqs[i];
  r.belief_particles = belief;
  r.n_belief = n_belief;
  r.params.seed = seed;
  r.params.step = step;
  PlanView& P = b->views[i];
  P.e.belief = belief;
  P.e.n_belief = n_belief;
  P.seed_lo = (uint32_t)seed;
  P.seed_hi = (uint32_t)(seed >> 32);
  P.step = step;
  hipError_t e = hipMemcpy(b->views_dev + i, &P, sizeof(PlanView), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch request update");
  return VOPP_OK;
}

extern "C" vopp_status vopp_batch_run(vopp_batch* b, void* stream, int32_t mode,
                                      vopp_result* results, double* device_ms) {
  clear_error();
  if (!b || !results) return fail(VOPP_E_INVALID, "null argument");
  if (mode != VOPP_BATCH_EAGER && mode != VOPP_BATCH_GRAPH && mode != VOPP_BATCH_PERSISTENT &&
      mode != VOPP_BATCH_AUTO)
    return fail(VOPP_E_INVALID, "unknown batch mode %d", mode);
  if (mode == VOPP_BATCH_AUTO) mode = b->auto_mode;
  hipError_t e = hipEventRecord(b->ev_in, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
  if (e == hipSuccess) e = hipEventRecord(b->ev0, b->stream);
  if (e == hipSuccess) {
    if (mode == VOPP_BATCH_PERSISTENT) e = hipGraphLaunch(b->pexec, b->stream);
    else if (mode == VOPP_BATCH_GRAPH) e = hipGraphLaunch(b->exec, b->stream);
    else e = enqueue_launches(b, b->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(b->ev1, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->out_host, b->out_dev, (size_t)b->n * kOutStride * sizeof(double),
                       hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    // The tables of every instance are in an unknown state now.
    const unsigned long long one = 1ull;
    for (vopp_workspace* w : b->ws) (void)hipMemcpy(&w->tree.counters[3], &one, 8, hipMemcpyHostToDevice);
    return hip_fail(e, "batch execution");
  }
  if (device_ms) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
    *device_ms = ms;
  }
  parse_results(b, results);
  for (int i = 0; i < b->n; ++i)
    if (results[i].status == VOPP_E_INTERNAL)
      return fail(VOPP_E_INTERNAL, "request %d: belief table overflow", i);
    else if (results[i].status != VOPP_OK)
      return fail(VOPP_E_INVALID, "request %d: a belief particle holds a state outside [0, nS)", i);
  return VOPP_OK;
}

extern "C" int32_t vopp_batch_num_launches(const vopp_batch* b) {
  return b ? (int32_t)b->launch_items.size() : 0;
}

extern "C" int32_t vopp_batch_auto_mode(const vopp_batch* b) {
  return b ? (int32_t)b->auto_mode : -1;
}

// Times `mode` on the batch's present schedule: the best of reps runs after
// one warm-up run.  Every run must reproduce ref (or sets it when have_ref is
// false): a launch shape or mode never changes a result.
static vopp_status time_mode(vopp_batch* b, void* stream, int32_t mode, int reps,
                             std::vector<vopp_result>& ref, bool& have_ref, double* best_ms) {
  std::vector<vopp_result> cur(b->n);
  double ms_min = 1e30;
  for (int r = 0; r < reps + 1; ++r) {
    double ms = 0.0;
    vopp_status st = vopp_batch_run(b, stream, mode, cur.data(), &ms);
    if (st != VOPP_OK) return st;
    if (r > 0) ms_min = std::min(ms_min, ms);
  }
  if (!have_ref) {
    ref = cur;
    have_ref = true;
  } else {
    for (int i = 0; i < b->n; ++i)
      if (std::memcmp(&ref[i], &cur[i], sizeof(vopp_result)) != 0)
        return fail(VOPP_E_INTERNAL,
                    "tuning (%d, %d, %d, %d, %d) in mode %d changed the result of request %d",
                    b->tuning.accum_cap, b->tuning.backup_cap, b->tuning.blocks_per_cu,
                    b->tuning.forward_group, b->tuning.sweep_group, mode, i);
  }
  *best_ms = ms_min;
  return VOPP_OK;
}

extern "C" vopp_status vopp_batch_autotune(vopp_batch* b, void* stream, int32_t reps,
                                           vopp_tuning* chosen) {
  clear_error();
  if (!b) return fail(VOPP_E_INVALID, "null batch");
  if (reps < 1) reps = 1;
  std::vector<vopp_result> ref(b->n);
  bool have_ref = false;
  vopp_status st = VOPP_OK;
  // 1. The persistent launch: tile sizes -- chunks of 256 belief positions or
  //    trace items per sweep tile, blocks of 256 episodes per forward tile --
  //    and persistent blocks per CU.  Its phases ignore the block caps.
  const int sweep_cands[] = {1, 2, 4, 8};
  const int fwd_cands[] = {1, 4};
  const int per_cu = persistent_blocks_per_cu(b->amax);
  std::vector<int> cu_cands{per_cu};
  if (per_cu > 1) cu_cands.push_back(1);
  double best_persist = 1e30;
  vopp_tuning best = b->tuning;
  for (int sg : sweep_cands) {
    for (int fg : fwd_cands) {
      for (int bc : cu_cands) {
        b->tuning.sweep_group = sg;
        b->tuning.forward_group = fg;
        b->tuning.blocks_per_cu = bc;
        st = build_schedule(b);
        if (st == VOPP_OK) st = capture(b);
        double ms = 0.0;
        if (st == VOPP_OK) st = time_mode(b, stream, VOPP_BATCH_PERSISTENT, reps, ref, have_ref, &ms);
        if (st != VOPP_OK) return st;
        if (ms < best_persist) {
          best_persist = ms;
          best = b->tuning;
        }
      }
    }
  }
  // 2. The per-phase graph: blocks per accumulate and backup sweep of an
  //    instance (few blocks let more instances share a launch; many let a
  //    large instance fill the GPU).
  const int cap_cands[][2] = {{256, 256}, {kAccumCap, kBackupCap}};
  double best_phase = 1e30;
  for (const auto& cc : cap_cands) {
    b->tuning = best;
    b->tuning.accum_cap = cc[0];
    b->tuning.backup_cap = cc[1];
    st = build_schedule(b);
    if (st == VOPP_OK) st = capture(b);
    double ms = 0.0;
    if (st == VOPP_OK) st = time_mode(b, stream, VOPP_BATCH_GRAPH, reps, ref, have_ref, &ms);
    if (st != VOPP_OK) return st;
    if (ms < best_phase) {
      best_phase = ms;
      best.accum_cap = cc[0];
      best.backup_cap = cc[1];
    }
  }
  b->tuning = best;
  b->auto_mode = best_phase < best_persist ? VOPP_BATCH_GRAPH : VOPP_BATCH_PERSISTENT;
  st = build_schedule(b);
  if (st == VOPP_OK) st = capture(b);
  if (st != VOPP_OK) return st;
  if (chosen) *chosen = best;
  return VOPP_OK;
}

extern "C" vopp_status vopp_plan_batch(const vopp_request* reqs, int32_t n, void* stream,
                                       vopp_result* results) {
  vopp_batch* b = nullptr;
  vopp_status st = vopp_batch_create(reqs, n, nullptr, &b);
  if (st != VOPP_OK) return st;
  st = vopp_batch_run(b, stream, VOPP_BATCH_PERSISTENT, results, nullptr);
  vopp_batch_free(b);
  return st;
}
