// vopp_internal.hpp -- host-side handle types shared by the library's
// translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/vopp.h"
#include "vopp_device.hpp"

struct vopp_pomdp {
  int kind = 0;
  int nA = 0;
  int device = 0;
  double r_max = 0.0, h_max = 0.0, gamma = 0.0;
  double branch = 1.0;           // |A| * |O| (observation keys per action)
  void* arena = nullptr;
  size_t bytes = 0;
  vopp::ModelView view{};
  vopp_workspace* own_ws = nullptr;
  // Scratch of vopp_env_step / vopp_belief_update (grown on demand).
  void* filt = nullptr;
  size_t filt_bytes = 0;
};

namespace vopp {
struct WsSizes {
  int n_p = 0, steps = 0, K = 0, depth = 0, Apad = 0, rs = 0;
  long long cap_b = 0;
  uint64_t hcap = 0;
};
}  // namespace vopp

struct vopp_workspace {
  vopp::WsSizes z;
  int device = 0;
  void* arena = nullptr;
  size_t bytes = 0;
  vopp::TreeView tree{};
  int* step_base_dev = nullptr;
  int* step_host = nullptr;       // pinned
  double* out_dev = nullptr;
  double* out_host = nullptr;     // pinned
  // Depth of the beliefs each level step of the last plan's tree holds (the
  // steps of a kept subtree first, then the plan's own).
  std::vector<int> step_depth;
  // A kept subtree written by vopp_reroot: its layout by depth, and whether
  // the next plan starts from it.  `carried` says the last plan's tree holds
  // these steps.
  struct Carry {
    bool pending = false;
    int n_p = 0, n_steps = 0;
    int first[vopp::kMaxDepth + 1] = {0}, count[vopp::kMaxDepth + 1] = {0};
    long long beliefs[vopp::kMaxDepth + 1] = {0}, nodes[vopp::kMaxDepth + 1] = {0};
    long long root_visits = 0;
    int shift = 0;               // fixed-point shift the kept sums were scaled to
    int budget = 0;              // iterations that shift allows
  } carry;
  bool carried = false;
  int* carry_rng_dev = nullptr;   // [kMaxDepth + 1][2] device copy of first, count
  // Anytime plans: pinned coherent host word written by the device at the end
  // of each iteration (iterations run | stop << 32), and its device address.
  unsigned long long* gate_host = nullptr;
  unsigned long long* gate_dev = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool hash_dirty = true;
  int n_prev_beliefs = 0, n_prev_actions = 0;
  int last_A = 0, last_apad = 0, last_steps = 0, last_n_p = 0, last_K = 0,
      last_depth = 0, last_schedule = 0;
  double last_fix_inv64 = 0.0;
  // Per-kernel event timing (vopp_profile_enable).
  bool prof_on = false;
  uint32_t prof_mask = 0;                // kinds bracketed with events
  bool prof_open = false;                // current launch is bracketed
  std::vector<hipEvent_t> prof_events;   // pool, two per bracketed launch
  std::vector<int> prof_kinds;           // kind of each bracketed launch
  size_t prof_used = 0;                  // events used by the current plan
  double prof_ms[VOPP_KERNEL_KINDS] = {0};
  int64_t prof_count[VOPP_KERNEL_KINDS] = {0};
};

namespace vopp {
// One phase of one plan or served request, in execution order.
struct Phase {
  int kind, a0, a1, nblk;
};
// The planning phases of a plan (set-up ... select) for the given block caps
// of the accumulate and backup sweeps.
std::vector<Phase> plan_phases(const vopp_pomdp* p, const PlanView& P, int accum_cap,
                               int backup_cap);

vopp_status fail(vopp_status st, const char* fmt, ...);
vopp_status hip_fail(hipError_t e, const char* what);
void clear_error();
int sum_depths(int K, int depth, int schedule);
vopp_status check_params(const vopp_pomdp* p, const vopp_params* prm, int32_t budget,
                         int32_t depth);
vopp_status ws_alloc(const WsSizes& z, vopp_workspace** out);
vopp_status ensure_ws(const vopp_pomdp* p, vopp_workspace** ws, const vopp_params* prm,
                      int K, int depth);
PlanView make_view(const vopp_pomdp* p, vopp_workspace* w, const void* belief,
                   int n_belief, int K, int depth, const vopp_params* prm);
// Blocks of a backup sweep over the beliefs of depth dep after iteration k;
// extra: level steps of a kept subtree holding that depth.
int backup_grid(const vopp_pomdp* p, int n_p, const int* D, int dep, int k,
                int cap, int extra = 0, bool wide = false);
// Sizes of a plan; extra_steps: level steps of a kept subtree in front.
WsSizes sizes_for(const vopp_pomdp* p, int n_p, int K, int depth, int schedule,
                  int extra_steps = 0);
// Fixed-point shift S of the sums for visits root visits in one plan.
int fixed_shift(const vopp_pomdp* p, double visits);
bool fits(const WsSizes& have, const WsSizes& need);
size_t bytes_for(const WsSizes& z);
size_t out_len(const WsSizes& z);
vopp_status enqueue_plan(const vopp_pomdp* p, vopp_workspace* w, const PlanView& P,
                         hipStream_t s, int* n_steps_out);
// Event brackets around one launch when profiling is on.
hipError_t prof_begin(vopp_workspace* w, int kind, hipStream_t s);
hipError_t prof_end(vopp_workspace* w, hipStream_t s);
// Fold the current plan's event pairs into the totals (after a sync).
void prof_collect(vopp_workspace* w);
}  // namespace vopp
