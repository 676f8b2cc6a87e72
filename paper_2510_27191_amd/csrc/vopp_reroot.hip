// vopp_reroot.hip -- tree re-rooting between real steps (host side).
//
// After a planning step, Alg. 1 executes the chosen action, perceives an
// observation and updates the belief.  vopp_reroot keeps the part of the tree
// that stays relevant: the belief reached from the root by that action and
// observation becomes the root of the next plan, and its descendants keep
// their records (preference rows, C, N, V, N_b), one level shallower.  The
// kept records are packed by depth into level steps at the front of the
// destination workspace, so the next plan's sweeps find them exactly like
// the level steps of its own iterations, and they are inserted into the
// destination's belief table under their new parents.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "../../include/vopp.h"
#include "vopp_device.hpp"
#include "vopp_internal.hpp"
#include "vopp_launch.hpp"

using namespace vopp;

namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Temporary device memory of one re-rooting.
struct Scratch {
  void* base = nullptr;
  ~Scratch() {
    if (base) (void)hipFree(base);
  }
};

}  // namespace

extern "C" vopp_status vopp_reroot(const vopp_pomdp* p, vopp_workspace* src, int32_t action,
                                   int32_t obs, const vopp_params* next, int32_t next_budget,
                                   int32_t next_depth, vopp_workspace* dst, void* stream,
                                   int64_t* kept_out) {
  clear_error();
  if (!p || !src || !dst) return fail(VOPP_E_INVALID, "null argument");
  if (src == dst) return fail(VOPP_E_INVALID, "source and destination workspaces must differ");
  vopp_status st = check_params(p, next, next_budget, next_depth);
  if (st != VOPP_OK) return st;
  if (next_budget > kMaxCarryBudget)
    return fail(VOPP_E_INVALID, "a plan from a kept subtree allows at most %d iterations",
                kMaxCarryBudget);
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != p->device || src->device != dev || dst->device != dev)
    return fail(VOPP_E_INVALID, "model and workspaces must live on the current device");
  if (src->n_prev_beliefs <= 0)
    return fail(VOPP_E_INVALID, "no plan has run in the source workspace");
  if (src->last_A != p->nA) return fail(VOPP_E_INVALID, "the source tree is of another model");
  if (action < 0 || action >= p->nA) return fail(VOPP_E_INVALID, "action out of range");
  if (obs < 0) return fail(VOPP_E_INVALID, "negative observation");
  hipStream_t s = (hipStream_t)stream;
  if (kept_out) *kept_out = 0;
  dst->carry.pending = false;
  if (obs >= (1 << p->view.obs_bits)) return VOPP_OK;   // no belief can have that key

  // Source level steps grouped by depth.
  const int n_src_steps = src->last_steps;
  if ((int)src->step_depth.size() != n_src_steps)
    return fail(VOPP_E_INTERNAL, "source tree layout is inconsistent");
  int max_d = 0;
  for (int d : src->step_depth) max_d = std::max(max_d, d);
  std::vector<int> steps_host, off(max_d + 2, 0);
  for (int d = 1; d <= max_d; ++d) {
    off[d] = (int)steps_host.size();
    for (int t = 0; t < n_src_steps; ++t)
      if (src->step_depth[t] == d) steps_host.push_back(t);
  }
  off[max_d + 1] = (int)steps_host.size();

  // Scratch: kept flags, new record ids, counters, step lists, the found record.
  const size_t n_rec = (size_t)src->z.cap_b;
  const size_t n_cnt = 4 * (size_t)kRerootCnt + 1;
  const size_t b_kept = align256(n_rec), b_new = align256(n_rec * 4),
               b_cnt = align256(n_cnt * 8), b_steps = align256(steps_host.size() * 4 + 4);
  Scratch sc;
  hipError_t e = hipMalloc(&sc.base, b_kept + b_new + b_cnt + b_steps + 256);
  if (e != hipSuccess) return fail(VOPP_E_NOMEM, "re-rooting scratch: %s", hipGetErrorString(e));
  char* q = (char*)sc.base;
  unsigned char* kept = (unsigned char*)q;
  int* new_id = (int*)(q + b_kept);
  unsigned long long* cnt = (unsigned long long*)(q + b_kept + b_new);
  int* steps_dev = (int*)(q + b_kept + b_new + b_cnt);
  int* found_dev = (int*)(q + b_kept + b_new + b_cnt + b_steps);
  e = hipMemsetAsync(kept, 0, n_rec, s);
  if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, n_cnt * 8, s);
  if (e == hipSuccess && !steps_host.empty())
    e = hipMemcpyAsync(steps_dev, steps_host.data(), steps_host.size() * 4,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_reroot_find(src->tree, action, obs, p->view.obs_bits, found_dev, s);
  int root_rec = -1;
  if (e == hipSuccess) e = hipMemcpyAsync(&root_rec, found_dev, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "re-rooting: find");
  if (root_rec <= 0) return VOPP_OK;            // not in the tree: the next plan starts fresh

  // Mark the kept subtree depth by depth and count it.
  RerootView V;
  std::memset(&V, 0, sizeof(V));
  V.src = src->tree;
  V.src_n_p = src->last_n_p;
  V.A = p->nA;
  V.obs_bits = p->view.obs_bits;
  V.root_rec = root_rec;
  V.kept = kept;
  V.new_id = new_id;
  V.cnt = cnt;
  for (int d = 1; d <= max_d && e == hipSuccess; ++d) {
    V.steps = steps_dev + off[d];
    V.n_steps = off[d + 1] - off[d];
    V.src_depth = d;
    e = launch_reroot_mark(V, s);
  }
  std::vector<unsigned long long> c(n_cnt);
  if (e == hipSuccess) e = hipMemcpyAsync(c.data(), cnt, 3 * kRerootCnt * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "re-rooting: mark");

  // Layout of the kept subtree in the destination: new depth d holds the
  // source's depth d + 1, packed into ceil(count / n_p) level steps.
  const int n_p = next->n_particles;
  vopp_workspace::Carry cy;
  cy.n_p = n_p;
  int carry_steps = 0;
  long long kept_total = 1;
  for (int d = 1; d + 1 <= max_d; ++d) {
    const long long nb = (long long)c[d + 1];
    const int k = (int)((nb + n_p - 1) / n_p);
    if (k > kMaxBudget)
      return fail(VOPP_E_INVALID, "kept subtree too wide at depth %d for n_particles = %d", d, n_p);
    cy.first[d] = carry_steps;
    cy.count[d] = k;
    cy.beliefs[d] = nb;
    cy.nodes[d] = (long long)c[kRerootCnt + d + 1];
    carry_steps += k;
    kept_total += nb;
  }
  cy.n_steps = carry_steps;
  cy.root_visits = (long long)c[2 * kRerootCnt + 1];
  cy.budget = next_budget;
  cy.shift = fixed_shift(p, (double)n_p * (double)next_budget + (double)cy.root_visits);
  if ((long long)n_p * (carry_steps + sum_depths(next_budget, next_depth, next->schedule)) + 1 >
      kMaxBeliefs)
    return fail(VOPP_E_INVALID, "kept subtree and plan exceed 2^28 beliefs");

  // The destination must hold the kept subtree and the next plan, with the
  // source's record layout.
  WsSizes need = sizes_for(p, n_p, next_budget, next_depth, next->schedule, carry_steps);
  need.Apad = src->z.Apad;
  need.rs = src->z.rs;
  if (!fits(dst->z, need) || dst->z.Apad != src->z.Apad) {
    vopp_workspace* grown = nullptr;
    st = ws_alloc(need, &grown);
    if (st != VOPP_OK) return st;
    std::swap(*dst, *grown);
    vopp_workspace_free(grown);
  }
  dst->n_prev_beliefs = 0;                      // its old tree is gone
  dst->hash_dirty = true;                       // until the copy has finished

  // Clear the destination's table and the kept steps' lists, then copy.
  const size_t hcap = (size_t)dst->tree.h_mask + 1;
  e = launch_fill16(dst->tree.h_slot, hcap, make_uint4(~0u, ~0u, ~0u, ~0u), s);
  if (e == hipSuccess && carry_steps > 0)
    e = hipMemsetAsync(dst->tree.list, 0, (size_t)carry_steps * n_p * sizeof(int), s);
  V.dst = dst->tree;
  V.dst_n_p = n_p;
  V.rescale = std::ldexp(1.0, cy.shift) * src->last_fix_inv64;
  for (int d = 1; d <= max_d && e == hipSuccess; ++d) {
    V.steps = steps_dev + off[d];
    V.n_steps = off[d + 1] - off[d];
    V.src_depth = d;
    V.first_step = d >= 2 ? cy.first[d - 1] : 0;
    e = launch_reroot_copy(V, s);
  }
  int rng[2 * (kMaxDepth + 1)] = {0};
  for (int d = 1; d <= kMaxDepth; ++d) {
    rng[2 * d] = cy.first[d];
    rng[2 * d + 1] = cy.count[d];
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->carry_rng_dev, rng, sizeof(rng), hipMemcpyHostToDevice, s);
  unsigned long long err = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&err, cnt + 4 * kRerootCnt, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "re-rooting: copy");
  if (err) return fail(VOPP_E_INTERNAL, "re-rooting: a kept belief could not be inserted");
  cy.pending = true;
  dst->carry = cy;
  dst->hash_dirty = false;
  if (kept_out) *kept_out = kept_total;
  return VOPP_OK;
}
