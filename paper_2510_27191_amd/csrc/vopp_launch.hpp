// vopp_launch.hpp -- host-side launchers of the planning kernels.
#pragma once

#include <hip/hip_runtime.h>
#include "vopp_device.hpp"

namespace vopp {

// Events that the calling thread's next plan-kernel launches (launch_setup
// ... launch_select) take as the start and end timestamps of their own
// dispatch (hipExtLaunchKernel), rather than stream markers around it.  The
// first launch takes `start`, every launch takes `stop`, so a bracket over
// two launches spans both.  `used` says whether any launch took them.  Only
// the plan's per-kernel profiling sets them, between its bracket's begin and
// end.
struct LaunchTiming {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
  bool used = false;
};
LaunchTiming& launch_timing();

int setup_blocks(const PlanView& P);
int forward_blocks(const PlanView& P);
// Blocks of a sweep over the trace of an iteration with D levels (at most cap).
int accum_blocks(const PlanView& P, int D, int cap);
hipError_t launch_setup(const PlanView& P, hipStream_t s);
hipError_t launch_forward(const PlanView& P, int k, int D, hipStream_t s);
hipError_t launch_accum(const PlanView& P, int D, int grid, hipStream_t s);
hipError_t launch_backup_leaf(const PlanView& P, int dep, int k, int grid, hipStream_t s);
hipError_t launch_backup_level(const PlanView& P, int dep, int k, int grid, hipStream_t s);
hipError_t launch_backup_root(const PlanView& P, int k, hipStream_t s);
hipError_t launch_select(const PlanView& P, hipStream_t s);
hipError_t launch_env(const PlanView& P, int t, hipStream_t s);
// SIR update of P.f: weight, scan, resample (three launches).
hipError_t launch_pf(const PlanView& P, int t, hipStream_t s);
// One of the three: 0 weight, 1 scan, 2 resample.
hipError_t launch_pf_part(const PlanView& P, int part, int t, hipStream_t s);
// Copy the records of beliefs ids[0..n) (device) to out[n * rs] (device).
hipError_t launch_gather(const TreeView& t, const int* ids, int n, unsigned char* out,
                         hipStream_t s);
// Tree re-rooting between real steps.  One launch of the mark or copy pass
// covers the source beliefs of one depth (src_depth), in the source's level
// steps steps[0 .. n_steps).
struct RerootView {
  TreeView src, dst;
  int src_n_p, dst_n_p;
  int A;
  int obs_bits;               // observation field of the belief keys
  const int* steps;
  int n_steps;
  int src_depth;
  int root_rec;               // source record of the new root (depth 1)
  int first_step;             // copy: first destination step of depth src_depth-1
  double rescale;             // copy: 2^(S_dst - S_src) for the fixed-point sums
  unsigned char* kept;        // [source records] 1: in the kept subtree
  int* new_id;                // [source records] destination record
  // [4][kMaxDepth + 1]: kept beliefs, their action nodes, the root's visits
  // (depth 1) and the copy's fill counters; [4 * (kMaxDepth + 1)] error flags.
  unsigned long long* cnt;
};
constexpr int kRerootCnt = kMaxDepth + 1;
// Record of the root's child belief for (a, obs) in a finished plan's table,
// or -1 (one thread; out is a device int).
hipError_t launch_reroot_find(const TreeView& t, int a, int obs, int ob, int* out,
                              hipStream_t s);
hipError_t launch_reroot_mark(const RerootView& V, hipStream_t s);
hipError_t launch_reroot_copy(const RerootView& V, hipStream_t s);
// Fill n 16-byte words at p with v.
hipError_t launch_fill16(void* p, size_t n, uint4 v, hipStream_t s);

// The persistent batched launch (one reset kernel, then n_blocks blocks that
// drain V's queue); the most blocks of it one CU holds at once.
hipError_t launch_persistent(const PlanView* views, const PersistView& V, int n_blocks,
                             int amax, hipStream_t s);
int persistent_blocks_per_cu(int amax);
// One batched launch: n_blocks blocks over n_items phase items (device arrays).
hipError_t launch_batch(const PlanView* views, const BatchItem* items, int n_items,
                        int n_blocks, int amax, hipStream_t s);

}  // namespace vopp
