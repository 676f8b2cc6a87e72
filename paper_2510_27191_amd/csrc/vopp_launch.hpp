// vopp_launch.hpp -- host-side launchers of the planning kernels.
#pragma once

#include <hip/hip_runtime.h>
#include "vopp_device.hpp"

namespace vopp {

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
// Copy the records of beliefs ids[0..n) (device) to out[n * rs] (device).
hipError_t launch_gather(const TreeView& t, const int* ids, int n, unsigned char* out,
                         hipStream_t s);
// One batched launch: n_blocks blocks over n_items phase items (device arrays).
hipError_t launch_batch(const PlanView* views, const BatchItem* items, int n_items,
                        int n_blocks, int amax, hipStream_t s);

}  // namespace vopp
