// vopp_launch.hpp -- host-side launchers of the planning kernels.
#pragma once

#include <hip/hip_runtime.h>
#include "vopp_device.hpp"

namespace vopp {

int setup_blocks(const PlanView& P);
hipError_t launch_setup(const PlanView& P, hipStream_t s);
hipError_t launch_expand(const PlanView& P, int k, int d, hipStream_t s);
hipError_t launch_resolve(const PlanView& P, int t, hipStream_t s);
hipError_t launch_finish(const PlanView& P, hipStream_t s);
hipError_t launch_backup_leaf(const PlanView& P, int dep, int k, int grid, hipStream_t s);
hipError_t launch_backup_level(const PlanView& P, int dep, int k, int grid, hipStream_t s);
hipError_t launch_backup_root(const PlanView& P, hipStream_t s);
hipError_t launch_select(const PlanView& P, int last_step, hipStream_t s);
hipError_t launch_env(const PlanView& P, int t, hipStream_t s);
// SIR update of P.f: weight, scan, resample (three launches).
hipError_t launch_pf(const PlanView& P, int t, hipStream_t s);
// One batched launch: n_blocks blocks over n_items phase items (device arrays).
hipError_t launch_batch(const PlanView* views, const BatchItem* items, int n_items,
                        int n_blocks, int amax, hipStream_t s);

}  // namespace vopp
