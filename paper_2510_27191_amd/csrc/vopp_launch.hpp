// vopp_launch.hpp -- host-side launchers of the planning kernels.
#pragma once

#include <hip/hip_runtime.h>
#include "vopp_device.hpp"

namespace vopp {

hipError_t launch_expand(const PlanView& P, int k, int d, hipStream_t s);
hipError_t launch_resolve(const PlanView& P, int t, hipStream_t s);
hipError_t launch_finish(const PlanView& P, hipStream_t s);
hipError_t launch_backup_leaf(const PlanView& P, int dep, int k, int grid, hipStream_t s);
hipError_t launch_backup_level(const PlanView& P, int dep, int k, int grid, hipStream_t s);
hipError_t launch_backup_root(const PlanView& P, hipStream_t s);
hipError_t launch_clear_slots(const PlanView& P, int n_prev, hipStream_t s);
hipError_t launch_fill32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_init_root(const PlanView& P, hipStream_t s);
hipError_t launch_select(const PlanView& P, int last_step, double* out, hipStream_t s);

}  // namespace vopp
