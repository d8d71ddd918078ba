// rr_kernels.hpp -- launchers for the kernels in rr_kernels.hip.
#pragma once

#include <hip/hip_runtime_api.h>

#include "rr_plan.hpp"

namespace rr {

// Enqueue the kernel a plan selects on `st`.  Returns the launch status.
hipError_t launch_plan(const Plan& p, hipStream_t st);

}  // namespace rr
