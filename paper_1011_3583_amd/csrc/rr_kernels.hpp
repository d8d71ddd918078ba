// rr_kernels.hpp -- launchers for the kernels in rr_kernels.hip and rr_batch_kernels.hip.
#pragma once

#include <hip/hip_runtime_api.h>

#include "rr_batch.hpp"
#include "rr_plan.hpp"

namespace rr {

// Enqueue the kernel a plan selects on `st`.  Returns the launch status.
hipError_t launch_plan(const Plan& p, hipStream_t st);

// Enqueue the 2-D stencil kernel for radius 1..4 and shape 0/1.
hipError_t launch_stencil(const StencilArgs& a, hipStream_t st);

// Enqueue one batch group whose table (argument blocks + prefix sums) is
// resident in device memory at `table`.  grid = 0 launches one workgroup per
// block of work; a smaller grid makes the launch persistent (grid-stride).
hipError_t launch_batch_group(const BatchGroup& g, const uint8_t* table, uint32_t grid, hipStream_t st);

}  // namespace rr
