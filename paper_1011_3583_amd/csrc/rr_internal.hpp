// rr_internal.hpp -- helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

#include "rr_batch.hpp"
#include "rr_plan.hpp"

namespace rr {

rr_status fail(rr_status s, const std::string& why);
void clear_error();
rr_status hip_fail(hipError_t e, const char* what);
bool ranges_overlap(uint64_t a, uint64_t na, uint64_t b, uint64_t nb);
// Validate and canonicalise one permute request (no launch).
rr_status validate_permute(const void* dst, const void* src, int ndim, const int64_t* dims,
                           const int* perm, int elem_size, Canon* c);

// Launch every group of a batch whose table is resident at dev_table.
rr_status launch_batch_plan(const BatchPlan& p, const uint8_t* dev_table, bool persistent, int device,
                            hipStream_t st);

}  // namespace rr
