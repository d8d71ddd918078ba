// rr_internal.hpp -- helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

#include "rr_batch.hpp"
#include "rr_plan.hpp"

namespace rr {

// Diagnostics on stderr by level, from the RR_LOG environment variable (read
// once): 0 or unset silent, 1 every error a call returns, 2 also the plan of
// every single launch and the groups of every batch, 3 also the server's batch
// and admission events.
int log_level();
void log_line(int level, const std::string& msg);

rr_status fail(rr_status s, const std::string& why);
void clear_error();
rr_status hip_fail(hipError_t e, const char* what);
// The tuning-cache context of this process (device architecture and HIP
// runtime version), set on first use from the current device.
void ensure_tune_context();
bool ranges_overlap(uint64_t a, uint64_t na, uint64_t b, uint64_t nb);
// Validate and canonicalise one permute request (no launch).
rr_status validate_permute(const void* dst, const void* src, int ndim, const int64_t* dims,
                           const int* perm, int elem_size, Canon* c);

// Side streams that let the groups of one batch run side by side.  Groups touch
// disjoint memory, so each may start once the work queued before the batch is
// done; the caller's stream continues after all of them.  Streams keep the
// default priority.
constexpr int FANOUT_SIDE = 3;
struct GroupFanout {
    hipStream_t side[FANOUT_SIDE] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[FANOUT_SIDE] = {};
};
rr_status fanout_init(GroupFanout* f);
void fanout_destroy(GroupFanout* f);

// Launch every group of a batch whose table is resident at dev_table: one after
// another on st, or (with a fanout) spread over st and the side streams, largest
// groups first, each to the stream with the least work queued so far.
rr_status launch_batch_plan(const BatchPlan& p, const uint8_t* dev_table, bool persistent, int device,
                            hipStream_t st, GroupFanout* fan = nullptr);

}  // namespace rr
