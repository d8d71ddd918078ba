// rr_noalloc.hip -- rr_permute_batched_noalloc: batched permutes that allocate no
// memory, for callers that cannot allocate (tight serving loops, harnesses that
// forbid hipMalloc).
//
// rr_permute_batched stages each batch's job table (argument blocks, prefix sums,
// bucket index, entry ranges) through pinned host and device buffers it grows on
// demand.  This variant keeps the table in a fixed device array instead: the
// array below, one copy per GPU for the life of the process.  Host code never
// uses the array's name as an address (on the host it only names the symbol):
// the device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current, and is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "rr_batch.hpp"
#include "rr_internal.hpp"

namespace rr {
namespace {

// Largest job table the variant accepts: 4096 tiled jobs take about 2.8 MB.
constexpr size_t NOALLOC_TABLE_BYTES = size_t(4) << 20;

__device__ __align__(256) uint8_t scratch[NOALLOC_TABLE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `device`'s copy of the table array (device is current).
rr_status scratch_address(int device, void** out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(RR_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return RR_OK;
}

}  // namespace
}  // namespace rr

using namespace rr;

extern "C" rr_status rr_permute_batched_noalloc(const rr_job* jobs, int njobs, rr_stream_t stream) {
    clear_error();
    // planned on the calling thread into buffers it keeps (host memory only)
    static thread_local BatchPlan bp;
    std::string why;
    int bad = -1;
    rr_status st = plan_batch(jobs, njobs, current_tile_options(), &bp, &why, &bad);
    if (st != RR_OK) {
        if (bad >= 0) why = "job " + std::to_string(bad) + ": " + why;
        return fail(st, why);
    }
    if (bp.groups.empty()) return RR_OK;
    if (bp.table.size() > NOALLOC_TABLE_BYTES)
        return fail(RR_ERR_UNSUPPORTED, "job table of " + std::to_string(bp.table.size()) +
                                            " bytes exceeds the 4 MiB static table (split the batch)");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void* table = nullptr;
    st = scratch_address(device, &table);
    if (st != RR_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    // A copy from pageable host memory waits for the work queued on the stream
    // before it (so an earlier call's kernels on this stream have finished with
    // the table) and has consumed the host buffer when it returns.
    e = hipMemcpyAsync(table, bp.table.data(), bp.table.size(), hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "job table upload");
    return launch_batch_plan(bp, (const uint8_t*)table, false, device, hs, nullptr);
}
