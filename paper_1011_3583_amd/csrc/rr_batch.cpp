// rr_batch.cpp -- batched permutes (placeholder until the persistent kernel lands).
#include "rr_internal.hpp"

extern "C" rr_status rr_permute_batched(const rr_job* jobs, int njobs, rr_stream_t stream) {
    (void)jobs; (void)njobs; (void)stream;
    return rr::fail(RR_ERR_UNSUPPORTED, "batched launch not built yet");
}
