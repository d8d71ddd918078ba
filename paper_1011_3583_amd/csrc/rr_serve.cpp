// rr_serve.cpp -- serving loop (placeholder until the server lands).
#include "rr_internal.hpp"

extern "C" {
rr_status rr_serve_create(const rr_serve_config*, rr_server**) { return rr::fail(RR_ERR_UNSUPPORTED, "server not built yet"); }
rr_status rr_serve_alloc(rr_server*, uint64_t, void**) { return RR_ERR_UNSUPPORTED; }
rr_status rr_serve_free(rr_server*, void*) { return RR_ERR_UNSUPPORTED; }
rr_status rr_serve_submit(rr_server*, const rr_job*, uint64_t*) { return RR_ERR_UNSUPPORTED; }
rr_status rr_serve_poll(rr_server*, uint64_t, rr_job_result*) { return RR_ERR_UNSUPPORTED; }
rr_status rr_serve_release(rr_server*, uint64_t) { return RR_ERR_UNSUPPORTED; }
rr_status rr_serve_destroy(rr_server*) { return RR_ERR_UNSUPPORTED; }
rr_status rr_serve_get_stats(rr_server*, rr_serve_stats*) { return RR_ERR_UNSUPPORTED; }
}
