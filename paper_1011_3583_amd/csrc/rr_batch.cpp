// rr_batch.cpp -- batched permutes: one-shot rr_permute_batched and reusable
// rr_batch handles (resident job table, optional hipGraph replay, autotuning).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rr_batch.hpp"
#include "rr_internal.hpp"
#include "rr_kernels.hpp"

namespace rr {

namespace {

// Staging ring of pinned host + device buffers for one-shot batches.
struct Slot {
    void* host = nullptr;
    void* dev = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};
constexpr int RING = 4;
// One-shot batches of at least this many jobs are planned and launched in chunks.
constexpr int PIPE_MIN_JOBS = 2048;
struct Ring {
    Slot slots[RING];
    int next = 0;
    GroupFanout fan;                // side streams the groups of one-shot batched calls fan out on
    hipStream_t upload = nullptr;   // table copies of pipelined calls
    hipEvent_t ready[RING] = {};    // slot k's table is in place (pipelined calls)
};

// Take the ring's next slot (ring lock held): wait for the batch that last used
// it, grow its pinned and device buffers to `need` bytes.
rr_status take_slot(Ring& ring, size_t need, int* index) {
    const int k = ring.next;
    Slot& s = ring.slots[k];
    ring.next = (ring.next + 1) % RING;
    if (s.used) {
        hipError_t e = hipEventSynchronize(s.done);
        if (e != hipSuccess) return hip_fail(e, "waiting for a staging slot");
        s.used = false;
    }
    if (need > s.cap) {
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        s.host = s.dev = nullptr;
        s.cap = 0;
        size_t cap = std::max<size_t>(need, 1 << 20);
        if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess)
            return fail(RR_ERR_NO_MEMORY, "pinned staging buffer");
        if (hipMalloc(&s.dev, cap) != hipSuccess) {
            (void)hipHostFree(s.host);
            s.host = nullptr;
            return fail(RR_ERR_NO_MEMORY, "device job table");
        }
        s.cap = cap;
    }
    if (!s.done && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
        return fail(RR_ERR_HIP, "hipEventCreate");
    *index = k;
    return RR_OK;
}
std::mutex g_ring_mu;
std::map<int, Ring> g_rings;

int cu_count(int device) {
    static std::map<int, int> cache;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(device);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) n = 256;
    cache[device] = n;
    return n;
}

uint32_t group_grid(const BatchGroup& g, bool persistent, int device) {
    if (!persistent) return g.total_blocks;
    const uint32_t per_cu = g.kind == K_TILE ? (g.lds_bytes > 32768 ? 2u : 4u) : 8u;
    return std::min<uint32_t>(g.total_blocks, (uint32_t)cu_count(device) * per_cu);
}


rr_status plan_or_fail(const rr_job* jobs, int njobs, const TileOptions& opt, BatchPlan* bp) {
    std::string why;
    int bad = -1;
    rr_status st = plan_batch(jobs, njobs, opt, bp, &why, &bad);
    if (st != RR_OK) {
        if (bad >= 0) why = "job " + std::to_string(bad) + ": " + why;
        return fail(st, why);
    }
    return RR_OK;
}

}  // namespace

rr_status fanout_init(GroupFanout* f) {
    if (f->fork) return RR_OK;
    for (int k = 0; k < FANOUT_SIDE; ++k) {
        if (hipStreamCreateWithFlags(&f->side[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&f->join[k], hipEventDisableTiming) != hipSuccess) {
            fanout_destroy(f);
            return fail(RR_ERR_HIP, "side streams for batch groups");
        }
    }
    if (hipEventCreateWithFlags(&f->fork, hipEventDisableTiming) != hipSuccess) {
        fanout_destroy(f);
        return fail(RR_ERR_HIP, "side streams for batch groups");
    }
    return RR_OK;
}

void fanout_destroy(GroupFanout* f) {
    for (int k = 0; k < FANOUT_SIDE; ++k) {
        if (f->side[k]) (void)hipStreamDestroy(f->side[k]);
        if (f->join[k]) (void)hipEventDestroy(f->join[k]);
        f->side[k] = nullptr;
        f->join[k] = nullptr;
    }
    if (f->fork) (void)hipEventDestroy(f->fork);
    f->fork = nullptr;
}

// Estimated run time of a group, for placing groups on streams: its workgroups,
// a tile workgroup (up to 16 KiB through LDS in two dependent phases) weighted as
// eight copy or run workgroups (4 KiB streamed each), the ratio of their average
// durations in the 4096-job batch's kernel trace.  Bytes alone rank odd-extent
// tile groups far too cheap: they move a byte 2-5x slower than copies.
static uint64_t group_cost(const BatchGroup& g) {
    return (uint64_t)std::max<uint32_t>(g.total_blocks, 1) * (g.kind == K_TILE ? 8 : 1);
}

// Groups of one or more batch plans spread over a stream and the side streams
// of a fanout, each plan's groups costliest first, each group to the stream
// with the least estimated work queued so far (over every plan added).  A
// stream starts a plan's groups only after that plan's `ready` event (its table
// in place, the caller's earlier work done); end() makes the caller's stream
// wait for every side stream used.
class FanSession {
   public:
    FanSession(GroupFanout* fan, hipStream_t st) : st_(st) {
        streams_[0] = st;
        for (int k = 0; k < FANOUT_SIDE; ++k) streams_[k + 1] = fan->side[k];
        fan_ = fan;
    }
    rr_status add(const BatchPlan& p, const uint8_t* dev_table, bool persistent, int device, hipEvent_t ready) {
        std::vector<size_t> order(p.groups.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return group_cost(p.groups[a]) > group_cost(p.groups[b]); });
        bool waited[FANOUT_SIDE + 1] = {};
        for (size_t i : order) {
            int s = 0;
            for (int k = 1; k <= FANOUT_SIDE; ++k) if (load_[k] < load_[s]) s = k;
            if (!waited[s]) {
                hipError_t e = hipStreamWaitEvent(streams_[s], ready, 0);
                if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
                waited[s] = true;
                used_[s] = true;
            }
            const BatchGroup& g = p.groups[i];
            hipError_t e = launch_batch_group(g, dev_table, group_grid(g, persistent, device), streams_[s]);
            if (e != hipSuccess) return hip_fail(e, "batched launch");
            load_[s] += group_cost(g);
        }
        return RR_OK;
    }
    rr_status end() {
        for (int k = 1; k <= FANOUT_SIDE; ++k) {
            if (!used_[k]) continue;
            hipError_t e = hipEventRecord(fan_->join[k - 1], streams_[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st_, fan_->join[k - 1], 0);
            if (e != hipSuccess) return hip_fail(e, "joining batch groups");
        }
        return RR_OK;
    }

   private:
    hipStream_t st_;
    GroupFanout* fan_;
    hipStream_t streams_[FANOUT_SIDE + 1];
    uint64_t load_[FANOUT_SIDE + 1] = {};
    bool used_[FANOUT_SIDE + 1] = {};
};

rr_status launch_batch_plan(const BatchPlan& p, const uint8_t* dev_table, bool persistent, int device,
                            hipStream_t st, GroupFanout* fan) {
    if (!fan || !fan->fork || p.groups.size() < 2) {
        for (const BatchGroup& g : p.groups) {
            hipError_t e = launch_batch_group(g, dev_table, group_grid(g, persistent, device), st);
            if (e != hipSuccess) return hip_fail(e, "batched launch");
        }
        return RR_OK;
    }
    hipError_t e = hipEventRecord(fan->fork, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    FanSession fs(fan, st);
    rr_status rs = fs.add(p, dev_table, persistent, device, fan->fork);
    const rr_status re = fs.end();
    return rs != RR_OK ? rs : re;
}

}  // namespace rr

using namespace rr;

struct rr_batch {
    int device = 0;
    int flags = 0;
    std::vector<rr_job> jobs;
    BatchPlan plan;
    TileOptions opt;
    bool persistent = false;
    void* dev_table = nullptr;
    size_t dev_cap = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GroupFanout fan;      // groups run side by side on these
    double tuned_us = 0.0;
};

namespace {

// Side streams of a handle, or none when its groups run one after another.
GroupFanout* fan_of(rr_batch* b) { return (b->flags & RR_BATCH_SERIAL) ? nullptr : &b->fan; }

rr_status upload_table(rr_batch* b) {
    const size_t need = std::max<size_t>(b->plan.table.size(), 256);
    if (need > b->dev_cap) {
        if (b->dev_table) (void)hipFree(b->dev_table);
        b->dev_table = nullptr;
        b->dev_cap = 0;
        hipError_t e = hipMalloc(&b->dev_table, need);
        if (e != hipSuccess) return fail(RR_ERR_NO_MEMORY, "cannot allocate the batch table");
        b->dev_cap = need;
    }
    if (!b->plan.table.empty()) {
        hipError_t e = hipMemcpy(b->dev_table, b->plan.table.data(), b->plan.table.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "batch table upload");
    }
    return RR_OK;
}

void drop_graph(rr_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Time one launch of the batch as planned now (median of 3 after a warm-up).
rr_status time_batch(rr_batch* b, hipStream_t st, double* us) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RR_ERR_HIP, "hipEventCreate failed");
    std::vector<float> ts;
    rr_status rs = RR_OK;
    for (int r = 0; r < 4 && rs == RR_OK; ++r) {
        (void)hipEventRecord(e0, st);
        rs = launch_batch_plan(b->plan, (const uint8_t*)b->dev_table, b->persistent, b->device, st, fan_of(b));
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0) ts.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rs != RR_OK) return rs;
    std::sort(ts.begin(), ts.end());
    *us = ts[ts.size() / 2] * 1e3;
    return RR_OK;
}

rr_status tune(rr_batch* b) {
    // row targets, traversal order, persistent grid, tile size (KiB), unaligned
    // micro-tiles, cache policy (-1: each job's own by line alignment), odd-extent
    // refit (-1: built-in), G = 1 rows of any alignment for every tile job
    struct Cand { int in_rb, out_rb, order; bool persistent; int kib = 0, umt = 0, cache = -1, fill = -1, ragged = 0; };
    const Cand cands[] = {{0, 0, 0, false}, {0, 0, 1, false}, {0, 0, 0, true}, {256, 512, 0, false},
                          {512, 256, 0, false}, {512, 512, 0, false}, {1024, 256, 0, false},
                          {256, 1024, 0, false}, {512, 256, 1, false}, {128, 256, 0, false},
                          {0, 0, 0, false, 0, 1}, {512, 512, 0, false, 32, 0},
                          {0, 0, 0, false, 0, 0, 0}, {0, 0, 0, false, 0, 0, 1}, {0, 0, 0, false, 0, 0, 2},
                          {0, 0, 0, false, 0, 0, -1, 0}, {512, 256, 1, false, 0, 0, -1, 0},
                          {512, 256, 1, false, 0, 0, -1, -1, 1}, {512, 256, 1, false, 0, 0, 3, -1, 1},
                          {0, 0, -1, false, 0, 0, -1, -1, 1}};
    // the candidates run the batch on a stream of their own: let whatever the
    // caller has queued on the device finish first
    hipError_t se = hipDeviceSynchronize();
    if (se != hipSuccess) return hip_fail(se, "hipDeviceSynchronize before tuning");
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return fail(RR_ERR_HIP, "stream");
    double best = 1e300;
    Cand bestc = cands[0];
    rr_status rs = RR_OK;
    for (const Cand& c : cands) {
        TileOptions o;
        o.in_row_bytes = c.in_rb;
        o.out_row_bytes = c.out_rb;
        o.order_out = c.order;
        o.tile_kib = c.kib;
        o.umt = c.umt;
        o.cache = c.cache;
        o.fill = c.fill;
        o.force_ragged = c.ragged;
        BatchPlan p;
        std::string why;
        int bad;
        if (plan_batch(b->jobs.data(), (int)b->jobs.size(), o, &p, &why, &bad) != RR_OK) continue;
        b->plan = std::move(p);
        b->persistent = c.persistent;
        if ((rs = upload_table(b)) != RR_OK) break;
        double us = 0;
        if ((rs = time_batch(b, st, &us)) != RR_OK) break;
        if (us < best) { best = us; bestc = c; }
    }
    (void)hipStreamDestroy(st);
    if (rs != RR_OK) return rs;
    b->opt = TileOptions();
    b->opt.in_row_bytes = bestc.in_rb;
    b->opt.out_row_bytes = bestc.out_rb;
    b->opt.order_out = bestc.order;
    b->opt.tile_kib = bestc.kib;
    b->opt.umt = bestc.umt;
    b->opt.cache = bestc.cache;
    b->opt.fill = bestc.fill;
    b->opt.force_ragged = bestc.ragged;
    b->persistent = bestc.persistent;
    b->tuned_us = best;
    rs = plan_or_fail(b->jobs.data(), (int)b->jobs.size(), b->opt, &b->plan);
    if (rs != RR_OK) return rs;
    return upload_table(b);
}

// Large one-shot batches: every job is validated first (an invalid batch
// enqueues nothing), then the jobs are planned, staged and launched in up to
// RING contiguous chunks (a sixteenth, three sixteenths, a quarter, the rest:
// small first, so the GPU starts early, larger later), so the GPU
// runs the first chunks while the host plans the next.  The chunks' groups
// share one fan-out over the caller's stream and the side streams; each
// chunk's table goes up on the ring's upload stream after the caller's earlier
// work, and a stream starts a chunk's groups once that chunk's table is in place.
rr_status permute_batched_pipelined(const rr_job* jobs, int njobs, hipStream_t hs) {
    std::string why;
    int bad = -1;
    rr_status st = validate_batch(jobs, njobs, &why, &bad);
    if (st != RR_OK) {
        if (bad >= 0) why = "job " + std::to_string(bad) + ": " + why;
        return fail(st, why);
    }
    const TileOptions opt = current_tile_options();
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ring_mu);
    Ring& ring = g_rings[device];
    st = fanout_init(&ring.fan);
    if (st != RR_OK) return st;
    for (hipEvent_t& ev : ring.ready)
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
            return fail(RR_ERR_HIP, "hipEventCreate");
        }
    if (!ring.upload && hipStreamCreateWithFlags(&ring.upload, hipStreamNonBlocking) != hipSuccess) {
        ring.upload = nullptr;
        return fail(RR_ERR_HIP, "table upload stream");
    }
    // uploads (and so every chunk's start) follow the caller's earlier work
    e = hipEventRecord(ring.fan.fork, hs);
    if (e == hipSuccess) e = hipStreamWaitEvent(ring.upload, ring.fan.fork, 0);
    if (e != hipSuccess) return hip_fail(e, "ordering the table uploads");
    static thread_local BatchPlan cp;
    FanSession fs(&ring.fan, hs);
    std::vector<int> slots;
    const int64_t n = njobs;
    const int64_t bounds[RING + 1] = {0, n / 16, n / 4, n / 2, n};
    for (int c = 0; c < RING && st == RR_OK; ++c) {
        const int lo = (int)bounds[c], hi = (int)bounds[c + 1];
        if (hi <= lo) continue;
        st = plan_or_fail(jobs + lo, hi - lo, opt, &cp);
        if (st != RR_OK) break;
        if (cp.groups.empty()) continue;
        int k = 0;
        if ((st = take_slot(ring, cp.table.size(), &k)) != RR_OK) break;
        Slot& s = ring.slots[k];
        std::memcpy(s.host, cp.table.data(), cp.table.size());
        e = hipMemcpyAsync(s.dev, s.host, cp.table.size(), hipMemcpyHostToDevice, ring.upload);
        if (e == hipSuccess) e = hipEventRecord(ring.ready[k], ring.upload);
        if (e != hipSuccess) { st = hip_fail(e, "job table upload"); break; }
        slots.push_back(k);
        st = fs.add(cp, (const uint8_t*)s.dev, false, device, ring.ready[k]);
    }
    if (cp.table.capacity() > (size_t(32) << 20)) std::vector<uint8_t>().swap(cp.table);
    const rr_status je = fs.end();
    // a slot is free again once the caller's stream, which now follows every
    // group, gets past this point
    for (int k : slots) {
        e = hipEventRecord(ring.slots[k].done, hs);
        ring.slots[k].used = true;
        if (e != hipSuccess && st == RR_OK) st = hip_fail(e, "hipEventRecord");
    }
    return st != RR_OK ? st : je;
}

}  // namespace

extern "C" {

rr_status rr_permute_batched(const rr_job* jobs, int njobs, rr_stream_t stream) {
    clear_error();
    hipStream_t hs = (hipStream_t)stream;
    if (njobs >= PIPE_MIN_JOBS) return permute_batched_pipelined(jobs, njobs, hs);
    // the plan's table is copied to the staging ring below: each calling thread
    // keeps one plan so its multi-megabyte table is not allocated per call
    static thread_local BatchPlan bp;
    rr_status st = plan_or_fail(jobs, njobs, current_tile_options(), &bp);
    if (st != RR_OK) return st;
    if (bp.groups.empty()) return RR_OK;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ring_mu);
    Ring& ring = g_rings[device];
    st = fanout_init(&ring.fan);
    if (st != RR_OK) return st;
    const size_t need = bp.table.size();
    int k = 0;
    st = take_slot(ring, need, &k);
    if (st != RR_OK) return st;
    Slot& s = ring.slots[k];
    std::memcpy(s.host, bp.table.data(), need);
    if (bp.table.capacity() > (size_t(32) << 20)) std::vector<uint8_t>().swap(bp.table);   // keep at most 32 MB
    e = hipMemcpyAsync(s.dev, s.host, need, hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "job table upload");
    st = launch_batch_plan(bp, (const uint8_t*)s.dev, false, device, hs, &ring.fan);
    e = hipEventRecord(s.done, hs);
    s.used = true;
    if (st != RR_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return RR_OK;
}

rr_status rr_batch_create(const rr_job* jobs, int njobs, int flags, rr_batch** out) {
    clear_error();
    if (!out) return fail(RR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (flags & ~(RR_BATCH_GRAPH | RR_BATCH_TUNE | RR_BATCH_PERSISTENT | RR_BATCH_SERIAL))
        return fail(RR_ERR_INVALID_ARG, "unknown flags");
    rr_batch* b = new rr_batch();
    b->flags = flags;
    b->persistent = (flags & RR_BATCH_PERSISTENT) != 0;
    if (njobs > 0 && jobs) b->jobs.assign(jobs, jobs + njobs);
    hipError_t e = hipGetDevice(&b->device);
    rr_status st = e == hipSuccess ? RR_OK : hip_fail(e, "hipGetDevice");
    b->opt = current_tile_options();   // the override if set, else built-in shapes + tuning cache
    if (st == RR_OK) st = plan_or_fail(jobs, njobs, b->opt, &b->plan);
    if (st == RR_OK) st = fanout_init(&b->fan);
    if (st == RR_OK) st = upload_table(b);
    if (st == RR_OK && (flags & RR_BATCH_TUNE) && !b->plan.groups.empty()) st = tune(b);
    if (st != RR_OK) {
        if (b->dev_table) (void)hipFree(b->dev_table);
        fanout_destroy(&b->fan);
        delete b;
        return st;
    }
    *out = b;
    return RR_OK;
}

rr_status rr_batch_launch(rr_batch* b, rr_stream_t stream) {
    clear_error();
    if (!b) return fail(RR_ERR_INVALID_ARG, "NULL batch");
    if (b->plan.groups.empty()) return RR_OK;
    hipStream_t hs = (hipStream_t)stream;
    if (!(b->flags & RR_BATCH_GRAPH))
        return launch_batch_plan(b->plan, (const uint8_t*)b->dev_table, b->persistent, b->device, hs, fan_of(b));
    if (!b->exec) {
        if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(RR_ERR_HIP, "capture stream");
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        rr_status st = launch_batch_plan(b->plan, (const uint8_t*)b->dev_table, b->persistent, b->device, b->cap_stream,
                                         fan_of(b));
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap_stream, &g);
        if (st != RR_OK) { if (g) (void)hipGraphDestroy(g); return st; }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { drop_graph(b); return hip_fail(e, "hipGraphInstantiate"); }
    }
    hipError_t e = hipGraphLaunch(b->exec, hs);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return RR_OK;
}

rr_status rr_batch_get_info(const rr_batch* b, rr_batch_info* out) {
    clear_error();
    if (!b || !out) return fail(RR_ERR_INVALID_ARG, "NULL argument");
    std::memset(out, 0, sizeof *out);
    out->njobs = (int32_t)b->plan.njobs;
    out->ngroups = (int32_t)b->plan.groups.size();
    out->in_row_bytes = b->opt.in_row_bytes;
    out->out_row_bytes = b->opt.out_row_bytes;
    out->order_out = b->opt.order_out;
    out->persistent = b->persistent ? 1 : 0;
    out->bytes = b->plan.bytes;
    out->tuned_us = b->tuned_us;
    out->tile_kib = b->opt.tile_kib;
    out->cache = b->opt.cache;
    out->fill = b->opt.fill;
    out->force_ragged = b->opt.force_ragged;
    return RR_OK;
}

rr_status rr_batch_describe(const rr_batch* b, char* buf, int buflen) {
    clear_error();
    if (!b || !buf || buflen < 1) return fail(RR_ERR_INVALID_ARG, "NULL argument");
    std::string text;
    for (const BatchGroup& g : b->plan.groups) {
        std::string k;
        if (g.kind == K_COPY) k = "k_batch_copy<" + std::to_string(g.variant) + ">";
        else if (g.kind == K_RUN) k = "k_batch_run<" + std::to_string(g.variant) + ">";
        else k = "k_batch_tile<" + std::to_string(g.variant / 100) + "," + std::to_string(g.variant % 100) + ">";
        text += "kernel=" + k + " jobs=" + std::to_string(g.njobs) + " workgroups=" + std::to_string(g.total_blocks) +
                " bytes=" + std::to_string(g.bytes) + " lds=" + std::to_string(g.lds_bytes) + "\n";
    }
    if ((int)text.size() + 1 > buflen) return fail(RR_ERR_INVALID_ARG, "buffer too short");
    std::memcpy(buf, text.c_str(), text.size() + 1);
    return RR_OK;
}

rr_status rr_batch_destroy(rr_batch* b) {
    clear_error();
    if (!b) return RR_OK;
    drop_graph(b);
    fanout_destroy(&b->fan);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->dev_table) (void)hipFree(b->dev_table);
    delete b;
    return RR_OK;
}

}  // extern "C"
