// rr_serve.cpp -- continuous-batching server for permute jobs.
//
// One server thread owns admission, batching and completion:
//   * submissions wait in a FIFO queue; a job is admitted when its output (if the
//     server allocates it) fits in the HBM budget -- jobs that need no memory may
//     pass a job that is waiting for memory;
//   * while fewer than max_inflight batches are on the device, the thread forms
//     the next batch from the admitted jobs (at most max_batch_jobs);
//   * a large job (output above chunk_bytes) with max_inflight >= 2 goes whole,
//     in a launch of its own on its own stream: the device runs the small jobs'
//     batches beside it (workgroups of kernels on several hardware queues share
//     the CUs), so it delays them only by the bandwidth it takes, and large jobs
//     hold at most max_inflight - 1 slots.  With one slot a batch blocks the
//     device while it runs, so a large job is cut into ranges of its own
//     workgroups (pieces of chunk_bytes of output and up), each batched with
//     the jobs that arrived meanwhile;
//   * each batch goes on the stream with the fewest batches in flight, so
//     batches overlap on the device; completion is observed with events and
//     published to a completion queue;
//   * jobs are validated and planned by the submitting thread, outside the
//     server's lock (a job whose output the server allocates is planned for a
//     256-byte aligned placeholder and moved to its buffer at admission); when
//     the server is idle, the submitting thread also admits and launches the
//     job itself, sparing it the hand-over to the server thread;
//   * the HBM budget caps the device memory the server has reserved (its arena
//     slabs), not only the bytes in use; slabs with nothing left in them are
//     given back when a job would otherwise not fit.
// A simulated backend (RR_SERVE_SIMULATED) replaces memory and launches with
// virtual addresses and synthetic durations, so the same policy code runs on a
// machine without a GPU.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rr_batch.hpp"
#include "rr_internal.hpp"
#include "rr_kernels.hpp"

namespace rr {
namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// ----------------------------------------------------------------- backends
struct Backend {
    virtual ~Backend() {}
    virtual rr_status init(int device, int nslots, int nstreams) = 0;
    virtual void bind_thread() {}
    // launch_single from a thread other than the server's (its own current device kept)
    virtual rr_status launch_single_from_caller(int slot, int stream, const Plan& p) {
        return launch_single(slot, stream, p);
    }
    virtual void* reserve(uint64_t bytes) = 0;
    virtual void release(void* p) = 0;
    // stage the table and launch a batch in slot `slot` on stream `stream`
    virtual rr_status launch(int slot, int stream, const BatchPlan& bp) = 0;
    // launch one job exactly as rr_permute does
    virtual rr_status launch_single(int slot, int stream, const Plan& p) = 0;
    virtual bool done(int slot) = 0;
};

class HipBackend : public Backend {
   public:
    ~HipBackend() override {
        for (Slot& s : slots_) {
            if (s.ev) (void)hipEventSynchronize(s.ev);
            if (s.ev) (void)hipEventDestroy(s.ev);
            if (s.host) (void)hipHostFree(s.host);
            if (s.dev) (void)hipFree(s.dev);
        }
        for (hipStream_t st : streams_) (void)hipStreamDestroy(st);
    }
    rr_status init(int device, int nslots, int nstreams) override {
        device_ = device;
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        slots_.resize((size_t)nslots);
        for (Slot& s : slots_) {
            if ((e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "hipEventCreate");
            // job-table staging for batches of up to a few thousand jobs, allocated
            // here: growing it while serving frees and pins memory, which waits for
            // the whole device
            if ((e = hipHostMalloc(&s.host, TABLE_BYTES, hipHostMallocDefault)) != hipSuccess)
                return hip_fail(e, "pinned staging");
            if ((e = hipMalloc(&s.dev, TABLE_BYTES)) != hipSuccess) return hip_fail(e, "device job table");
            s.cap = TABLE_BYTES;
        }
        streams_.resize((size_t)nstreams);
        for (hipStream_t& st : streams_)
            if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreate");
        return RR_OK;
    }
    void bind_thread() override { (void)hipSetDevice(device_); }
    void* reserve(uint64_t bytes) override {
        // allocate on the server's device without changing the caller's current device
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device_);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
        (void)hipSetDevice(prev);
        return p;
    }
    void release(void* p) override { (void)hipFree(p); }
    rr_status launch(int slot, int stream, const BatchPlan& bp) override {
        Slot& s = slots_[(size_t)slot];
        const size_t need = bp.table.size();
        if (need > s.cap) {
            if (s.host) (void)hipHostFree(s.host);
            if (s.dev) (void)hipFree(s.dev);
            s.host = s.dev = nullptr;
            s.cap = 0;
            const size_t cap = std::max<size_t>(round_up(need, 1 << 20), 1 << 20);
            if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess)
                return fail(RR_ERR_NO_MEMORY, "pinned staging");
            if (hipMalloc(&s.dev, cap) != hipSuccess) return fail(RR_ERR_NO_MEMORY, "device job table");
            s.cap = cap;
        }
        hipStream_t st = streams_[(size_t)stream];
        std::memcpy(s.host, bp.table.data(), need);
        hipError_t e = hipMemcpyAsync(s.dev, s.host, need, hipMemcpyHostToDevice, st);
        rr_status rs = e == hipSuccess ? launch_batch_plan(bp, (const uint8_t*)s.dev, false, device_, st)
                                       : hip_fail(e, "server table upload");
        e = hipEventRecord(s.ev, st);
        if (rs == RR_OK && e != hipSuccess) rs = hip_fail(e, "hipEventRecord");
        // A failed launch may have queued the table copy and some groups: let them
        // finish before the caller reuses the slot's buffers or the jobs' outputs.
        if (rs != RR_OK) drain_stream(st, s.ev, e == hipSuccess);
        return rs;
    }
    rr_status launch_single(int slot, int stream, const Plan& p) override {
        hipStream_t st = streams_[(size_t)stream];
        hipEvent_t ev = slots_[(size_t)slot].ev;
        hipError_t e = launch_plan(p, st);
        rr_status rs = e == hipSuccess ? RR_OK : hip_fail(e, "server direct launch");
        e = hipEventRecord(ev, st);
        if (rs == RR_OK && e != hipSuccess) rs = hip_fail(e, "hipEventRecord");
        if (rs != RR_OK) drain_stream(st, ev, e == hipSuccess);
        return rs;
    }
    rr_status launch_single_from_caller(int slot, int stream, const Plan& p) override {
        int prev = 0;
        const bool have_prev = hipGetDevice(&prev) == hipSuccess;
        if (!have_prev || prev != device_) (void)hipSetDevice(device_);
        const rr_status rs = launch_single(slot, stream, p);
        if (have_prev && prev != device_) (void)hipSetDevice(prev);
        return rs;
    }
    bool done(int slot) override { return hipEventQuery(slots_[(size_t)slot].ev) != hipErrorNotReady; }

   private:
    static constexpr size_t TABLE_BYTES = 2u << 20;
    static void drain_stream(hipStream_t st, hipEvent_t ev, bool recorded) {
        if (!recorded || hipEventSynchronize(ev) != hipSuccess) (void)hipStreamSynchronize(st);
    }
    struct Slot {
        void* host = nullptr;
        void* dev = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
    };
    int device_ = 0;
    std::vector<Slot> slots_;
    std::vector<hipStream_t> streams_;
};

class SimBackend : public Backend {
   public:
    // device_bytes: memory of the simulated device (0: unlimited); a reservation
    // beyond it fails as hipMalloc would
    SimBackend(double bytes_per_us, uint64_t device_bytes)
        : bpus_(bytes_per_us > 0 ? bytes_per_us : 4e6), cap_(device_bytes) {}
    rr_status init(int, int nslots, int) override {
        left_.assign((size_t)nslots, 0.0);
        return RR_OK;
    }
    void* reserve(uint64_t bytes) override {
        std::lock_guard<std::mutex> lk(mu_);
        if (cap_ && taken_ + bytes > cap_) return nullptr;
        const uint64_t p = next_;
        next_ += round_up(bytes, 1 << 20) + (1 << 20);
        taken_ += bytes;
        sizes_[p] = bytes;
        return reinterpret_cast<void*>(p);
    }
    void release(void* p) override {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = sizes_.find((uint64_t)p);
        if (it == sizes_.end()) return;
        taken_ -= it->second;
        sizes_.erase(it);
    }
    rr_status launch(int slot, int, const BatchPlan& bp) override { return occupy(slot, bp.bytes); }
    rr_status launch_single(int slot, int, const Plan& p) override { return occupy(slot, p.bytes); }
    bool done(int slot) override {
        std::lock_guard<std::mutex> lk(mu_);
        advance(now_ns());
        return left_[(size_t)slot] <= 0.0;
    }

   private:
    // One device whose bandwidth the batches in flight share equally (as
    // workgroups of kernels on several streams share the CUs): a batch costs
    // reading and writing its bytes plus 2 us of launch at the full rate.
    rr_status occupy(int slot, uint64_t bytes) {
        std::lock_guard<std::mutex> lk(mu_);
        advance(now_ns());
        left_[(size_t)slot] = 2.0 * (double)bytes + 2.0 * bpus_;
        return RR_OK;
    }
    // run the simulated device up to time t (ns)
    void advance(uint64_t t) {
        if (t_ == 0 || t < t_) { t_ = t; return; }
        const double per_ns = bpus_ * 1e-3;
        while (t_ < t) {
            int n = 0;
            double first = 0.0;
            for (double l : left_)
                if (l > 0.0) { first = n == 0 ? l : std::min(first, l); ++n; }
            if (n == 0) { t_ = t; break; }
            const double rate = per_ns / n;               // bytes per ns for each batch
            const double dt = std::min((double)(t - t_), first / rate);
            for (double& l : left_)
                if (l > 0.0) { l -= rate * dt; if (l < 1e-6 * bpus_) l = 0.0; }
            t_ += std::max<uint64_t>(1, (uint64_t)dt);
        }
    }
    double bpus_;
    uint64_t cap_;
    std::mutex mu_;
    uint64_t taken_ = 0;
    std::unordered_map<uint64_t, uint64_t> sizes_;
    uint64_t next_ = 0x200000000000ull;
    uint64_t t_ = 0;                  // simulated time reached (ns)
    std::vector<double> left_;        // bytes each slot's batch has still to move
};

// ----------------------------------------------------------------- arena
// First-fit allocator with coalescing over slabs reserved from the backend.  The
// slabs themselves (not only what is handed out of them) stay within the budget:
// a new slab takes at most what the budget has left, and when that is too little
// the slabs with nothing allocated in them are given back first.
enum class AllocFail { NONE, NO_ROOM, BACKEND };

class Arena {
   public:
    Arena(Backend* be, uint64_t budget) : be_(be), budget_(budget) {}
    ~Arena() {
        for (auto& s : slabs_) be_->release(reinterpret_cast<void*>(s.base));
    }
    // NO_ROOM: would take the reserved memory past the budget (wait for frees);
    // BACKEND: the device refused memory although the budget had room
    void* alloc(uint64_t bytes, AllocFail* why) {
        *why = AllocFail::NONE;
        bytes = round_up(std::max<uint64_t>(bytes, 1), 256);
        if (void* p = fit(bytes)) return p;
        for (int attempt = 0; attempt < 2; ++attempt) {
            const uint64_t room = budget_ > reserved_ ? budget_ - reserved_ : 0;
            if (room >= bytes) {
                uint64_t slab = std::max<uint64_t>(bytes, std::min<uint64_t>(256ull << 20, room));
                void* p = be_->reserve(slab);
                if (!p && slab > bytes) p = be_->reserve(slab = bytes);   // the device is short: just this job
                if (!p) { *why = AllocFail::BACKEND; return nullptr; }
                reserved_ += slab;
                slabs_.push_back(Slab{(uint64_t)p, slab, {}, 0});
                Slab& s = slabs_.back();
                if (slab > bytes) s.free[bytes] = slab - bytes;
                used_[s.base] = bytes;
                s.live = 1;
                return p;
            }
            if (attempt == 0 && !trim()) break;
        }
        *why = AllocFail::NO_ROOM;
        return nullptr;
    }
    // returns the bytes freed (0 if p is not an allocation of this arena)
    uint64_t free(void* p) {
        auto u = used_.find((uint64_t)p);
        if (u == used_.end()) return 0;
        const uint64_t addr = u->first, len = u->second;
        used_.erase(u);
        for (Slab& s : slabs_) {
            if (addr < s.base || addr >= s.base + s.size) continue;
            s.live--;
            uint64_t off = addr - s.base, n = len;
            auto next = s.free.lower_bound(off);
            if (next != s.free.end() && next->first == off + n) { n += next->second; next = s.free.erase(next); }
            if (next != s.free.begin()) {
                auto prev = std::prev(next);
                if (prev->first + prev->second == off) { prev->second += n; return len; }
            }
            s.free[off] = n;
            return len;
        }
        return len;
    }
    uint64_t reserved() const { return reserved_; }

   private:
    struct Slab {
        uint64_t base, size;
        std::map<uint64_t, uint64_t> free;  // offset -> length
        uint64_t live;                      // allocations handed out of it
    };
    void* fit(uint64_t bytes) {
        for (Slab& s : slabs_) {
            for (auto it = s.free.begin(); it != s.free.end(); ++it) {
                if (it->second >= bytes) {
                    const uint64_t off = it->first, len = it->second;
                    s.free.erase(it);
                    if (len > bytes) s.free[off + bytes] = len - bytes;
                    used_[s.base + off] = bytes;
                    s.live++;
                    return reinterpret_cast<void*>(s.base + off);
                }
            }
        }
        return nullptr;
    }
    // give the slabs with no allocation back to the backend; whether any was
    bool trim() {
        bool any = false;
        for (size_t i = 0; i < slabs_.size();) {
            if (slabs_[i].live == 0) {
                be_->release(reinterpret_cast<void*>(slabs_[i].base));
                reserved_ -= slabs_[i].size;
                slabs_.erase(slabs_.begin() + (long)i);
                any = true;
            } else {
                ++i;
            }
        }
        return any;
    }
    Backend* be_;
    uint64_t budget_;
    uint64_t reserved_ = 0;
    std::vector<Slab> slabs_;
    std::unordered_map<uint64_t, uint64_t> used_;
};

// ----------------------------------------------------------------- server
struct JobState {
    uint64_t ticket = 0;
    rr_job job{};
    Plan plan;
    bool own_dst = false;
    uint64_t out_bytes = 0;
    uint32_t next_block = 0;     // first workgroup not yet put in a batch
    uint32_t chunk_blocks = 0;   // workgroups per chunk (0: whole job)
    uint32_t piece_mult = 1;     // chunks per piece: doubles while no other job waits
    uint32_t outstanding = 0;    // batches in flight holding a piece of this job
    int32_t chunks = 0;
    int32_t status = RR_OK;
    bool done = false;
    uint64_t t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
};

struct InFlight {
    int slot;
    int stream;
    std::vector<JobState*> jobs;
    uint64_t bytes;
    bool launched;   // false while a submitting thread is still launching it
    bool large;      // a large job launched whole, alone
};

// Placeholder output address a job is planned for when the server allocates its
// output: arena blocks are 256-byte aligned, so the plan is the same as for the
// real buffer up to the base address (moved at admission by rebase_dst).
constexpr uint64_t PLACEHOLDER_DST = 256;

void rebase_dst(Plan& p, uint64_t dst) {
    switch (p.kind) {
        case K_COPY: p.copy.dst = p.copy.dst - PLACEHOLDER_DST + dst; break;
        case K_RUN: p.run.dst = p.run.dst - PLACEHOLDER_DST + dst; break;
        case K_TILE: p.tile.dst = p.tile.dst - PLACEHOLDER_DST + dst; break;
        case K_SELECT: p.select.dst = p.select.dst - PLACEHOLDER_DST + dst; break;
        default: break;
    }
}

enum class Admit { OK, WAIT, NO_MEMORY };

}  // namespace
}  // namespace rr

using namespace rr;

struct rr_server {
    rr_serve_config cfg{};
    std::unique_ptr<Backend> be;
    std::unique_ptr<Arena> arena;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<JobState*> pending;
    std::deque<JobState*> large;
    std::unordered_map<uint64_t, std::unique_ptr<JobState>> jobs;
    std::deque<uint64_t> completions;
    std::vector<InFlight> inflight;
    std::vector<bool> slot_busy;
    std::unordered_map<uint64_t, uint64_t> user_allocs;
    uint64_t next_ticket = 1;
    uint64_t budget_used = 0;
    bool stopping = false;
    bool fail_next = false;
    int next_stream = 0;
    int nstreams = 1;
    std::vector<int> stream_load;   // batches in flight (or being launched) per stream
    int large_inflight = 0;         // large jobs launched whole, not yet retired
    uint64_t last_activity = 0;   // last submission or launch (server thread's spin window)
    rr_serve_stats stats{};
    std::thread th;

    void complete(JobState* j, uint64_t t) {
        j->done = true;
        j->t_done = t;
        if (j->status == RR_OK) stats.completed++; else stats.failed++;
        completions.push_back(j->ticket);
    }

    // Admit planned job j (lock held): allocate its output if the server owns it.
    // WAIT: the budget has no room now (a release may make some); NO_MEMORY: the
    // device refused memory within the budget while nothing was in flight, so no
    // completion can change that -- the job fails instead of waiting forever.
    Admit admit(JobState* j) {
        if (j->own_dst) {
            AllocFail why;
            void* p = arena->alloc(j->out_bytes, &why);
            if (!p) {
                if (why == AllocFail::BACKEND && inflight.empty()) {
                    j->status = RR_ERR_NO_MEMORY;
                    return Admit::NO_MEMORY;
                }
                return Admit::WAIT;
            }
            budget_used += round_up(j->out_bytes, 256);
            stats.budget_peak = std::max(stats.budget_peak, budget_used);
            j->job.dst = p;
            rebase_dst(j->plan, (uint64_t)p);
        }
        j->t_admit = now_ns();
        return Admit::OK;
    }

    // The stream with the fewest batches in flight, in turn among equals (lock
    // held): a batch queued behind a long one on its stream would wait for it
    // even with other streams idle.
    int take_stream() {
        int best = next_stream;
        for (int i = 1; i < nstreams; ++i) {
            const int s = (next_stream + i) % nstreams;
            if (stream_load[(size_t)s] < stream_load[(size_t)best]) best = s;
        }
        next_stream = (best + 1) % nstreams;
        stream_load[(size_t)best]++;
        return best;
    }

    int free_slot() const {
        if ((int)inflight.size() >= std::max(1, cfg.max_inflight)) return -1;
        for (int s = 0; s < std::max(1, cfg.max_inflight); ++s) if (!slot_busy[(size_t)s]) return s;
        return -1;
    }

    // Finish a batch whose launch failed (lock held): release its slot, fail its jobs.
    void fail_batch(int slot, int stream, bool large_launch, std::vector<JobState*>& members) {
        slot_busy[(size_t)slot] = false;
        stream_load[(size_t)stream]--;
        if (large_launch) large_inflight--;
        const uint64_t t = now_ns();
        for (JobState* j : members) {
            j->status = RR_ERR_HIP;
            j->outstanding--;
            // stop issuing the rest of a failed large job
            auto it = std::find(large.begin(), large.end(), j);
            if (it != large.end()) large.erase(it);
            if (j->outstanding == 0 && !j->done) complete(j, t);
        }
    }

    void loop() {
        be->bind_thread();
        const bool direct = (cfg.flags & RR_SERVE_DIRECT) != 0;
        const size_t maxjobs = direct ? 1 : (size_t)std::max(1, cfg.max_batch_jobs);
        for (;;) {
            std::vector<BatchEntry> entries;
            std::vector<JobState*> members;
            int slot = -1, stream = 0;
            bool fail_this = false;
            bool launch_large = false;
            {
                std::unique_lock<std::mutex> lk(mu);
                // retire finished batches
                const uint64_t t = now_ns();
                for (size_t i = 0; i < inflight.size();) {
                    if (!inflight[i].launched || !be->done(inflight[i].slot)) { ++i; continue; }
                    InFlight f = std::move(inflight[i]);
                    inflight.erase(inflight.begin() + (long)i);
                    slot_busy[(size_t)f.slot] = false;
                    stream_load[(size_t)f.stream]--;
                    if (f.large) large_inflight--;
                    stats.bytes_moved += f.bytes;
                    for (JobState* j : f.jobs) {
                        j->outstanding--;
                        const bool all_launched = j->status != RR_OK || j->next_block >= j->plan.grid;
                        if (j->outstanding == 0 && all_launched && !j->done) complete(j, t);
                    }
                }
                if (stopping && pending.empty() && large.empty() && inflight.empty()) break;
                // Shutting down with nothing in flight: a job still waiting for memory
                // would wait for a release that cannot come any more -- it fails.
                const bool drain = stopping && large.empty() && inflight.empty();
                slot = free_slot();
                if (slot >= 0) {
                    const int nslots = std::max(1, cfg.max_inflight);
                    if (nslots > 1) {
                        // Several slots: the device runs batches of different streams side
                        // by side (their workgroups share the CUs), so a large job goes
                        // whole, in a launch of its own, and the small jobs' batches run
                        // beside it.  New jobs first; a large one is admitted and queued.
                        // Large jobs hold at most nslots - 1 slots: one stays for the rest.
                        bool head_blocked = false;
                        for (auto it = pending.begin(); it != pending.end() && entries.size() < maxjobs;) {
                            JobState* j = *it;
                            if (head_blocked && j->own_dst && !drain) { ++it; continue; }
                            const Admit a = admit(j);
                            if (a == Admit::WAIT && !drain) { head_blocked = true; ++it; continue; }
                            it = pending.erase(it);
                            if (a == Admit::WAIT) j->status = RR_ERR_NO_MEMORY;
                            if (j->status != RR_OK) { complete(j, now_ns()); continue; }
                            if (j->plan.kind == K_EMPTY || j->plan.grid == 0) { complete(j, now_ns()); continue; }
                            if (j->chunk_blocks) { large.push_back(j); continue; }
                            entries.push_back({&j->plan, 0, j->plan.grid, j->plan.bytes});
                            members.push_back(j);
                            j->next_block = j->plan.grid;
                            j->outstanding++;
                            j->chunks++;
                        }
                        if (entries.empty() && !large.empty() && large_inflight + 1 < nslots) {
                            JobState* j = large.front();
                            large.pop_front();
                            entries.push_back({&j->plan, j->next_block, j->plan.grid - j->next_block,
                                               j->plan.bytes});
                            members.push_back(j);
                            j->next_block = j->plan.grid;
                            j->outstanding++;
                            j->chunks++;
                            launch_large = true;
                        }
                    } else {
                    // One slot: a batch blocks the device until it ends, so a large job
                    // goes in pieces, each in a batch with the jobs that arrived meanwhile.
                    // One piece of every large job in progress, oldest first.  A piece is
                    // piece_mult chunks: while no other job is waiting the pieces double
                    // (up to 16 chunks), since a lone large job gains nothing from fine
                    // pieces and pays a batch launch for each; any waiting job brings the
                    // pieces back to one chunk, so it is launched after at most one.
                    const bool others_waiting = !pending.empty() || large.size() > 1;
                    for (size_t k = 0; k < large.size() && entries.size() < maxjobs;) {
                        JobState* j = large[k];
                        j->piece_mult = others_waiting ? 1u : std::min<uint32_t>(j->piece_mult * 2, 16);
                        const uint32_t n = (uint32_t)std::min<uint64_t>((uint64_t)j->chunk_blocks * j->piece_mult,
                                                                        j->plan.grid - j->next_block);
                        const uint64_t bytes = (uint64_t)((double)j->plan.bytes * n / j->plan.grid);
                        entries.push_back({&j->plan, j->next_block, n, bytes});
                        members.push_back(j);
                        j->next_block += n;
                        j->outstanding++;
                        j->chunks++;
                        if (j->next_block >= j->plan.grid) large.erase(large.begin() + (long)k);
                        else ++k;
                    }
                    // newly admitted jobs, FIFO; jobs needing no memory may pass one that waits
                    bool head_blocked = false;
                    for (auto it = pending.begin(); it != pending.end() && entries.size() < maxjobs;) {
                        JobState* j = *it;
                        if (head_blocked && j->own_dst && !drain) { ++it; continue; }
                        const Admit a = admit(j);
                        if (a == Admit::WAIT && !drain) { head_blocked = true; ++it; continue; }
                        it = pending.erase(it);
                        if (a == Admit::WAIT) j->status = RR_ERR_NO_MEMORY;
                        if (j->status != RR_OK) { complete(j, now_ns()); continue; }
                        if (j->plan.kind == K_EMPTY || j->plan.grid == 0) { complete(j, now_ns()); continue; }
                        const uint32_t n = j->chunk_blocks ? j->chunk_blocks : j->plan.grid;
                        const uint64_t bytes = (uint64_t)((double)j->plan.bytes * n / j->plan.grid);
                        entries.push_back({&j->plan, 0, n, bytes});
                        members.push_back(j);
                        j->next_block = n;
                        j->outstanding++;
                        j->chunks++;
                        if (j->next_block < j->plan.grid) large.push_back(j);
                    }
                    }
                    if (entries.empty()) {
                        slot = -1;
                    } else {
                        slot_busy[(size_t)slot] = true;
                        stream = take_stream();
                        if (launch_large) large_inflight++;
                        fail_this = fail_next;
                        fail_next = false;
                        const uint64_t tl = now_ns();
                        for (JobState* j : members) if (!j->t_launch) j->t_launch = tl;
                        stats.batches++;
                        stats.chunks += entries.size();
                    }
                }
                if (slot < 0) {
                    // Nothing to launch now.  While batches are in flight or work arrived
                    // recently, poll without sleeping (a timed sleep costs tens of
                    // microseconds of timer slack per poll); otherwise block until a
                    // submission arrives or tick_us * 50 passes.
                    const uint64_t tnow = now_ns();
                    if (!inflight.empty() || tnow - last_activity < 2'000'000ull) {
                        lk.unlock();
                        std::this_thread::yield();
                        continue;
                    }
                    cv.wait_for(lk, std::chrono::microseconds(std::max<uint32_t>(cfg.tick_us, 1) * 50));
                    continue;
                }
                last_activity = now_ns();
            }
            // build and launch outside the lock
            BatchPlan bp;
            std::string why;
            rr_status st = RR_ERR_HIP;
            // a batch of one whole job needs no job table: launch it with its
            // arguments by value (what one launch per request does)
            const bool one_whole = entries.size() == 1 && entries[0].first_block == 0 &&
                                   entries[0].nblocks == entries[0].plan->grid;
            if (!fail_this && (direct || one_whole)) {
                st = be->launch_single(slot, stream, *entries[0].plan);
                bp.bytes = entries[0].bytes;
            } else if (!fail_this) {
                st = build_batch(entries, &bp, &why);
                if (st == RR_OK) st = be->launch(slot, stream, bp);
            }
            std::lock_guard<std::mutex> lk(mu);
            if (st != RR_OK) fail_batch(slot, stream, launch_large, members);
            else inflight.push_back(InFlight{slot, stream, std::move(members), bp.bytes, true, launch_large});
            if (log_level() >= 3)
                log_line(3, "serve: batch of " + std::to_string(entries.size()) + " entries, " +
                                std::to_string(bp.bytes) + " bytes per side, slot " + std::to_string(slot) +
                                (st == RR_OK ? "" : " (launch failed)"));
        }
    }
};

extern "C" {

rr_status rr_serve_create(const rr_serve_config* cfg, rr_server** out) {
    clear_error();
    if (!cfg || !out) return fail(RR_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (cfg->max_inflight < 1 || cfg->max_inflight > 64 || cfg->max_batch_jobs < 1 ||
        cfg->queue_capacity < 1 || cfg->hbm_budget_bytes == 0)
        return fail(RR_ERR_INVALID_ARG, "bad server configuration");
    auto s = std::make_unique<rr_server>();
    s->cfg = *cfg;
    if (cfg->flags & RR_SERVE_SIMULATED)
        s->be = std::make_unique<SimBackend>(cfg->sim_bytes_per_us, cfg->sim_device_bytes);
    else s->be = std::make_unique<HipBackend>();
    s->nstreams = std::min(cfg->max_inflight, 4);
    s->stream_load.assign((size_t)s->nstreams, 0);
    rr_status st = s->be->init(cfg->device, cfg->max_inflight, s->nstreams);
    if (st != RR_OK) return st;
    s->arena = std::make_unique<Arena>(s->be.get(), cfg->hbm_budget_bytes);
    s->slot_busy.assign((size_t)cfg->max_inflight, false);
    rr_server* raw = s.release();
    raw->th = std::thread([raw] { raw->loop(); });
    *out = raw;
    return RR_OK;
}

rr_status rr_serve_alloc(rr_server* s, uint64_t bytes, void** dptr) {
    clear_error();
    if (!s || !dptr || bytes == 0) return fail(RR_ERR_INVALID_ARG, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    const uint64_t b = round_up(bytes, 256);
    AllocFail why;
    void* p = s->arena->alloc(bytes, &why);
    if (!p) return fail(RR_ERR_NO_MEMORY, why == AllocFail::BACKEND ? "device allocation failed" : "over the HBM budget");
    s->budget_used += b;
    s->stats.budget_peak = std::max(s->stats.budget_peak, s->budget_used);
    s->user_allocs[(uint64_t)p] = b;
    *dptr = p;
    return RR_OK;
}

rr_status rr_serve_free(rr_server* s, void* dptr) {
    clear_error();
    if (!s) return fail(RR_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->user_allocs.find((uint64_t)dptr);
    if (it == s->user_allocs.end()) return fail(RR_ERR_INVALID_ARG, "not a server allocation");
    s->arena->free(dptr);
    s->budget_used -= it->second;
    s->user_allocs.erase(it);
    return RR_OK;
}

rr_status rr_serve_submit(rr_server* s, const rr_job* job, uint64_t* ticket) {
    clear_error();
    if (!s || !job || !ticket) return fail(RR_ERR_INVALID_ARG, "NULL argument");
    Canon c;
    std::string why;
    rr_status st = canonicalize(job->ndim, job->dims, job->perm, job->elem_size, &c, &why);
    if (st != RR_OK) return fail(st, why);
    const uint64_t nb = (uint64_t)c.total_bytes;
    if (nb > 0 && !job->src) return fail(RR_ERR_INVALID_ARG, "NULL source");
    if (job->dst && ranges_overlap((uint64_t)job->dst, nb, (uint64_t)job->src, nb))
        return fail(RR_ERR_ALIAS, "source and destination overlap");
    const bool own = job->dst == nullptr && nb > 0;
    if (own && round_up(nb, 256) > s->cfg.hbm_budget_bytes) return fail(RR_ERR_NO_MEMORY, "job exceeds the budget");
    // plan here, on the submitting thread, outside the server's lock
    auto j = std::make_unique<JobState>();
    j->job = *job;
    j->own_dst = own;
    j->out_bytes = nb;
    if (nb > 0) {
        const uint64_t dst = own ? PLACEHOLDER_DST : (uint64_t)job->dst;
        st = plan_permute(dst, (uint64_t)job->src, c, batch_job_options(current_tile_options(), c.total_bytes),
                          &j->plan, &why);
        if (st != RR_OK) return fail(st, why);
        if (!(s->cfg.flags & RR_SERVE_DIRECT) && s->cfg.chunk_bytes > 0 && j->plan.grid > 1 &&
            j->plan.bytes > s->cfg.chunk_bytes) {
            const uint64_t per_block = std::max<uint64_t>(1, j->plan.bytes / j->plan.grid);
            j->chunk_blocks = (uint32_t)std::max<uint64_t>(1, s->cfg.chunk_bytes / per_block);
        }
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stopping) return fail(RR_ERR_INVALID_ARG, "server is shutting down");
    if (nb > 0 && (int)s->pending.size() >= s->cfg.queue_capacity) return fail(RR_ERR_BUSY, "queue full");
    j->ticket = s->next_ticket++;
    j->t_submit = now_ns();
    JobState* raw = j.get();
    s->jobs[j->ticket] = std::move(j);
    s->stats.submitted++;
    *ticket = raw->ticket;
    if (nb == 0 || raw->plan.kind == K_EMPTY || raw->plan.grid == 0) {
        s->complete(raw, raw->t_submit);
        return RR_OK;
    }
    s->last_activity = raw->t_submit;
    // Idle fast path: nothing queued or in flight, no chunking -- admit and launch
    // here instead of handing the job to the server thread.  Only when the server
    // is idle: under load the launch would cost the submitting thread its time
    // while the server thread batches it just as fast.
    int slot = -1;
    const bool whole_large = s->cfg.max_inflight > 1;   // large jobs launch whole (see the server loop)
    if (s->pending.empty() && s->large.empty() && s->inflight.empty() && (raw->chunk_blocks == 0 || whole_large) &&
        !s->fail_next && (slot = s->free_slot()) >= 0) {
        const Admit a = s->admit(raw);
        if (a == Admit::NO_MEMORY) {
            s->complete(raw, now_ns());
            return RR_OK;
        }
        if (a == Admit::OK) {
            s->slot_busy[(size_t)slot] = true;
            const int stream = s->take_stream();
            const bool is_large = raw->chunk_blocks != 0;
            if (is_large) s->large_inflight++;
            raw->next_block = raw->plan.grid;
            raw->outstanding = 1;
            raw->chunks = 1;
            raw->t_launch = now_ns();
            s->stats.batches++;
            s->stats.chunks++;
            s->inflight.push_back(InFlight{slot, stream, {raw}, raw->plan.bytes, false, is_large});
            lk.unlock();
            const rr_status ls = s->be->launch_single_from_caller(slot, stream, raw->plan);
            lk.lock();
            for (size_t i = 0; i < s->inflight.size(); ++i) {
                if (s->inflight[i].slot != slot || s->inflight[i].launched) continue;
                if (ls == RR_OK) {
                    s->inflight[i].launched = true;
                } else {
                    std::vector<JobState*> members = std::move(s->inflight[i].jobs);
                    s->inflight.erase(s->inflight.begin() + (long)i);
                    s->fail_batch(slot, stream, is_large, members);
                }
                break;
            }
            s->cv.notify_one();
            return RR_OK;
        }
    }
    s->pending.push_back(raw);
    s->cv.notify_one();
    return RR_OK;
}

rr_status rr_serve_poll(rr_server* s, uint64_t ticket, rr_job_result* out) {
    if (!s || !out) return fail(RR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return fail(RR_ERR_INVALID_ARG, "unknown ticket");
    const JobState& j = *it->second;
    if (!j.done) return RR_ERR_NOT_READY;
    out->status = j.status;
    out->chunks = j.chunks;
    out->dst = j.job.dst;
    out->t_submit_ns = j.t_submit;
    out->t_admit_ns = j.t_admit;
    out->t_launch_ns = j.t_launch;
    out->t_done_ns = j.t_done;
    return RR_OK;
}

rr_status rr_serve_completions(rr_server* s, uint64_t* out, int max, int* n) {
    if (!s || !n || (max > 0 && !out)) return fail(RR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    int k = 0;
    while (k < max && !s->completions.empty()) {
        out[k++] = s->completions.front();
        s->completions.pop_front();
    }
    *n = k;
    return RR_OK;
}

rr_status rr_serve_release(rr_server* s, uint64_t ticket) {
    if (!s) return fail(RR_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return fail(RR_ERR_INVALID_ARG, "unknown ticket");
    JobState& j = *it->second;
    if (!j.done) return fail(RR_ERR_NOT_READY, "ticket still pending");
    if (j.own_dst && j.job.dst) {
        s->arena->free(j.job.dst);
        s->budget_used -= round_up(j.out_bytes, 256);
    }
    s->jobs.erase(it);
    return RR_OK;
}

rr_status rr_serve_destroy(rr_server* s) {
    clear_error();
    if (!s) return RR_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    s->arena.reset();
    s->be.reset();
    delete s;
    return RR_OK;
}

rr_status rr_serve_get_stats(rr_server* s, rr_serve_stats* out) {
    if (!s || !out) return fail(RR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->budget_used = s->budget_used;
    out->reserved = s->arena->reserved();
    return RR_OK;
}

rr_status rr_serve_fail_next_batch(rr_server* s) {
    if (!s) return fail(RR_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    s->fail_next = true;
    return RR_OK;
}

}  // extern "C"
