// rr_batch_plan.cpp -- validation, per-job planning and grouping of batched
// permutes (host only; shared by the library and its CPU emulator).
#include <unistd.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>

#include "rr_batch.hpp"

namespace rr {

namespace {

struct Interval {
    uint64_t lo, hi;  // [lo, hi)
    int job;
};

// Destinations must not overlap any other job's source or destination.
bool find_overlap(std::vector<Interval>& dsts, std::vector<Interval>& srcs, int* a, int* b) {
    std::sort(dsts.begin(), dsts.end(), [](const Interval& x, const Interval& y) { return x.lo < y.lo; });
    for (size_t i = 1; i < dsts.size(); ++i)
        if (dsts[i].lo < dsts[i - 1].hi) { *a = dsts[i - 1].job; *b = dsts[i].job; return true; }
    for (const Interval& s : srcs) {
        // last destination starting before the source ends
        auto it = std::lower_bound(dsts.begin(), dsts.end(), s.hi,
                                   [](const Interval& d, uint64_t v) { return d.lo < v; });
        if (it == dsts.begin()) continue;
        --it;
        if (it->hi > s.lo && it->job != s.job) { *a = it->job; *b = s.job; return true; }
    }
    return false;
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace

static rr_status validate_job(const rr_job& j, Canon* c, std::string* why) {
    rr_status st = canonicalize(j.ndim, j.dims, j.perm, j.elem_size, c, why);
    if (st != RR_OK) return st;
    if (c->total_bytes > 0) {
        if (!j.dst || !j.src) { *why = "NULL buffer for a non-empty job"; return RR_ERR_INVALID_ARG; }
        const uint64_t d = (uint64_t)j.dst, s = (uint64_t)j.src, n = (uint64_t)c->total_bytes;
        if (d < s + n && s < d + n) { *why = "job source and destination overlap"; return RR_ERR_ALIAS; }
    }
    return RR_OK;
}

rr_status plan_job(const rr_job& j, const TileOptions& opt, Plan* p, std::string* why) {
    Canon c;
    rr_status st = validate_job(j, &c, why);
    if (st != RR_OK) return st;
    return plan_permute((uint64_t)j.dst, (uint64_t)j.src, c, batch_job_options(opt, c.total_bytes), p, why);
}

// Host threads that plan (or validate) a batch of njobs: one below 256 jobs,
// else one per 128 jobs up to 8 and the host's cores.
static int planning_threads(int njobs) {
    if (njobs < 256) return 1;
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    return std::max(1, std::min({8, hw, njobs / 128}));
}

// Worker threads kept for the life of the process to run the slices of a
// validation or planning pass.  Starting and joining a thread per slice cost
// 30-100 us per thread on every call (7 threads: 0.2-0.7 ms, about what
// validating 4096 jobs takes on one core), and a one-shot batch waits for that
// before its first chunk runs.  One pass at a time uses the workers; a caller
// that finds them busy, or runs in a child forked after they started, starts
// threads of its own as before.  The pool is never destroyed: its workers are
// detached and sleep until the next pass, and the process ends them at exit.
class SlicePool {
   public:
    static constexpr int MAXW = 7;   // slices 1..7; slice 0 runs on the caller

    static SlicePool* get() {
        static SlicePool* pool = [] {
            SlicePool* p = new SlicePool();
            for (int w = 1; w <= MAXW; ++w) {
                try {
                    std::thread(&SlicePool::worker, p, w).detach();
                } catch (...) {
                    break;
                }
                p->nworkers_ = w;
            }
            return p;
        }();
        return pool->nworkers_ > 0 && pool->pid_ == getpid() ? pool : nullptr;
    }

    // Run body(t) for t in [0, nt) with slices 1..nworkers on the workers and
    // the rest on the caller; false (nothing run) if another pass holds them.
    bool try_run(int nt, const std::function<void(int)>& body) {
        std::unique_lock<std::mutex> pass(pass_mu_, std::try_to_lock);
        if (!pass.owns_lock()) return false;
        const int use = std::min(nt, nworkers_ + 1);
        {
            std::lock_guard<std::mutex> lk(mu_);
            body_ = &body;
            nt_ = use;
            pending_ = use - 1;
            ++gen_;
        }
        cv_.notify_all();
        // the workers use `body` until they report back: wait for them even if
        // the caller's own slices throw
        std::exception_ptr err;
        try {
            body(0);
            for (int t = use; t < nt; ++t) body(t);
        } catch (...) {
            err = std::current_exception();
        }
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return pending_ == 0; });
        body_ = nullptr;
        lk.unlock();
        if (err) std::rethrow_exception(err);
        return true;
    }

   private:
    void worker(int w) {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (w >= nt_) continue;   // not part of this pass
            const std::function<void(int)>* b = body_;
            lk.unlock();
            (*b)(w);
            lk.lock();
            if (--pending_ == 0) done_.notify_one();
        }
    }

    const pid_t pid_ = getpid();
    int nworkers_ = 0;
    std::mutex pass_mu_;   // held by the pass using the workers
    std::mutex mu_;        // guards the fields below
    std::condition_variable cv_, done_;
    const std::function<void(int)>* body_ = nullptr;
    int nt_ = 0, pending_ = 0;
    uint64_t gen_ = 0;
};

// Run body(t) for t in [0, nt): t = 0 on the calling thread, the others on the
// pool's workers, or on threads of their own when those are busy (or here,
// where no thread can be started).
template <class Body>
static void run_slices(int nt, Body body) {
    if (nt <= 1) {
        body(0);
        return;
    }
    if (SlicePool* pool = SlicePool::get()) {
        const std::function<void(int)> f = [&](int t) { body(t); };
        if (pool->try_run(nt, f)) return;
    }
    std::vector<std::thread> th;
    std::vector<int> inline_slices;
    for (int t = 1; t < nt; ++t) {
        try {
            th.emplace_back(body, t);
        } catch (...) {
            inline_slices.push_back(t);
        }
    }
    body(0);
    for (int t : inline_slices) body(t);
    for (std::thread& x : th) x.join();
}

rr_status plan_batch(const rr_job* jobs, int njobs, const TileOptions& opt, BatchPlan* out,
                     std::string* why, int* bad_job) {
    *bad_job = -1;
    out->table.clear();
    out->groups.clear();
    out->bytes = 0;
    out->njobs = 0;
    if (njobs < 0) { *why = "njobs < 0"; return RR_ERR_INVALID_ARG; }
    if (njobs > 0 && !jobs) { *why = "jobs is NULL"; return RR_ERR_INVALID_ARG; }

    // A Plan is over a kilobyte: a fresh array for thousands of jobs costs more in
    // page faults and zero fill than planning them, so each calling thread keeps
    // its array (grown on demand; only the members a plan's kind uses are read).
    // A batch larger than KEEP_PLANS jobs gives its array back when it is done.
    constexpr size_t KEEP_PLANS = 16384;   // about 20 MB
    static thread_local std::vector<Plan> tl_plans;
    if (tl_plans.size() < (size_t)njobs) tl_plans.resize((size_t)njobs);
    struct Release {
        ~Release() {
            if (tl_plans.size() > KEEP_PLANS) std::vector<Plan>().swap(tl_plans);
        }
    } release;
    Plan* const plans = tl_plans.data();   // the planning threads fill this thread's array
    // Jobs plan independently (about a microsecond each): large batches split
    // them into contiguous slices over a few host threads.  The lowest failing
    // job is reported, as in a sequential pass.
    const int nt = planning_threads(njobs);
    std::vector<int> bad((size_t)nt, -1);
    std::vector<rr_status> sts((size_t)nt, RR_OK);
    std::vector<std::string> whys((size_t)nt);
    auto slice = [&](int t) {
        const int lo = (int)((int64_t)njobs * t / nt), hi = (int)((int64_t)njobs * (t + 1) / nt);
        for (int i = lo; i < hi; ++i) {
            const rr_status st = plan_job(jobs[i], opt, &plans[i], &whys[(size_t)t]);
            if (st != RR_OK) { sts[(size_t)t] = st; bad[(size_t)t] = i; return; }
        }
    };
    run_slices(nt, slice);
    for (int t = 0; t < nt; ++t)
        if (sts[(size_t)t] != RR_OK) { *why = whys[(size_t)t]; *bad_job = bad[(size_t)t]; return sts[(size_t)t]; }
    std::vector<Interval> dsts, srcs;
    dsts.reserve((size_t)njobs);
    srcs.reserve((size_t)njobs);
    for (int i = 0; i < njobs; ++i) {
        const uint64_t n = plans[i].bytes;
        if (plans[i].kind != K_EMPTY && n > 0) {
            const uint64_t d = (uint64_t)jobs[i].dst, s = (uint64_t)jobs[i].src;
            dsts.push_back({d, d + n, i});
            srcs.push_back({s, s + n, i});
        }
    }
    int ja, jb;
    if (find_overlap(dsts, srcs, &ja, &jb)) {
        *why = "jobs " + std::to_string(ja) + " and " + std::to_string(jb) + " overlap";
        *bad_job = -1;
        return RR_ERR_ALIAS;
    }
    std::vector<BatchEntry> entries;
    entries.reserve((size_t)njobs);
    for (int i = 0; i < njobs; ++i) {   // the array may be longer than this batch
        const Plan& p = plans[i];
        if (p.kind != K_EMPTY && p.grid > 0) entries.push_back({&p, 0, p.grid, p.bytes});
    }
    return build_batch(entries, out, why);
}

rr_status validate_batch(const rr_job* jobs, int njobs, std::string* why, int* bad_job) {
    *bad_job = -1;
    if (njobs < 0) { *why = "njobs < 0"; return RR_ERR_INVALID_ARG; }
    if (njobs > 0 && !jobs) { *why = "jobs is NULL"; return RR_ERR_INVALID_ARG; }
    // contiguous slices on a few host threads; the lowest failing job is reported
    const int nt = planning_threads(njobs);
    std::vector<std::vector<Interval>> tdst((size_t)nt), tsrc((size_t)nt);
    std::vector<int> bad((size_t)nt, -1);
    std::vector<rr_status> sts((size_t)nt, RR_OK);
    std::vector<std::string> whys((size_t)nt);
    run_slices(nt, [&](int t) {
        const int lo = (int)((int64_t)njobs * t / nt), hi = (int)((int64_t)njobs * (t + 1) / nt);
        for (int i = lo; i < hi; ++i) {
            Canon c;
            const rr_status st = validate_job(jobs[i], &c, &whys[(size_t)t]);
            if (st != RR_OK) { sts[(size_t)t] = st; bad[(size_t)t] = i; return; }
            if (c.total_bytes > 0) {
                const uint64_t d = (uint64_t)jobs[i].dst, s = (uint64_t)jobs[i].src, n = (uint64_t)c.total_bytes;
                tdst[(size_t)t].push_back({d, d + n, i});
                tsrc[(size_t)t].push_back({s, s + n, i});
            }
        }
    });
    for (int t = 0; t < nt; ++t)
        if (sts[(size_t)t] != RR_OK) { *why = whys[(size_t)t]; *bad_job = bad[(size_t)t]; return sts[(size_t)t]; }
    std::vector<Interval> dsts, srcs;
    dsts.reserve((size_t)njobs);
    srcs.reserve((size_t)njobs);
    for (int t = 0; t < nt; ++t) {
        dsts.insert(dsts.end(), tdst[(size_t)t].begin(), tdst[(size_t)t].end());
        srcs.insert(srcs.end(), tsrc[(size_t)t].begin(), tsrc[(size_t)t].end());
    }
    int ja, jb;
    if (find_overlap(dsts, srcs, &ja, &jb)) {
        *why = "jobs " + std::to_string(ja) + " and " + std::to_string(jb) + " overlap";
        return RR_ERR_ALIAS;
    }
    return RR_OK;
}

rr_status build_batch(const std::vector<BatchEntry>& entries, BatchPlan* out, std::string* why) {
    out->table.clear();
    out->groups.clear();
    out->bytes = 0;
    out->njobs = 0;
    // group by kernel family and, for tiles, by LDS size class (a group launches
    // with its largest tile's LDS, which sets how many workgroups share a CU),
    // keeping entry order within a group
    using Key = std::tuple<int, int, int>;
    std::map<Key, std::vector<size_t>> fam;
    for (size_t i = 0; i < entries.size(); ++i) {
        const Plan& p = *entries[i].plan;
        if (p.kind == K_EMPTY || entries[i].nblocks == 0) continue;
        if (p.kind != K_COPY && p.kind != K_RUN && p.kind != K_TILE) {   // dense jobs plan to these only
            *why = "batch entry of a kind the batched kernels do not run";
            return RR_ERR_UNSUPPORTED;
        }
        int variant = 0;
        if (p.kind == K_COPY) variant = (int)p.copy.wbytes;
        else if (p.kind == K_RUN) variant = (int)p.run.wbytes;
        else variant = (int)(p.tile.unit * 100 + p.tile.g);
        int lds_class = 0;
        if (p.kind == K_TILE) lds_class = p.tile.lds_bytes <= 16384 ? 0 : p.tile.lds_bytes <= 32768 ? 1 : 2;
        fam[Key{(int)p.kind, variant, lds_class}].push_back(i);
        out->bytes += entries[i].bytes;
        out->njobs++;
    }
    uint64_t off = 0;
    for (auto& kv : fam) {
        BatchGroup g;
        std::memset(&g, 0, sizeof g);
        g.kind = std::get<0>(kv.first);
        g.variant = std::get<1>(kv.first);
        g.njobs = (uint32_t)kv.second.size();
        size_t asz = g.kind == K_COPY ? sizeof(CopyArgs) : g.kind == K_RUN ? sizeof(RunArgs) : sizeof(TileArgs);
        g.args_off = off;
        off = align_up(off + asz * g.njobs, 256);
        uint64_t blocks = 0;
        for (size_t m : kv.second) blocks += entries[m].nblocks;
        g.prefix_off = off;
        off = align_up(off + 4ull * (g.njobs + 1) + 4ull * batch_buckets(blocks), 256);
        g.range_off = off;
        off = align_up(off + sizeof(EntryRange) * g.njobs, 256);
        out->groups.push_back(g);
    }
    out->table.assign(off, 0);
    size_t gi = 0;
    for (auto& kv : fam) {
        BatchGroup& g = out->groups[gi++];
        const std::vector<size_t>& members = kv.second;
        uint32_t* prefix = reinterpret_cast<uint32_t*>(out->table.data() + g.prefix_off);
        EntryRange* ranges = reinterpret_cast<EntryRange*>(out->table.data() + g.range_off);
        uint8_t* argp = out->table.data() + g.args_off;
        uint64_t acc = 0;
        for (size_t m = 0; m < members.size(); ++m) {
            const BatchEntry& e = entries[members[m]];
            const Plan& p = *e.plan;
            prefix[m] = (uint32_t)acc;
            ranges[m].first = e.first_block;
            ranges[m].job_blocks = p.grid;
            ranges[m].start = (uint32_t)acc;
            ranges[m].count = e.nblocks;
            acc += e.nblocks;
            g.bytes += e.bytes;
            if (g.kind == K_COPY) std::memcpy(argp + m * sizeof(CopyArgs), &p.copy, sizeof(CopyArgs));
            else if (g.kind == K_RUN) std::memcpy(argp + m * sizeof(RunArgs), &p.run, sizeof(RunArgs));
            else {
                std::memcpy(argp + m * sizeof(TileArgs), &p.tile, sizeof(TileArgs));
                g.lds_bytes = std::max(g.lds_bytes, p.tile.lds_bytes);
            }
        }
        if (acc > 0x7fffffffULL) { *why = "batch group exceeds 2^31 workgroups"; return RR_ERR_UNSUPPORTED; }
        prefix[members.size()] = (uint32_t)acc;
        g.total_blocks = (uint32_t)acc;
        // bucket index: the job of every BATCH_BUCKET-th workgroup
        uint32_t* bucket = prefix + members.size() + 1;
        const uint64_t nbk = batch_buckets(acc);
        uint32_t j = 0;
        for (uint64_t k = 0; k < nbk; ++k) {
            const uint64_t first = k * BATCH_BUCKET;
            if (first >= acc) { bucket[k] = g.njobs - 1; continue; }
            while (j + 1 < g.njobs && prefix[j + 1] <= first) ++j;
            bucket[k] = j;
        }
    }
    return RR_OK;
}

}  // namespace rr
