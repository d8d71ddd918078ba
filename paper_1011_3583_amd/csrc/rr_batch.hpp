// rr_batch.hpp -- planning of batched permutes (host side, no HIP).
//
// Jobs are validated and planned one by one exactly as rr_permute would plan
// them, then grouped by kernel family (copy / run / tile with a given unit and
// micro-tile).  Each group becomes one device table: the jobs' argument blocks
// plus an exclusive prefix sum of their workgroup counts, so one launch of the
// family's batched kernel covers every job of the group; workgroup b finds its
// job by binary search over the prefix sums.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "rr_plan.hpp"

namespace rr {

struct BatchGroup {
    int32_t kind;          // K_COPY / K_RUN / K_TILE
    int32_t variant;       // vector bytes (copy, run) or unit*100 + g (tile)
    uint32_t njobs;        // entries (whole jobs or chunks of jobs)
    uint32_t total_blocks;
    uint32_t lds_bytes;    // largest tile of the group
    uint32_t pad_;
    uint64_t args_off;     // byte offset of the argument array in the table
    uint64_t prefix_off;   // byte offset of the njobs+1 prefix sums (uint32), followed
                           // by the group's bucket index (batch_buckets entries)
    uint64_t range_off;    // byte offset of njobs EntryRange records
    uint64_t bytes;        // bytes per side moved by the group
};

// Bucket index after a group's prefix sums: entry k is the job that holds
// workgroup k * BATCH_BUCKET (the last job where that is past the end), so a
// workgroup's job lies between its bucket's entry and the next one's.
#ifndef RR_BATCH_BUCKET
#define RR_BATCH_BUCKET 32
#endif
constexpr uint32_t BATCH_BUCKET = RR_BATCH_BUCKET;
constexpr uint64_t batch_buckets(uint64_t total_blocks) {
    return total_blocks ? (total_blocks - 1) / BATCH_BUCKET + 2 : 1;
}

// Which of its job's workgroups an entry runs: blocks [first, first + count)
// of a launch of `job_blocks` workgroups, taken by the group's workgroups
// [start, start + count).  A whole job is {0, grid, start, grid}.  One 16-byte
// record, so a workgroup reads everything it maps by in a single load once it
// knows its entry.
struct EntryRange {
    uint32_t first;
    uint32_t job_blocks;
    uint32_t start;
    uint32_t count;
};

// One entry of a batch: a planned job, or a contiguous range of its workgroups.
struct BatchEntry {
    const Plan* plan;
    uint32_t first_block;
    uint32_t nblocks;
    uint64_t bytes;        // bytes per side this entry moves (for accounting)
};

struct BatchPlan {
    std::vector<uint8_t> table;        // argument arrays and prefix sums, 256-byte aligned pieces
    std::vector<BatchGroup> groups;
    uint64_t bytes = 0;                // bytes per side over all jobs
    uint32_t njobs = 0;
};

// Validate and plan `njobs` jobs.  On error *bad_job is the index of the first
// failing job (or -1 for a cross-job overlap) and nothing is planned.
rr_status plan_batch(const rr_job* jobs, int njobs, const TileOptions& opt, BatchPlan* out,
                     std::string* why, int* bad_job);

// Validate every job (shape, buffers, its own aliasing) and the overlaps between
// jobs, without planning them: what plan_batch reports, before any planning.
rr_status validate_batch(const rr_job* jobs, int njobs, std::string* why, int* bad_job);

// Validate one job and plan it (no overlap check against other jobs).
rr_status plan_job(const rr_job& j, const TileOptions& opt, Plan* p, std::string* why);

// Group already planned entries into a batch table.
rr_status build_batch(const std::vector<BatchEntry>& entries, BatchPlan* out, std::string* why);

}  // namespace rr
