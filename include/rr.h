/*
 * rr.h -- C ABI of librr, an MI355X (gfx950) library of data-rearrangement
 * kernels: N-D permute/transpose/reorder (also of a box, N-to-M), index-set and
 * range reads, interlace and de-interlace, a 2-D stencil, a batched launch for
 * many uneven permutes, and a continuous-batching server.
 *
 * The operations are those of "Fast GPGPU Data Rearrangement Kernels using
 * CUDA" (arXiv:1011.3583): Sec. III.A (read/write kernels with access
 * patterns), Sec. III.B (re-ordering an N-dimensional array under a given order
 * of its axes, N-to-N and N-to-M), Sec. III.C (interlace / de-interlace) and
 * Sec. III.D (generic 2-D stencil).
 *
 * Conventions
 *  - Arrays are dense and row-major ("linearized storage", Sec. III.B): the LAST
 *    axis varies fastest.  Axis permutations use the row-major (NumPy) reading:
 *    the output has shape out_dims[j] = dims[perm[j]] and
 *        out[J] = in[I]  with  I[perm[j]] = J[j].
 *    The paper lists orders fastest-dimension-first; rr_order_to_perm converts.
 *  - Elements are opaque runs of elem_size bytes (1..16).  Apart from the
 *    stencil (fp32 arithmetic, see rr_stencil2d) no arithmetic is ever done on
 *    values: results are bit-exact copies (NaN payloads survive).
 *  - Device pointers are plain HIP device addresses (hipMalloc, or any torch
 *    CUDA tensor's data_ptr()).  The caller owns every buffer passed in; the
 *    library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Calls are stream-ordered and asynchronous: they return after enqueueing.
 *  - Argument validation happens synchronously, before anything is enqueued;
 *    on any error nothing is written and nothing is launched.
 *  - Source and destination byte ranges must not overlap (no in-place).
 *  - A problem with zero elements returns RR_OK and does nothing.
 *  - Error detail for the calling thread is available from rr_last_error().
 */
#ifndef RR_H
#define RR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RR_MAX_DIMS   8   /* input rank accepted by rr_permute */
#define RR_MAX_PLANES 16  /* data sets accepted by rr_interlace / rr_deinterlace */

typedef enum {
    RR_OK = 0,
    RR_ERR_INVALID_ARG = 1,  /* bad rank, perm, elem_size, count or NULL pointer   */
    RR_ERR_OVERFLOW = 2,     /* element count * elem_size does not fit in int64     */
    RR_ERR_ALIAS = 3,        /* source and destination byte ranges overlap          */
    RR_ERR_UNSUPPORTED = 4,  /* valid request outside what this build handles       */
    RR_ERR_NO_MEMORY = 5,    /* device/host allocation or server HBM budget refused */
    RR_ERR_BUSY = 6,         /* server queue full, retry later                      */
    RR_ERR_NOT_READY = 7,    /* server ticket still pending                         */
    RR_ERR_HIP = 8           /* a HIP runtime call failed; see rr_last_error()      */
} rr_status;

typedef void* rr_stream_t; /* a hipStream_t */

/* -------------------------------------------------------------------------
 * Permute (Sec. III.B, 3D Permute Kernel and generic Reorder Kernel).
 *   dst     device buffer of prod(dims)*elem_size bytes, written in the output
 *           order (row-major over out_dims[j] = dims[perm[j]]).
 *   src     device buffer of prod(dims)*elem_size bytes, row-major over dims.
 *   ndim    1..RR_MAX_DIMS.  dims[k] >= 0.  Size-1 axes are allowed anywhere.
 *   perm    a permutation of 0..ndim-1 (row-major reading above).
 *   elem_size 1..16 bytes.
 * Any alignment of src/dst is accepted; 16-byte aligned buffers take the
 * widest vector path.
 * Errors: RR_ERR_INVALID_ARG, RR_ERR_OVERFLOW, RR_ERR_ALIAS, RR_ERR_UNSUPPORTED,
 * RR_ERR_HIP (launch failure).
 */
rr_status rr_permute(void* dst, const void* src, int ndim, const int64_t* dims,
                     const int* perm, int elem_size, rr_stream_t stream);

/* -------------------------------------------------------------------------
 * N-to-M reorder with base and range (Sec. III.B, the reorder kernel's N-to-M
 * form): a box of the input, fewer dimensions out.
 *   Output axis j (0 <= j < out_ndim) runs over input axis order[j] from
 *   base[order[j]] for range[order[j]] steps; every input axis d not listed in
 *   order stays fixed at base[d]:
 *     dst[J] = src[I],  I[order[j]] = base[order[j]] + J[j],  I[d] = base[d].
 *   dst     device buffer of prod_j range[order[j]] * elem_size bytes, row-major
 *           over (range[order[0]], ..., range[order[out_ndim-1]]).
 *   src     device buffer of prod(dims)*elem_size bytes, row-major over dims
 *           (only the box is read).
 *   ndim    1..RR_MAX_DIMS; out_ndim 0..ndim (0: the single element at base).
 *   base    host array of ndim offsets, or NULL for all zeros; a fixed axis
 *           needs 0 <= base < dims.
 *   range   host array of ndim extents (entries of fixed axes are ignored), or
 *           NULL for "to the end"; a kept axis needs base + range <= dims.
 *   order   host array of out_ndim distinct axes of 0..ndim-1.
 * A box whose fastest input axis is kept and contiguous is tiled like
 * rr_permute; one that drops or cuts the input's fastest axis is gathered
 * element by element (reads cannot be coalesced there).
 * Errors: RR_ERR_INVALID_ARG, RR_ERR_OVERFLOW, RR_ERR_ALIAS (dst overlaps the
 * byte range spanned by the box), RR_ERR_UNSUPPORTED, RR_ERR_HIP.
 */
rr_status rr_reorder(void* dst, const void* src, int ndim, const int64_t* dims, const int64_t* base,
                     const int64_t* range, int out_ndim, const int* order, int elem_size,
                     rr_stream_t stream);

/* -------------------------------------------------------------------------
 * Read kernel over an index set (Sec. III.A, read/write kernels with an access
 * pattern given as a set of indices):
 *   dst[i] = src[idx[i]]   for 0 <= i < count, elements of elem_size bytes.
 *   dst        device buffer of count*elem_size bytes.
 *   src        device buffer of src_count elements.
 *   idx        device array of count int64 indices (any order, repeats allowed).
 *   bad_count  optional device uint64 (may be NULL): incremented by the number of
 *              indices outside [0, src_count); such elements are written as zeros.
 * Four elements per thread; each element is read with the widest access its
 * size and the pointers allow.  Host-side validation cannot see the indices
 * (they live on the device), hence the counter instead of an error status.
 * Errors: RR_ERR_INVALID_ARG, RR_ERR_OVERFLOW, RR_ERR_ALIAS (dst overlaps src,
 * idx or the counter), RR_ERR_HIP.
 */
rr_status rr_gather(void* dst, const void* src, int64_t src_count, const int64_t* idx, int64_t count,
                    int elem_size, uint64_t* bad_count, rr_stream_t stream);

/* -------------------------------------------------------------------------
 * Read kernel over a range (Sec. III.A, access based on a specified range):
 *   dst[i] = src[start + i*stride]   for 0 <= i < count (stride may be negative
 *   or zero); every index read must lie in [0, src_count).
 *   dst  device buffer of count*elem_size bytes; src device buffer of src_count
 *        elements.  stride 1 is a plain copy of the range.
 * Errors: RR_ERR_INVALID_ARG (range outside the source, bad sizes, NULL),
 * RR_ERR_OVERFLOW, RR_ERR_ALIAS (dst overlaps the bytes read), RR_ERR_HIP.
 */
rr_status rr_copy_range(void* dst, const void* src, int64_t src_count, int64_t start, int64_t stride,
                        int64_t count, int elem_size, rr_stream_t stream);

/* -------------------------------------------------------------------------
 * 2-D stencil (Sec. III.D, generic stencil kernel; its measured case is a
 * finite-difference stencil of orders I-IV on single-precision grids).  Each
 * point of a rows x cols float grid (row-major) becomes a weighted sum of its
 * neighbours, evaluated with fp32 fused multiply-adds:
 *   RR_STENCIL_STAR: weights[0..radius]; out = w0*x[i][j] + sum_{k=1..radius}
 *     wk * ((x[i-k][j] + x[i+k][j]) + (x[i][j-k] + x[i][j+k])).
 *   RR_STENCIL_BOX: weights[(2*radius+1)^2], row-major over dy = -r..r,
 *     dx = -r..r; out = sum w[dy][dx] * x[i+dy][j+dx].
 * Points closer than radius to an edge keep their input value.
 *   dst, src   device grids of rows*cols floats, 4-byte aligned, not overlapping.
 *   radius     1..4.  weights: host array (copied at the call).
 * Each workgroup produces a 32 x 128 tile (16 x 128 on grids above 2^24 points)
 * from LDS holding it plus its halo.
 * Errors: RR_ERR_INVALID_ARG, RR_ERR_OVERFLOW, RR_ERR_ALIAS, RR_ERR_UNSUPPORTED,
 * RR_ERR_HIP.
 */
#define RR_STENCIL_STAR 0
#define RR_STENCIL_BOX 1
rr_status rr_stencil2d(float* dst, const float* src, int64_t rows, int64_t cols, int radius, int shape,
                       const float* weights, rr_stream_t stream);

/* -------------------------------------------------------------------------
 * Interlace (Sec. III.C): join n equally long data sets, set index fastest:
 *   dst[i*n + c] = srcs[c][i]    for 0 <= i < count, 0 <= c < n.
 *   dst   device buffer of n*count*elem_size bytes.
 *   srcs  host array of n device pointers, each count*elem_size bytes.
 *   n     1..RR_MAX_PLANES.  count >= 0.  elem_size 1..16.
 * Errors: as rr_permute (RR_ERR_ALIAS if dst overlaps any source plane).
 */
rr_status rr_interlace(void* dst, const void* const* srcs, int n, int64_t count,
                       int elem_size, rr_stream_t stream);

/* -------------------------------------------------------------------------
 * De-interlace (Sec. III.C): split one interlaced set into n data sets:
 *   dsts[c][i] = src[i*n + c]    (e.g. complex numbers into real and
 *                                 imaginary planes with n = 2).
 *   dsts  host array of n device pointers, each count*elem_size bytes; the
 *         planes must not overlap each other or src.
 * Errors: as rr_interlace.
 */
rr_status rr_deinterlace(void* const* dsts, const void* src, int n, int64_t count,
                         int elem_size, rr_stream_t stream);

/* -------------------------------------------------------------------------
 * Batched permutes: many independent, unevenly shaped rr_permute jobs run with
 * one launch per kernel family (the paper's "batched 2D data movement",
 * Sec. III.B, applied across jobs): the jobs are planned as rr_permute would
 * plan them, grouped by kernel, and each group's launch walks the concatenated
 * work of all its jobs.  Each job's result is identical to running it alone.
 *   jobs   host array of njobs descriptors (copied before return; the array may
 *          be reused immediately).  Job buffers must not overlap each other.
 *   njobs  >= 0.
 * The job table is staged through pinned host and device buffers the library
 * owns (a small ring per device, grown on demand and held until process exit);
 * a call waits only if it would reuse a slot whose batch is still running.
 * The groups run side by side on `stream` and three side streams per device
 * that the library owns (default priority, held until process exit): they start
 * after the work queued on `stream` before the call, and work queued on `stream`
 * after the call waits for all of them.  Calls on one device share those side
 * streams, so batched calls issued on different streams may run one after the
 * other.  A batch of 2048 jobs or more is validated whole first, then planned,
 * staged and launched in up to four chunks of consecutive jobs (the first a
 * sixteenth of them), so the device runs the first chunks while the host plans the
 * rest; each chunk takes a ring slot, and its table goes up on a fourth stream of
 * the library.  Batches of 256 jobs or more are validated and planned in slices
 * on up to seven host worker threads that the library starts on first use and
 * keeps, asleep between calls, until process exit (a call that finds them busy
 * starts threads of its own for that call).
 * Errors: the first invalid job's error (nothing is launched), RR_ERR_NO_MEMORY,
 * RR_ERR_HIP.
 */
typedef struct {
    void* dst;
    const void* src;
    int32_t ndim;
    int32_t elem_size;
    int64_t dims[RR_MAX_DIMS];
    int32_t perm[RR_MAX_DIMS];
} rr_job;

rr_status rr_permute_batched(const rr_job* jobs, int njobs, rr_stream_t stream);

/* -------------------------------------------------------------------------
 * rr_permute_batched without any memory allocation, for callers that cannot
 * allocate device or pinned host memory (serving loops that must not call
 * hipMalloc, harnesses that forbid it).  Same jobs, validation, planning and
 * kernels as rr_permute_batched, and the same result for every job; the
 * differences:
 *  - the job table lives in a fixed 4 MiB device array of the library (one copy
 *    per GPU, held until the process ends) instead of a staging ring; a batch
 *    whose table exceeds it (about 5700 tiled jobs) fails with
 *    RR_ERR_UNSUPPORTED before anything is enqueued;
 *  - the table is copied from pageable host memory with a stream-ordered copy
 *    on `stream` (the call may block until the work already queued on `stream`
 *    has finished), and every group runs on `stream` itself (no side streams);
 *  - all calls on one GPU share that GPU's table: calls on the same stream are
 *    ordered, but calls that overlap in time on different streams of one GPU
 *    race on the table and must be ordered by the caller (events or one
 *    stream).  Not for graph capture (the copy would be recorded as a node that
 *    reads the calling thread's staging buffer).
 * Host planning uses per-thread buffers kept across calls and, for 256 jobs or
 * more, the host worker threads described under rr_permute_batched.
 * Errors: the first invalid job's error (nothing is launched), RR_ERR_UNSUPPORTED,
 * RR_ERR_HIP.
 */
rr_status rr_permute_batched_noalloc(const rr_job* jobs, int njobs, rr_stream_t stream);

/* -------------------------------------------------------------------------
 * Reusable batch: validate, plan and group the jobs once, keep the job table
 * resident in device memory owned by the handle, launch many times.
 *   flags  RR_BATCH_GRAPH      launches replay a hipGraph captured on the
 *                              first rr_batch_launch (one graph launch per call);
 *          RR_BATCH_TUNE       rr_batch_create times candidate tile shapes and
 *                              grid modes (running the batch, so it writes the
 *                              job outputs) on the current device and keeps the
 *                              fastest; needs the job buffers to be valid; it
 *                              first waits for all work queued on the device
 *                              (hipDeviceSynchronize), so the candidates never
 *                              overlap work that still uses the job buffers;
 *          RR_BATCH_PERSISTENT persistent grids (a few workgroups per CU that
 *                              loop over the group's work) instead of one
 *                              workgroup per block of work;
 *          RR_BATCH_SERIAL     the groups run one after another on the
 *                              launch stream alone (no side streams), in the
 *                              order rr_batch_describe lists them: each group's
 *                              kernel time can then be read on its own.
 * Jobs are planned like rr_permute (the tile override if one is set, else the
 * built-in shapes and the tuning cache).  The handle's device is the current
 * HIP device at creation.  A launch runs its groups side by side on `stream`
 * and three streams the handle owns (default priority): they start after the
 * work queued on `stream` before the call, and work queued on `stream` after
 * the call waits for all of them.  Launches on different streams must not
 * overlap in time (they write the same outputs), and one handle is launched
 * from one thread at a time.
 * Errors: as rr_permute_batched; RR_ERR_NO_MEMORY if the table cannot be
 * allocated.
 */
typedef struct rr_batch rr_batch;
#define RR_BATCH_GRAPH 1
#define RR_BATCH_TUNE 2
#define RR_BATCH_PERSISTENT 4
#define RR_BATCH_SERIAL 8

typedef struct {
    int32_t njobs;             /* jobs with a non-empty problem                */
    int32_t ngroups;           /* groups (kernel family x LDS size class) =
                                  launches per batch                           */
    int32_t in_row_bytes;      /* tile shape chosen (0 = built-in)              */
    int32_t out_row_bytes;
    int32_t order_out;         /* tile traversal in output order                */
    int32_t persistent;        /* persistent grids chosen                       */
    uint64_t bytes;            /* bytes per side moved by one launch            */
    double tuned_us;           /* best measured time of one launch (0 if untuned) */
    int32_t tile_kib;          /* tile LDS size the planner shrinks to (0 = 16) */
    int32_t cache;             /* tile cache policy, -1 = each job's own         */
    int32_t fill;              /* odd-extent refit, -1 = built-in                */
    int32_t force_ragged;      /* G = 1 rows of any alignment for every tile job */
} rr_batch_info;

rr_status rr_batch_create(const rr_job* jobs, int njobs, int flags, rr_batch** out);
rr_status rr_batch_launch(rr_batch* b, rr_stream_t stream);
rr_status rr_batch_get_info(const rr_batch* b, rr_batch_info* out);
/* One text line per kernel group of the batch as currently planned, in the order
 * the groups are stored (and launched under RR_BATCH_SERIAL):
 *   "kernel=k_batch_tile<8,1> jobs=622 workgroups=194744 bytes=2179800000 lds=16384"
 * (bytes per side moved by the group).  Host only.  Errors: RR_ERR_INVALID_ARG
 * (NULL argument, or buf shorter than the text; buflen counts the final NUL). */
rr_status rr_batch_describe(const rr_batch* b, char* buf, int buflen);
rr_status rr_batch_destroy(rr_batch* b);

/* -------------------------------------------------------------------------
 * Serving: a background thread that owns HIP streams and an HBM budget. It
 * admits submitted permute jobs as budget and in-flight slots free up, and
 * keeps forming batches from whatever has arrived while earlier batches are
 * still running (continuous batching); each batch goes to the stream with the
 * fewest batches in flight, so their work overlaps on the device.  A job with
 * more than chunk_bytes of output is large: with max_inflight >= 2 it is
 * launched whole, alone, on a stream of its own, beside the small jobs' batches
 * (kernels on several streams share the device's compute units), and large
 * jobs hold at most max_inflight - 1 slots; with max_inflight == 1 it is cut
 * into ranges of its own workgroups (each rewrites a disjoint part of the
 * output), one range per batch, so small jobs keep flowing past it.  Results
 * are identical to rr_permute run alone.
 * Jobs are validated and planned by rr_serve_submit on the calling thread.  When
 * the server is idle (nothing queued, nothing in flight), rr_serve_submit also
 * admits and launches the job itself (on the server's streams and device) unless
 * it is to be cut into ranges.  The budget caps the device memory the server reserves (slabs of its
 * arena, up to 256 MiB each, kept for reuse and given back when a job would
 * otherwise not fit), not only the bytes handed out.  A job whose output the
 * device refuses to allocate within the budget while no batch is in flight
 * completes with RR_ERR_NO_MEMORY; rr_serve_destroy fails every job still
 * waiting for memory once nothing is in flight.
 */
typedef struct rr_server rr_server;

#define RR_SERVE_SIMULATED 1u  /* no GPU: memory is virtual, and the batches in
                                  flight share a simulated sim_bytes_per_us of
                                  read+write bandwidth equally, each costing its
                                  bytes plus 2 us of launch; exercises admission
                                  and batching on a host. */
#define RR_SERVE_DIRECT 2u     /* baseline: every job is launched alone, in arrival
                                  order, exactly as rr_permute launches it (no
                                  batching, no chunking). */

typedef struct {
    int32_t device;             /* HIP device ordinal                               */
    int32_t max_inflight;       /* batches on the GPU at once (>= 1)                 */
    int32_t max_batch_jobs;     /* whole jobs or chunks per batch (>= 1)             */
    int32_t queue_capacity;     /* pending submissions before RR_ERR_BUSY            */
    uint64_t hbm_budget_bytes;  /* cap on server-allocated device memory             */
    uint64_t chunk_bytes;       /* output bytes above which a job is large (0 = none);
                                   with one slot, bytes per range of a large job    */
    uint32_t tick_us;           /* longest idle wait of the server thread            */
    uint32_t flags;             /* RR_SERVE_SIMULATED                                */
    double sim_bytes_per_us;    /* simulated read+write bandwidth (simulated mode)   */
    uint64_t sim_device_bytes;  /* simulated device memory, 0 = unlimited: a
                                   reservation past it fails as hipMalloc would     */
} rr_serve_config;

typedef struct {
    int32_t status;          /* rr_status of the job                                 */
    int32_t chunks;          /* batches the job was spread over                      */
    void* dst;               /* output buffer (server-allocated when job.dst == NULL) */
    uint64_t t_submit_ns;    /* steady-clock (CLOCK_MONOTONIC) timestamps             */
    uint64_t t_admit_ns;
    uint64_t t_launch_ns;    /* first batch holding the job was launched             */
    uint64_t t_done_ns;      /* server thread saw the job's last batch complete      */
} rr_job_result;

/* Create a server; *out receives the handle.  Errors: RR_ERR_INVALID_ARG, RR_ERR_HIP. */
rr_status rr_serve_create(const rr_serve_config* cfg, rr_server** out);
/* Allocate device memory counted against the budget (for resident inputs). */
rr_status rr_serve_alloc(rr_server* s, uint64_t bytes, void** dptr);
rr_status rr_serve_free(rr_server* s, void* dptr);
/* Submit a job.  job->dst == NULL asks the server to allocate the output at
 * admission (counted against the budget, freed by rr_serve_release).
 * Errors: validation errors of rr_permute, RR_ERR_NO_MEMORY (job larger than the
 * whole budget), RR_ERR_BUSY (queue full). */
rr_status rr_serve_submit(rr_server* s, const rr_job* job, uint64_t* ticket);
/* RR_ERR_NOT_READY while pending; otherwise fills *out and returns RR_OK (the
 * job's own status is out->status). */
rr_status rr_serve_poll(rr_server* s, uint64_t ticket, rr_job_result* out);
/* Completion queue: tickets finished since the previous call, oldest first;
 * up to max are written to out, *n receives the count. */
rr_status rr_serve_completions(rr_server* s, uint64_t* out, int max, int* n);
/* Forget a completed ticket and free its server-allocated output
 * (RR_ERR_NOT_READY if it is still pending). */
rr_status rr_serve_release(rr_server* s, uint64_t ticket);
/* Drain every admitted and queued job, stop the thread, free the server. */
rr_status rr_serve_destroy(rr_server* s);
/* Counters since creation. */
typedef struct {
    uint64_t submitted, completed, failed, batches, chunks, bytes_moved, budget_peak, budget_used;
    uint64_t reserved;   /* device memory the server holds (arena slabs), <= the budget */
} rr_serve_stats;
rr_status rr_serve_get_stats(rr_server* s, rr_serve_stats* out);
/* Failure-handling hook: the next batch the server forms is not launched and
 * its jobs complete with RR_ERR_HIP, as if the launch had failed; the server
 * keeps serving.  For the tests of that path. */
rr_status rr_serve_fail_next_batch(rr_server* s);

/* -------------------------------------------------------------------------
 * Paper notation (Sec. III.B): an order vector lists dimensions fastest first
 * and sizes are given fastest first.  For sizes listed fastest first, the
 * row-major dims are the reversed list, and
 *   perm[j] = ndim-1 - paper_order[ndim-1-j].
 * Errors: RR_ERR_INVALID_ARG if paper_order is not a permutation.
 */
rr_status rr_order_to_perm(int ndim, const int* paper_order, int* perm_out);

/* -------------------------------------------------------------------------
 * Host-only plan introspection (no GPU needed): the canonical form and kernel
 * plan rr_permute would use for this problem, written as one line of text
 * "class=... rank=... dims=... perm=... esize_bytes=... unit=... ..." into buf.
 * Alignment is taken from the two pointer values (which need not be valid).
 */
/* The same for the plan rr_reorder would use (alignment from dst and from src
 * plus the box's offset). */
rr_status rr_reorder_describe(const void* dst, const void* src, int ndim, const int64_t* dims,
                              const int64_t* base, const int64_t* range, int out_ndim, const int* order,
                              int elem_size, char* buf, int buflen);
rr_status rr_plan_describe(const void* dst, const void* src, int ndim, const int64_t* dims,
                           const int* perm, int elem_size, char* buf, int buflen);
/* The same for the plan rr_interlace (de = 0) or rr_deinterlace (de = 1) would
 * use with these pointers (flat: the joined buffer; planes: host array of n
 * plane pointers, read for their values only).  Arguments are checked as by
 * those calls; count = 0 describes an empty plan. */
rr_status rr_interlace_describe(const void* flat, const void* const* planes, int n, int64_t count,
                                int elem_size, int de, char* buf, int buflen);

/* Tile-shape override (the autotuner's knobs): row targets in bytes for the
 * input and output sides of the tiled kernel (0 = built-in choice, max 4096),
 * the order in which tiles are assigned to workgroups (flags:
 * RR_TILE_ORDER_OUT / RR_TILE_ORDER_IN, neither = built-in choice by element
 * size), a cap on the register micro-tile edge G (RR_TILE_MAX_G(g), g one of
 * 1, 2, 4, 8, 16; 0 = no cap) and the LDS size tiles are shrunk to
 * (RR_TILE_KIB(k), 4..64 KiB; 0 = 16); RR_TILE_XCD hands each of the 8 XCDs a
 * contiguous range of tiles instead of every 8th one, RR_TILE_NO_XCD never does
 * (neither: where tile rows share 128-byte lines with neighbouring tiles and a
 * side goes through the caches); RR_TILE_CACHE(p) fixes how tiles access global
 * memory: p = 0 both sides non-temporal, 1 reads cached, 2 writes cached, 3 both
 * cached (0 in those bits: the planner's choice -- writes cached where tile
 * rows share 128-byte lines, so neighbouring tiles' parts of a line meet in L2;
 * both sides non-temporal where every row starts on a line, and for interlace).  Process-wide; affects plans
 * made after the call.  RR_ERR_INVALID_ARG for row targets outside 0..4096, a
 * bad cap, a bad tile size or both XCD flags.
 * RR_TILE_FILL / RR_TILE_NO_FILL switch the odd-extent refit on or off (neither:
 * the built-in choice, on): where a tile does not divide an outer tile axis, the
 * planner evens out both outer extents for the fewest tiles that fit the tile size,
 * keeping each side's rows at least half their target, one 128-byte line and a
 * multiple of 16 bytes (or the whole axis).  RR_ERR_INVALID_ARG also for both fill
 * flags.  RR_TILE_NO_WEAVE sends every interlace and de-interlace through the LDS
 * tile (by default 2-8 sets of 1-, 2-, 4- or 8-byte elements, every pointer on a
 * 16-byte boundary and every set a whole number of 16-byte vectors, are joined or
 * split in registers, one 16-byte vector of each set per thread; the cache bits
 * then say whether the joined side goes through the caches, streamed by
 * default).  RR_TILE_DIAG / RR_TILE_NO_DIAG switch the diagonal tile order on or
 * off everywhere; with neither the planner uses it for 2-D transposes of 1-8-byte
 * elements whose rows are a power of two of at least 4 KiB on both sides
 * (RR_ERR_INVALID_ARG for both flags). */
#define RR_TILE_ORDER_OUT 1
#define RR_TILE_ORDER_IN 2
#define RR_TILE_FORCE_RAGGED 4  /* use the odd-shape (ragged) tile path everywhere (testing) */
#define RR_TILE_XCD 8           /* each XCD takes a contiguous range of tiles (per job in batches) */
#define RR_TILE_UMT 16          /* odd shapes: unaligned G x G micro-tiles instead of G = 1 rows */
#define RR_TILE_UMT_ALWAYS 32   /* unaligned micro-tiles even where aligned ones fit (testing) */
#define RR_TILE_NO_XCD 64       /* never hand XCDs contiguous tile ranges */
#define RR_TILE_DIAG 128        /* diagonal tile order: consecutive tiles step along both tile-grid axes */
#define RR_TILE_NO_DIAG (1 << 30) /* never the diagonal order (neither diag flag: the built-in choice) */
#define RR_TILE_FILL (1 << 27)  /* odd extents: refit tile extents for the fewest tiles within the tile size */
#define RR_TILE_NO_FILL (1 << 28) /* keep the row-target tile extents on odd extents */
#define RR_TILE_NO_WEAVE (1 << 29) /* interlace through the LDS tile only */
#define RR_TILE_MAX_G(g) ((g) << 8)
#define RR_TILE_KIB(k) ((k) << 16)
#define RR_TILE_CACHE(p) (((p) + 1) << 24)
rr_status rr_set_tile_override(int in_row_bytes, int out_row_bytes, int flags);

/* -------------------------------------------------------------------------
 * Autotuner for single permutes: runs the problem (writing dst, so the buffers
 * must be valid) once per candidate tile shape, traversal order and
 * global-access policy on `stream`, times each with HIP events after writing a
 * 512 MiB scratch buffer the call allocates and frees (so no run finds the
 * problem in the caches; without that memory it times warm runs), and caches
 * the fastest for the problem's canonical form and pointer-alignment class.  Every later plan with the same
 * key (rr_permute, rr_permute_batched, batch handles, the server) uses it,
 * unless rr_set_tile_override is active.  Problems that plan to a copy or run
 * copy have nothing to tune and return at once.
 *   best_us, default_us (either may be NULL): best and built-in-choice times.
 * Errors: as rr_permute; RR_ERR_HIP if timing fails.
 */
rr_status rr_tune_permute(void* dst, const void* src, int ndim, const int64_t* dims, const int* perm,
                          int elem_size, rr_stream_t stream, double* best_us, double* default_us);
/* Persist / restore / forget the tuning cache (one text line per key).  Every
 * key starts with the process's tuning context, "<gcnArchName>@hip<runtime
 * version>|" (the device current at the first tuning-cache call and the HIP
 * runtime loaded): a shape was timed on one device and runtime, so rr_tune_load
 * skips lines of another context (RR_LOG=1 reports how many) and stores the
 * others; a malformed line fails the whole load (RR_ERR_INVALID_ARG) and stores
 * nothing. */
rr_status rr_tune_save(const char* path);
rr_status rr_tune_load(const char* path);
rr_status rr_tune_clear(void);
/* The tuning context of this process as a NUL-terminated string (for building
 * or checking tuning files).  Errors: RR_ERR_INVALID_ARG (NULL or short buffer). */
rr_status rr_tune_context(char* buf, int buflen);

const char* rr_status_string(rr_status s);
/* Detail of the last error on the calling thread ("" if none).  With the
 * environment variable RR_LOG set, the library also writes diagnostics to stderr:
 * 1 every error a call returns, 2 also the plan of every single launch and the
 * kernel groups of every batch handle, 3 also the server's admission and batch
 * events. */
const char* rr_last_error(void);
/* Library version string. */
const char* rr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RR_H */
