// rr_plan.hpp -- problem canonicalisation and kernel plans (host side), plus the
// plain-data argument blocks the HIP kernels read.  No HIP types appear here so
// the planner can be exercised on a machine without a GPU.
#pragma once

#include <cstdint>
#include <string>

#include "../../include/rr.h"

namespace rr {

constexpr int MAXR = RR_MAX_DIMS;  // canonical rank never exceeds the input rank
constexpr int MAXS = 4;            // axes on one side of a tile
constexpr int NT = 256;            // threads per workgroup of the tiled kernels
// Vectors of W bytes each thread of the copy and run kernels moves.  16-byte
// vectors go one per thread (a workgroup moves 4 KiB: 6.3 TB/s against 5.9 TB/s
// at four per thread); narrower vectors keep several loads in flight per thread
// (one-byte runs lose 40 % at one per thread).
constexpr int copy_vpt(int W) { return W >= 16 ? 1 : W >= 8 ? 2 : 4; }

// Unsigned division by an invariant 32-bit divisor d >= 1 (Granlund & Montgomery,
// "Division by Invariant Integers using Multiplication", PLDI 1994):
//   l = ceil(log2 d),  mul = floor(2^32 * (2^l - d) / d) + 1,
//   x / d = (mulhi(x, mul) + x) >> l   with a 33-bit intermediate sum.
struct Magic {
    uint32_t mul;
    uint32_t shift;
};
Magic make_magic(uint32_t d);
inline uint32_t magic_div_host(uint32_t x, Magic m) {
    uint32_t hi = (uint32_t)(((uint64_t)x * m.mul) >> 32);
    return (uint32_t)(((uint64_t)hi + x) >> m.shift);
}

// A permute problem after squeezing size-1 axes, fusing axes that stay adjacent
// and in order, and folding the trailing unpermuted axis into the element.
struct Canon {
    int rank = 0;              // 0 means "plain copy of elem_bytes * count bytes"
    int64_t dims[MAXR] = {};   // input extents, slowest axis first
    int perm[MAXR] = {};       // out axis j reads input axis perm[j]
    int64_t sinb[MAXR] = {};   // input byte stride of each axis (row-major for a dense input)
    bool strided = false;      // sinb differs from the dense row-major strides of dims
    int64_t elem_bytes = 0;    // bytes per canonical element (run length)
    int64_t count = 0;         // canonical elements (product of dims)
    int64_t total_bytes = 0;   // bytes per side
};

enum Kind : int32_t { K_EMPTY = 0, K_COPY = 1, K_RUN = 2, K_TILE = 3, K_GATHER = 4, K_SELECT = 5, K_WEAVE = 6 };

// ---------------------------------------------------------------- kernel args
struct CopyArgs {
    uint64_t src, dst;
    uint64_t nvec;      // W-byte vectors in the body
    uint32_t head;      // bytes copied one by one before the body
    uint32_t tail;      // bytes copied one by one after the body
    uint32_t wbytes;    // W
    uint32_t pad_;
};

// Index-set or range read, one element per index (Sec. III.A):
//   dst[i] = src[ix(i)],  ix(i) = idx[i] (idx != 0) or start + i*stride.
// An index outside [0, src_count) reads as zeros and is counted in *bad.
struct GatherArgs {
    uint64_t src, dst;
    uint64_t idx;          // device array of count int64 indices (0: range mode)
    uint64_t bad;          // device uint64 counter of rejected indices (0: none)
    int64_t count, src_count, start, stride;
    uint32_t esize;        // bytes per element
    uint32_t wbytes;       // W: bytes per access
    uint32_t k;            // accesses per element (esize / W)
    uint32_t pad_;
};

// 2-D stencil over a rows x cols float grid (Sec. III.D).  shape 0 (star):
// w[0] center, w[k] the four points at distance k along the axes; shape 1
// (box): w[(dy+r)*(2r+1) + dx+r].  Points closer than r to an edge keep
// their input.  Output tiles are th x ST_TW points, tile t at row
// (t / tiles_x) * th, column (t % tiles_x) * ST_TW.
constexpr int ST_TW = 128;                  // output tile columns
// Output tile rows: 32 up to 2^24 grid points (Table 4's 4096 x 4096 grid), 16 on
// larger grids.  Shorter tiles use less LDS, so more workgroups overlap their loads
// and stores on a CU; with each XCD taking a contiguous range of tiles, the extra
// halo rows are mostly found in L2 (measured: 4096^2 +7 % at 32 rows over 64,
// 16384^2 +8.5 % at 16 rows).
inline int stencil_tile_rows(int64_t rows, int64_t cols) {
    return rows * cols > (int64_t(1) << 24) ? 16 : 32;
}
constexpr int ST_HALO = 4;                  // columns loaded on each side (>= radius)
constexpr int ST_PITCH = ST_TW + 2 * ST_HALO;   // floats per LDS row
constexpr int ST_MAXR = 4;
struct StencilArgs {
    uint64_t src, dst;
    int64_t rows, cols;
    uint32_t tiles_x, ntiles;
    int32_t radius, shape;
    int32_t th, pad_;      // tile rows (16 or 32)
    float w[(2 * ST_MAXR + 1) * (2 * ST_MAXR + 1)];
};

struct RunArgs {
    uint64_t src, dst;
    uint32_t nvec;        // total W-byte vectors
    uint32_t vpr;         // vectors per run (run_bytes / W)
    Magic mvpr;
    uint32_t wbytes;      // W
    int32_t nax;          // output axes (canonical rank)
    uint32_t on[MAXR];    // output extents, slowest first
    Magic om[MAXR];
    uint64_t sin[MAXR];   // input byte stride of output axis j
    uint64_t run_bytes;
    uint32_t ua;          // runs move as 16-byte vectors at any alignment, the last one
                          // ending at the run's end (overlapping its neighbour: same bytes)
    uint32_t cached;      // runs share 128-byte input lines: loads through the caches, and
                          // in batches each XCD takes a contiguous range of the job's blocks
};

// Strided select (a box that keeps the input's fastest axis but not every element
// along it, e.g. one component of interleaved pixels): output rows of n elements
// of R bytes, contiguous, whose input elements lie S = M * R bytes apart.  Each
// thread reads the M 16-byte vectors that span 16 / R consecutive elements and
// keeps one R-byte piece of every S bytes (M in 2..4, R in 1, 2, 4, 8).
struct SelectArgs {
    uint64_t src, dst;        // first element of the box; output
    uint64_t src_end;         // one past the box's last byte: no load reaches beyond
    uint32_t n;               // elements per output row (along the strided axis)
    uint32_t vpr;             // 16-byte output vectors per row, ceil(n * R / 16)
    Magic mvpr;
    uint32_t nvec;            // output vectors in all rows
    int32_t nax;              // outer axes (rows are their combinations)
    uint32_t on[MAXR];        // outer output extents, slowest first
    Magic om[MAXR];
    uint64_t sin[MAXR];       // input byte stride of outer output axis j
    uint32_t S;               // input byte stride of the strided axis
    uint32_t R;               // bytes per element
    uint32_t M;               // S / R
    uint32_t pad_;
};

// Interlace / de-interlace in registers: N planes of U-byte elements (N in
// 2..WEAVE_MAX_SETS, U in 1, 2, 4, 8), every pointer 16-byte aligned and every
// plane a whole number of 16-byte vectors.  Thread v joins (or splits) vector v
// of each plane and the N consecutive 16-byte vectors of the joined array that
// hold the same elements.
constexpr int WEAVE_MAX_SETS = 8;
struct WeaveArgs {
    uint64_t planes[WEAVE_MAX_SETS];   // interlace: the sets read; de-interlace: the sets written
    uint64_t joined;          // interlace: output; de-interlace: input
    uint64_t bstride;         // bytes from one batch to the next on both sides (permutes of
                              // (batch, n, L) <-> (batch, L, n)); 0 for one batch
    uint32_t nvec;            // 16-byte vectors per plane
    uint32_t n;               // planes
    uint32_t unit;            // element bytes
    uint32_t de;              // 1: de-interlace
    uint32_t cached;          // 1: the joined side goes through the caches, 0: streamed
    uint32_t chunks;          // chunks of 64 groups per wave (1 or 2)
    uint32_t bpb;             // workgroups per batch
    uint32_t pad_;
};

enum TileFlags : uint32_t {
    TF_IN_TABLE = 1u,    // input rows are absolute plane pointers (interlace)
    TF_OUT_TABLE = 2u,   // output rows are absolute plane pointers (de-interlace)
    TF_IN_FLAT = 4u,     // input tile is one contiguous range, LDS rows unpadded
    TF_OUT_MERGE = 8u,   // a micro-tile's G output rows are back to back (TB == G)
    TF_RAGGED_IN = 16u,  // input rows move as 16-byte vectors at any element alignment
                         // plus a per-element tail
    TF_OUT_FLAT = 32u,   // output tile is one contiguous range of short rows: written as
                         // 16-byte vectors gathered across row boundaries
    TF_RAGGED_OUT = 64u, // output rows written as 16-byte vectors at any alignment,
                         // gathered element by element from LDS, plus a tail
    TF_STACK = 128u,     // tile = cO_t whole TA x TB transposes stacked along axis C,
                         // each contiguous (msub bytes) in input and output
    TF_XCD = 256u,       // each XCD takes a contiguous range of the tiles (of each batch entry)
    TF_UMT = 512u,       // G x G micro-tiles on rows of any alignment: unaligned 16-byte row
                         // reads, unaligned G*U-byte stores, element-wise partial micro-tiles
    TF_LD_CACHED = 1024u,   // read through the caches (rows share 128-byte lines with
                            // neighbouring tiles); default: non-temporal
    TF_ST_CACHED = 2048u,   // write through the caches; default: non-temporal
    TF_DIAG = 4096u,        // diagonal tile order over the two fastest tile-grid axes
};

struct TileArgs {
    uint64_t src, dst;        // byte base addresses (0 in table mode)
    uint32_t ntiles;
    int32_t ngrid;            // tile-grid axes, slowest first
    uint32_t gn[MAXR];        // tiles along each grid axis
    Magic gm[MAXR];
    uint64_t gsin[MAXR];      // input byte step per tile step
    uint64_t gsout[MAXR];     // output byte step per tile step
    int32_t grid_aO, grid_bO; // grid index of the partial outer A / B axis (-1: none)
    uint32_t aO_len, aO_t;    // extent and tile extent of the outer A axis
    uint32_t bO_len, bO_t;
    uint32_t TAinner, TBinner;
    uint32_t TA, TB;          // tile extents (elements): row length, row count
    int32_t nA, nB;
    uint32_t tA[MAXS];        // tile extent of each A axis (fastest first)
    Magic mA[MAXS];
    uint64_t soutA[MAXS];     // output byte stride of each A axis
    uint32_t tB[MAXS];
    Magic mB[MAXS];
    uint64_t sinB[MAXS];      // input byte stride of each B axis
    uint32_t R;               // bytes per element
    uint32_t k;               // units per element
    Magic mk;
    uint32_t pitch;           // LDS row pitch in bytes (multiple of 16)
    uint32_t nch16;           // pitch / 16
    uint32_t rotmask;         // (largest power of two <= nch16) - 1
    uint32_t win;             // read vector bytes
    uint32_t rch;             // read chunks per row
    Magic mrch;
    uint32_t nmb;             // write micro-tiles per output row (TB / G); unit path: TB*k
    Magic mnmb;
    uint32_t nwork;           // write work items per tile
    Magic mtb;                // divide by TB (flat output)
    uint32_t flags;
    uint32_t lds_bytes;
    uint32_t unit;            // U
    uint32_t g;               // G
    int32_t grid_cO;          // stacked: grid index of the C axis (-1: none)
    uint32_t cO_len, cO_t;    // extent of C and sub-tiles per tile (cO_t = 1 unless stacked)
    uint32_t msub;            // stacked: bytes of one sub-tile (TA * TB * R)
    uint32_t msubp;           // stacked: LDS bytes per sub-tile (msub if back to back in
                              // the input, else msub rounded up to 16)
    Magic msubel;             // stacked: divide by TA * TB
    uint64_t sinC, soutC;     // stacked: byte stride of C in input and output
    uint64_t table[RR_MAX_PLANES];
};

struct TileOptions {
    int in_row_bytes = 0;   // 0 = default
    int out_row_bytes = 0;
    int order_out = -1;     // 1: traverse tiles in output order, 0: input order, -1: by unit size
    int force_ragged = 0;   // plan odd-shape (ragged) tiles even where aligned micro-tiles fit
    int max_g = 0;          // cap on the micro-tile edge G (0 = none)
    int tile_kib = 0;       // tile size the planner shrinks to (KiB of LDS; 0 = 16)
    int xcd = -1;           // 1: contiguous tile range per XCD (per entry in batches), 0: never,
                            // -1: where the cache policy reads or writes through the caches
    int diag = -1;          // diagonal tile order (the paper's answer to partition camping): 1 on,
                            // 0 off, -1 built-in (on for 2-D transposes at power-of-two pitches)
    int cache = -1;         // global accesses of tiles: 0 non-temporal, 1 loads cached,
                            // 2 stores cached, 3 both; -1: by line alignment (cache_policy)
    int umt = 0;            // unaligned micro-tiles: 1 where aligned ones do not fit (instead
                            // of the G = 1 ragged paths), 2 everywhere (testing)
    int fill = -1;          // refit odd extents for fewer, fuller tiles: 1 on, 0 off, -1 built-in
    int weave = 1;          // interlace of 2-4 aligned sets of 1-8-byte elements in registers (0: LDS tile)
    int max_lds = 65536;    // hard limit
    bool use_tuned = false; // a tuned shape cached for the problem replaces these options
};

bool valid_max_g(int g);      // 0 or a power of two up to 16
bool valid_tile_kib(int k);   // 0 or 4..64
constexpr int DEFAULT_TILE_KIB = 16;

// Process-wide override (autotuner hook), read and written under a lock.
// current_tile_options() is a snapshot: the override if one is set, else the
// built-in defaults with use_tuned (tuning-cache lookups) enabled.
TileOptions current_tile_options();
void set_tile_override(const TileOptions& o);
bool override_active(const TileOptions& o);

// Options for a job planned into a batch group (batched calls and handles, the
// serving loop).  The register interlace is off: the batch kernels run copies,
// runs and tiles.  Unless opt is an override (or a tuner candidate), a job of at
// most BATCH_SMALL_JOB_BYTES per side gets 512-byte input and 256-byte output
// row targets, output-order tile traversal and cached tile accesses.  That is
// the shape the batch tuner picks for many small odd-shaped jobs, whose
// neighbours in a group share lines and run from L2.
constexpr int64_t BATCH_SMALL_JOB_BYTES = 128ll << 20;
TileOptions batch_job_options(const TileOptions& opt, int64_t bytes_per_side);

// Tuning cache: device architecture and HIP runtime version (the context, one per
// process) + canonical problem + alignment class -> tile options.  Keys read
//   <arch>@hip<version>|r<rank>:e<bytes>:a<src align>/<dst align>:d<dims>:p<perm>[:s<strides>]
// A tuned shape was timed on one device and runtime, so lines of another context
// are skipped when a file is loaded.
void tune_set_context(const std::string& ctx);   // first call wins
std::string tune_context();
std::string tune_key(const Canon& c, uint64_t dst, uint64_t src);
// The tuned options cached for a canonical problem at these pointer
// alignments, if any (the key is formatted on the stack: no allocation).
bool tune_lookup(const Canon& c, uint64_t dst, uint64_t src, TileOptions* out);
void tune_store(const std::string& key, const TileOptions& o);
void tune_clear();
std::string tune_dump();
// Entries of this process's context are stored; *skipped (if given) counts the
// well-formed lines of another context.  Returns the entries stored, -1 if a line
// is malformed.
int tune_parse(const std::string& text, int* skipped = nullptr);

// Validation + canonicalisation.  Writes a human-readable reason on failure.
rr_status canonicalize(int ndim, const int64_t* dims, const int* perm, int elem_size,
                       Canon* out, std::string* why);
// N-to-M reorder: the box of a dense input given by base and range (NULL base =
// zeros, NULL range = up to the end) with only the axes listed in order kept.
// On success *src_off is the byte offset of the box's first element and *span
// the byte length from there to the end of its last element.
rr_status canonicalize_view(int ndim, const int64_t* dims, const int64_t* base, const int64_t* range,
                            int out_ndim, const int* order, int elem_size, Canon* out, uint64_t* src_off,
                            uint64_t* span, std::string* why);

// Alignment (largest power of two <= 16 dividing the address).
inline int addr_align(uint64_t p) {
    int a = 16;
    while (a > 1 && (p % (uint64_t)a)) a >>= 1;
    return a;
}

// Runs at least this long (bytes) are copied run by run without LDS.
constexpr int64_t RUN_MIN_BYTES = 64;

struct Plan {
    Kind kind = K_EMPTY;
    Canon c;
    CopyArgs copy;
    RunArgs run;
    TileArgs tile;
    GatherArgs gather;
    SelectArgs select;
    WeaveArgs weave;
    uint32_t grid = 0;       // workgroups to launch
    uint64_t bytes = 0;      // bytes per side
};

rr_status plan_permute(uint64_t dst, uint64_t src, const Canon& c, const TileOptions& opt,
                       Plan* p, std::string* why);
// Index-set read (idx != 0) or range read (idx == 0: start, stride).
void plan_gather(uint64_t dst, uint64_t src, uint64_t idx, uint64_t bad, int64_t count, int64_t src_count,
                 int64_t start, int64_t stride, int esize, Plan* p);
// flat = joined buffer (interlace output / de-interlace input); planes = the n sets.
rr_status plan_interlace(uint64_t flat, const uint64_t* planes, int n, int64_t count, int esize,
                         bool deinterlace, const TileOptions& opt, Plan* p, std::string* why);
void plan_copy(uint64_t dst, uint64_t src, uint64_t nbytes, Plan* p);

std::string describe(const Plan& p);

}  // namespace rr
