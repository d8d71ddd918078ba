// rr_plan.cpp -- validation, canonicalisation and kernel planning (host only).
//
// A permute (Sec. III.B) is reduced to the smallest equivalent problem before a
// kernel is chosen:
//   1. axes of extent 1 are dropped (Table 2 of the paper carries such axes);
//   2. input axes that stay adjacent and in the same order in the output are
//      fused into one axis (the offset/stride representation only needs one
//      stride per fused axis);
//   3. if the fastest input axis is also the fastest output axis it is folded
//      into the element, which becomes a contiguous run of bytes.
// What is left is either a plain copy, a copy of long runs, or a true
// transpose between the input's fastest axis and the output's fastest axis --
// the paper's choice of the 2-D plane "of the fastest changing dimensions of
// the input and desired order" (Sec. III.B), here widened to several axes per
// side when extents are short.
#include "rr_plan.hpp"

#include <algorithm>
#include <atomic>
#include <charconv>
#include <cstring>
#include <numeric>
#include <string_view>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <sstream>
#include <vector>

namespace rr {

Magic make_magic(uint32_t d) {
    if (d == 0) d = 1;
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    uint64_t mul = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    return Magic{(uint32_t)mul, l};
}

namespace {
std::mutex g_override_mu;
TileOptions g_override;
}  // namespace

bool override_active(const TileOptions& o) {
    return o.in_row_bytes != 0 || o.out_row_bytes != 0 || o.order_out != -1 || o.force_ragged ||
           o.max_g != 0 || o.tile_kib != 0 || o.xcd != -1 || o.umt != 0 || o.cache != -1 || o.diag != -1 ||
           o.fill != -1 || o.weave != 1;
}

TileOptions batch_job_options(const TileOptions& opt, int64_t bytes_per_side) {
    TileOptions o = opt;
    o.weave = 0;
    if (!override_active(opt) && bytes_per_side <= BATCH_SMALL_JOB_BYTES) {
        o.in_row_bytes = 512;
        o.out_row_bytes = 256;
        o.order_out = 1;
        o.cache = 3;
    }
    return o;
}

TileOptions current_tile_options() {
    std::lock_guard<std::mutex> lk(g_override_mu);
    TileOptions o = g_override;
    o.use_tuned = !override_active(o);
    return o;
}

void set_tile_override(const TileOptions& o) {
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_override = o;
    g_override.use_tuned = false;
}

namespace {
std::shared_mutex g_tune_mu;   // lookups share it (batches plan on several threads)
std::atomic<size_t> g_tune_entries{0};   // lets lookups skip building a key while empty
// transparent comparison: lookups pass a string_view formatted on the stack
std::map<std::string, TileOptions, std::less<>>& tune_cache() {
    static std::map<std::string, TileOptions, std::less<>> m;
    return m;
}

// Context prefix of every key ("<arch>@hip<version>|"), fixed once per process.
std::mutex g_ctx_mu;
char g_ctx[128] = "";
size_t g_ctx_len = 0;

// The key of a canonical problem, written into buf (no allocation):
// <context>|r<rank>:e<bytes>:a<src align>/<dst align>:d<dims>:p<perm>[:s<input strides>]
std::string_view format_tune_key(const Canon& c, uint64_t dst, uint64_t src, char (&buf)[768]) {
    char* p = buf;
    char* const end = buf + sizeof buf;
    auto put = [&](char ch) { if (p < end) *p++ = ch; };
    auto num = [&](int64_t v) { p = std::to_chars(p, end, v).ptr; };
    for (size_t i = 0; i < g_ctx_len; ++i) put(g_ctx[i]);
    put('|');
    put('r'); num(c.rank); put(':'); put('e'); num(c.elem_bytes); put(':'); put('a');
    num(addr_align(src)); put('/'); num(addr_align(dst)); put(':'); put('d');
    for (int i = 0; i < c.rank; ++i) { if (i) put(','); num(c.dims[i]); }
    put(':'); put('p');
    for (int i = 0; i < c.rank; ++i) { if (i) put(','); num(c.perm[i]); }
    if (c.strided) {
        put(':'); put('s');
        for (int i = 0; i < c.rank; ++i) { if (i) put(','); num(c.sinb[i]); }
    }
    return std::string_view(buf, (size_t)(p - buf));
}
}  // namespace

void tune_set_context(const std::string& ctx) {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if (g_ctx_len) return;
    g_ctx_len = std::min(ctx.size(), sizeof g_ctx - 1);
    std::memcpy(g_ctx, ctx.data(), g_ctx_len);
    g_ctx[g_ctx_len] = 0;
}

std::string tune_context() {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    return std::string(g_ctx, g_ctx_len);
}

std::string tune_key(const Canon& c, uint64_t dst, uint64_t src) {
    char buf[768];
    return std::string(format_tune_key(c, dst, src, buf));
}

bool tune_lookup(const Canon& c, uint64_t dst, uint64_t src, TileOptions* out) {
    if (g_tune_entries.load(std::memory_order_relaxed) == 0) return false;
    char buf[768];
    const std::string_view key = format_tune_key(c, dst, src, buf);
    std::shared_lock<std::shared_mutex> lk(g_tune_mu);
    auto& m = tune_cache();
    auto it = m.find(key);
    if (it == m.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string& key, const TileOptions& o) {
    std::lock_guard<std::shared_mutex> lk(g_tune_mu);
    tune_cache()[key] = o;
    g_tune_entries.store(tune_cache().size(), std::memory_order_relaxed);
}

void tune_clear() {
    std::lock_guard<std::shared_mutex> lk(g_tune_mu);
    tune_cache().clear();
    g_tune_entries.store(0, std::memory_order_relaxed);
}

std::string tune_dump() {
    std::lock_guard<std::shared_mutex> lk(g_tune_mu);
    std::ostringstream o;
    for (const auto& kv : tune_cache())
        o << kv.first << " " << kv.second.in_row_bytes << " " << kv.second.out_row_bytes << " "
          << kv.second.order_out << " " << kv.second.max_g << " " << kv.second.tile_kib << " "
          << kv.second.xcd << " " << kv.second.umt << " " << kv.second.cache << " " << kv.second.diag << " "
          << kv.second.fill << "\n";
    return o.str();
}

bool valid_max_g(int g) { return g == 0 || g == 1 || g == 2 || g == 4 || g == 8 || g == 16; }
bool valid_tile_kib(int k) { return k == 0 || (k >= 4 && k <= 64); }

// One entry per line:
//   key in_row_bytes out_row_bytes order_out [max_g [tile_kib [xcd [umt [cache [diag [fill]]]]]]]
// (an entry without the xcd field never uses XCD ranges, one without cache plans
// its accesses by line alignment, one without diag keeps the plain tile order,
// one without fill takes the built-in refit; diag -1 is the built-in choice)
int tune_parse(const std::string& text, int* skipped) {
    std::istringstream lines(text);
    std::string line;
    int n = 0, other = 0;
    const std::string prefix = tune_context() + "|";
    std::vector<std::pair<std::string, TileOptions>> keep;
    while (std::getline(lines, line)) {
        std::istringstream in(line);
        std::string key;
        if (!(in >> key)) continue;   // blank line
        TileOptions o;
        o.diag = 0;   // lines written before the built-in diagonal rule were timed without it
        if (!(in >> o.in_row_bytes >> o.out_row_bytes >> o.order_out)) return -1;
        if (!(in >> o.max_g)) { o.max_g = 0; o.xcd = 0; }
        else if (!(in >> o.tile_kib)) { o.tile_kib = 0; o.xcd = 0; }
        else if (!(in >> o.xcd)) o.xcd = 0;
        else if (!(in >> o.umt)) o.umt = 0;
        else if (!(in >> o.cache)) o.cache = -1;
        else if (!(in >> o.diag)) o.diag = 0;
        else if (!(in >> o.fill)) o.fill = -1;
        std::string extra;
        if (in >> extra) return -1;
        if (o.in_row_bytes < 0 || o.in_row_bytes > 4096 || o.out_row_bytes < 0 || o.out_row_bytes > 4096 ||
            o.order_out < -1 || o.order_out > 1 || !valid_max_g(o.max_g) || !valid_tile_kib(o.tile_kib) ||
            o.xcd < -1 || o.xcd > 1 || o.umt < 0 || o.umt > 2 || o.cache < -1 || o.cache > 3 || o.diag < -1 ||
            o.diag > 1 || o.fill < -1 || o.fill > 1)
            return -1;
        if (key.find('|') == std::string::npos) return -1;   // no context
        if (key.compare(0, prefix.size(), prefix) != 0) { ++other; continue; }
        keep.emplace_back(key, o);
    }
    for (const auto& kv : keep) { tune_store(kv.first, kv.second); ++n; }   // all or nothing
    if (skipped) *skipped = other;
    return n;
}

static bool mul_ovf(int64_t a, int64_t b, int64_t* r) { return __builtin_mul_overflow(a, b, r); }

rr_status canonicalize(int ndim, const int64_t* dims, const int* perm, int elem_size,
                       Canon* out, std::string* why) {
    if (ndim > RR_MAX_DIMS) {
        *why = "ndim exceeds RR_MAX_DIMS";
        return RR_ERR_UNSUPPORTED;
    }
    if (ndim < 1) { *why = "ndim must be >= 1"; return RR_ERR_INVALID_ARG; }
    if (!dims || !perm) { *why = "dims and perm must be non-NULL"; return RR_ERR_INVALID_ARG; }
    if (elem_size < 1 || elem_size > 16) { *why = "elem_size must be 1..16"; return RR_ERR_INVALID_ARG; }
    bool seen[MAXR] = {};
    for (int j = 0; j < ndim; ++j) {
        if (perm[j] < 0 || perm[j] >= ndim || seen[perm[j]]) {
            *why = "perm is not a permutation of 0..ndim-1";
            return RR_ERR_INVALID_ARG;
        }
        seen[perm[j]] = true;
    }
    int64_t count = 1;
    for (int k = 0; k < ndim; ++k) {
        if (dims[k] < 0) { *why = "negative extent"; return RR_ERR_INVALID_ARG; }
        if (mul_ovf(count, dims[k], &count)) { *why = "element count overflows int64"; return RR_ERR_OVERFLOW; }
    }
    int64_t bytes;
    if (mul_ovf(count, elem_size, &bytes)) { *why = "byte count overflows int64"; return RR_ERR_OVERFLOW; }

    Canon c;
    c.total_bytes = bytes;
    if (count == 0) {
        c.rank = 0; c.count = 0; c.elem_bytes = elem_size;
        *out = c;
        return RR_OK;
    }
    // 1. squeeze extent-1 axes
    int newidx[MAXR];
    int64_t d[MAXR];
    int r = 0;
    for (int k = 0; k < ndim; ++k) {
        if (dims[k] != 1) { newidx[k] = r; d[r++] = dims[k]; } else newidx[k] = -1;
    }
    int p[MAXR];
    int j2 = 0;
    for (int j = 0; j < ndim; ++j)
        if (dims[perm[j]] != 1) p[j2++] = newidx[perm[j]];
    // 2. fuse runs of input axes that stay consecutive in the output
    int gstart[MAXR], glen[MAXR];
    int ng = 0;
    for (int j = 0; j < r; ++j) {
        if (j > 0 && p[j] == p[j - 1] + 1) glen[ng - 1]++;
        else { gstart[ng] = p[j]; glen[ng] = 1; ++ng; }
    }
    // groups are listed in output order; rank them by input position
    int rank_of[MAXR];
    for (int g = 0; g < ng; ++g) {
        int rk = 0;
        for (int h = 0; h < ng; ++h) if (gstart[h] < gstart[g]) ++rk;
        rank_of[g] = rk;
    }
    int64_t cd[MAXR];
    int cp[MAXR];
    for (int g = 0; g < ng; ++g) {
        int64_t e = 1;
        for (int a = 0; a < glen[g]; ++a) e *= d[gstart[g] + a];
        cd[rank_of[g]] = e;
        cp[g] = rank_of[g];
    }
    // 3. fold a trailing axis that is fastest on both sides into the element
    int64_t R = elem_size;
    int rc = ng;
    while (rc >= 1 && cp[rc - 1] == rc - 1) {
        R *= cd[rc - 1];
        --rc;
    }
    c.rank = rc;
    c.elem_bytes = R;
    c.count = 1;
    for (int k = 0; k < rc; ++k) { c.dims[k] = cd[k]; c.perm[k] = cp[k]; c.count *= cd[k]; }
    int64_t s = R;
    for (int k = rc - 1; k >= 0; --k) { c.sinb[k] = s; s *= cd[k]; }
    *out = c;
    return RR_OK;
}

rr_status canonicalize_view(int ndim, const int64_t* dims, const int64_t* base, const int64_t* range,
                            int out_ndim, const int* order, int elem_size, Canon* out, uint64_t* src_off,
                            uint64_t* span, std::string* why) {
    if (ndim > RR_MAX_DIMS) { *why = "ndim exceeds RR_MAX_DIMS"; return RR_ERR_UNSUPPORTED; }
    if (ndim < 1) { *why = "ndim must be >= 1"; return RR_ERR_INVALID_ARG; }
    if (out_ndim < 0 || out_ndim > ndim) { *why = "out_ndim must be 0..ndim"; return RR_ERR_INVALID_ARG; }
    if (!dims || (out_ndim > 0 && !order)) { *why = "dims and order must be non-NULL"; return RR_ERR_INVALID_ARG; }
    if (elem_size < 1 || elem_size > 16) { *why = "elem_size must be 1..16"; return RR_ERR_INVALID_ARG; }
    bool kept[MAXR] = {};
    for (int j = 0; j < out_ndim; ++j) {
        if (order[j] < 0 || order[j] >= ndim || kept[order[j]]) {
            *why = "order must list distinct axes of 0..ndim-1";
            return RR_ERR_INVALID_ARG;
        }
        kept[order[j]] = true;
    }
    int64_t b[MAXR], ext[MAXR];
    int64_t total_in = 1;
    for (int d = 0; d < ndim; ++d) {
        if (dims[d] < 0) { *why = "negative extent"; return RR_ERR_INVALID_ARG; }
        if (mul_ovf(total_in, dims[d], &total_in)) { *why = "element count overflows int64"; return RR_ERR_OVERFLOW; }
        b[d] = base ? base[d] : 0;
        if (b[d] < 0) { *why = "negative base"; return RR_ERR_INVALID_ARG; }
        if (kept[d]) {
            ext[d] = range ? range[d] : dims[d] - b[d];
            if (ext[d] < 0 || b[d] > dims[d] || ext[d] > dims[d] - b[d]) {
                *why = "base + range exceeds the extent of a kept axis";
                return RR_ERR_INVALID_ARG;
            }
        } else {
            ext[d] = 1;
            if (b[d] >= dims[d]) { *why = "base of a fixed axis is outside its extent"; return RR_ERR_INVALID_ARG; }
        }
    }
    int64_t in_bytes;
    if (mul_ovf(total_in, elem_size, &in_bytes)) { *why = "byte count overflows int64"; return RR_ERR_OVERFLOW; }
    int64_t st[MAXR];   // element strides of the whole input
    {
        int64_t s = 1;
        for (int d = ndim - 1; d >= 0; --d) { st[d] = s; s *= std::max<int64_t>(dims[d], 1); }
    }
    int64_t count = 1;
    for (int j = 0; j < out_ndim; ++j) count *= ext[order[j]];
    Canon c;
    c.total_bytes = count * elem_size;
    *src_off = 0;
    *span = 0;
    if (count == 0) {
        c.rank = 0; c.count = 0; c.elem_bytes = elem_size;
        *out = c;
        return RR_OK;
    }
    int64_t off = 0, last = 0;
    for (int d = 0; d < ndim; ++d) {
        off += b[d] * st[d];
        last += (ext[d] - 1) * st[d];
    }
    *src_off = (uint64_t)(off * elem_size);
    *span = (uint64_t)((last + 1) * elem_size);
    // kept axes of extent > 1, in input order, with their strides
    int newidx[MAXR];
    int64_t d2[MAXR], s2[MAXR];
    int r = 0;
    for (int d = 0; d < ndim; ++d) {
        if (kept[d] && ext[d] != 1) { newidx[d] = r; d2[r] = ext[d]; s2[r] = st[d]; ++r; } else newidx[d] = -1;
    }
    int p[MAXR];
    int j2 = 0;
    for (int j = 0; j < out_ndim; ++j)
        if (newidx[order[j]] >= 0) p[j2++] = newidx[order[j]];
    // fuse output-consecutive axes that are input-consecutive and contiguous in the box
    int gstart[MAXR], glen[MAXR];
    int ng = 0;
    for (int j = 0; j < r; ++j) {
        if (j > 0 && p[j] == p[j - 1] + 1 && s2[p[j - 1]] == s2[p[j]] * d2[p[j]]) glen[ng - 1]++;
        else { gstart[ng] = p[j]; glen[ng] = 1; ++ng; }
    }
    int rank_of[MAXR];
    for (int g = 0; g < ng; ++g) {
        int rk = 0;
        for (int h = 0; h < ng; ++h) if (gstart[h] < gstart[g]) ++rk;
        rank_of[g] = rk;
    }
    int64_t cd[MAXR], cs[MAXR];
    int cp[MAXR];
    for (int g = 0; g < ng; ++g) {
        int64_t e = 1;
        for (int a = 0; a < glen[g]; ++a) e *= d2[gstart[g] + a];
        cd[rank_of[g]] = e;
        cs[rank_of[g]] = s2[gstart[g] + glen[g] - 1] * elem_size;   // innermost member's stride
        cp[g] = rank_of[g];
    }
    // fold trailing axes that are fastest on both sides and contiguous into the element
    int64_t R = elem_size;
    int rc = ng;
    while (rc >= 1 && cp[rc - 1] == rc - 1 && cs[rc - 1] == R) {
        R *= cd[rc - 1];
        --rc;
    }
    c.rank = rc;
    c.elem_bytes = R;
    c.count = 1;
    int64_t dense = R;
    c.strided = false;
    for (int k = rc - 1; k >= 0; --k) {
        c.dims[k] = cd[k]; c.perm[k] = cp[k]; c.sinb[k] = cs[k]; c.count *= cd[k];
        if (cs[k] != dense) c.strided = true;
        dense *= cd[k];
    }
    *out = c;
    return RR_OK;
}

void plan_gather(uint64_t dst, uint64_t src, uint64_t idx, uint64_t bad, int64_t count, int64_t src_count,
                 int64_t start, int64_t stride, int esize, Plan* p) {
    p->kind = K_GATHER;
    p->bytes = (uint64_t)count * (uint64_t)esize;
    GatherArgs& a = p->gather;
    std::memset(&a, 0, sizeof(a));
    uint32_t W = 16;
    while (W > 1 && (esize % W || src % W || dst % W)) W >>= 1;
    a.src = src; a.dst = dst; a.idx = idx; a.bad = bad;
    a.count = count; a.src_count = src_count; a.start = start; a.stride = stride;
    a.esize = (uint32_t)esize; a.wbytes = W; a.k = (uint32_t)esize / W;
    uint64_t per_block = (uint64_t)NT * 4;
    uint64_t g = ((uint64_t)count + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 0x7fffffffULL) g = 0x7fffffffULL;   // grid-stride beyond this
    p->grid = (uint32_t)g;
}

void plan_copy(uint64_t dst, uint64_t src, uint64_t nbytes, Plan* p) {
    p->kind = K_COPY;
    p->bytes = nbytes;
    CopyArgs& a = p->copy;
    std::memset(&a, 0, sizeof(a));
    uint32_t W = 16;
    while (W > 1 && ((src - dst) % W)) W >>= 1;
    uint64_t head = (W - (dst % W)) % W;
    if (head > nbytes) head = nbytes;
    uint64_t body = (nbytes - head) / W;
    uint64_t tail = nbytes - head - body * W;
    a.src = src; a.dst = dst; a.nvec = body; a.head = (uint32_t)head; a.tail = (uint32_t)tail; a.wbytes = W;
    uint64_t per_block = (uint64_t)NT * copy_vpt((int)W);
    uint64_t g = (body + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 0x7fffffffULL) g = 0x7fffffffULL;  // grid-stride beyond this
    p->grid = (uint32_t)g;
}

static int pow2_divisor_cap16(int64_t x) {
    int u = 1;
    while (u < 16 && (x % (u * 2)) == 0) u <<= 1;
    return u;
}

static rr_status plan_run(uint64_t dst, uint64_t src, const Canon& c, Plan* p, std::string* why) {
    p->kind = K_RUN;
    RunArgs& a = p->run;
    std::memset(&a, 0, sizeof(a));
    const int r = c.rank;
    const int64_t R = c.elem_bytes;
    uint32_t W = 16;
    auto strides_ok = [&](uint32_t w) {
        for (int k = 0; k < r; ++k) if (c.sinb[k] % w) return false;
        return true;
    };
    while (W > 1 && (src % W || dst % W || R % W || !strides_ok(W))) W >>= 1;
    // Runs that aligned 16-byte vectors do not fit (odd lengths or starts): 16-byte
    // vectors at any alignment, the run's last vector ending at its last byte.
    const bool ua = W < 16 && R >= 16;
    if (ua) W = 16;
    int64_t vpr = ua ? (R + 15) / 16 : R / W;
    int64_t nvec = c.count * vpr;
    if (vpr > 0xffffffffLL || nvec > 0xffffffffLL) {
        *why = "run-copy problem exceeds 2^32 vectors per launch";
        return RR_ERR_UNSUPPORTED;
    }
    a.src = src; a.dst = dst; a.nvec = (uint32_t)nvec; a.vpr = (uint32_t)vpr;
    a.mvpr = make_magic((uint32_t)vpr); a.wbytes = W; a.nax = r; a.run_bytes = (uint64_t)R;
    a.ua = ua ? 1u : 0u;
    // Runs shorter than a 128-byte line that start or end inside lines share
    // those lines with the runs beside them in the input: loads through the
    // caches (with XCD-contiguous block ranges, so a line's second reader is on
    // the same L2) find them there instead of fetching them again.  Measured
    // +14-21 % on runs of 66-72 bytes; longer runs gain nothing and a 256-byte
    // run at a 4-byte offset lost 40 %, so they stay streamed.
    bool shared = (src % 128) != 0 || (R % 128) != 0;
    for (int k = 0; k < r; ++k) shared = shared || (c.sinb[k] % 128) != 0;
    a.cached = shared && R < 128 ? 1u : 0u;
    for (int j = 0; j < r; ++j) {
        a.on[j] = (uint32_t)c.dims[c.perm[j]];
        a.om[j] = make_magic(a.on[j]);
        a.sin[j] = (uint64_t)c.sinb[c.perm[j]];
    }
    uint64_t per_block = (uint64_t)NT * copy_vpt((int)W);
    uint64_t g = ((uint64_t)nvec + per_block - 1) / per_block;
    if (g > 0x7fffffffULL) { *why = "grid too large"; return RR_ERR_UNSUPPORTED; }
    p->grid = (uint32_t)std::max<uint64_t>(1, g);
    p->bytes = (uint64_t)c.total_bytes;
    return RR_OK;
}

// Strided select: the fastest output axis is the fastest input axis, whose input
// stride S is 2..4 elements of R = 1, 2, 4 or 8 bytes.  Returns false (nothing
// planned) for any other shape, alignment or size.
static bool plan_select(uint64_t dst, uint64_t src, const Canon& c, Plan* p) {
    const int r = c.rank;
    const int64_t R = c.elem_bytes, S = c.sinb[r - 1];
    if (!(R == 1 || R == 2 || R == 4 || R == 8) || S % R != 0) return false;
    const int64_t M = S / R;
    if (M < 2 || M > 4 || addr_align(src) < R || addr_align(dst) < R) return false;
    const int64_t n = c.dims[r - 1];
    const int64_t V = 16 / R;
    const int64_t vpr = (n + V - 1) / V;
    const int64_t rows = c.count / n;
    if (n > 0xffffffffLL || vpr * rows > 0x7fffffffLL) return false;
    SelectArgs& a = p->select;
    std::memset(&a, 0, sizeof a);
    int64_t last = 0;   // byte offset of the box's last element
    for (int k = 0; k < r; ++k) last += (c.dims[k] - 1) * c.sinb[k];
    a.src = src; a.dst = dst; a.src_end = src + (uint64_t)(last + R);
    a.n = (uint32_t)n; a.vpr = (uint32_t)vpr; a.mvpr = make_magic((uint32_t)vpr);
    a.nvec = (uint32_t)(vpr * rows);
    a.nax = r - 1;
    for (int j = 0; j < r - 1; ++j) {   // outer output axes read input axes perm[j] (perm[r-1] = r-1)
        a.on[j] = (uint32_t)c.dims[c.perm[j]];
        a.om[j] = make_magic(a.on[j]);
        a.sin[j] = (uint64_t)c.sinb[c.perm[j]];
    }
    a.S = (uint32_t)S; a.R = (uint32_t)R; a.M = (uint32_t)M;
    p->kind = K_SELECT;
    p->grid = (a.nvec + NT - 1) / NT;
    p->bytes = (uint64_t)c.total_bytes;
    return true;
}

static int default_row_bytes(int U, bool in_side) {
    switch (U) {
        case 1: return 128;
        case 2: return in_side ? 256 : 128;
        case 4: return 256;
        case 8: return in_side ? 256 : 512;
        default: return 512;
    }
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Whether plan_tile refits odd extents for fewer, fuller tiles (TileOptions::fill).
static bool fill_refit(const TileOptions& o) { return o.fill != 0; }

// Share of each 128-byte line touched by one wave's store instruction that the
// instruction writes, for a tile whose output rows hold TB units of U bytes,
// row_stride bytes apart (0: rows lie in unrelated places, e.g. separate planes).
// G > 1: lanes take micro-tiles B-fastest, so a wave writes runs of
// min(TB / G, 64) * G * U contiguous bytes, one per micro-tile row, G output rows
// apart; merged micro-tiles (TB == G, rows back to back) store their G rows as
// 16-byte vectors, one vector per lane and instruction.  G == 1: 16-byte vectors
// along each row, rows back to back when row_stride == TB * U.
static double store_line_fill(int U, int G, uint32_t TB, uint64_t row_stride, bool merge) {
    constexpr uint64_t LINE = 128, LANES = 64;
    const uint64_t W = (uint64_t)U * G;
    uint64_t run, nrun, step;
    if (G == 1) {
        const uint64_t rowb = (uint64_t)TB * U;
        run = std::min<uint64_t>(rowb, 16 * LANES);
        nrun = std::max<uint64_t>(1, 16 * LANES / rowb);
        step = row_stride;
    } else if (merge) {
        run = 16; nrun = LANES; step = W * G;
    } else {
        const uint64_t nmb = TB / G;
        run = std::min<uint64_t>(nmb, LANES) * W;
        nrun = std::max<uint64_t>(1, LANES / nmb);
        step = row_stride * G;
    }
    uint64_t lines;
    if (nrun == 1 || step == 0 || step >= LINE) lines = nrun * ((run + LINE - 1) / LINE);
    else lines = ((nrun - 1) * step + run + LINE - 1) / LINE;
    if (step != 0 && step < run) lines = (nrun * run + LINE - 1) / LINE;   // runs overlap: contiguous
    return (double)(nrun * run) / (double)(lines * LINE);
}

// Register micro-tiles on short output rows store partial lines (a 4 x 4 tile of
// 4-byte elements whose output rows are 16 bytes writes one quarter of each line
// it touches per instruction), which costs up to 3x against the G = 1 paths that
// write whole 16-byte vectors along the output.  Walk G down while the best line
// fill so far is poor and a smaller G fills strictly more; 4..16-byte elements
// need more than half-filled lines, 1- and 2-byte elements (whose G = 1 paths
// assemble vectors byte by byte from LDS) accept half.
static int line_friendly_g(int U, int G, uint32_t TB, int nA, uint64_t row_stride, bool out_table) {
    if (G <= 1) return G;
    auto fill = [&](int g) {
        const bool merge = g > 1 && !out_table && nA == 1 && TB == (uint32_t)g && row_stride == (uint64_t)U * g &&
                           U * g >= 4 && (U * g * g) % 16 == 0;
        return store_line_fill(U, g, TB, out_table ? 0 : row_stride, merge);
    };
    auto good = [&](double f) { return U >= 4 ? f > 0.5 : f >= 0.5; };
    int best = G;
    double fb = fill(G);
    for (int g = G >> 1; g >= 1 && !good(fb); g >>= 1) {
        const double f = fill(g);
        if (f > fb) { best = g; fb = f; }
    }
    return best;
}

// Global access flavour and XCD ranges of a finished tile plan (TF_LD_CACHED,
// TF_ST_CACHED, TF_XCD).  Rows that start or end inside 128-byte lines share
// those lines with the neighbouring tile.  With non-temporal stores each tile
// writes its part of such a line to HBM on its own; written through the caches,
// with neighbouring tiles on one XCD (contiguous tile ranges, one L2), the parts
// meet in L2 and leave as whole lines (in a batch launch each entry's tiles are
// grouped so).  Measured with cold caches on odd shapes of 1..16-byte elements:
// 1.1-2.6x over non-temporal stores, +3.6 % on a 4096-job batch of small odd
// jobs (few tiles per XCD); cached loads lose
// (their apparent gains came from inputs still resident in the 256 MB Infinity
// Cache).  Where every row starts on a line, and for interlace and de-interlace
// (plane tables), both sides stream non-temporally.
// Whether one side of a tile shares 128-byte lines with other tiles.  Rows of
// row_bytes at offsets sum(idx[i] * stride[i]) over nax row axes (t[i] values
// each) form blocks: an axis whose stride equals the block built so far extends
// it.  Lines are shared where a block starts (base, tile grid steps, strides of
// the axes left over) or ends off a line.
static bool shares_lines(uint64_t starts, uint64_t row_bytes, int nax, const uint32_t* t,
                         const uint64_t* stride) {
    uint64_t block = row_bytes;
    bool used[MAXS] = {};
    for (bool grew = true; grew;) {
        grew = false;
        for (int i = 0; i < nax; ++i)
            if (!used[i] && stride[i] == block) { used[i] = true; block *= t[i]; grew = true; }
    }
    for (int i = 0; i < nax; ++i) if (!used[i]) starts |= stride[i];
    return ((starts | block) % 128) != 0;
}

static void cache_policy(TileArgs& a, const TileOptions& opt) {
    uint64_t in_starts = a.src, out_starts = a.dst;
    for (int g = 0; g < a.ngrid; ++g) { in_starts |= a.gsin[g]; out_starts |= a.gsout[g]; }
    bool split;
    if (a.flags & TF_STACK) {   // cO_t sub-tiles of msub bytes, each contiguous on both sides
        split = shares_lines(in_starts, a.msub, 1, &a.cO_t, &a.sinC) ||
                shares_lines(out_starts, a.msub, 1, &a.cO_t, &a.soutC);
    } else {
        const uint64_t in_rb = (uint64_t)a.TA * a.R, out_rb = (uint64_t)a.TB * a.R;
        if (a.flags & TF_IN_TABLE) {
            for (uint32_t c = 0; c < a.TB; ++c) in_starts |= a.table[c];
            split = shares_lines(in_starts, in_rb, 0, nullptr, nullptr);
        } else {
            split = shares_lines(in_starts, in_rb, a.nB, a.tB, a.sinB);
        }
        if (a.flags & TF_OUT_TABLE) {
            for (uint32_t c = 0; c < a.TA; ++c) out_starts |= a.table[c];
            split = split || shares_lines(out_starts, out_rb, 0, nullptr, nullptr);
        } else {
            split = split || shares_lines(out_starts, out_rb, a.nA, a.tA, a.soutA);
        }
    }
    const bool table = (a.flags & (TF_IN_TABLE | TF_OUT_TABLE)) != 0;
    int pol = opt.cache;
    if (pol < 0) pol = split && !table ? 2 : 0;
    if (pol & 1) a.flags |= TF_LD_CACHED;
    if (pol & 2) a.flags |= TF_ST_CACHED;
    const bool xcd = opt.xcd >= 0 ? opt.xcd > 0 : split && pol != 0 && !table;
    if (xcd) a.flags |= TF_XCD;
}

// Fill the LDS / read / write geometry of a tile plan whose extents are set.
//   row_align_in : OR of every input row start offset (alignment probe)
//   flat_ok      : input rows are back to back (row stride == row bytes), so a
//                  tile's input is one contiguous range starting at flat_base
//                  plus a multiple of TB rows; total_rows is the row axis's whole
//                  extent when slower axes follow it (0 when none do)
static rr_status finish_tile(TileArgs& a, int U, int G, int k, uint64_t row_align_in, bool flat_ok,
                             uint64_t flat_base, uint64_t total_rows, const TileOptions& opt,
                             std::string* why) {
    a.unit = U; a.g = G; a.k = k;
    a.mk = make_magic(k);
    if (a.flags & TF_STACK) {
        a.pitch = a.TA * a.R;
        a.nch16 = 0xffffffffu;
        a.rotmask = 0;
        a.lds_bytes = (a.cO_t * a.msubp + 15) / 16 * 16;
        if (a.lds_bytes > (uint32_t)opt.max_lds) { *why = "tile does not fit LDS"; return RR_ERR_UNSUPPORTED; }
        a.win = 16;
        a.mtb = make_magic(a.TB);
        a.msubel = make_magic(a.TA * a.TB);
        a.nmb = a.TB;
        a.mnmb = make_magic(a.nmb);
        return RR_OK;
    }
    const uint64_t rowbytes = (uint64_t)a.TA * a.R;
    // every tile's range starts on a 16-byte boundary (also across slower axes);
    // the input's last tile may end inside a vector (its tail moves byte by byte)
    const bool flat = flat_ok && (rowbytes % 16 != 0 || rowbytes < 64) && (flat_base % 16) == 0 &&
                      ((uint64_t)a.TB * rowbytes) % 16 == 0 && (total_rows * rowbytes) % 16 == 0;
    if (flat) {
        a.flags |= TF_IN_FLAT;
        a.pitch = (uint32_t)rowbytes;
        a.nch16 = 0xffffffffu;   // no chunk rotation
        a.rotmask = 0;
    } else {
        a.pitch = (uint32_t)((rowbytes + 15) / 16 * 16);
        a.nch16 = a.pitch / 16;
        uint32_t pw = 1;
        while (pw * 2 <= a.nch16) pw <<= 1;
        a.rotmask = pw - 1;
    }
    a.lds_bytes = (a.pitch * a.TB + 15) / 16 * 16;
    if (a.lds_bytes > (uint32_t)opt.max_lds) { *why = "tile does not fit LDS"; return RR_ERR_UNSUPPORTED; }
    uint32_t win = 16;
    if (!flat)
        while (win > (uint32_t)U && ((row_align_in % win) || (rowbytes % win))) win >>= 1;
    if (win < (uint32_t)U) win = U;
    a.win = win;
    a.rch = (uint32_t)(rowbytes / win);
    a.mrch = make_magic(a.rch);
    a.mtb = make_magic(a.TB);
    if (k == 1 && (a.flags & TF_UMT)) {
        a.nmb = (a.TB + G - 1) / G;
        a.nwork = a.nmb * ((a.TA + G - 1) / G);
    } else if (k == 1) {
        a.nmb = a.TB / G;
        a.nwork = a.nmb * (a.TA / G);
        const uint32_t W = (uint32_t)(U * G);
        if (a.nmb == 1 && a.nA == 1 && !(a.flags & TF_OUT_TABLE) && a.soutA[0] == W && W >= 4 &&
            (W * G) % 16 == 0)
            a.flags |= TF_OUT_MERGE;
        // G == 1 because extents or strides are odd: move rows as 16-byte vectors at any
        // alignment instead of one element per access.  Short back-to-back output rows
        // (interlace of a few sets) are written as one contiguous range.
        if (G == 1 && U < 16) {
            const bool out_rows_adjacent = a.nA == 1 && !(a.flags & TF_OUT_TABLE) &&
                                           a.soutA[0] == (uint64_t)a.TB * a.R;
            const bool tb_whole = a.grid_bO < 0;   // every tile holds all TB output columns
            if (out_rows_adjacent && tb_whole && (uint64_t)a.TB * a.R < 64) a.flags |= TF_OUT_FLAT;
            else a.flags |= TF_RAGGED_OUT;
            if ((a.flags & TF_IN_FLAT) == 0) a.flags |= TF_RAGGED_IN;
        }
    } else {
        a.nmb = a.TB * k;      // units per output row
        a.nwork = a.nmb * a.TA;
        // Elements of k > 1 units (6, 12, 24 ... bytes): rows of any length move as
        // 16-byte vectors at any alignment instead of one unit per access.
        if (G == 1 && U < 16 && !(a.flags & (TF_OUT_TABLE | TF_IN_TABLE))) {
            a.flags |= TF_RAGGED_OUT;
            if ((a.flags & TF_IN_FLAT) == 0) a.flags |= TF_RAGGED_IN;
        }
    }
    a.mnmb = make_magic(a.nmb);
    return RR_OK;
}

// Built-in diagonal tile order: 2-D transposes of 1-8-byte elements whose rows
// are a power of two of at least 4 KiB on both sides.  Concurrent tiles then
// start on rows 2^k bytes apart, which the HBM3E address hashing still piles
// onto few channels (the partition camping of Sec. II); the skew spreads them.
// Measured from cold caches on 4096^2-16384^2 and 16384 x 4096 transposes
// (16 MiB and more per side): +1-41 %, one case -1 %.  At other pitches
// (16000^2, 8320 x 8192, 12288^2) and for 16-byte elements it lost up to 23 %,
// so those keep the plain order, as do smaller problems (not measured).
static bool diag_by_default(const Canon& c) {
    if (c.rank != 2 || c.perm[0] != 1 || c.strided || c.elem_bytes > 8 || c.total_bytes < (16ll << 20)) return false;
    auto pow2 = [](int64_t x) { return x >= 4096 && (x & (x - 1)) == 0; };
    return pow2(c.dims[0] * c.elem_bytes) && pow2(c.dims[1] * c.elem_bytes);
}

static rr_status plan_tile(uint64_t dst, uint64_t src, const Canon& c, const TileOptions& opt,
                           Plan* p, std::string* why) {
    p->kind = K_TILE;
    TileArgs& a = p->tile;
    std::memset(&a, 0, sizeof(a));
    const int r = c.rank;
    const int64_t* d = c.dims;
    const int* pm = c.perm;
    const int64_t R = c.elem_bytes;
    const int64_t* sinb = c.sinb;   // input byte strides (the fastest axis's is R)
    int64_t sout_el[MAXR];
    {
        int64_t s = 1;
        for (int j = r - 1; j >= 0; --j) { sout_el[pm[j]] = s; s *= d[pm[j]]; }
    }
    int U = pow2_divisor_cap16(R);
    U = std::min(U, std::min(addr_align(src), addr_align(dst)));
    for (int q = 0; q < r; ++q) U = std::min(U, addr_align((uint64_t)sinb[q]));
    const int k = (int)(R / U);
    const int a1 = r - 1, b1 = pm[r - 1];
    // every input row starts at a multiple of this (plus the tile's column offset)
    uint64_t row_starts = 0;
    for (int q = 0; q < r; ++q) if (q != a1) row_starts |= (uint64_t)sinb[q];
    int G = 1;
    bool umt = false;
    if (k == 1 && !opt.force_ragged) {
        // 1- and 2-byte elements default to 8-byte micro-tile rows: 16 KiB tiles
        // then still give every thread a micro-tile, and the transpose stays small
        // enough in registers for six waves per SIMD.
        const int Gdef = opt.max_g > 0 ? std::min(16 / U, opt.max_g) : (U <= 2 ? 8 / U : 16 / U);
        G = Gdef;
        while (G > 1 && ((d[a1] % G) || (d[b1] % G) || addr_align(src) < U * G ||
                         addr_align(dst) < U * G || (row_starts % (uint64_t)(U * G))))
            G >>= 1;
        // Odd extents or pointers rule out aligned micro-tiles: on request keep them
        // anyway with unaligned vector accesses when both fastest extents hold one
        // (the ragged G = 1 paths measured faster on most shapes, so this is a
        // tuner candidate, not the default).
        if (((G == 1 && opt.umt == 1) || opt.umt == 2) && Gdef > 1 && d[a1] >= Gdef && d[b1] >= Gdef) {
            G = Gdef;
            umt = true;
        }
    }
    // a micro-tile's G outputs along B must be one contiguous run: with unaligned
    // micro-tiles on an extent that G does not divide, B stays a single axis
    const bool b_single = umt && (d[b1] % G) != 0;
    const int in_rb = opt.in_row_bytes > 0 ? opt.in_row_bytes : default_row_bytes(U, true);
    const int out_rb = opt.out_row_bytes > 0 ? opt.out_row_bytes : default_row_bytes(U, false);
    int64_t targetA = std::max<int64_t>(G, cdiv(in_rb, R));
    int64_t targetB = std::max<int64_t>(G, cdiv(out_rb, R));
    const int64_t soft_bytes = (int64_t)(opt.tile_kib > 0 ? opt.tile_kib : DEFAULT_TILE_KIB) * 1024;
    const int64_t tile_el = std::max<int64_t>(1, soft_bytes / R);

    // A: trailing input axes, B: trailing output axes; each grows by whole
    // axes (the slowest one partially) until its row target is met or the next
    // axis belongs to the other side.
    int A[MAXS], B[MAXS];
    int nA = 0, nB = 0;
    bool inA[MAXR] = {}, inB[MAXR] = {};
    A[nA++] = a1; inA[a1] = true;
    B[nB++] = b1; inB[b1] = true;
    int64_t prodA = d[a1], prodB = d[b1];
    int nxA = r - 2, nxB = r - 2;
    auto growA = [&]() {   // A's axes must stay one contiguous input run
        for (; prodA < targetA && nxA >= 0 && !inB[nxA] && nA < MAXS && sinb[nxA] == prodA * R; --nxA) {
            A[nA++] = nxA; inA[nxA] = true; prodA *= d[nxA];
        }
    };
    auto growB = [&]() {
        for (; !b_single && prodB < targetB && nxB >= 0 && !inA[pm[nxB]] && nB < MAXS; --nxB) {
            B[nB++] = pm[nxB]; inB[pm[nxB]] = true; prodB *= d[pm[nxB]];
        }
    };
    growA();
    growB();
    // A side that ran out of axes short of its target leaves a thin tile (few
    // elements per input row): the other side then grows to keep about
    // soft_bytes per tile, so short rows come in long runs of the long side.
    const bool shortA = prodA < targetA, shortB = prodB < targetB;
    if (shortA && !shortB) {
        targetB = std::max(targetB, cdiv(tile_el, prodA));
        growB();
    } else if (shortB && !shortA) {
        targetA = std::max(targetA, cdiv(tile_el, prodB));
        growA();
    }
    int64_t t[MAXR];
    for (int i = 0; i < r; ++i) t[i] = 1;
    int64_t innerA = 1, innerB = 1;
    for (int i = 0; i < nA - 1; ++i) { t[A[i]] = d[A[i]]; innerA *= d[A[i]]; }
    for (int i = 0; i < nB - 1; ++i) { t[B[i]] = d[B[i]]; innerB *= d[B[i]]; }
    const int aO = A[nA - 1], bO = B[nB - 1];
    auto set_outer = [&](int ax, int64_t target, int64_t inner, bool single) {
        int64_t v = std::min<int64_t>(d[ax], cdiv(target, inner));
        if (single) v = std::min<int64_t>(d[ax], (v + G - 1) / G * G);
        t[ax] = std::max<int64_t>(1, v);
    };
    set_outer(aO, targetA, innerA, nA == 1);
    set_outer(bO, targetB, innerB, nB == 1);
    // Short output rows whose next output axis sits on the input side: with the
    // whole B side in the tile, consecutive values of that axis are adjacent
    // output rows, so taking it whole turns short rows into one long output run.
    // (The input side needs no such step: when A is whole and B starts at the
    // next input axis, input rows are already back to back.)
    if (nB < r && t[bO] == d[bO] && innerB * d[bO] * R < out_rb) {
        const int x = pm[r - 1 - nB];
        if (x == aO) t[aO] = d[aO];
    }
    // shrink toward the soft tile size (an LDS row is padded to 16 bytes)
    const int64_t soft_lds = std::min<int64_t>(soft_bytes, opt.max_lds);
    for (int guard = 0; guard < 64; ++guard) {
        int64_t TA = innerA * t[aO], TB = innerB * t[bO];
        int64_t bytes = TB * ((TA * R + 15) / 16 * 16);
        if (bytes <= soft_lds) break;
        int64_t stepA = nA == 1 ? G : 1, stepB = nB == 1 ? G : 1;
        bool canA = t[aO] > stepA, canB = t[bO] > stepB;
        if (!canA && !canB) {
            if (bytes <= opt.max_lds) break;
            *why = "cannot fit a tile in LDS";
            return RR_ERR_UNSUPPORTED;
        }
        bool shrinkA = canA && (!canB || TA * R >= TB * R);
        if (shrinkA) t[aO] = std::max(stepA, (t[aO] / 2 + stepA - 1) / stepA * stepA);
        else t[bO] = std::max(stepB, (t[bO] / 2 + stepB - 1) / stepB * stepB);
    }
    // Fill refit for odd extents.  Halving toward the soft size and splitting an
    // outer axis at its row target leave the last tile along it mostly empty on
    // extents that the tile does not divide (an A axis of 39 at a target of 32
    // gives tiles of 32 and 7), and small problems then spend most of their
    // workgroups on thin tiles.  Where an outer axis ends in such a partial tile,
    // try every extent of A's outer axis that leaves B room for half its row
    // target, give B's outer axis the longest even split that keeps the tile
    // within the soft size, and keep the shape with the fewest tiles (evened out
    // along A) if that saves at least an eighth of them.  Rows on either side stay
    // at least half their target and one 128-byte line (or whole) and a multiple
    // of 16 bytes, so they end in no per-element tail (which costs
    // up to 15 one-byte accesses per row for 1-byte units); a whole axis may end
    // in one where units are 4..16 bytes (at most three accesses) or where the
    // row-target shape already held it whole.  Evenly divided axes are left alone.
    if (fill_refit(opt) && !umt) {
        const int64_t stepA = nA == 1 ? G : 1, stepB = nB == 1 ? G : 1;
        auto quantum = [&](int64_t step, int64_t inner) {   // tile extents with 16-byte rows
            const int64_t b = inner * step * R;
            return step * (16 / std::gcd<int64_t>(b, 16));
        };
        const int64_t qA = quantum(stepA, innerA), qB = quantum(stepB, innerB);
        const bool wholeA_ok = U >= 4 || (innerA * d[aO] * R) % 16 == 0 || t[aO] == d[aO];
        const bool wholeB_ok = U >= 4 || (innerB * d[bO] * R) % 16 == 0 || t[bO] == d[bO];
        // an extent covering len in n pieces: a multiple of q, or the whole axis
        // where allowed; 0 if neither
        auto split = [&](int64_t len, int64_t n, int64_t q, bool whole_ok) -> int64_t {
            const int64_t v = cdiv(cdiv(len, n), q) * q;
            if (v < len) return v;
            return whole_ok ? len : 0;
        };
        auto lds_of = [&](int64_t ta, int64_t tb) { return innerB * tb * ((innerA * ta * R + 15) / 16 * 16); };
        const bool ragged = (d[aO] % t[aO]) != 0 || (d[bO] % t[bO]) != 0;
        if (ragged && lds_of(t[aO], t[bO]) <= soft_lds) {
            // rows of at least half their target and at least one 128-byte line
            const int64_t minA = std::min<int64_t>(
                d[aO], std::max<int64_t>(stepA, cdiv(std::max(in_rb / 2, 128), innerA * R)));
            const int64_t minB = std::min<int64_t>(
                d[bO], std::max<int64_t>(stepB, cdiv(std::max(out_rb / 2, 128), innerB * R)));
            const int64_t cur = cdiv(d[aO], t[aO]) * cdiv(d[bO], t[bO]);
            int64_t best = cur, bestA = t[aO], bestB = t[bO];
            // tiles for A extent ta: B takes the longest even split that fits
            auto consider = [&](int64_t ta) {
                const int64_t row = innerB * ((innerA * ta * R + 15) / 16 * 16);
                const int64_t fit = soft_lds / row;   // B extent that fits the soft size
                int64_t tb;
                if (fit >= d[bO] && wholeB_ok) {
                    tb = d[bO];
                } else {
                    const int64_t cap = std::min<int64_t>(fit, d[bO] - 1) / qB * qB;
                    if (cap < qB) return;
                    tb = split(d[bO], cdiv(d[bO], cap), qB, false);
                    if (tb == 0) return;
                }
                if (tb < minB || lds_of(ta, tb) > soft_lds) return;
                const int64_t n = cdiv(d[aO], ta) * cdiv(d[bO], tb);
                if (n < best) { best = n; bestA = ta; bestB = tb; }
            };
            // A extents that leave B at least minB rows: the whole axis (where
            // allowed), then every multiple of qA from the longest down (longer
            // input rows win ties) -- at most a few thousand steps, whatever
            // the extent
            const int64_t amax_row = soft_lds / (innerB * minB);   // padded A row bytes
            if (wholeA_ok && d[aO] >= minA && (innerA * d[aO] * R + 15) / 16 * 16 <= amax_row) consider(d[aO]);
            int64_t ta = std::min<int64_t>(d[aO] - 1, amax_row / (innerA * R)) / qA * qA;
            for (; ta >= std::max<int64_t>(qA, minA); ta -= qA) consider(ta);
            // same tile count, evened out along A (never longer, so it still fits)
            if (bestA != t[aO] || bestB != t[bO]) {
                const int64_t even = split(d[aO], cdiv(d[aO], bestA), qA, wholeA_ok);
                if (even != 0 && even >= minA && even <= bestA) bestA = even;
            }
            if (best * 8 <= cur * 7) {   // at least an eighth fewer tiles
                t[aO] = bestA;
                t[bO] = bestB;
            }
        }
    }
    // Stacked tiles: when the last two axes are swapped and the tile holds both
    // whole, a tile would be one small transpose; the next slower input axis C
    // (whose stride is exactly one such transpose) then stacks several of them,
    // so a tile reads one contiguous range and writes one contiguous run per
    // transpose (one range when C is also the next output axis).
    int cax = -1;
    {
        const int64_t msub = innerA * t[aO] * innerB * t[bO] * R;
        if (k == 1 && U < 16 && r >= 3 && nA == 1 && nB == 1 && t[a1] == d[a1] && t[b1] == d[b1] &&
            b1 == r - 2 && pm[r - 2] == a1 && sinb[b1] == d[a1] * R && msub * 2 <= soft_bytes) {
            cax = r - 3;
            G = 1;
            umt = false;
            t[cax] = std::min<int64_t>(d[cax], std::max<int64_t>(1, soft_bytes / msub));
            a.flags |= TF_STACK;
            a.msub = a.msubp = (uint32_t)msub;
            a.sinC = (uint64_t)sinb[cax];
            a.soutC = (uint64_t)(sout_el[cax] * R);
        }
    }
    // Rows back to back (A whole, B the next slower input axis): a tile's input is
    // one range, read as 16-byte vectors when every tile starts on a 16-byte
    // boundary, so short rows take B in multiples of 16 / gcd(row bytes, 16).
    if (cax < 0 && !umt && nB == 1 && t[aO] == d[aO] && b1 == r - 1 - nA && sinb[b1] == innerA * t[aO] * R) {
        const int64_t rowb = innerA * t[aO] * R;
        if (rowb % 16 != 0 || rowb < 64) {
            const int64_t low = std::min<int64_t>(rowb & -rowb, 16);
            const int64_t m = std::max<int64_t>(G, 16 / low);
            if (t[b1] < d[b1] && t[b1] >= m) t[b1] = t[b1] / m * m;
        }
    }
    a.grid_cO = -1;
    a.cO_len = 1;
    a.cO_t = 1;
    a.TA = (uint32_t)(innerA * t[aO]);
    a.TB = (uint32_t)(innerB * t[bO]);
    a.TAinner = (uint32_t)innerA;
    a.TBinner = (uint32_t)innerB;
    a.nA = nA; a.nB = nB;
    for (int i = 0; i < nA; ++i) {
        a.tA[i] = (uint32_t)t[A[i]]; a.mA[i] = make_magic(a.tA[i]);
        a.soutA[i] = (uint64_t)(sout_el[A[i]] * R);
    }
    for (int i = 0; i < nB; ++i) {
        a.tB[i] = (uint32_t)t[B[i]]; a.mB[i] = make_magic(a.tB[i]);
        a.sinB[i] = (uint64_t)sinb[B[i]];
    }
    a.R = (uint32_t)R;
    a.src = src; a.dst = dst;
    // tile grid
    int order[MAXR];
    for (int i = 0; i < r; ++i) order[i] = i;
    // Tiles of 4..16-byte elements are walked in output order (neighbouring
    // workgroups then write neighbouring output segments); 1- and 2-byte
    // elements keep input order, which measured slightly faster for them.
    const bool order_out = opt.order_out < 0 ? U >= 4 : opt.order_out != 0;
    if (order_out) for (int j = 0; j < r; ++j) order[j] = pm[j];
    a.ngrid = 0; a.grid_aO = -1; a.grid_bO = -1;
    uint64_t ntiles = 1;
    for (int oi = 0; oi < r; ++oi) {
        int s = order[oi];
        bool tiled = inA[s] || inB[s] || s == cax;
        int64_t n = tiled ? cdiv(d[s], t[s]) : d[s];
        if (n <= 1) continue;
        int g = a.ngrid++;
        a.gn[g] = (uint32_t)n; a.gm[g] = make_magic((uint32_t)n);
        int64_t step = tiled ? t[s] : 1;
        a.gsin[g] = (uint64_t)(step * sinb[s]);
        a.gsout[g] = (uint64_t)(step * sout_el[s] * R);
        if (s == aO) a.grid_aO = g;
        if (s == bO) a.grid_bO = g;
        if (s == cax) a.grid_cO = g;
        ntiles *= (uint64_t)n;
        if (ntiles > 0x7fffffffULL) { *why = "too many tiles for one launch"; return RR_ERR_UNSUPPORTED; }
    }
    a.aO_len = (uint32_t)d[aO]; a.aO_t = (uint32_t)t[aO];
    a.bO_len = (uint32_t)d[bO]; a.bO_t = (uint32_t)t[bO];
    if (cax >= 0) { a.cO_len = (uint32_t)d[cax]; a.cO_t = (uint32_t)t[cax]; }
    a.ntiles = (uint32_t)ntiles;
    // input rows start at multiples of the other axes' strides plus the tile's column offset
    uint64_t ra = src | row_starts;
    if (nA == 1) ra |= (uint64_t)(t[a1] * R);
    // rows are back to back when every A axis is whole and the single B axis is
    // the next slower input axis, adjacent to them
    const bool flat_ok = nB == 1 && t[aO] == d[aO] && b1 == r - 1 - nA && sinb[b1] == innerA * t[aO] * R;
    if (umt) a.flags |= TF_UMT;
    else G = line_friendly_g(U, G, a.TB, nA, a.soutA[0], false);
    rr_status st = finish_tile(a, U, G, k, ra, flat_ok && !umt, src, b1 > 0 ? (uint64_t)d[b1] : 0, opt, why);
    if (st != RR_OK) return st;
    cache_policy(a, opt);
    if (a.ngrid >= 2 && (opt.diag == 1 || (opt.diag == -1 && diag_by_default(c)))) a.flags |= TF_DIAG;
    p->grid = a.ntiles;
    p->bytes = (uint64_t)c.total_bytes;
    return RR_OK;
}

// 2-8 sets of 1-8-byte elements on 16-byte boundaries, a whole number of
// 16-byte vectors each: joined and split in registers, vectors swapped between
// lanes through a wave-private LDS region (no tile, no workgroup barrier).
// nbatch problems lie bstride bytes apart on both sides.  False (nothing
// planned) where these conditions do not hold.
static bool plan_weave(uint64_t flat, const uint64_t* planes, int n, int64_t count, int esize, bool de,
                       int64_t nbatch, uint64_t bstride, const TileOptions& opt, Plan* p) {
    const bool pow2_unit = esize == 1 || esize == 2 || esize == 4 || esize == 8;
    if (!opt.weave || !pow2_unit || n < 2 || n > WEAVE_MAX_SETS || count <= 0 || nbatch < 1) return false;
    // eight-set de-interlaces, and interlaces of eight sets of 4-8-byte
    // elements, stay on the tile (measured 4-10 % faster from cold caches)
    if (n == 8 && (de || esize >= 4)) return false;
    bool aligned = flat % 16 == 0 && (count * esize) % 16 == 0 && bstride % 16 == 0;
    for (int c = 0; c < n; ++c) aligned = aligned && planes[c] % 16 == 0;
    const int64_t nvec = count * esize / 16;
    if (!aligned || nvec > 0x7fffffffLL) return false;
    // two chunks per wave (2 * n loads in flight per lane) up to three sets and
    // for a four-set de-interlace; one from four sets on (two would take 32 KiB
    // or more of LDS per workgroup, cutting the waves per CU to 20 or fewer)
    const uint32_t chunks = n <= 3 || (n == 4 && de) ? 2u : 1u;
    const int64_t bpb = (nvec + (int64_t)NT * chunks - 1) / ((int64_t)NT * chunks);
    if (bpb * nbatch > 0x7fffffffLL) return false;
    p->kind = K_WEAVE;
    WeaveArgs& w = p->weave;
    std::memset(&w, 0, sizeof(w));
    for (int c = 0; c < n; ++c) w.planes[c] = planes[c];
    w.joined = flat;
    w.bstride = nbatch > 1 ? bstride : 0;
    w.nvec = (uint32_t)nvec;
    w.n = (uint32_t)n;
    w.unit = (uint32_t)esize;
    w.de = de ? 1u : 0u;
    // cache override: bit 0 cached reads, bit 1 cached writes (joined side
    // only).  Built in: streamed, except the joined stores of an interlace of an
    // odd number of sets, which measured 0.5-7 % faster through the caches from
    // cold caches (even numbers of sets 0-5 % slower; cached joined loads of a
    // de-interlace 15-40 % slower)
    w.cached = opt.cache >= 0 ? (uint32_t)((opt.cache >> (de ? 0 : 1)) & 1) : (!de && n % 2 == 1) ? 1u : 0u;
    w.chunks = chunks;
    w.bpb = (uint32_t)bpb;
    p->grid = (uint32_t)(bpb * nbatch);
    return true;
}

// A dense permute that swaps the two fastest axes where one of them has 2-8
// entries -- (n, L) -> (L, n), an interlace of n sets, or (L, n) -> (n, L), a
// de-interlace -- optionally under one unpermuted slower axis (a batch of them):
// the register interlace above with the sets at a fixed stride.  Batched sets
// of fewer than 256 vectors (4 KiB) stay on the tile kernel, whose stacked
// tiles hold several small transposes each; the register path would give each
// one a whole workgroup.
static bool plan_weave_permute(uint64_t dst, uint64_t src, const Canon& c, const TileOptions& opt, Plan* p) {
    if (c.strided || !(c.elem_bytes == 1 || c.elem_bytes == 2 || c.elem_bytes == 4 || c.elem_bytes == 8)) return false;
    const bool r2 = c.rank == 2 && c.perm[0] == 1 && c.perm[1] == 0;
    const bool r3 = c.rank == 3 && c.perm[0] == 0 && c.perm[1] == 2 && c.perm[2] == 1;
    if (!r2 && !r3) return false;
    const int64_t e = c.elem_bytes;
    const int64_t A = c.dims[c.rank - 2], B = c.dims[c.rank - 1];   // input: A rows of B elements
    const int64_t nbatch = r3 ? c.dims[0] : 1;
    const uint64_t bstride = (uint64_t)(A * B * e);
    if (nbatch > 1 && std::max(A, B) * e < (int64_t)NT * 16) return false;
    uint64_t planes[WEAVE_MAX_SETS];
    if (A >= 2 && A <= WEAVE_MAX_SETS) {   // A sets of B elements -> joined
        for (int k = 0; k < (int)A; ++k) planes[k] = src + (uint64_t)(k * B * e);
        if (plan_weave(dst, planes, (int)A, B, (int)e, false, nbatch, bstride, opt, p)) return true;
    }
    if (B >= 2 && B <= WEAVE_MAX_SETS) {   // joined (A groups of B) -> B sets of A elements
        for (int k = 0; k < (int)B; ++k) planes[k] = dst + (uint64_t)(k * A * e);
        if (plan_weave(src, planes, (int)B, A, (int)e, true, nbatch, bstride, opt, p)) return true;
    }
    return false;
}

rr_status plan_permute(uint64_t dst, uint64_t src, const Canon& c, const TileOptions& opt,
                       Plan* p, std::string* why) {
    p->c = c;
    p->bytes = (uint64_t)c.total_bytes;
    if (c.count == 0 || c.total_bytes == 0) { p->kind = K_EMPTY; p->grid = 0; return RR_OK; }
    if (c.rank == 0) { plan_copy(dst, src, (uint64_t)c.total_bytes, p); return RR_OK; }
    if (c.elem_bytes >= RUN_MIN_BYTES) return plan_run(dst, src, c, p, why);
    // a box whose fastest input axis is kept but strided (one component of
    // interleaved records): whole records read with 16-byte vectors
    if (c.perm[c.rank - 1] == c.rank - 1 && plan_select(dst, src, c, p)) return RR_OK;
    // a box whose fastest input axis is not contiguous (a dropped or cut innermost
    // axis) has no input rows to tile: gather its elements (one run each)
    if (c.sinb[c.rank - 1] != c.elem_bytes || c.perm[c.rank - 1] == c.rank - 1) return plan_run(dst, src, c, p, why);
    // small-axis transposes: the register interlace, for an interlace only where
    // the tile would not merge its short output rows into whole 16-byte stores
    Plan wv;
    wv.c = c;
    wv.bytes = p->bytes;
    const bool weave = plan_weave_permute(dst, src, c, opt, &wv);
    if (weave && wv.weave.de) { *p = wv; return RR_OK; }
    // a tuned shape for this problem replaces the built-in choice (not an explicit override)
    TileOptions tuned;
    rr_status st;
    if (opt.use_tuned && tune_lookup(c, dst, src, &tuned)) {
        tuned.max_lds = opt.max_lds;
        st = plan_tile(dst, src, c, tuned, p, why);
    } else {
        st = plan_tile(dst, src, c, opt, p, why);
    }
    if (st == RR_OK && weave && p->kind == K_TILE && !(p->tile.flags & TF_OUT_MERGE)) *p = wv;
    return st;
}

// The tile plan of an interlace (plane-pointer table on the set side).
static rr_status plan_interlace_tile(uint64_t flat, const uint64_t* planes, int n, int64_t count, int esize,
                                     bool de, const TileOptions& opt, Plan* p, std::string* why) {
    const uint64_t dst = flat;
    p->kind = K_TILE;
    TileArgs& a = p->tile;
    std::memset(&a, 0, sizeof(a));
    const int64_t R = esize;
    int al = addr_align(dst);
    for (int c = 0; c < n; ++c) al = std::min(al, addr_align(planes[c]));
    int U = std::min(pow2_divisor_cap16(R), al);
    const int k = (int)(R / U);
    int G = 1;
    if (k == 1) {
        G = 16 / U;
        while (G > 1 && ((count % G) || (n % G) || al < U * G)) G >>= 1;
    }
    const int in_rb = opt.in_row_bytes > 0 ? opt.in_row_bytes : default_row_bytes(U, true);
    const int out_rb = opt.out_row_bytes > 0 ? opt.out_row_bytes : default_row_bytes(U, false);
    // aim for ~16 KiB tiles: the plane axis is short
    const int64_t tile_target = 16384;
    int64_t L = std::max<int64_t>(cdiv(de ? out_rb : in_rb, R), cdiv(tile_target, n * R));
    L = std::min<int64_t>(count, (L + 15) / 16 * 16);  // whole 16-byte vectors per row
    while (L > G && (int64_t)((L * R + 15) / 16 * 16) * n > opt.max_lds && !de) L = std::max<int64_t>(G, L / 2 / G * G);
    while (L > G && (int64_t)(((int64_t)n * R + 15) / 16 * 16) * L > opt.max_lds && de) L = std::max<int64_t>(G, L / 2 / G * G);
    // interlaced output rows are n elements: keep micro-tiles only where they
    // still write well-filled lines (de-interlace writes long plane rows)
    if (!de) G = line_friendly_g(U, G, (uint32_t)n, 1, (uint64_t)(n * R), false);
    a.R = (uint32_t)R;
    a.ngrid = 0; a.grid_aO = -1; a.grid_bO = -1; a.grid_cO = -1;
    a.cO_len = 1; a.cO_t = 1;
    int64_t nt = cdiv(count, L);
    if (nt > 0x7fffffffLL) { *why = "too many tiles"; return RR_ERR_UNSUPPORTED; }
    if (!de) {
        // A = element axis (length L per tile), B = plane axis (n, full)
        a.flags = TF_IN_TABLE;
        a.src = 0; a.dst = dst;
        a.TA = (uint32_t)L; a.TB = (uint32_t)n; a.TAinner = 1; a.TBinner = 1;
        a.nA = 1; a.tA[0] = (uint32_t)L; a.mA[0] = make_magic((uint32_t)L); a.soutA[0] = (uint64_t)(n * R);
        a.nB = 1; a.tB[0] = (uint32_t)n; a.mB[0] = make_magic((uint32_t)n); a.sinB[0] = 0;
        if (nt > 1) {
            a.ngrid = 1; a.gn[0] = (uint32_t)nt; a.gm[0] = make_magic((uint32_t)nt);
            a.gsin[0] = (uint64_t)(L * R); a.gsout[0] = (uint64_t)(L * n * R); a.grid_aO = 0;
        }
        a.aO_len = (uint32_t)count; a.aO_t = (uint32_t)L;
        a.bO_len = (uint32_t)n; a.bO_t = (uint32_t)n;
        for (int c = 0; c < n; ++c) a.table[c] = planes[c];
        uint64_t ra = (uint64_t)(L * R) | (uint64_t)(count * R);
        for (int c = 0; c < n; ++c) ra |= planes[c];
        rr_status st = finish_tile(a, U, G, k, ra, false, 0, 0, opt, why);
        if (st != RR_OK) return st;
    } else {
        // A = plane axis (n, full), B = element axis (length L per tile)
        a.flags = TF_OUT_TABLE;
        a.src = flat;
        a.dst = 0;
        a.TA = (uint32_t)n; a.TB = (uint32_t)L; a.TAinner = 1; a.TBinner = 1;
        a.nA = 1; a.tA[0] = (uint32_t)n; a.mA[0] = make_magic((uint32_t)n); a.soutA[0] = 0;
        a.nB = 1; a.tB[0] = (uint32_t)L; a.mB[0] = make_magic((uint32_t)L); a.sinB[0] = (uint64_t)(n * R);
        if (nt > 1) {
            a.ngrid = 1; a.gn[0] = (uint32_t)nt; a.gm[0] = make_magic((uint32_t)nt);
            a.gsin[0] = (uint64_t)(L * n * R); a.gsout[0] = (uint64_t)(L * R); a.grid_bO = 0;
        }
        a.aO_len = (uint32_t)n; a.aO_t = (uint32_t)n;
        a.bO_len = (uint32_t)count; a.bO_t = (uint32_t)L;
        for (int c = 0; c < n; ++c) a.table[c] = planes[c];
        uint64_t ra = a.src | (uint64_t)(n * R);
        rr_status st = finish_tile(a, U, G, k, ra, true, a.src, 0, opt, why);
        if (st != RR_OK) return st;
    }
    cache_policy(a, opt);
    a.ntiles = (uint32_t)nt;
    p->grid = a.ntiles;
    return RR_OK;
}

// Interlace: virtual input (n planes, count) -> output (count, n).
// De-interlace: input (count, n) -> virtual output (n planes, count).
rr_status plan_interlace(uint64_t flat, const uint64_t* planes, int n, int64_t count, int esize,
                         bool de, const TileOptions& opt, Plan* p, std::string* why) {
    p->c = Canon{};
    p->bytes = (uint64_t)(count * n * esize);
    if (count == 0) { p->kind = K_EMPTY; p->grid = 0; return RR_OK; }
    if (n == 1) { plan_copy(de ? planes[0] : flat, de ? flat : planes[0], (uint64_t)(count * esize), p); return RR_OK; }
    if (de && plan_weave(flat, planes, n, count, esize, de, 1, 0, opt, p)) return RR_OK;
    rr_status st = plan_interlace_tile(flat, planes, n, count, esize, de, opt, p, why);
    if (st == RR_OK && !de && !(p->tile.flags & TF_OUT_MERGE)) plan_weave(flat, planes, n, count, esize, de, 1, 0, opt, p);
    return st;
}

std::string describe(const Plan& p) {
    std::ostringstream o;
    static const char* names[] = {"empty", "copy", "run", "tile", "gather", "select", "weave"};
    o << "class=" << names[p.kind];
    const Canon& c = p.c;
    o << " rank=" << c.rank << " dims=";
    for (int k = 0; k < c.rank; ++k) o << (k ? "," : "") << c.dims[k];
    o << " perm=";
    for (int k = 0; k < c.rank; ++k) o << (k ? "," : "") << c.perm[k];
    o << " esize_bytes=" << c.elem_bytes << " bytes=" << p.bytes << " grid=" << p.grid;
    if (p.kind == K_COPY) o << " vec=" << p.copy.wbytes << " head=" << p.copy.head << " tail=" << p.copy.tail;
    if (p.kind == K_RUN)
        o << " vec=" << p.run.wbytes << " vpr=" << p.run.vpr << " ua=" << p.run.ua << " cached=" << p.run.cached;
    if (p.kind == K_WEAVE)
        o << " n=" << p.weave.n << " unit=" << p.weave.unit << " de=" << p.weave.de << " nvec=" << p.weave.nvec
          << " cached=" << p.weave.cached << " chunks=" << p.weave.chunks
          << " batches=" << (p.weave.bpb ? p.grid / p.weave.bpb : 0);
    if (p.kind == K_GATHER) o << " vec=" << p.gather.wbytes << " k=" << p.gather.k << " indexed=" << (p.gather.idx != 0);
    if (p.kind == K_SELECT) o << " vec=16 stride=" << p.select.S << " m=" << p.select.M << " n=" << p.select.n;
    if (p.kind == K_TILE) {
        const TileArgs& a = p.tile;
        o << " unit=" << a.unit << " g=" << a.g << " k=" << a.k << " TA=" << a.TA << " TB=" << a.TB
          << " nA=" << a.nA << " nB=" << a.nB << " win=" << a.win << " pitch=" << a.pitch
          << " lds=" << a.lds_bytes << " ntiles=" << a.ntiles << " ngrid=" << a.ngrid
          << " tc=" << a.cO_t << " flags=" << a.flags;
    }
    return o.str();
}

}  // namespace rr
