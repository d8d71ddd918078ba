// rr_emu.cpp -- CPU execution of librr's kernel bodies, for tests only.
//
// Builds the product's planner (rr_plan.cpp) and per-thread kernel bodies
// (rr_device.hpp) for the host and runs every workgroup and thread of a launch
// sequentially: the read phase of all threads, then (after what is a barrier on
// the GPU) the write phase.  Every buffer -- source, destination, each plane and
// each LDS tile -- is a separate heap allocation of exactly its size, so under
// AddressSanitizer any out-of-bounds access of the GPU index arithmetic aborts
// here instead of faulting a GPU.  LDS tiles are filled with a poison byte so a
// read of a never-written LDS byte shows up as a wrong output byte.
//
// Input: a manifest, one job per line:
//   permute  ndim d0..d{n-1} p0..p{n-1} esize src_off dst_off in_rb out_rb order max_g ragged xcd umt diag fill weave infile outfile
//   reorder  ndim d.. base.. range.. m order.. esize src_off dst_off umt max_g infile outfile
//   gather   src_count count esize indexed start stride src_off dst_off infile idxfile outfile
//   stencil  rows cols radius shape nweights w... infile outfile             (float grids)
//   interlace   n count esize off in_rb out_rb weave infile outfile    (infile: n planes back to back)
//   deinterlace n count esize off in_rb out_rb weave infile outfile    (outfile: n planes back to back)
// (interlace buffers start on 64-byte boundaries before the offset, as GPU
// allocations do, so the aligned register path is planned where it applies)
// Prints one line per job: "ok <plan description>" or "err <status> <reason>".
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <thread>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../paper_1011_3583_amd/csrc/rr_batch.hpp"
#include "../../paper_1011_3583_amd/csrc/rr_device.hpp"
#include "../../paper_1011_3583_amd/csrc/rr_plan.hpp"

using namespace rr;

static std::vector<uint8_t> read_file(const std::string& path) {
    std::ifstream f(path, std::ios::binary);
    return std::vector<uint8_t>((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
}

static void write_file(const std::string& path, const uint8_t* p, size_t n) {
    std::ofstream f(path, std::ios::binary);
    f.write(reinterpret_cast<const char*>(p), (std::streamsize)n);
}

template <int U, int G>
static void run_tile_ug(const TileArgs& a, uint32_t grid) {
    std::vector<uint8_t> seen(grid, 0);
    for (uint32_t b = 0; b < grid; ++b) {
        const uint32_t tile = block_to_tile(a, b);
        if (tile >= grid || seen[tile]++) { std::fprintf(stderr, "block %u -> bad tile %u\n", b, tile); std::abort(); }
        uint8_t* lds = new uint8_t[a.lds_bytes];
        std::memset(lds, 0xA5, a.lds_bytes);
        const TileCtx t = tile_decode(a, tile);
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) read_dispatch<U, G>(a, t, lds, tid);
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) write_phase<U, G>(a, t, lds, tid);
        delete[] lds;
    }
}

static bool run_tile(const TileArgs& a, uint32_t grid) {
    switch (a.unit * 100 + a.g) {
        case 101: run_tile_ug<1, 1>(a, grid); return true;
        case 102: run_tile_ug<1, 2>(a, grid); return true;
        case 104: run_tile_ug<1, 4>(a, grid); return true;
        case 108: run_tile_ug<1, 8>(a, grid); return true;
        case 116: run_tile_ug<1, 16>(a, grid); return true;
        case 201: run_tile_ug<2, 1>(a, grid); return true;
        case 202: run_tile_ug<2, 2>(a, grid); return true;
        case 204: run_tile_ug<2, 4>(a, grid); return true;
        case 208: run_tile_ug<2, 8>(a, grid); return true;
        case 401: run_tile_ug<4, 1>(a, grid); return true;
        case 402: run_tile_ug<4, 2>(a, grid); return true;
        case 404: run_tile_ug<4, 4>(a, grid); return true;
        case 801: run_tile_ug<8, 1>(a, grid); return true;
        case 802: run_tile_ug<8, 2>(a, grid); return true;
        case 1601: run_tile_ug<16, 1>(a, grid); return true;
    }
    return false;
}

template <int W>
static void run_copy_w(const CopyArgs& a, uint32_t grid) {
    for (uint32_t b = 0; b < grid; ++b)
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) copy_thread<W>(a, b, grid, tid);
}

template <int W>
static void run_run_w(const RunArgs& a, uint32_t grid) {
    for (uint32_t b = 0; b < grid; ++b)
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) run_thread<W>(a, b, tid);
}

template <int U, int G>
static void run_batch_tile_ug(const BatchGroup& g, const uint8_t* table) {
    const TileArgs* args = reinterpret_cast<const TileArgs*>(table + g.args_off);
    const uint32_t* prefix = reinterpret_cast<const uint32_t*>(table + g.prefix_off);
    const EntryRange* ranges = reinterpret_cast<const EntryRange*>(table + g.range_off);
    std::vector<std::vector<uint8_t>> seen(g.njobs);   // each entry's tiles taken once
    for (uint32_t j = 0; j < g.njobs; ++j) {
        seen[j].assign(prefix[j + 1] - prefix[j], 0);
        // the record repeats the entry's workgroup range from the prefix sums
        if (ranges[j].start != prefix[j] || ranges[j].count != prefix[j + 1] - prefix[j]) {
            std::fprintf(stderr, "entry %u: record (%u, %u) != prefix range (%u, %u)\n", j, ranges[j].start,
                         ranges[j].count, prefix[j], prefix[j + 1] - prefix[j]);
            std::abort();
        }
    }
    for (uint32_t b = 0; b < g.total_blocks; ++b) {
        const uint32_t j = find_job(prefix, g.njobs, b);
        const TileArgs& a = args[j];
        const uint32_t tile = batch_block_to_tile(a.flags, ranges[j], b);
        const uint32_t rel = tile - ranges[j].first;
        if (tile < ranges[j].first || rel >= seen[j].size() || seen[j][rel]++) {
            std::fprintf(stderr, "batch block %u (entry %u) -> bad tile %u\n", b, j, tile);
            std::abort();
        }
        uint8_t* lds = new uint8_t[g.lds_bytes];
        std::memset(lds, 0xA5, g.lds_bytes);
        const TileCtx t = tile_decode(a, tile);
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) read_dispatch<U, G>(a, t, lds, tid);
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) write_phase<U, G>(a, t, lds, tid);
        delete[] lds;
    }
}

template <int W>
static void run_batch_small(const BatchGroup& g, const uint8_t* table) {
    const uint32_t* prefix = reinterpret_cast<const uint32_t*>(table + g.prefix_off);
    const EntryRange* ranges = reinterpret_cast<const EntryRange*>(table + g.range_off);
    for (uint32_t b = 0; b < g.total_blocks; ++b)
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) {
            if (g.kind == K_COPY)
                batch_copy_block<W>(reinterpret_cast<const CopyArgs*>(table + g.args_off), prefix, ranges,
                                    g.njobs, b, tid);
            else
                batch_run_block<W>(reinterpret_cast<const RunArgs*>(table + g.args_off), prefix, ranges,
                                   g.njobs, b, tid);
        }
}

static bool emulate_group(const BatchGroup& g, const uint8_t* table) {
    if (g.kind != K_TILE) {
        switch (g.variant) {
            case 16: run_batch_small<16>(g, table); return true;
            case 8: run_batch_small<8>(g, table); return true;
            case 4: run_batch_small<4>(g, table); return true;
            case 2: run_batch_small<2>(g, table); return true;
            default: run_batch_small<1>(g, table); return true;
        }
    }
    switch (g.variant) {
        case 101: run_batch_tile_ug<1, 1>(g, table); return true;
        case 102: run_batch_tile_ug<1, 2>(g, table); return true;
        case 104: run_batch_tile_ug<1, 4>(g, table); return true;
        case 108: run_batch_tile_ug<1, 8>(g, table); return true;
        case 116: run_batch_tile_ug<1, 16>(g, table); return true;
        case 201: run_batch_tile_ug<2, 1>(g, table); return true;
        case 202: run_batch_tile_ug<2, 2>(g, table); return true;
        case 204: run_batch_tile_ug<2, 4>(g, table); return true;
        case 208: run_batch_tile_ug<2, 8>(g, table); return true;
        case 401: run_batch_tile_ug<4, 1>(g, table); return true;
        case 402: run_batch_tile_ug<4, 2>(g, table); return true;
        case 404: run_batch_tile_ug<4, 4>(g, table); return true;
        case 801: run_batch_tile_ug<8, 1>(g, table); return true;
        case 802: run_batch_tile_ug<8, 2>(g, table); return true;
        case 1601: run_batch_tile_ug<16, 1>(g, table); return true;
    }
    return false;
}

template <int R, int SHAPE, int TH>
static void run_stencil_rs(const StencilArgs& a) {
    const size_t nl = (size_t)(TH + 2 * R) * ST_PITCH;
    std::vector<uint8_t> seen(a.ntiles, 0);   // the workgroup -> tile map takes each tile once
    for (uint32_t b = 0; b < a.ntiles; ++b) {
        const uint32_t tile = xcd_range(b, a.ntiles);
        if (tile >= a.ntiles || seen[tile]++) {
            std::fprintf(stderr, "stencil block %u -> bad tile %u\n", b, tile);
            std::abort();
        }
        uint32_t* lds = new uint32_t[nl];
        std::memset(lds, 0xA5, nl * 4);
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) stencil_load<R, TH>(a, tile, lds, tid);
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) stencil_compute<R, SHAPE, TH>(a, tile, lds, tid);
        delete[] lds;
    }
}

template <int TH>
static bool run_stencil_th(const StencilArgs& a) {
    switch (a.radius * 2 + a.shape) {
        case 2: run_stencil_rs<1, 0, TH>(a); return true;
        case 3: run_stencil_rs<1, 1, TH>(a); return true;
        case 4: run_stencil_rs<2, 0, TH>(a); return true;
        case 5: run_stencil_rs<2, 1, TH>(a); return true;
        case 6: run_stencil_rs<3, 0, TH>(a); return true;
        case 7: run_stencil_rs<3, 1, TH>(a); return true;
        case 8: run_stencil_rs<4, 0, TH>(a); return true;
        case 9: run_stencil_rs<4, 1, TH>(a); return true;
    }
    return false;
}

static bool run_stencil(const StencilArgs& a) {
    switch (a.th) {
        case 16: return run_stencil_th<16>(a);
        case 32: return run_stencil_th<32>(a);
    }
    return false;
}

static uint64_t g_bad = 0;   // rejected indices of the last gather

template <int W>
static void run_gather_w(const GatherArgs& a, uint32_t grid) {
    for (uint32_t b = 0; b < grid; ++b)
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) g_bad += gather_thread<W>(a, b, grid, tid);
}

template <int R, int M>
static void run_select_rm(const SelectArgs& a, uint32_t grid) {
    for (uint32_t b = 0; b < grid; ++b) {
        if (a.nax == 0) {
            std::vector<uint8_t> lds(NT * 16 * M, 0xA5);
            for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) select_stage<R, M>(a, b, lds.data(), tid);
            for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) select_pack_store<R, M>(a, b, lds.data(), tid);
        } else {
            for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) select_thread<R, M>(a, b, tid);
        }
    }
}

template <int U, int N, bool DE, int R>
static void run_weave_undr(const WeaveArgs& a, uint32_t grid) {
    for (uint32_t g = 0; g < grid; ++g) {
        const uint32_t batch = g / a.bpb, b = g - batch * a.bpb;
        const uint64_t off = (uint64_t)batch * a.bstride;
        std::vector<uint8_t> lds((size_t)R * NT * N * 16, 0xA5);
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) weave_stage<U, N, DE, false, R>(a, b, off, lds.data(), tid);
        for (uint32_t tid = 0; tid < (uint32_t)NT; ++tid) weave_finish<U, N, DE, false, R>(a, b, off, lds.data(), tid);
    }
}

template <int U, int N>
static bool run_weave_un(const WeaveArgs& a, uint32_t grid) {
    if (a.chunks == 1) {
        if (a.de) run_weave_undr<U, N, true, 1>(a, grid);
        else run_weave_undr<U, N, false, 1>(a, grid);
        return true;
    }
    if constexpr (N <= 4) {
        if (a.chunks == 2) {
            if (a.de) run_weave_undr<U, N, true, 2>(a, grid);
            else run_weave_undr<U, N, false, 2>(a, grid);
            return true;
        }
    }
    return false;
}

template <int U>
static bool run_weave_u(const WeaveArgs& a, uint32_t grid) {
    switch (a.n) {
        case 2: return run_weave_un<U, 2>(a, grid);
        case 3: return run_weave_un<U, 3>(a, grid);
        case 4: return run_weave_un<U, 4>(a, grid);
        case 5: return run_weave_un<U, 5>(a, grid);
        case 6: return run_weave_un<U, 6>(a, grid);
        case 7: return run_weave_un<U, 7>(a, grid);
        case 8: return run_weave_un<U, 8>(a, grid);
    }
    return false;
}

static bool run_weave(const WeaveArgs& a, uint32_t grid) {
    switch (a.unit) {
        case 1: return run_weave_u<1>(a, grid);
        case 2: return run_weave_u<2>(a, grid);
        case 4: return run_weave_u<4>(a, grid);
        case 8: return run_weave_u<8>(a, grid);
    }
    return false;
}

template <int R>
static bool run_select_r(const SelectArgs& a, uint32_t grid) {
    switch (a.M) {
        case 2: run_select_rm<R, 2>(a, grid); return true;
        case 3: run_select_rm<R, 3>(a, grid); return true;
        case 4: run_select_rm<R, 4>(a, grid); return true;
    }
    return false;
}

static bool emulate(const Plan& p) {
    switch (p.kind) {
        case K_EMPTY: return true;
        case K_COPY:
            switch (p.copy.wbytes) {
                case 16: run_copy_w<16>(p.copy, p.grid); return true;
                case 8: run_copy_w<8>(p.copy, p.grid); return true;
                case 4: run_copy_w<4>(p.copy, p.grid); return true;
                case 2: run_copy_w<2>(p.copy, p.grid); return true;
                default: run_copy_w<1>(p.copy, p.grid); return true;
            }
        case K_RUN:
            switch (p.run.wbytes) {
                case 16: run_run_w<16>(p.run, p.grid); return true;
                case 8: run_run_w<8>(p.run, p.grid); return true;
                case 4: run_run_w<4>(p.run, p.grid); return true;
                case 2: run_run_w<2>(p.run, p.grid); return true;
                default: run_run_w<1>(p.run, p.grid); return true;
            }
        case K_TILE:
            return run_tile(p.tile, p.grid);
        case K_SELECT:
            switch (p.select.R) {
                case 1: return run_select_r<1>(p.select, p.grid);
                case 2: return run_select_r<2>(p.select, p.grid);
                case 4: return run_select_r<4>(p.select, p.grid);
                case 8: return run_select_r<8>(p.select, p.grid);
            }
            return false;
        case K_WEAVE:
            return run_weave(p.weave, p.grid);
        case K_GATHER:
            switch (p.gather.wbytes) {
                case 16: run_gather_w<16>(p.gather, p.grid); return true;
                case 8: run_gather_w<8>(p.gather, p.grid); return true;
                case 4: run_gather_w<4>(p.gather, p.grid); return true;
                case 2: run_gather_w<2>(p.gather, p.grid); return true;
                default: run_gather_w<1>(p.gather, p.grid); return true;
            }
    }
    return false;
}

int main(int argc, char** argv) {
    if (argc < 2) { std::fprintf(stderr, "usage: rr_emu manifest\n"); return 2; }
    std::ifstream mf(argv[1]);
    std::string line;
    while (std::getline(mf, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string op;
        is >> op;
        TileOptions opt;
        Plan plan;
        std::string why;
        if (op == "permute") {
            int ndim; is >> ndim;
            std::vector<int64_t> dims(ndim);
            std::vector<int> perm(ndim);
            for (auto& d : dims) is >> d;
            for (auto& q : perm) is >> q;
            int esize, soff, doff, order; std::string inf, outf;
            is >> esize >> soff >> doff >> opt.in_row_bytes >> opt.out_row_bytes >> order >> opt.max_g >>
                opt.force_ragged >> opt.xcd >> opt.umt >> opt.diag >> opt.fill >> opt.weave >> inf >> outf;
            opt.order_out = order;
            Canon c;
            rr_status st = canonicalize(ndim, dims.data(), perm.data(), esize, &c, &why);
            if (st != RR_OK) { std::printf("err %d %s\n", (int)st, why.c_str()); continue; }
            std::vector<uint8_t> in = read_file(inf);
            const size_t nb = (size_t)c.total_bytes;
            // 16-byte-aligned bases, as GPU allocations are (at least)
            uint8_t* sbuf = static_cast<uint8_t*>(::operator new[](soff + nb + 1, std::align_val_t{16}));
            uint8_t* dbuf = static_cast<uint8_t*>(::operator new[](doff + nb + 1, std::align_val_t{16}));
            // exact-size views: the +1 keeps zero-byte buffers valid; nothing may touch it
            if (nb) std::memcpy(sbuf + soff, in.data(), nb);
            std::memset(dbuf, 0x5A, doff + nb + 1);
            st = plan_permute((uint64_t)(dbuf + doff), (uint64_t)(sbuf + soff), c, opt, &plan, &why);
            auto release = [&] {
                ::operator delete[](sbuf, std::align_val_t{16});
                ::operator delete[](dbuf, std::align_val_t{16});
            };
            if (st != RR_OK) { std::printf("err %d %s\n", (int)st, why.c_str()); release(); continue; }
            if (!emulate(plan)) { std::printf("err -1 no kernel for plan\n"); release(); continue; }
            if (dbuf[doff + nb] != 0x5A) { std::printf("err -2 wrote past the end\n"); return 3; }
            for (int i = 0; i < doff; ++i) if (dbuf[i] != 0x5A) { std::printf("err -2 wrote before the start\n"); return 3; }
            write_file(outf, dbuf + doff, nb);
            std::printf("ok %s\n", describe(plan).c_str());
            release();
        } else if (op == "stencil") {
            // stencil rows cols radius shape nweights w... infile outfile  (float grids)
            int64_t rows, cols; int radius, shape, nw; std::string inf, outf;
            is >> rows >> cols >> radius >> shape >> nw;
            StencilArgs a;
            std::memset(&a, 0, sizeof a);
            for (int k = 0; k < nw; ++k) is >> a.w[k];
            is >> inf >> outf;
            std::vector<uint8_t> in = read_file(inf);
            const size_t nb = (size_t)(rows * cols * 4);
            uint32_t* sbuf = new uint32_t[nb / 4 + 1];
            uint32_t* dbuf = new uint32_t[nb / 4 + 1];
            if (nb) std::memcpy(sbuf, in.data(), nb);
            std::memset(dbuf, 0x5A, nb + 4);
            a.src = (uint64_t)sbuf; a.dst = (uint64_t)dbuf; a.rows = rows; a.cols = cols;
            a.radius = radius; a.shape = shape;
            a.tiles_x = (uint32_t)((cols + ST_TW - 1) / ST_TW);
            // both tile heights, whichever the grid size picks: the results must agree
            std::vector<uint8_t> first;
            for (int th : {16, 32}) {
                a.th = th;
                a.ntiles = (uint32_t)(a.tiles_x * ((rows + th - 1) / th));
                std::memset(dbuf, 0x5A, nb + 4);
                if (nb && !run_stencil(a)) { std::printf("err -1 no kernel\n"); return 3; }
                if (reinterpret_cast<uint8_t*>(dbuf)[nb] != 0x5A) { std::printf("err -2 wrote past the end\n"); return 3; }
                if (th == 16) first.assign(reinterpret_cast<uint8_t*>(dbuf), reinterpret_cast<uint8_t*>(dbuf) + nb);
                else if (nb && std::memcmp(first.data(), dbuf, nb) != 0) { std::printf("err -3 tile heights differ\n"); return 3; }
            }
            write_file(outf, reinterpret_cast<uint8_t*>(dbuf), nb);
            std::printf("ok stencil tiles=%u\n", a.ntiles);
            delete[] sbuf;
            delete[] dbuf;
        } else if (op == "gather") {
            // gather src_count count esize indexed start stride src_off dst_off infile idxfile outfile
            int64_t src_count, count, start, stride; int esize, indexed, soff, doff; std::string inf, idxf, outf;
            is >> src_count >> count >> esize >> indexed >> start >> stride >> soff >> doff >> inf >> idxf >> outf;
            std::vector<uint8_t> in = read_file(inf);
            std::vector<uint8_t> ix = indexed ? read_file(idxf) : std::vector<uint8_t>();
            const size_t nb = (size_t)(count * esize);
            uint8_t* sbuf = new uint8_t[soff + in.size() + 1];
            uint8_t* dbuf = new uint8_t[doff + nb + 1];
            uint8_t* ibuf = new uint8_t[ix.size() + 1];
            if (!in.empty()) std::memcpy(sbuf + soff, in.data(), in.size());
            if (!ix.empty()) std::memcpy(ibuf, ix.data(), ix.size());
            std::memset(dbuf, 0x5A, doff + nb + 1);
            plan_gather((uint64_t)(dbuf + doff), (uint64_t)(sbuf + soff), indexed ? (uint64_t)ibuf : 0, 0, count,
                        src_count, start, stride, esize, &plan);
            g_bad = 0;
            if (count > 0 && !emulate(plan)) { std::printf("err -1 no kernel for plan\n"); return 3; }
            if (dbuf[doff + nb] != 0x5A) { std::printf("err -2 wrote past the end\n"); return 3; }
            for (int i = 0; i < doff; ++i) if (dbuf[i] != 0x5A) { std::printf("err -2 wrote before the start\n"); return 3; }
            write_file(outf, dbuf + doff, nb);
            std::printf("ok %s bad=%llu\n", describe(plan).c_str(), (unsigned long long)g_bad);
            delete[] sbuf;
            delete[] dbuf;
            delete[] ibuf;
        } else if (op == "reorder") {
            int ndim; is >> ndim;
            std::vector<int64_t> dims(ndim), base(ndim), range(ndim);
            for (auto& d : dims) is >> d;
            for (auto& d : base) is >> d;
            for (auto& d : range) is >> d;
            int m; is >> m;
            std::vector<int> order(std::max(m, 1));
            for (int j = 0; j < m; ++j) is >> order[j];
            int esize, soff, doff; std::string inf, outf;
            is >> esize >> soff >> doff >> opt.umt >> opt.max_g >> inf >> outf;
            Canon c;
            uint64_t off = 0, span = 0;
            rr_status st = canonicalize_view(ndim, dims.data(), base.data(), range.data(), m, order.data(), esize, &c,
                                             &off, &span, &why);
            if (st != RR_OK) { std::printf("err %d %s\n", (int)st, why.c_str()); continue; }
            std::vector<uint8_t> in = read_file(inf);
            const size_t ni = in.size();
            const size_t nb = (size_t)c.total_bytes;
            uint8_t* sbuf = new uint8_t[soff + ni + 1];
            uint8_t* dbuf = new uint8_t[doff + nb + 1];
            if (ni) std::memcpy(sbuf + soff, in.data(), ni);
            std::memset(dbuf, 0x5A, doff + nb + 1);
            if (nb && off + span > ni) { std::printf("err -3 box outside the input\n"); return 3; }
            st = plan_permute((uint64_t)(dbuf + doff), (uint64_t)(sbuf + soff) + off, c, opt, &plan, &why);
            auto release = [&] {
                ::operator delete[](sbuf, std::align_val_t{16});
                ::operator delete[](dbuf, std::align_val_t{16});
            };
            if (st != RR_OK) { std::printf("err %d %s\n", (int)st, why.c_str()); release(); continue; }
            if (!emulate(plan)) { std::printf("err -1 no kernel for plan\n"); release(); continue; }
            if (dbuf[doff + nb] != 0x5A) { std::printf("err -2 wrote past the end\n"); return 3; }
            for (int i = 0; i < doff; ++i) if (dbuf[i] != 0x5A) { std::printf("err -2 wrote before the start\n"); return 3; }
            write_file(outf, dbuf + doff, nb);
            std::printf("ok %s\n", describe(plan).c_str());
            delete[] sbuf;
            delete[] dbuf;
        } else if (op == "interlace" || op == "deinterlace") {
            const bool de = op == "deinterlace";
            int n, esize, off; int64_t count; std::string inf, outf;
            is >> n >> count >> esize >> off >> opt.in_row_bytes >> opt.out_row_bytes >> opt.weave >> inf >> outf;
            std::vector<uint8_t> in = read_file(inf);
            const size_t pb = (size_t)count * esize;
            const std::align_val_t A64{64};
            std::vector<uint8_t*> planes(n);
            for (int c = 0; c < n; ++c) {
                planes[c] = static_cast<uint8_t*>(::operator new[](off + pb + 1, A64));
                std::memset(planes[c], 0x5A, off + pb + 1);
            }
            uint8_t* flat = static_cast<uint8_t*>(::operator new[](off + pb * n + 1, A64));
            std::memset(flat, 0x5A, off + pb * n + 1);
            if (!de) {
                for (int c = 0; c < n; ++c) std::memcpy(planes[c] + off, in.data() + c * pb, pb);
            } else {
                std::memcpy(flat + off, in.data(), pb * n);
            }
            std::vector<uint64_t> pl(n);
            for (int c = 0; c < n; ++c) pl[c] = (uint64_t)(planes[c] + off);
            rr_status st = plan_interlace((uint64_t)(flat + off), pl.data(), n, count, esize, de, opt, &plan, &why);
            if (st != RR_OK) { std::printf("err %d %s\n", (int)st, why.c_str()); continue; }
            if (!emulate(plan)) { std::printf("err -1 no kernel for plan\n"); continue; }
            if (!de) {
                write_file(outf, flat + off, pb * n);
            } else {
                std::ofstream f(outf, std::ios::binary);
                for (int c = 0; c < n; ++c) f.write(reinterpret_cast<const char*>(planes[c] + off), (std::streamsize)pb);
            }
            // nothing written before or after any output buffer
            bool clean = true;
            for (int c = 0; c < n && de; ++c)
                for (size_t i = 0; i < (size_t)off; ++i) clean = clean && planes[c][i] == 0x5A;
            for (int c = 0; c < n && de; ++c) clean = clean && planes[c][off + pb] == 0x5A;
            for (size_t i = 0; i < (size_t)off && !de; ++i) clean = clean && flat[i] == 0x5A;
            if (!de) clean = clean && flat[off + pb * n] == 0x5A;
            if (!clean) std::printf("err -2 wrote outside the output\n");
            else std::printf("ok %s\n", describe(plan).c_str());
            for (int c = 0; c < n; ++c) ::operator delete[](planes[c], A64);
            ::operator delete[](flat, A64);
        } else if (op == "batched") {
            // batched k in_rb out_rb order chunk max_g ragged umt : then k lines
            //   "job ndim dims.. perm.. esize infile outfile"
            int k, order, chunk = 0;
            is >> k >> opt.in_row_bytes >> opt.out_row_bytes >> order >> chunk >> opt.max_g >> opt.force_ragged >>
                opt.umt;
            opt.order_out = order;
            std::vector<rr_job> jobs((size_t)k);
            std::vector<uint8_t*> bufs;
            std::vector<std::string> outs((size_t)k);
            std::vector<size_t> sizes((size_t)k);
            for (int i = 0; i < k; ++i) {
                std::string jl;
                std::getline(mf, jl);
                std::istringstream js(jl);
                std::string tag;
                js >> tag;
                rr_job& j = jobs[(size_t)i];
                std::memset(&j, 0, sizeof j);
                js >> j.ndim;
                int64_t n = 1;
                for (int d = 0; d < j.ndim; ++d) { js >> j.dims[d]; n *= j.dims[d]; }
                for (int d = 0; d < j.ndim; ++d) js >> j.perm[d];
                std::string inf;
                js >> j.elem_size >> inf >> outs[(size_t)i];
                const size_t nb = (size_t)n * (size_t)j.elem_size;
                sizes[(size_t)i] = nb;
                std::vector<uint8_t> in = read_file(inf);
                uint8_t* sb = new uint8_t[nb + 1];
                uint8_t* db = new uint8_t[nb + 1];
                if (nb) std::memcpy(sb, in.data(), nb);
                std::memset(db, 0x5A, nb + 1);
                bufs.push_back(sb);
                bufs.push_back(db);
                j.src = sb;
                j.dst = db;
            }
            BatchPlan bp;
            int bad = -1;
            rr_status st = RR_OK;
            std::vector<Plan> plans((size_t)k);
            if (chunk > 0) {
                // every job cut into ranges of `chunk` workgroups, ranges of all jobs interleaved
                std::vector<BatchEntry> entries;
                for (int i = 0; i < k && st == RR_OK; ++i) {
                    st = plan_job(jobs[(size_t)i], opt, &plans[(size_t)i], &why);
                    if (st != RR_OK) bad = i;
                }
                for (uint32_t round = 0; st == RR_OK; ++round) {
                    bool any = false;
                    for (int i = 0; i < k; ++i) {
                        const Plan& p = plans[(size_t)i];
                        const uint64_t first = (uint64_t)round * (uint64_t)chunk;
                        if (p.kind == K_EMPTY || first >= p.grid) continue;
                        const uint32_t n = (uint32_t)std::min<uint64_t>((uint64_t)chunk, p.grid - first);
                        entries.push_back({&p, (uint32_t)first, n, 0});
                        any = true;
                    }
                    if (!any) break;
                }
                if (st == RR_OK) st = build_batch(entries, &bp, &why);
            } else {
                st = plan_batch(jobs.data(), k, opt, &bp, &why, &bad);
            }
            // chunk < 0: -chunk host threads plan the same batch at once, 6 times
            // each, while the library's planning workers are shared among them;
            // every plan must equal the one above byte for byte
            int differ = 0;
            if (st == RR_OK && chunk < 0) {
                std::atomic<int> diffs{0};
                std::vector<std::thread> th;
                for (int t = 0; t < -chunk; ++t)
                    th.emplace_back([&] {
                        for (int r = 0; r < 6; ++r) {
                            BatchPlan q;
                            std::string w;
                            int b2 = -1;
                            if (plan_batch(jobs.data(), k, opt, &q, &w, &b2) != RR_OK || q.table != bp.table ||
                                q.groups.size() != bp.groups.size())
                                ++diffs;
                        }
                    });
                for (std::thread& x : th) x.join();
                differ = diffs.load();
            }
            if (st != RR_OK) {
                std::printf("err %d job %d %s\n", (int)st, bad, why.c_str());
            } else if (differ) {
                std::printf("err -3 %d concurrent plans differ\n", differ);
            } else {
                bool ok = true;
                for (const BatchGroup& g : bp.groups) ok = ok && emulate_group(g, bp.table.data());
                for (int i = 0; i < k; ++i) {
                    uint8_t* db = (uint8_t*)jobs[(size_t)i].dst;
                    if (db[sizes[(size_t)i]] != 0x5A) { std::printf("err -2 wrote past the end\n"); return 3; }
                    write_file(outs[(size_t)i], db, sizes[(size_t)i]);
                }
                std::string variants;
                for (const BatchGroup& g : bp.groups)
                    variants += (variants.empty() ? "" : ",") + std::to_string(g.kind) + ":" + std::to_string(g.variant);
                std::printf(ok ? "ok groups=%zu jobs=%u bytes=%llu variants=%s\n" : "err -1 no kernel\n",
                            bp.groups.size(), bp.njobs, (unsigned long long)bp.bytes, variants.c_str());
            }
            for (uint8_t* q : bufs) delete[] q;
        } else {
            std::printf("err -1 unknown op %s\n", op.c_str());
        }
        std::fflush(stdout);
    }
    return 0;
}
