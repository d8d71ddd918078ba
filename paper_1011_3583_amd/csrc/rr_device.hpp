// rr_device.hpp -- per-thread bodies of the rearrangement kernels.
//
// Everything here is plain C++ that compiles both for gfx950 (inside the
// __global__ kernels of rr_kernels.hip) and for the host, where a CPU build runs
// the very same index arithmetic thread by thread under AddressSanitizer to
// prove every global and LDS access in bounds before a kernel ever reaches the
// GPU.  The only device-specific code is the vector load/store, which issues a
// single 16/8/4/2/1-byte access on the GPU and a memcpy on the host.
#pragma once

#include <cstdint>
#include <cstring>

#include "rr_batch.hpp"
#include "rr_plan.hpp"

#if defined(__HIPCC__)
#define RR_HD __host__ __device__ __forceinline__
#else
#define RR_HD inline
#endif

namespace rr {

RR_HD uint32_t mdiv(uint32_t x, Magic m) {
    const uint32_t hi = (uint32_t)(((uint64_t)x * m.mul) >> 32);
    return (uint32_t)(((uint64_t)hi + x) >> m.shift);
}

RR_HD uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

template <int W>
struct NWords { static constexpr int value = (W + 3) / 4; };

#if defined(__HIP_DEVICE_COMPILE__)
typedef uint32_t rr_u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t rr_u32x2 __attribute__((ext_vector_type(2)));
#endif

// ----------------------------------------------------------------- vector I/O
// Global memory is streamed: every byte is read once and written once, so both
// sides use non-temporal accesses (they keep the streams from displacing each
// other in L2 and the Infinity Cache).  LDS accesses are ordinary.
#ifndef RR_RB_U1
#define RR_RB_U1 16
#endif
#ifndef RR_RB_U2
#define RR_RB_U2 8
#endif
#ifndef RR_RB_U4
#define RR_RB_U4 4
#endif
#ifndef RR_NT_LOAD
#define RR_NT_LOAD 1
#endif
#ifndef RR_NT_STORE
#define RR_NT_STORE 1
#endif

template <int W, bool NT_ACCESS>
RR_HD void vload_t(const uint8_t* p, uint32_t (&w)[NWords<W>::value]) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (W == 16) {
        const rr_u32x4* q = reinterpret_cast<const rr_u32x4*>(p);
        rr_u32x4 v = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else if constexpr (W == 8) {
        const rr_u32x2* q = reinterpret_cast<const rr_u32x2*>(p);
        rr_u32x2 v = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
        w[0] = v.x; w[1] = v.y;
    } else if constexpr (W == 4) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
        w[0] = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
    } else if constexpr (W == 2) {
        const uint16_t* q = reinterpret_cast<const uint16_t*>(p);
        w[0] = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
    } else {
        w[0] = NT_ACCESS ? __builtin_nontemporal_load(p) : *p;
    }
#else
    uint8_t tmp[4 * NWords<W>::value] = {};
    std::memcpy(tmp, p, W);
    std::memcpy(w, tmp, sizeof tmp);
#endif
}

template <int W, bool NT_ACCESS>
RR_HD void vstore_t(uint8_t* p, const uint32_t (&w)[NWords<W>::value]) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (W == 16) {
        rr_u32x4 v; v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
        rr_u32x4* q = reinterpret_cast<rr_u32x4*>(p);
        if (NT_ACCESS) __builtin_nontemporal_store(v, q); else *q = v;
    } else if constexpr (W == 8) {
        rr_u32x2 v; v.x = w[0]; v.y = w[1];
        rr_u32x2* q = reinterpret_cast<rr_u32x2*>(p);
        if (NT_ACCESS) __builtin_nontemporal_store(v, q); else *q = v;
    } else if constexpr (W == 4) {
        uint32_t* q = reinterpret_cast<uint32_t*>(p);
        if (NT_ACCESS) __builtin_nontemporal_store(w[0], q); else *q = w[0];
    } else if constexpr (W == 2) {
        uint16_t* q = reinterpret_cast<uint16_t*>(p);
        if (NT_ACCESS) __builtin_nontemporal_store((uint16_t)w[0], q); else *q = (uint16_t)w[0];
    } else {
        if (NT_ACCESS) __builtin_nontemporal_store((uint8_t)w[0], p); else *p = (uint8_t)w[0];
    }
#else
    std::memcpy(p, w, W);
#endif
}

// global memory (streamed) and LDS (ordinary)
template <int W>
RR_HD void gload(const uint8_t* p, uint32_t (&w)[NWords<W>::value]) { vload_t<W, RR_NT_LOAD != 0>(p, w); }
template <int W>
RR_HD void gstore(uint8_t* p, const uint32_t (&w)[NWords<W>::value]) { vstore_t<W, RR_NT_STORE != 0>(p, w); }
template <int W>
RR_HD void sload(const uint8_t* p, uint32_t (&w)[NWords<W>::value]) { vload_t<W, false>(p, w); }
template <int W>
RR_HD void sstore(uint8_t* p, const uint32_t (&w)[NWords<W>::value]) { vstore_t<W, false>(p, w); }

// GxG transpose of U-byte elements held as G rows of W = U*G bytes:
//   out[i] element j  =  in[j] element i.
template <int U, int G>
RR_HD void xpose(const uint32_t (&r)[G][NWords<U * G>::value], uint32_t (&o)[G][NWords<U * G>::value]) {
    constexpr int W = U * G;
    if constexpr (U >= 4) {
        constexpr int EW = U / 4;
#pragma unroll
        for (int i = 0; i < G; ++i)
#pragma unroll
            for (int j = 0; j < G; ++j)
#pragma unroll
                for (int q = 0; q < EW; ++q) o[i][j * EW + q] = r[j][i * EW + q];
    } else {
        constexpr int EPW = (W >= 4 ? 4 : W) / U;  // elements per output word
        constexpr int NWO = NWords<W>::value;
        constexpr uint32_t MASK = U == 1 ? 0xffu : 0xffffu;
#pragma unroll
        for (int i = 0; i < G; ++i)
#pragma unroll
            for (int q = 0; q < NWO; ++q) {
                uint32_t acc = 0;
#pragma unroll
                for (int b = 0; b < EPW; ++b) {
                    const int j = q * EPW + b;
                    const uint32_t e = (r[j][(i * U) / 4] >> (8 * ((i * U) % 4))) & MASK;
                    acc |= e << (8 * U * b);
                }
                o[i][q] = acc;
            }
    }
}

// ----------------------------------------------------------------- copy
// One thread's share of a grid-stride streaming copy (4 vectors in flight).
template <int W>
RR_HD void copy_thread(const CopyArgs& a, uint32_t block, uint32_t nblocks, uint32_t tid) {
    constexpr int NW = NWords<W>::value;
    const uint8_t* s = reinterpret_cast<const uint8_t*>(a.src) + a.head;
    uint8_t* d = reinterpret_cast<uint8_t*>(a.dst) + a.head;
    const uint64_t stride = (uint64_t)nblocks * NT * 4;
    for (uint64_t i = (uint64_t)block * NT * 4 + tid; i < a.nvec; i += stride) {
        uint32_t w[4][NW];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t v = i + (uint64_t)u * NT;
            if (v < a.nvec) gload<W>(s + v * W, w[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t v = i + (uint64_t)u * NT;
            if (v < a.nvec) gstore<W>(d + v * W, w[u]);
        }
    }
    if (block == 0) {
        const uint8_t* s0 = reinterpret_cast<const uint8_t*>(a.src);
        uint8_t* d0 = reinterpret_cast<uint8_t*>(a.dst);
        if (tid < a.head) d0[tid] = s0[tid];
        if (tid < a.tail) {
            const uint64_t off = a.head + a.nvec * W + tid;
            d0[off] = s0[off];
        }
    }
}

// ----------------------------------------------------------------- run copy
// Output is written contiguously; each W-byte vector is read from the input run
// its output run maps to.
template <int W>
RR_HD void run_thread(const RunArgs& a, uint32_t block, uint32_t tid) {
    constexpr int NW = NWords<W>::value;
    const uint8_t* src = reinterpret_cast<const uint8_t*>(a.src);
    uint8_t* dst = reinterpret_cast<uint8_t*>(a.dst);
    const uint32_t base = block * (uint32_t)(NT * 4) + tid;
    uint32_t w[4][NW];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t v = base + u * NT;
        if (v < a.nvec) {
            const uint32_t run = mdiv(v, a.mvpr);
            const uint32_t part = v - run * a.vpr;
            uint64_t off = 0;
            uint32_t rem = run;
#pragma unroll
            for (int j = MAXR - 1; j >= 1; --j) {
                if (j < a.nax) {
                    const uint32_t q = mdiv(rem, a.om[j]);
                    off += (uint64_t)(rem - q * a.on[j]) * a.sin[j];
                    rem = q;
                }
            }
            off += (uint64_t)rem * a.sin[0];
            gload<W>(src + off + (uint64_t)part * W, w[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t v = base + u * NT;
        if (v < a.nvec) gstore<W>(dst + (uint64_t)v * W, w[u]);
    }
}

// ----------------------------------------------------------------- tiles
struct TileCtx {
    uint64_t bin, bout;   // byte bases of the tile (absolute unless in table mode)
    uint32_t TAv, TBv;    // valid row length / row count of this tile
};

RR_HD TileCtx tile_decode(const TileArgs& a, uint32_t tile) {
    TileCtx t;
    t.bin = a.src;
    t.bout = a.dst;
    t.TAv = a.TA;
    t.TBv = a.TB;
    uint32_t rem = tile;
#pragma unroll
    for (int g = MAXR - 1; g >= 0; --g) {
        if (g < a.ngrid) {
            const uint32_t q = mdiv(rem, a.gm[g]);
            const uint32_t c = rem - q * a.gn[g];
            rem = q;
            t.bin += (uint64_t)c * a.gsin[g];
            t.bout += (uint64_t)c * a.gsout[g];
            if (g == a.grid_aO) t.TAv = a.TAinner * umin(a.aO_t, a.aO_len - c * a.aO_t);
            if (g == a.grid_bO) t.TBv = a.TBinner * umin(a.bO_t, a.bO_len - c * a.bO_t);
        }
    }
    return t;
}

RR_HD uint64_t row_in(const TileArgs& a, uint32_t ib) {
    if (a.flags & TF_IN_TABLE) return a.table[ib];
    if (a.nB == 1) return (uint64_t)ib * a.sinB[0];
    uint64_t off = 0;
    uint32_t rem = ib;
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        if (i < a.nB) {
            if (i == a.nB - 1) {
                off += (uint64_t)rem * a.sinB[i];
            } else {
                const uint32_t q = mdiv(rem, a.mB[i]);
                off += (uint64_t)(rem - q * a.tB[i]) * a.sinB[i];
                rem = q;
            }
        }
    }
    return off;
}

RR_HD uint64_t row_out(const TileArgs& a, uint32_t ia) {
    if (a.flags & TF_OUT_TABLE) return a.table[ia];
    if (a.nA == 1) return (uint64_t)ia * a.soutA[0];
    uint64_t off = 0;
    uint32_t rem = ia;
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        if (i < a.nA) {
            if (i == a.nA - 1) {
                off += (uint64_t)rem * a.soutA[i];
            } else {
                const uint32_t q = mdiv(rem, a.mA[i]);
                off += (uint64_t)(rem - q * a.tA[i]) * a.soutA[i];
                rem = q;
            }
        }
    }
    return off;
}

// LDS byte address of (row ib, byte x): the 16-byte chunks of a row are rotated
// by (ib / G) so that the G-row column reads of the write phase, made by lanes
// on consecutive row groups, fall on different banks.
template <int G>
RR_HD uint32_t lds_pos(const TileArgs& a, uint32_t ib, uint32_t x) {
    const uint32_t rot = (ib / G) & a.rotmask;
    uint32_t cc = (x >> 4) + rot;
    if (cc >= a.nch16) cc -= a.nch16;
    return ib * a.pitch + (cc << 4) + (x & 15u);
}

// Loads each thread keeps in flight before writing any of them to LDS.  Tiles
// are planned to need 16/U loads per thread for U = 1, 2 (64 and 32 KiB tiles,
// where LDS already limits occupancy) and 4 for U >= 4 (16 KiB tiles, where the
// register budget decides how many waves fit).
template <int U>
struct ReadBatch { static constexpr int value = U == 1 ? RR_RB_U1 : (U == 2 ? RR_RB_U2 : RR_RB_U4); };

// Read phase: rows of the tile (contiguous along the input's fastest axes) are
// loaded with WIN-byte vectors and parked in LDS.
template <int WIN, int G, int B>
RR_HD void read_phase(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    constexpr int NWI = NWords<WIN>::value;
    const uint32_t total = a.TB * a.rch;
    const uint32_t rowvalid = t.TAv * a.R;
    for (uint32_t base = 0; base < total; base += NT * B) {
        uint32_t w[B][NWI];
        uint32_t lo[B];
        bool ok[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t f = base + u * NT + tid;
            const uint32_t ib = mdiv(f, a.mrch);
            const uint32_t x = (f - ib * a.rch) * WIN;
            ok[u] = f < total && ib < t.TBv && x < rowvalid;
            lo[u] = 0;
            if (ok[u]) {
                const uint8_t* p = reinterpret_cast<const uint8_t*>(t.bin + row_in(a, ib) + x);
                gload<WIN>(p, w[u]);
                lo[u] = lds_pos<G>(a, ib, x);
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (ok[u]) sstore<WIN>(lds + lo[u], w[u]);
    }
}

// Flat read: the tile's input rows are back to back in memory (a contiguous
// byte range), and LDS holds them unpadded, so the whole range moves with
// 16-byte vectors however short or oddly sized a row is (de-interlace).
template <int B>
RR_HD void read_flat(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    const uint32_t nbytes = t.TBv * a.pitch;
    const uint32_t nvec = nbytes / a.win;
    for (uint32_t base = 0; base < nvec; base += NT * B) {
        uint32_t w[B][4];
        bool ok[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t v = base + u * NT + tid;
            ok[u] = v < nvec;
            if (ok[u]) gload<16>(reinterpret_cast<const uint8_t*>(t.bin) + (uint64_t)v * 16, w[u]);
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (ok[u]) sstore<16>(lds + (base + u * NT + tid) * 16, w[u]);
    }
}

template <int U, int G>
RR_HD void read_dispatch(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    constexpr int B = ReadBatch<U>::value;
    if (a.flags & TF_IN_FLAT) { read_flat<4>(a, t, lds, tid); return; }
    switch (a.win) {
        case 16: read_phase<16, G, B>(a, t, lds, tid); break;
        case 8: read_phase<8, G, B>(a, t, lds, tid); break;
        case 4: read_phase<4, G, 4>(a, t, lds, tid); break;
        case 2: read_phase<2, G, 4>(a, t, lds, tid); break;
        default: read_phase<1, G, 4>(a, t, lds, tid); break;
    }
}

// Write phase: each work item is a GxG micro-tile (G rows of the LDS tile, G
// elements each), transposed in registers into G output vectors that lie along
// the output's fastest axis.  Elements of k > 1 units go one unit at a time.
template <int U, int G>
RR_HD void write_phase(const TileArgs& a, const TileCtx& t, const uint8_t* lds, uint32_t tid) {
    constexpr int W = U * G;
    constexpr int NW = NWords<W>::value;
    if (G > 1 || a.k == 1) {
        for (uint32_t gi = tid; gi < a.nwork; gi += NT) {
            const uint32_t ma = mdiv(gi, a.mnmb);
            const uint32_t mb = gi - ma * a.nmb;
            const uint32_t ia0 = ma * G, ib0 = mb * G;
            if (ia0 < t.TAv && ib0 < t.TBv) {
                uint32_t r[G][NW];
#pragma unroll
                for (int j = 0; j < G; ++j) sload<W>(lds + lds_pos<G>(a, ib0 + j, ia0 * U), r[j]);
                uint32_t o[G][NW];
                xpose<U, G>(r, o);
                if (a.flags & TF_OUT_TABLE) {
#pragma unroll
                    for (int i = 0; i < G; ++i)
                        gstore<W>(reinterpret_cast<uint8_t*>(a.table[ia0 + i] + t.bout + (uint64_t)ib0 * U), o[i]);
                } else if (W >= 4 && W * G >= 16 && (a.flags & TF_OUT_MERGE)) {
                    // the G output rows are back to back: store them as 16-byte vectors
                    constexpr int NV = (W * G >= 16) ? W * G / 16 : 1;
                    constexpr int PER = W >= 4 ? W / 4 : 1;
                    uint8_t* q = reinterpret_cast<uint8_t*>(t.bout + row_out(a, ia0));
                    uint32_t flat[NV * 4];
#pragma unroll
                    for (int i = 0; i < G; ++i)
#pragma unroll
                        for (int c = 0; c < PER; ++c)
                            if (i * PER + c < NV * 4) flat[i * PER + c] = o[i][c];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const uint32_t(&fv)[4] = *reinterpret_cast<const uint32_t(*)[4]>(&flat[v * 4]);
                        gstore<16>(q + v * 16, fv);
                    }
                } else {
                    uint8_t* q = reinterpret_cast<uint8_t*>(t.bout + row_out(a, ia0) + (uint64_t)ib0 * U);
#pragma unroll
                    for (int i = 0; i < G; ++i) gstore<W>(q + (uint64_t)i * a.soutA[0], o[i]);
                }
            }
        }
    } else {
        for (uint32_t gi = tid; gi < a.nwork; gi += NT) {
            const uint32_t ia = mdiv(gi, a.mnmb);
            const uint32_t m = gi - ia * a.nmb;
            const uint32_t ib = mdiv(m, a.mk);
            const uint32_t s = m - ib * a.k;
            if (ia < t.TAv && ib < t.TBv) {
                uint32_t v[NWords<U>::value];
                sload<U>(lds + lds_pos<1>(a, ib, (ia * a.k + s) * U), v);
                gstore<U>(reinterpret_cast<uint8_t*>(t.bout + row_out(a, ia) + (uint64_t)m * U), v);
            }
        }
    }
}

// ----------------------------------------------------------------- batches
// Job of workgroup b in a batch group: the largest j with prefix[j] <= b
// (prefix holds njobs+1 exclusive sums of the jobs' workgroup counts).
RR_HD uint32_t find_job(const uint32_t* prefix, uint32_t njobs, uint32_t b) {
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

template <int W>
RR_HD void batch_copy_block(const CopyArgs* args, const uint32_t* prefix, const EntryRange* ranges,
                            uint32_t njobs, uint32_t b, uint32_t tid) {
    const uint32_t j = find_job(prefix, njobs, b);
    copy_thread<W>(args[j], b - prefix[j] + ranges[j].first, ranges[j].job_blocks, tid);
}

template <int W>
RR_HD void batch_run_block(const RunArgs* args, const uint32_t* prefix, const EntryRange* ranges,
                           uint32_t njobs, uint32_t b, uint32_t tid) {
    const uint32_t j = find_job(prefix, njobs, b);
    run_thread<W>(args[j], b - prefix[j] + ranges[j].first, tid);
}

}  // namespace rr
