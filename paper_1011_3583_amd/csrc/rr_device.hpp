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
template <int W>
RR_HD void vload(const uint8_t* p, uint32_t (&w)[NWords<W>::value]) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (W == 16) {
        rr_u32x4 v = *reinterpret_cast<const rr_u32x4*>(p);
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else if constexpr (W == 8) {
        rr_u32x2 v = *reinterpret_cast<const rr_u32x2*>(p);
        w[0] = v.x; w[1] = v.y;
    } else if constexpr (W == 4) {
        w[0] = *reinterpret_cast<const uint32_t*>(p);
    } else if constexpr (W == 2) {
        w[0] = *reinterpret_cast<const uint16_t*>(p);
    } else {
        w[0] = *p;
    }
#else
    uint8_t tmp[4 * NWords<W>::value] = {};
    std::memcpy(tmp, p, W);
    std::memcpy(w, tmp, sizeof tmp);
#endif
}

template <int W>
RR_HD void vstore(uint8_t* p, const uint32_t (&w)[NWords<W>::value]) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (W == 16) {
        rr_u32x4 v; v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
        *reinterpret_cast<rr_u32x4*>(p) = v;
    } else if constexpr (W == 8) {
        rr_u32x2 v; v.x = w[0]; v.y = w[1];
        *reinterpret_cast<rr_u32x2*>(p) = v;
    } else if constexpr (W == 4) {
        *reinterpret_cast<uint32_t*>(p) = w[0];
    } else if constexpr (W == 2) {
        *reinterpret_cast<uint16_t*>(p) = (uint16_t)w[0];
    } else {
        *p = (uint8_t)w[0];
    }
#else
    std::memcpy(p, w, W);
#endif
}

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
            if (v < a.nvec) vload<W>(s + v * W, w[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t v = i + (uint64_t)u * NT;
            if (v < a.nvec) vstore<W>(d + v * W, w[u]);
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
            vload<W>(src + off + (uint64_t)part * W, w[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t v = base + u * NT;
        if (v < a.nvec) vstore<W>(dst + (uint64_t)v * W, w[u]);
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

// Read phase: rows of the tile (contiguous along the input's fastest axes) are
// loaded with WIN-byte vectors and parked in LDS.
template <int WIN, int G>
RR_HD void read_phase(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    constexpr int NWI = NWords<WIN>::value;
    constexpr int B = WIN >= 8 ? 8 : 4;
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
                vload<WIN>(p, w[u]);
                lo[u] = lds_pos<G>(a, ib, x);
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (ok[u]) vstore<WIN>(lds + lo[u], w[u]);
    }
}

template <int G>
RR_HD void read_dispatch(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    switch (a.win) {
        case 16: read_phase<16, G>(a, t, lds, tid); break;
        case 8: read_phase<8, G>(a, t, lds, tid); break;
        case 4: read_phase<4, G>(a, t, lds, tid); break;
        case 2: read_phase<2, G>(a, t, lds, tid); break;
        default: read_phase<1, G>(a, t, lds, tid); break;
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
                for (int j = 0; j < G; ++j) vload<W>(lds + lds_pos<G>(a, ib0 + j, ia0 * U), r[j]);
                uint32_t o[G][NW];
                xpose<U, G>(r, o);
                if (a.flags & TF_OUT_TABLE) {
#pragma unroll
                    for (int i = 0; i < G; ++i)
                        vstore<W>(reinterpret_cast<uint8_t*>(a.table[ia0 + i] + t.bout + (uint64_t)ib0 * U), o[i]);
                } else {
                    uint8_t* q = reinterpret_cast<uint8_t*>(t.bout + row_out(a, ia0) + (uint64_t)ib0 * U);
#pragma unroll
                    for (int i = 0; i < G; ++i) vstore<W>(q + (uint64_t)i * a.soutA[0], o[i]);
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
                vload<U>(lds + lds_pos<1>(a, ib, (ia * a.k + s) * U), v);
                vstore<U>(reinterpret_cast<uint8_t*>(t.bout + row_out(a, ia) + (uint64_t)m * U), v);
            }
        }
    }
}

}  // namespace rr
