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
// Global memory is streamed: every byte is read once and written once, so by
// default both sides use non-temporal accesses (they keep the streams from
// displacing each other in L2 and the Infinity Cache).  Tiles whose rows start
// or end inside 128-byte lines share those lines with their neighbours; a plan
// may then read (TF_LD_CACHED) or write (TF_ST_CACHED) through the caches so the
// neighbour finds the line there.  The access helpers take S = streamed.  LDS
// accesses are ordinary.
#ifndef RR_READ_BATCH
#define RR_READ_BATCH 4
#endif
#ifndef RR_NT_LOAD
#define RR_NT_LOAD 1
#endif
#ifndef RR_NT_STORE
#define RR_NT_STORE 1
#endif

// Device pointers here come from integers, so without help the compiler would
// use flat instructions, which also count against the LDS wait counter and make
// every LDS access wait for outstanding global stores.  Global accesses are
// therefore made through address-space-1 pointers (global_load/global_store).
#if defined(__HIP_DEVICE_COMPILE__)
#define RR_AS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const RR_AS_GLOBAL T* as_global(const uint8_t* p) {
    return (const RR_AS_GLOBAL T*)(reinterpret_cast<uintptr_t>(p));
}
template <typename T>
__device__ __forceinline__ RR_AS_GLOBAL T* as_global_mut(uint8_t* p) {
    return (RR_AS_GLOBAL T*)(reinterpret_cast<uintptr_t>(p));
}
#endif

template <int W, bool NT_ACCESS, bool GLOBAL>
RR_HD void vload_t(const uint8_t* p, uint32_t (&w)[NWords<W>::value]) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (GLOBAL) {
        if constexpr (W == 16) {
            const RR_AS_GLOBAL rr_u32x4* q = as_global<rr_u32x4>(p);
            rr_u32x4 v = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else if constexpr (W == 8) {
            const RR_AS_GLOBAL rr_u32x2* q = as_global<rr_u32x2>(p);
            rr_u32x2 v = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
            w[0] = v.x; w[1] = v.y;
        } else if constexpr (W == 4) {
            const RR_AS_GLOBAL uint32_t* q = as_global<uint32_t>(p);
            w[0] = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
        } else if constexpr (W == 2) {
            const RR_AS_GLOBAL uint16_t* q = as_global<uint16_t>(p);
            w[0] = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
        } else {
            const RR_AS_GLOBAL uint8_t* q = as_global<uint8_t>(p);
            w[0] = NT_ACCESS ? __builtin_nontemporal_load(q) : *q;
        }
    } else {
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
    }
#else
    uint8_t tmp[4 * NWords<W>::value] = {};
    std::memcpy(tmp, p, W);
    std::memcpy(w, tmp, sizeof tmp);
#endif
}

template <int W, bool NT_ACCESS, bool GLOBAL>
RR_HD void vstore_t(uint8_t* p, const uint32_t (&w)[NWords<W>::value]) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (GLOBAL) {
        if constexpr (W == 16) {
            rr_u32x4 v; v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
            RR_AS_GLOBAL rr_u32x4* q = as_global_mut<rr_u32x4>(p);
            if (NT_ACCESS) __builtin_nontemporal_store(v, q); else *q = v;
        } else if constexpr (W == 8) {
            rr_u32x2 v; v.x = w[0]; v.y = w[1];
            RR_AS_GLOBAL rr_u32x2* q = as_global_mut<rr_u32x2>(p);
            if (NT_ACCESS) __builtin_nontemporal_store(v, q); else *q = v;
        } else if constexpr (W == 4) {
            RR_AS_GLOBAL uint32_t* q = as_global_mut<uint32_t>(p);
            if (NT_ACCESS) __builtin_nontemporal_store(w[0], q); else *q = w[0];
        } else if constexpr (W == 2) {
            RR_AS_GLOBAL uint16_t* q = as_global_mut<uint16_t>(p);
            if (NT_ACCESS) __builtin_nontemporal_store((uint16_t)w[0], q); else *q = (uint16_t)w[0];
        } else {
            RR_AS_GLOBAL uint8_t* q = as_global_mut<uint8_t>(p);
            if (NT_ACCESS) __builtin_nontemporal_store((uint8_t)w[0], q); else *q = (uint8_t)w[0];
        }
    } else {
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
    }
#else
    std::memcpy(p, w, W);
#endif
}

// 16 bytes at any byte alignment: gfx950 issues one global_load/store_dwordx4
// whatever the address alignment (the memory system runs in unaligned mode).
#if defined(__HIP_DEVICE_COMPILE__)
typedef uint32_t rr_u32x4_u __attribute__((ext_vector_type(4), aligned(1)));
#endif
template <bool S = true>
RR_HD void gload16u(const uint8_t* p, uint32_t (&w)[4]) {
#if defined(__HIP_DEVICE_COMPILE__)
    const RR_AS_GLOBAL rr_u32x4_u* q = as_global<rr_u32x4_u>(p);
    rr_u32x4_u v = (S && RR_NT_LOAD) ? __builtin_nontemporal_load(q) : *q;
    w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
#else
    std::memcpy(w, p, 16);
#endif
}
template <bool S = true>
RR_HD void gstore16u(uint8_t* p, const uint32_t (&w)[4]) {
#if defined(__HIP_DEVICE_COMPILE__)
    rr_u32x4_u v; v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
    RR_AS_GLOBAL rr_u32x4_u* q = as_global_mut<rr_u32x4_u>(p);
    if (S && RR_NT_STORE) __builtin_nontemporal_store(v, q); else *q = v;
#else
    std::memcpy(p, w, 16);
#endif
}

// W bytes (2, 4, 8, 16) at any byte alignment.
#if defined(__HIP_DEVICE_COMPILE__)
typedef uint32_t rr_u32x2_u __attribute__((ext_vector_type(2), aligned(1)));
typedef uint32_t rr_u32_u __attribute__((aligned(1)));
typedef uint16_t rr_u16_u __attribute__((aligned(1)));
#endif
template <int W, bool S = true>
RR_HD void gstore_u(uint8_t* p, const uint32_t (&w)[NWords<W>::value]) {
    if constexpr (W == 16) {
        gstore16u<S>(p, w);
    } else {
#if defined(__HIP_DEVICE_COMPILE__)
        constexpr bool NTS = S && RR_NT_STORE;
        if constexpr (W == 8) {
            rr_u32x2_u v; v.x = w[0]; v.y = w[1];
            RR_AS_GLOBAL rr_u32x2_u* q = as_global_mut<rr_u32x2_u>(p);
            if (NTS) __builtin_nontemporal_store(v, q); else *q = v;
        } else if constexpr (W == 4) {
            RR_AS_GLOBAL rr_u32_u* q = as_global_mut<rr_u32_u>(p);
            if (NTS) __builtin_nontemporal_store((rr_u32_u)w[0], q); else *q = w[0];
        } else if constexpr (W == 2) {
            RR_AS_GLOBAL rr_u16_u* q = as_global_mut<rr_u16_u>(p);
            if (NTS) __builtin_nontemporal_store((rr_u16_u)w[0], q); else *q = (uint16_t)w[0];
        } else {
            vstore_t<1, NTS, true>(p, w);
        }
#else
        std::memcpy(p, w, W);
#endif
    }
}

// global memory (streamed unless S is false) and LDS (ordinary)
template <int W, bool S = true>
RR_HD void gload(const uint8_t* p, uint32_t (&w)[NWords<W>::value]) {
    vload_t<W, S && RR_NT_LOAD != 0, true>(p, w);
}
template <int W, bool S = true>
RR_HD void gstore(uint8_t* p, const uint32_t (&w)[NWords<W>::value]) {
    vstore_t<W, S && RR_NT_STORE != 0, true>(p, w);
}
template <int W>
RR_HD void sload(const uint8_t* p, uint32_t (&w)[NWords<W>::value]) { vload_t<W, false, false>(p, w); }
template <int W>
RR_HD void sstore(uint8_t* p, const uint32_t (&w)[NWords<W>::value]) { vstore_t<W, false, false>(p, w); }

// Byte permute of two words (gfx950 v_perm_b32): the eight bytes hi:lo are
// numbered 0..3 (lo) and 4..7 (hi); byte k of the result is the byte that
// selector byte k names.  Selector bytes here are 0..7, or 12 for a zero byte.
RR_HD uint32_t perm_b32(uint32_t hi, uint32_t lo, uint32_t sel) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_perm(hi, lo, sel);
#else
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    uint32_t out = 0;
    for (int k = 0; k < 4; ++k) {
        const uint32_t s = (sel >> (8 * k)) & 0xffu;
        const uint32_t byte = s < 8 ? (uint32_t)(v >> (8 * s)) & 0xffu : 0u;
        out |= byte << (8 * k);
    }
    return out;
#endif
}

// 4x4 byte transpose of the words a, b, c, d: result word k holds byte k of a,
// b, c and d, in that order.  Two rounds of byte permutes: pairs interleave
// (a0 b0 a1 b1 / a2 b2 a3 b3, likewise c with d), then the pairs combine.
RR_HD void xpose4x4_b8(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t& o0, uint32_t& o1, uint32_t& o2,
                       uint32_t& o3) {
    const uint32_t ab01 = perm_b32(b, a, 0x05010400u), ab23 = perm_b32(b, a, 0x07030602u);
    const uint32_t cd01 = perm_b32(d, c, 0x05010400u), cd23 = perm_b32(d, c, 0x07030602u);
    o0 = perm_b32(cd01, ab01, 0x05040100u);
    o1 = perm_b32(cd01, ab01, 0x07060302u);
    o2 = perm_b32(cd23, ab23, 0x05040100u);
    o3 = perm_b32(cd23, ab23, 0x07060302u);
}

// GxG transpose of U-byte elements held as G rows of W = U*G bytes:
//   out[i] element j  =  in[j] element i.
// 4..16-byte elements are whole words (register renaming); 2-byte elements take
// one byte permute per output word (half i of rows 2q and 2q+1), 1-byte
// elements a 4x4 byte transpose per four output words (eight permutes), so an
// 8x8 byte tile costs 32 permutes instead of masks, shifts and ors per byte.
template <int U, int G>
RR_HD void xpose(const uint32_t (&r)[G][NWords<U * G>::value], uint32_t (&o)[G][NWords<U * G>::value]) {
    if constexpr (U >= 4) {
        constexpr int EW = U / 4;
#pragma unroll
        for (int i = 0; i < G; ++i)
#pragma unroll
            for (int j = 0; j < G; ++j)
#pragma unroll
                for (int q = 0; q < EW; ++q) o[i][j * EW + q] = r[j][i * EW + q];
    } else if constexpr (U == 2) {
        // o[i][q] = { row 2q half i, row 2q+1 half i }; row j's half i sits in
        // word i/2, low half when i is even
        constexpr int NWO = NWords<2 * G>::value;
#pragma unroll
        for (int i = 0; i < G; ++i)
#pragma unroll
            for (int q = 0; q < NWO; ++q) {
                if constexpr (G == 1) {
                    o[i][q] = r[0][0];
                } else {
                    const uint32_t sel = (i & 1) ? 0x07060302u : 0x05040100u;
                    o[i][q] = perm_b32(r[2 * q + 1][i / 2], r[2 * q][i / 2], sel);
                }
            }
    } else if constexpr (G == 1) {
        o[0][0] = r[0][0];
    } else if constexpr (G == 2) {
        // two 2-byte rows: o[i] = { row 0 byte i, row 1 byte i }
        o[0][0] = perm_b32(r[1][0], r[0][0], 0x0c0c0400u);
        o[1][0] = perm_b32(r[1][0], r[0][0], 0x0c0c0501u);
    } else {
        // byte b of o[i][q] is byte i of row 4q+b, i.e. byte i%4 of word i/4 of
        // that row: for each (q, h = i/4) a 4x4 byte transpose of rows 4q..4q+3
        constexpr int NWO = G / 4;
#pragma unroll
        for (int q = 0; q < NWO; ++q)
#pragma unroll
            for (int h = 0; h < NWO; ++h)
                xpose4x4_b8(r[4 * q][h], r[4 * q + 1][h], r[4 * q + 2][h], r[4 * q + 3][h], o[4 * h][q],
                            o[4 * h + 1][q], o[4 * h + 2][q], o[4 * h + 3][q]);
    }
}

// ----------------------------------------------------------------- copy
// One thread's share of a grid-stride streaming copy (copy_vpt(W) vectors in flight).
template <int W>
RR_HD void copy_thread(const CopyArgs& a, uint32_t block, uint32_t nblocks, uint32_t tid) {
    constexpr int NW = NWords<W>::value;
    const uint8_t* s = reinterpret_cast<const uint8_t*>(a.src) + a.head;
    uint8_t* d = reinterpret_cast<uint8_t*>(a.dst) + a.head;
    constexpr int V = copy_vpt(W);
    const uint64_t stride = (uint64_t)nblocks * NT * V;
    for (uint64_t i = (uint64_t)block * NT * V + tid; i < a.nvec; i += stride) {
        uint32_t w[V][NW];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const uint64_t v = i + (uint64_t)u * NT;
            if (v < a.nvec) gload<W>(s + v * W, w[u]);
        }
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const uint64_t v = i + (uint64_t)u * NT;
            if (v < a.nvec) gstore<W>(d + v * W, w[u]);
        }
    }
    if (block == 0) {
        const uint8_t* s0 = reinterpret_cast<const uint8_t*>(a.src);
        uint8_t* d0 = reinterpret_cast<uint8_t*>(a.dst);
        uint32_t b[1];
        if (tid < a.head) {
            gload<1>(s0 + tid, b);
            gstore<1>(d0 + tid, b);
        }
        if (tid < a.tail) {
            const uint64_t off = a.head + a.nvec * W + tid;
            gload<1>(s0 + off, b);
            gstore<1>(d0 + off, b);
        }
    }
}

// ----------------------------------------------------------------- index-set / range read
// One thread's share of an index-set or range read: four elements per thread
// per step (indices first, then their elements, then the stores), grid-stride
// over the output.  Loads are unconditional at clamped in-bounds addresses
// (results masked afterwards) so the four of each kind are in flight together.
// Returns how many indices fell outside the source.
template <int W>
RR_HD uint32_t gather_thread(const GatherArgs& a, uint64_t block, uint64_t nblocks, uint32_t tid) {
    constexpr int NW = NWords<W>::value;
    const uint8_t* src = reinterpret_cast<const uint8_t*>(a.src);
    uint8_t* dst = reinterpret_cast<uint8_t*>(a.dst);
    const uint8_t* idx = reinterpret_cast<const uint8_t*>(a.idx);
    const uint64_t n = (uint64_t)a.count;   // >= 1 when launched
    uint32_t nbad = 0;
    for (uint64_t base = block * NT * 4 + tid; base < n; base += nblocks * NT * 4) {
        int64_t s[4];
        bool ok[4], valid[4];
        uint32_t w[4][2];
        if (a.idx) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t i = base + (uint64_t)u * NT;
                gload<8>(idx + (i < n ? i : n - 1) * 8, w[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t i = base + (uint64_t)u * NT;
            ok[u] = i < n;
            s[u] = a.idx ? (int64_t)(((uint64_t)w[u][1] << 32) | w[u][0]) : a.start + (int64_t)i * a.stride;
            valid[u] = ok[u] && s[u] >= 0 && s[u] < a.src_count;
            nbad += ok[u] && !valid[u];
            if (!valid[u]) s[u] = 0;   // element 0 is read instead and discarded
        }
        const bool any_src = a.src_count > 0;
        if (a.k == 1) {
            uint32_t v[4][NW];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (any_src) gload<W>(src + (uint64_t)s[u] * W, v[u]);
                else
#pragma unroll
                    for (int q = 0; q < NW; ++q) v[u][q] = 0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (!valid[u])
#pragma unroll
                    for (int q = 0; q < NW; ++q) v[u][q] = 0;
                if (ok[u]) gstore<W>(dst + (base + (uint64_t)u * NT) * W, v[u]);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (!ok[u]) continue;
                const uint8_t* ps = src + (uint64_t)s[u] * a.esize;
                uint8_t* pd = dst + (base + (uint64_t)u * NT) * a.esize;
                for (uint32_t q = 0; q < a.k; ++q) {
                    uint32_t v[NW];
#pragma unroll
                    for (int c = 0; c < NW; ++c) v[c] = 0;
                    if (valid[u]) gload<W>(ps + q * W, v);
                    gstore<W>(pd + q * W, v);
                }
            }
        }
    }
    return nbad;
}

// ----------------------------------------------------------------- 2-D stencil
RR_HD float bits_to_float(uint32_t u) { return __builtin_bit_cast(float, u); }
RR_HD uint32_t float_to_bits(float f) { return __builtin_bit_cast(uint32_t, f); }

// Load phase: the tile's rows plus R halo rows above and below, each as
// ST_PITCH floats starting ST_HALO columns left of the tile, into LDS as 16-byte
// vectors (element by element where a vector crosses the grid's edge; points
// outside the grid are zero and never used).
template <int R, int TH>
RR_HD void stencil_load(const StencilArgs& a, uint32_t tile, uint32_t* lds, uint32_t tid) {
    constexpr int LR = TH + 2 * R;
    constexpr int NV = ST_PITCH / 4;
    const int64_t ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int64_t i0 = ty * TH - R, j0 = tx * ST_TW - ST_HALO;
    const uint8_t* src = reinterpret_cast<const uint8_t*>(a.src);
    for (uint32_t v = tid; v < (uint32_t)(LR * NV); v += NT) {
        const int lr = (int)(v / NV), lc = (int)(v - (uint32_t)lr * NV) * 4;
        const int64_t gi = i0 + lr, gj = j0 + lc;
        uint32_t w[4] = {0, 0, 0, 0};
        if (gi >= 0 && gi < a.rows) {
            const uint8_t* row = src + (uint64_t)gi * (uint64_t)a.cols * 4;
            if (gj >= 0 && gj + 4 <= a.cols) {
                gload16u(row + gj * 4, w);
            } else {
                for (int e = 0; e < 4; ++e)
                    if (gj + e >= 0 && gj + e < a.cols) {
                        uint32_t one[1];
                        gload<4>(row + (gj + e) * 4, one);
                        w[e] = one[0];
                    }
            }
        }
        sstore<16>(reinterpret_cast<uint8_t*>(lds + lr * ST_PITCH + lc), w);
    }
}

// Compute phase: thread (cx = tid % 32, ry = tid / 32) produces the four points
// at columns 4cx..4cx+3 of tile rows ry, ry+8, ... (TH / 8 rows).  Every
// LDS read is an aligned 16-byte vector: three for the horizontal window, one
// per vertical neighbour row.  Accumulation is fp32 FMA: center first, then
// ring k = (up + down) + (left + right) for a star, row by row for a box.
template <int R, int SHAPE, int TH>
RR_HD void stencil_compute(const StencilArgs& a, uint32_t tile, const uint32_t* lds, uint32_t tid) {
    constexpr int N = 2 * R + 1;
    const int64_t ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const uint32_t cx = tid % 32, ry = tid / 32;
    const int64_t gj = tx * ST_TW + cx * 4;
    if (gj >= a.cols) return;
    const int lc = ST_HALO + (int)cx * 4;
    uint8_t* dst = reinterpret_cast<uint8_t*>(a.dst);
    for (int s = 0; s < TH / 8; ++s) {
        const int li = (int)ry + s * 8;
        const int64_t gi = ty * TH + li;
        if (gi >= a.rows) break;
        const uint32_t* c = lds + (li + R) * ST_PITCH + lc;   // first output point's center
        float acc[4];
        uint32_t ctr[4];
        sload<16>(reinterpret_cast<const uint8_t*>(c), ctr);
        if constexpr (SHAPE == 0) {
            uint32_t hw[12];   // columns lc-4 .. lc+7 of the center row
            sload<16>(reinterpret_cast<const uint8_t*>(c - 4), *reinterpret_cast<uint32_t(*)[4]>(&hw[0]));
            sload<16>(reinterpret_cast<const uint8_t*>(c + 4), *reinterpret_cast<uint32_t(*)[4]>(&hw[8]));
#pragma unroll
            for (int e = 0; e < 4; ++e) { hw[4 + e] = ctr[e]; acc[e] = a.w[0] * bits_to_float(ctr[e]); }
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                uint32_t up[4], dn[4];
                sload<16>(reinterpret_cast<const uint8_t*>(c - k * ST_PITCH), up);
                sload<16>(reinterpret_cast<const uint8_t*>(c + k * ST_PITCH), dn);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float ring = (bits_to_float(up[e]) + bits_to_float(dn[e])) +
                                       (bits_to_float(hw[4 + e - k]) + bits_to_float(hw[4 + e + k]));
                    acc[e] = __builtin_fmaf(a.w[k], ring, acc[e]);
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = 0.0f;
#pragma unroll
            for (int dy = -R; dy <= R; ++dy) {
                uint32_t hw[12];
                const uint32_t* rowp = c + dy * ST_PITCH;
                sload<16>(reinterpret_cast<const uint8_t*>(rowp - 4), *reinterpret_cast<uint32_t(*)[4]>(&hw[0]));
                sload<16>(reinterpret_cast<const uint8_t*>(rowp), *reinterpret_cast<uint32_t(*)[4]>(&hw[4]));
                sload<16>(reinterpret_cast<const uint8_t*>(rowp + 4), *reinterpret_cast<uint32_t(*)[4]>(&hw[8]));
#pragma unroll
                for (int dx = -R; dx <= R; ++dx)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[e] = __builtin_fmaf(a.w[(dy + R) * N + dx + R], bits_to_float(hw[4 + e + dx]), acc[e]);
            }
        }
        uint32_t o[4];
        const bool row_edge = gi < R || gi >= a.rows - R;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t j = gj + e;
            o[e] = (row_edge || j < R || j >= a.cols - R) ? ctr[e] : float_to_bits(acc[e]);
        }
        uint8_t* q = dst + ((uint64_t)gi * (uint64_t)a.cols + (uint64_t)gj) * 4;
        if (gj + 4 <= a.cols) {
            gstore16u(q, o);
        } else {
            for (int e = 0; e < 4; ++e)
                if (gj + e < a.cols) {
                    uint32_t one[1] = {o[e]};
                    gstore<4>(q + e * 4, one);
                }
        }
    }
}

// ----------------------------------------------------------------- run copy
// Output is written contiguously; each W-byte vector is read from the input run
// its output run maps to.  With a.ua (W = 16) runs of any length and alignment
// move as unaligned 16-byte vectors, vector `part` of a run at byte
// min(16 * part, run_bytes - 16): the last one overlaps its neighbour and
// rewrites the same bytes.
template <int W, bool S>
RR_HD void run_body(const RunArgs& a, uint32_t block, uint32_t tid) {
    constexpr int NW = NWords<W>::value;
    const uint8_t* src = reinterpret_cast<const uint8_t*>(a.src);
    uint8_t* dst = reinterpret_cast<uint8_t*>(a.dst);
    constexpr int V = copy_vpt(W);
    const uint32_t base = block * (uint32_t)(NT * V) + tid;
    uint32_t w[V][NW];
    uint64_t out[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
        const uint32_t v = base + u * NT;
        out[u] = (uint64_t)v * W;
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
            if constexpr (W == 16) {
                if (a.ua) {
                    const uint64_t pos = (uint64_t)part * 16u < a.run_bytes - 16u ? (uint64_t)part * 16u
                                                                                 : a.run_bytes - 16u;
                    out[u] = (uint64_t)run * a.run_bytes + pos;
                    gload16u<S>(src + off + pos, w[u]);
                    continue;
                }
            }
            gload<W, S>(src + off + (uint64_t)part * W, w[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < V; ++u) {
        const uint32_t v = base + u * NT;
        if (v < a.nvec) {
            if constexpr (W == 16) {
                if (a.ua) { gstore16u<true>(dst + out[u], w[u]); continue; }
            }
            gstore<W>(dst + out[u], w[u]);
        }
    }
}

// The load flavour is chosen once per launch (a uniform branch).
template <int W>
RR_HD void run_thread(const RunArgs& a, uint32_t block, uint32_t tid) {
    if (a.cached) run_body<W, false>(a, block, tid);
    else run_body<W, true>(a, block, tid);
}

// ----------------------------------------------------------------- interlace in registers
// One thread's share of an interlace of N sets of U-byte elements (Sec. III.C):
// vector v of every set (16 / U elements each) and the N consecutive 16-byte
// vectors of the joined array that hold the same elements, set index fastest.
// in[][] holds the sets' vectors (interlace) or the joined vectors
// (de-interlace); out[][] receives the other side.  Every byte position is a
// compile-time constant, so the loops unroll to word moves (U >= 4) or byte
// shifts the compiler folds into byte permutes (U = 1, 2).
template <int U, int N, bool DE>
RR_HD void weave_regs(const uint32_t (&in)[N][4], uint32_t (&out)[N][4]) {
    constexpr int P = U < 4 ? U : 4;   // bytes moved per piece
    constexpr uint32_t MASK = P == 4 ? 0xffffffffu : (1u << (8 * P)) - 1u;
#pragma unroll
    for (int ow = 0; ow < 4 * N; ++ow) {
        uint32_t word = 0;
#pragma unroll
        for (int bb = 0; bb < 4; bb += P) {
            const int ob = ow * 4 + bb;   // byte of the thread's output side
            int sv, sb;                   // its source vector and byte
            if constexpr (!DE) {
                const int k = ob / U;     // element of the joined span
                sv = k % N;
                sb = (k / N) * U + ob % U;
            } else {
                const int jb = ((ob % 16 / U) * N + ob / 16) * U + ob % U;
                sv = jb / 16;
                sb = jb % 16;
            }
            const uint32_t piece = (in[sv][sb / 4] >> (8 * (sb % 4))) & MASK;
            word |= P == 4 ? piece : piece << (8 * bb);
        }
        out[ow / 4][ow % 4] = word;
    }
}

// LDS slot of vector m (0 .. 64 * N - 1) of a wave's joined span.  For N = 2,
// 4, 8 the low three bits are XORed with the next three, so the lane-strided
// side (lane L at vector L * N + k) spreads over the banks; the consecutive side
// (lane L at vector k * 64 + L) permutes within aligned groups of eight.  Other
// N are odd or leave at most two lanes of eight on one bank unswizzled.
template <int N>
RR_HD uint32_t weave_slot(uint32_t m) {
    return (N & (N - 1)) == 0 ? m ^ ((m >> 3) & 7u) : m;
}

// Keeps the scheduler from moving instructions across this point: placed after
// a thread's independent global loads so they all issue before the first use of
// a result (otherwise a register reuse can make the second load wait for the
// first).
RR_HD void sched_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_sched_barrier(0);
#endif
}

// A wave's share of a weave: R chunks of 64 consecutive groups each (vector v of
// every set, v = first group of the chunk + lane) and the 64 * N consecutive
// joined vectors that hold them.  Both global sides are accessed one 16-byte
// vector per lane with consecutive lanes at consecutive addresses: the set side
// as group v, the joined side as vector k * 64 + lane of the chunk's span.  The
// two numberings meet in a wave-private LDS region per chunk (64 * N vectors):
// stage writes it, finish reads it back after a wave-level barrier (no
// workgroup barrier: waves never share a region).  Workgroup b covers groups
// [b * R * NT, (b + 1) * R * NT), chunk r of its wave w starting at
// (b * R + r) * NT + w * 64.  The joined side goes through the caches when C is
// true, else is streamed like the set side.  Only chunks that hold the last
// group check vector bounds.  `off` is added to every set and joined pointer
// (the batch's byte offset).  lds: R * NT * N * 16 bytes.
RR_HD uint64_t weave_chunk(uint32_t block, int r, uint32_t wave, int R) {
    return ((uint64_t)block * R + r) * NT + wave * 64u;
}

template <int U, int N, bool DE, bool C, int R>
RR_HD void weave_stage(const WeaveArgs& a, uint32_t block, uint64_t off, uint8_t* lds, uint32_t tid) {
    constexpr uint32_t WV = 64, NW = NT / WV;
    const uint32_t wave = tid / WV, lane = tid % WV;
    if constexpr (!DE) {
        uint32_t in[R][N][4];
        bool ok[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t v = weave_chunk(block, r, wave, R) + lane;
            ok[r] = v < a.nvec;
            if (ok[r])
#pragma unroll
                for (int s = 0; s < N; ++s)
                    gload<16>(reinterpret_cast<const uint8_t*>(a.planes[s]) + off + v * 16u, in[r][s]);
        }
        sched_fence();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            uint8_t* w = lds + (uint64_t)(r * NW + wave) * WV * N * 16u;
            uint32_t out[N][4];
            weave_regs<U, N, false>(in[r], out);
#pragma unroll
            for (int k = 0; k < N; ++k) sstore<16>(w + 16u * weave_slot<N>(lane * N + k), out[k]);
        }
    } else {
        const uint64_t total = (uint64_t)a.nvec * N;
        const uint8_t* joined = reinterpret_cast<const uint8_t*>(a.joined) + off;
        if (weave_chunk(block, R - 1, wave, R) + WV <= a.nvec) {
            uint32_t x[R][N][4];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < N; ++k)
                    gload<16, !C>(joined + (weave_chunk(block, r, wave, R) * N + k * WV + lane) * 16u, x[r][k]);
            sched_fence();
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < N; ++k)
                    sstore<16>(lds + (uint64_t)(r * NW + wave) * WV * N * 16u + 16u * weave_slot<N>(k * WV + lane),
                               x[r][k]);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const uint32_t m = k * WV + lane;
                    const uint64_t j = weave_chunk(block, r, wave, R) * N + m;
                    if (j < total) {
                        uint32_t x[4];
                        gload<16, !C>(joined + j * 16u, x);
                        sstore<16>(lds + (uint64_t)(r * NW + wave) * WV * N * 16u + 16u * weave_slot<N>(m), x);
                    }
                }
        }
    }
}

template <int U, int N, bool DE, bool C, int R>
RR_HD void weave_finish(const WeaveArgs& a, uint32_t block, uint64_t off, const uint8_t* lds, uint32_t tid) {
    constexpr uint32_t WV = 64, NW = NT / WV;
    const uint32_t wave = tid / WV, lane = tid % WV;
    if constexpr (!DE) {
        const uint64_t total = (uint64_t)a.nvec * N;
        uint8_t* joined = reinterpret_cast<uint8_t*>(a.joined) + off;
        if (weave_chunk(block, R - 1, wave, R) + WV <= a.nvec) {
            uint32_t x[R][N][4];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < N; ++k)
                    sload<16>(lds + (uint64_t)(r * NW + wave) * WV * N * 16u + 16u * weave_slot<N>(k * WV + lane),
                              x[r][k]);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < N; ++k)
                    gstore<16, !C>(joined + (weave_chunk(block, r, wave, R) * N + k * WV + lane) * 16u, x[r][k]);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const uint32_t m = k * WV + lane;
                    const uint64_t j = weave_chunk(block, r, wave, R) * N + m;
                    if (j < total) {
                        uint32_t x[4];
                        sload<16>(lds + (uint64_t)(r * NW + wave) * WV * N * 16u + 16u * weave_slot<N>(m), x);
                        gstore<16, !C>(joined + j * 16u, x);
                    }
                }
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t v = weave_chunk(block, r, wave, R) + lane;
            if (v >= a.nvec) continue;
            const uint8_t* w = lds + (uint64_t)(r * NW + wave) * WV * N * 16u;
            uint32_t in[N][4], out[N][4];
#pragma unroll
            for (int k = 0; k < N; ++k) sload<16>(w + 16u * weave_slot<N>(lane * N + k), in[k]);
            weave_regs<U, N, true>(in, out);
#pragma unroll
            for (int s = 0; s < N; ++s) gstore<16>(reinterpret_cast<uint8_t*>(a.planes[s]) + off + v * 16u, out[s]);
        }
    }
}

// ----------------------------------------------------------------- strided select
// Bytes of the R-byte element j of a span of M consecutive 16-byte vectors whose
// elements lie S = M * R bytes apart, packed into one 16-byte output vector
// (16 / R elements).  All positions are compile-time constants.
template <int R, int M>
RR_HD void select_pack(const uint32_t (&in)[4 * M], uint32_t (&o)[4]) {
    constexpr int V = 16 / R, S = M * R;
    if constexpr (R >= 4) {
#pragma unroll
        for (int j = 0; j < V; ++j)
#pragma unroll
            for (int t = 0; t < R / 4; ++t) o[j * (R / 4) + t] = in[(j * S) / 4 + t];
    } else {
        constexpr int PER_WORD = 4 / R;
        constexpr uint32_t MASK = R == 1 ? 0xffu : 0xffffu;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t acc = 0;
#pragma unroll
            for (int b = 0; b < PER_WORD; ++b) {
                const int byte = (q * PER_WORD + b) * S;   // element start in the span (never crosses a word)
                acc |= ((in[byte / 4] >> (8 * (byte % 4))) & MASK) << (8 * R * b);
            }
            o[q] = acc;
        }
    }
}

// One thread's output vector of a strided select: 16 / R consecutive elements of
// one output row, read as M 16-byte vectors at any alignment when the whole span
// lies inside the box (loads through the caches: neighbouring lanes' spans share
// lines), element by element at a row's end or the box's end.
template <int R, int M>
RR_HD void select_thread(const SelectArgs& a, uint32_t block, uint32_t tid) {
    constexpr int V = 16 / R, S = M * R;
    const uint32_t v = block * (uint32_t)NT + tid;
    if (v >= a.nvec) return;
    const uint32_t row = mdiv(v, a.mvpr);
    const uint32_t col = v - row * a.vpr;
    uint64_t off = 0;
    uint32_t rem = row;
#pragma unroll
    for (int j = MAXR - 1; j >= 1; --j) {
        if (j < a.nax) {
            const uint32_t q = mdiv(rem, a.om[j]);
            off += (uint64_t)(rem - q * a.on[j]) * a.sin[j];
            rem = q;
        }
    }
    if (a.nax >= 1) off += (uint64_t)rem * a.sin[0];
    const uint32_t e0 = col * V;
    const uint32_t cnt = umin(V, a.n - e0);
    const uint8_t* p = reinterpret_cast<const uint8_t*>(a.src) + off + (uint64_t)e0 * S;
    uint8_t* q = reinterpret_cast<uint8_t*>(a.dst) + ((uint64_t)row * a.n + e0) * R;
    if (cnt == (uint32_t)V && reinterpret_cast<uint64_t>(p) + 16u * M <= a.src_end) {
        uint32_t in[4 * M];
#pragma unroll
        for (int u = 0; u < M; ++u) gload16u<false>(p + 16 * u, *reinterpret_cast<uint32_t(*)[4]>(&in[4 * u]));
        uint32_t o[4];
        select_pack<R, M>(in, o);
        gstore16u<true>(q, o);
    } else {
        for (uint32_t j = 0; j < cnt; ++j) {
            uint32_t e[NWords<R>::value];
            gload<R, false>(p + (uint64_t)j * S, e);
            gstore<R>(q + (uint64_t)j * R, e);
        }
    }
}

// Workgroup-staged select for a box whose kept elements lie S bytes apart along
// one run (no outer rows: nax == 0).  Workgroup `block` covers elements
// [block * NT * V, +NT * V) of the run, whose input is one contiguous span of
// NT * 16 * M bytes: the stage phase loads it with 16-byte vectors, lane after
// lane (each load instruction of a wave reads 1 KiB of consecutive bytes), into
// LDS; after the barrier the pack phase reads each thread's M vectors back from
// LDS and writes its output vector.  Bytes of the span past the box's end are
// not loaded.  lds: NT * 16 * M bytes.
template <int R, int M>
RR_HD void select_stage(const SelectArgs& a, uint32_t block, uint8_t* lds, uint32_t tid) {
    const uint8_t* base = reinterpret_cast<const uint8_t*>(a.src) + (uint64_t)block * NT * 16u * M;
    const uint64_t end = a.src_end;
    uint32_t w[M][4];
    bool full[M];
    // Every lane loads when the run holds a 16-byte vector at all (a vector past
    // the end re-reads the run's last whole one, discarded): loads behind
    // per-lane branches left one load in flight at a time.
    if (end >= reinterpret_cast<uint64_t>(a.src) + 16u) {
#pragma unroll
        for (int u = 0; u < M; ++u) {
            const uint8_t* p = base + 16u * (u * NT + tid);
            full[u] = reinterpret_cast<uint64_t>(p) + 16u <= end;
            gload16u<true>(full[u] ? p : reinterpret_cast<const uint8_t*>(end - 16u), w[u]);
        }
        sched_fence();
    } else {
#pragma unroll
        for (int u = 0; u < M; ++u) full[u] = false;
    }
#pragma unroll
    for (int u = 0; u < M; ++u) {
        uint8_t* q = lds + 16u * (u * NT + tid);
        if (full[u]) {
            sstore<16>(q, w[u]);
        } else {
            const uint8_t* p = base + 16u * (u * NT + tid);
            for (uint32_t i = 0; i < 16u && reinterpret_cast<uint64_t>(p + i) < end; ++i) {
                uint32_t b[1];
                gload<1, true>(p + i, b);
                q[i] = (uint8_t)b[0];
            }
        }
    }
}

template <int R, int M>
RR_HD void select_pack_store(const SelectArgs& a, uint32_t block, const uint8_t* lds, uint32_t tid) {
    constexpr int V = 16 / R;
    const uint32_t v = block * (uint32_t)NT + tid;   // output vector of the run
    if (v >= a.nvec) return;
    const uint32_t e0 = v * V;
    const uint32_t cnt = umin(V, a.n - e0);
    const uint8_t* p = lds + 16u * M * tid;
    uint8_t* q = reinterpret_cast<uint8_t*>(a.dst) + (uint64_t)e0 * R;
    if (cnt == (uint32_t)V) {
        uint32_t in[4 * M];
#pragma unroll
        for (int u = 0; u < M; ++u) sload<16>(p + 16 * u, *reinterpret_cast<uint32_t(*)[4]>(&in[4 * u]));
        uint32_t o[4];
        select_pack<R, M>(in, o);
        gstore16u<true>(q, o);
    } else {
        for (uint32_t j = 0; j < cnt; ++j) {
            uint32_t e[NWords<R>::value];
            sload<R>(p + j * (uint32_t)(M * R), e);
            gstore<R>(q + (uint64_t)j * R, e);
        }
    }
}

// ----------------------------------------------------------------- tiles
struct TileCtx {
    uint64_t bin, bout;   // byte bases of the tile (absolute unless in table mode)
    uint32_t TAv, TBv;    // valid row length / row count of this tile
    uint32_t TCv;         // stacked sub-tiles in this tile (1 unless stacked)
};

RR_HD TileCtx tile_decode(const TileArgs& a, uint32_t tile) {
    TileCtx t;
    t.bin = a.src;
    t.bout = a.dst;
    t.TAv = a.TA;
    t.TBv = a.TB;
    t.TCv = a.cO_t;
    uint32_t rem = tile, cfast = 0;
#pragma unroll
    for (int g = MAXR - 1; g >= 0; --g) {
        if (g < a.ngrid) {
            const uint32_t q = mdiv(rem, a.gm[g]);
            uint32_t c = rem - q * a.gn[g];
            rem = q;
            // diagonal order: the second-fastest tile coordinate advances with the
            // fastest one, so consecutive tiles differ in both (a bijection per slab)
            if (g == a.ngrid - 1) cfast = c;
            else if (g == a.ngrid - 2 && (a.flags & TF_DIAG)) {
                const uint32_t s = c + cfast;
                c = s - mdiv(s, a.gm[g]) * a.gn[g];
            }
            t.bin += (uint64_t)c * a.gsin[g];
            t.bout += (uint64_t)c * a.gsout[g];
            if (g == a.grid_aO) t.TAv = a.TAinner * umin(a.aO_t, a.aO_len - c * a.aO_t);
            if (g == a.grid_bO) t.TBv = a.TBinner * umin(a.bO_t, a.bO_len - c * a.bO_t);
            if (g == a.grid_cO) t.TCv = umin(a.cO_t, a.cO_len - c * a.cO_t);
        }
    }
    return t;
}

// Workgroups of a launch are dispatched round-robin over the XCDs (8 on
// MI355X, each with its own L2).  Plain order gives XCD x every 8th tile; with
// TF_XCD it takes the contiguous range [x*q + min(x, r), +q + (x < r)) of the
// ntiles = 8q + r tiles instead.  Either way a bijection on [0, ntiles).
constexpr uint32_t NXCD = 8;
RR_HD uint32_t xcd_range(uint32_t b, uint32_t ntiles) {
    const uint32_t q = ntiles / NXCD, r = ntiles % NXCD;
    const uint32_t x = b % NXCD, k = b / NXCD;
    return x * q + umin(x, r) + k;
}
RR_HD uint32_t block_to_tile(const TileArgs& a, uint32_t b) {
    return (a.flags & TF_XCD) ? xcd_range(b, a.ntiles) : b;
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
// by (ib / RG) so that the column reads of the write phase, where each lane reads
// RG consecutive rows and neighbouring lanes the next groups of RG rows, fall on
// different banks.
template <int RG>
RR_HD uint32_t lds_pos(const TileArgs& a, uint32_t ib, uint32_t x) {
    const uint32_t rot = (ib / RG) & a.rotmask;
    uint32_t cc = (x >> 4) + rot;
    if (cc >= a.nch16) cc -= a.nch16;
    return ib * a.pitch + (cc << 4) + (x & 15u);
}

// Rows that share one chunk rotation in a tile of U-byte units and G x G
// micro-tiles: G rows for micro-tiles; 16 / U rows when G = 1, where a lane
// gathers one 16-byte output vector from 16 / U consecutive rows (with one row
// per rotation step, lanes 16 / U rows apart would meet on a few banks: 6-9
// conflict cycles per LDS read for 2- and 4-byte units).  Read and write phases
// of a kernel use the same value.
template <int U, int G>
constexpr int rot_group() { return G > 1 ? G : 16 / U; }

// Loads each thread keeps in flight before writing any of them to LDS.  Default
// tiles are 16 KiB, i.e. four 16-byte vectors per thread: one batch, and few
// enough registers that six waves fit per SIMD.  Larger tiles loop.
constexpr int READ_BATCH = RR_READ_BATCH;

// Read phase: rows of the tile (contiguous along the input's fastest axes) are
// loaded with WIN-byte vectors and parked in LDS.
template <int WIN, int RG, int B, bool S>
RR_HD void read_phase(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    constexpr int NWI = NWords<WIN>::value;
    const uint32_t total = a.TB * a.rch;
    const uint32_t rowvalid = t.TAv * a.R;
    for (uint32_t base = 0; base < total; base += NT * B) {
        uint32_t w[B][NWI];
        uint32_t lo[B];
        uint64_t src[B];
        bool ok[B];
        // Every lane loads (a lane past the tile's valid extent re-reads the tile's
        // first vector, which exists whenever the tile does): loads behind per-lane
        // branches are issued one at a time, each waited for before the next.  All
        // addresses are formed before the first load: address arithmetic between
        // the loads made the compiler wait for each load before the next (a
        // register it rewrote could still be the target of the previous round's
        // load), leaving one load in flight per lane.
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t f = base + u * NT + tid;
            uint32_t ib = mdiv(f, a.mrch);
            uint32_t x = (f - ib * a.rch) * WIN;
            ok[u] = f < total && ib < t.TBv && x < rowvalid;
            if (!ok[u]) { ib = 0; x = 0; }
            src[u] = t.bin + row_in(a, ib) + x;
            lo[u] = lds_pos<RG>(a, ib, x);
        }
        sched_fence();
#pragma unroll
        for (int u = 0; u < B; ++u) gload<WIN, S>(reinterpret_cast<const uint8_t*>(src[u]), w[u]);
        sched_fence();
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (ok[u]) sstore<WIN>(lds + lo[u], w[u]);
    }
}

// Flat read: the tile's input rows are back to back in memory (a contiguous
// byte range), and LDS holds them unpadded, so the whole range moves with
// 16-byte vectors however short or oddly sized a row is (de-interlace).
template <int B, bool S>
RR_HD void read_flat(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    const uint32_t nbytes = t.TBv * a.pitch;
    const uint32_t nvec = nbytes / a.win;
    for (uint32_t base = 0; base < nvec; base += NT * B) {
        uint32_t w[B][4];
        bool ok[B];
        // every lane loads (past the end: the range's first vector), so the B
        // loads issue back to back instead of each behind its own branch
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t v = base + u * NT + tid;
            ok[u] = v < nvec;
            gload<16, S>(reinterpret_cast<const uint8_t*>(t.bin) + (uint64_t)(ok[u] ? v : 0u) * 16, w[u]);
        }
        sched_fence();
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (ok[u]) sstore<16>(lds + (base + u * NT + tid) * 16, w[u]);
    }
    // the input's last tile may end inside a 16-byte vector: its last bytes one by one
    const uint32_t tail = nbytes - nvec * 16;
    if (tid < tail) {
        const uint32_t x = nvec * 16 + tid;
        lds[x] = reinterpret_cast<const uint8_t*>(t.bin)[x];
    }
}

// Walk n items laid out as rows of `per` items with NT threads: item f = tid +
// s*NT of a thread is (row, col); steps advance incrementally, no division per item.
struct RowWalk {
    uint32_t row, col, drow, dcol, per;
    RR_HD RowWalk(uint32_t tid, uint32_t per_row) : per(per_row) {
        row = tid / per_row;
        col = tid - row * per_row;
        drow = (uint32_t)NT / per_row;
        dcol = (uint32_t)NT - drow * per_row;
    }
    RR_HD void step() {
        row += drow;
        col += dcol;
        if (col >= per) { col -= per; ++row; }
    }
};

// Copy nrows rows of rowbytes bytes (a multiple of U, any alignment) from
// global memory into LDS: whole 16-byte vectors plus each row's last
// (rowbytes % 16) / U elements one by one, so nothing outside a row is touched.
//   src_row(r)      -> global byte address of row r
//   lds_at(r, x)    -> LDS byte offset of byte x of row r
template <int U, bool S, class SrcRow, class LdsAt>
RR_HD void read_rows(uint32_t nrows, uint32_t rowbytes, SrcRow src_row, LdsAt lds_at, uint8_t* lds,
                     uint32_t tid) {
    constexpr int B = READ_BATCH;
    const uint32_t nfull = rowbytes >> 4;
    const uint32_t per = nfull + ((rowbytes & 15u) / U);
    if (per == 0 || nrows == 0) return;
    RowWalk w(tid, per);
    using Elem = uint32_t[NWords<U>::value];
    while (w.row < nrows) {
        uint32_t v[B][4];
        uint32_t lo[B];
        uint64_t src[B];
        uint8_t kind[B];   // 0: none, 1: 16-byte vector, 2: one U-byte element
        // addresses first, then the loads back to back (an element lands in the
        // first words of its vector's registers, so no copy waits for it)
#pragma unroll
        for (int u = 0; u < B; ++u) {
            kind[u] = 0;
            lo[u] = 0;
            src[u] = 0;
            if (w.row < nrows) {
                const uint64_t rowp = src_row(w.row);
                const uint32_t x = w.col < nfull ? w.col << 4 : (nfull << 4) + (w.col - nfull) * U;
                src[u] = rowp + x;
                lo[u] = lds_at(w.row, x);
                kind[u] = w.col < nfull ? 1 : 2;
                w.step();
            }
        }
        sched_fence();
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (kind[u] == 1) gload16u<S>(reinterpret_cast<const uint8_t*>(src[u]), v[u]);
            else if (kind[u] == 2) gload<U, S>(reinterpret_cast<const uint8_t*>(src[u]), *reinterpret_cast<Elem*>(&v[u][0]));
        }
        sched_fence();
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (kind[u] == 1) sstore<16>(lds + lo[u], v[u]);
            else if (kind[u] == 2) sstore<U>(lds + lo[u], *reinterpret_cast<const Elem*>(&v[u][0]));
        }
    }
}

// Ragged read: each input row (TAv*R bytes at any element alignment) of the
// tile, into its padded LDS row.
template <int U, bool S>
RR_HD void read_ragged(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    read_rows<U, S>(
        t.TBv, t.TAv * a.R, [&](uint32_t r) { return t.bin + row_in(a, r); },
        [&](uint32_t r, uint32_t x) { return lds_pos<rot_group<U, 1>()>(a, r, x); }, lds, tid);
}

// Stacked read: TCv sub-tiles of msub input bytes each; when they are back to
// back in the input (sinC == msub) the whole range is one row.
template <int U, bool S>
RR_HD void read_stack(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    if (a.sinC == a.msub)
        read_rows<U, S>(
            1, t.TCv * a.msub, [&](uint32_t) { return t.bin; }, [&](uint32_t, uint32_t x) { return x; }, lds,
            tid);
    else
        read_rows<U, S>(
            t.TCv, a.msub, [&](uint32_t r) { return t.bin + (uint64_t)r * a.sinC; },
            [&](uint32_t r, uint32_t x) { return r * a.msubp + x; }, lds, tid);
}

template <int U, int G, bool S>
RR_HD void read_tile(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    constexpr int B = READ_BATCH;
    if constexpr (G == 1 && U < 16) {   // 16-byte units are always aligned vectors
        if (a.flags & TF_STACK) { read_stack<U, S>(a, t, lds, tid); return; }
        if (a.flags & TF_RAGGED_IN) { read_ragged<U, S>(a, t, lds, tid); return; }
    }
    if constexpr (G > 1 && U < 16) {
        if (a.flags & TF_UMT) {
            read_rows<U, S>(
                t.TBv, t.TAv * a.R, [&](uint32_t r) { return t.bin + row_in(a, r); },
                [&](uint32_t r, uint32_t x) { return lds_pos<G>(a, r, x); }, lds, tid);
            return;
        }
    }
    if (a.flags & TF_IN_FLAT) { read_flat<B, S>(a, t, lds, tid); return; }
    switch (a.win) {
        case 16: read_phase<16, rot_group<U, G>(), B, S>(a, t, lds, tid); break;
        case 8: read_phase<8, rot_group<U, G>(), B, S>(a, t, lds, tid); break;
        case 4: read_phase<4, rot_group<U, G>(), B, S>(a, t, lds, tid); break;
        case 2: read_phase<2, rot_group<U, G>(), B, S>(a, t, lds, tid); break;
        default: read_phase<1, rot_group<U, G>(), B, S>(a, t, lds, tid); break;
    }
}

// The access flavour is chosen once per tile (a uniform branch), so the loops
// below it carry no per-load condition.
template <int U, int G>
RR_HD void read_dispatch(const TileArgs& a, const TileCtx& t, uint8_t* lds, uint32_t tid) {
    if (a.flags & TF_LD_CACHED) read_tile<U, G, false>(a, t, lds, tid);
    else read_tile<U, G, true>(a, t, lds, tid);
}

// Write phase: each work item is a GxG micro-tile (G rows of the LDS tile, G
// elements each), transposed in registers into G output vectors that lie along
// the output's fastest axis.
// Ragged write: each output row (TBv elements of k units of U bytes along the
// output's fastest axis, any alignment) is written as 16-byte vectors gathered
// unit by unit from LDS, plus its last (bytes % 16) / U units one by one.  Unit
// q of an output row is unit q % k of element q / k (an LDS row).
template <int U, bool S>
RR_HD void write_ragged(const TileArgs& a, const TileCtx& t, const uint8_t* lds, uint32_t tid) {
    constexpr int EPV = 16 / U;   // units per 16-byte vector
    const uint32_t k = a.k;
    const uint32_t rowbytes = t.TBv * a.R;
    const uint32_t nfull = rowbytes >> 4;
    const uint32_t per = nfull + ((rowbytes & 15u) / U);
    if (per == 0 || t.TAv == 0) return;
    constexpr int RG = rot_group<U, 1>();   // == EPV: one output vector's rows share a rotation
    // LDS address of unit q of output row ia
    auto unit_at = [&](uint32_t ia, uint32_t q) {
        if (k == 1) return lds_pos<RG>(a, q, ia * U);
        const uint32_t ib = mdiv(q, a.mk);
        return lds_pos<RG>(a, ib, (ia * k + (q - ib * k)) * U);
    };
    // Items go B per round: each item's row address and LDS gather first, then
    // the round's stores back to back (an address formed between stores made
    // the compiler wait for every outstanding store).
    constexpr int B = U == 2 ? 2 : READ_BATCH;
    using Elem = uint32_t[NWords<U>::value];
    RowWalk w(tid, per);
    while (w.row < t.TAv) {
        uint32_t o[B][4];
        uint64_t dst[B];
        uint8_t kind[B];   // 0: none, 1: 16-byte vector, 2: one U-byte unit
#pragma unroll
        for (int u = 0; u < B; ++u) {
            kind[u] = 0;
            dst[u] = 0;
            if (w.row >= t.TAv) continue;
            const uint32_t ia = w.row;
            const uint64_t rowp = t.bout + row_out(a, ia);
            if (w.col < nfull) {
                const uint32_t q0 = w.col * EPV;
                // element j of the vector: rows q0 + j (single-unit elements, one
                // rotation group: one address, then a pitch per row) or unit q0 + j
                const uint32_t base0 = k == 1 ? lds_pos<RG>(a, q0, ia * U) : 0u;
                auto at = [&](uint32_t j) { return k == 1 ? base0 + j * a.pitch : unit_at(ia, q0 + j); };
                if constexpr (U >= 4) {
#pragma unroll
                    for (int j = 0; j < EPV; ++j) {
                        uint32_t e[NWords<U>::value];
                        sload<U>(lds + at(j), e);
#pragma unroll
                        for (int q = 0; q < U / 4; ++q) o[u][j * (U / 4) + q] = e[q];
                    }
                } else {
                    constexpr int PER_WORD = 4 / U;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        uint32_t acc = 0;
#pragma unroll
                        for (int b = 0; b < PER_WORD; ++b) {
                            uint32_t e[1];
                            sload<U>(lds + at(q * PER_WORD + b), e);
                            acc |= e[0] << (8 * U * b);
                        }
                        o[u][q] = acc;
                    }
                }
                dst[u] = rowp + (w.col << 4);
                kind[u] = 1;
            } else {
                const uint32_t q = nfull * EPV + (w.col - nfull);
                sload<U>(lds + unit_at(ia, q), *reinterpret_cast<Elem*>(&o[u][0]));
                dst[u] = rowp + (uint64_t)q * U;
                kind[u] = 2;
            }
            w.step();
        }
        sched_fence();
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (kind[u] == 1) gstore16u<S>(reinterpret_cast<uint8_t*>(dst[u]), o[u]);
            else if (kind[u] == 2) gstore<U, S>(reinterpret_cast<uint8_t*>(dst[u]), *reinterpret_cast<const Elem*>(&o[u][0]));
        }
    }
}

// Flat write: the tile's output rows are back to back (row_out(ia) = ia*TB*U),
// so the whole tile is one contiguous byte range, written as 16-byte vectors
// whose elements come from LDS across row boundaries, plus an element tail.
template <int U, bool S>
RR_HD void write_flat(const TileArgs& a, const TileCtx& t, const uint8_t* lds, uint32_t tid) {
    constexpr int EPV = 16 / U;
    const uint32_t nel = t.TAv * a.TB;            // output rows of the tile are full (TBv == TB)
    const uint32_t nbytes = nel * U;
    const uint32_t nfull = nbytes >> 4;
    const uint32_t per = nfull + ((nbytes & 15u) / U);
    uint8_t* base = reinterpret_cast<uint8_t*>(t.bout);
    for (uint32_t c = tid; c < per; c += NT) {
        if (c < nfull) {
            uint32_t o[4];
            const uint32_t q0 = c * EPV;
            if constexpr (U >= 4) {
#pragma unroll
                for (int j = 0; j < EPV; ++j) {
                    const uint32_t q = q0 + j;
                    const uint32_t ia = mdiv(q, a.mtb);
                    uint32_t e[NWords<U>::value];
                    sload<U>(lds + lds_pos<rot_group<U, 1>()>(a, q - ia * a.TB, ia * U), e);
#pragma unroll
                    for (int k = 0; k < U / 4; ++k) o[j * (U / 4) + k] = e[k];
                }
            } else {
                constexpr int PER_WORD = 4 / U;
#pragma unroll
                for (int w4 = 0; w4 < 4; ++w4) {
                    uint32_t acc = 0;
#pragma unroll
                    for (int b = 0; b < PER_WORD; ++b) {
                        const uint32_t q = q0 + w4 * PER_WORD + b;
                        const uint32_t ia = mdiv(q, a.mtb);
                        uint32_t e[1];
                        sload<U>(lds + lds_pos<rot_group<U, 1>()>(a, q - ia * a.TB, ia * U), e);
                        acc |= e[0] << (8 * U * b);
                    }
                    o[w4] = acc;
                }
            }
            gstore16u<S>(base + ((uint64_t)c << 4), o);
        } else {
            const uint32_t q = nfull * EPV + (c - nfull);
            const uint32_t ia = mdiv(q, a.mtb);
            uint32_t e[NWords<U>::value];
            sload<U>(lds + lds_pos<rot_group<U, 1>()>(a, q - ia * a.TB, ia * U), e);
            gstore<U, S>(base + (uint64_t)q * U, e);
        }
    }
}

// Stacked write: the output of sub-tile c is TA rows of TB elements back to
// back (msub bytes at c * soutC); when the sub-tiles are back to back too
// (soutC == msub) the whole tile is one row.  Element (c, ia, ib) of the output
// is element (c, ib, ia) of the input, at LDS c * msubp + (ib * TA + ia) * U.
// Each 16-byte output vector gathers its elements from LDS, walking (c, ia, ib)
// incrementally from one division per vector.
template <int U, bool S>
RR_HD void write_stack(const TileArgs& a, const TileCtx& t, const uint8_t* lds, uint32_t tid) {
    constexpr int EPV = 16 / U;
    const bool one = a.soutC == a.msub;
    const uint32_t nrows = one ? 1u : t.TCv;
    const uint32_t rowbytes = one ? t.TCv * a.msub : a.msub;
    const uint32_t row_el = rowbytes / U;
    const uint32_t nfull = rowbytes >> 4;
    const uint32_t per = nfull + ((rowbytes & 15u) / U);
    for (RowWalk w(tid, per); w.row < nrows; w.step()) {
        uint8_t* rowp = reinterpret_cast<uint8_t*>(t.bout + (uint64_t)w.row * a.soutC);
        const bool vec = w.col < nfull;
        const uint32_t q0 = vec ? w.col * EPV : nfull * EPV + (w.col - nfull);
        // element q of the whole tile -> (c, ia, ib)
        const uint32_t qg = w.row * row_el + q0;
        uint32_t c = mdiv(qg, a.msubel);
        const uint32_t rem = qg - c * (a.TA * a.TB);
        uint32_t ia = mdiv(rem, a.mtb);
        uint32_t ib = rem - ia * a.TB;
        auto at = [&]() { return lds + c * a.msubp + (ib * a.TA + ia) * U; };
        auto next = [&]() {
            if (++ib == a.TB) { ib = 0; if (++ia == a.TA) { ia = 0; ++c; } }
        };
        if (vec) {
            uint32_t o[4];
            if constexpr (U >= 4) {
#pragma unroll
                for (int j = 0; j < EPV; ++j) {
                    uint32_t e[NWords<U>::value];
                    sload<U>(at(), e);
#pragma unroll
                    for (int q = 0; q < U / 4; ++q) o[j * (U / 4) + q] = e[q];
                    next();
                }
            } else {
                constexpr int PER_WORD = 4 / U;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t acc = 0;
#pragma unroll
                    for (int b = 0; b < PER_WORD; ++b) {
                        uint32_t e[1];
                        sload<U>(at(), e);
                        acc |= e[0] << (8 * U * b);
                        next();
                    }
                    o[q] = acc;
                }
            }
            gstore16u<S>(rowp + (w.col << 4), o);
        } else {
            uint32_t e[NWords<U>::value];
            sload<U>(at(), e);
            gstore<U, S>(rowp + (uint64_t)q0 * U, e);
        }
    }
}

// Unaligned micro-tiles: full G x G micro-tiles are transposed in registers and
// stored as G unaligned W-byte vectors (row starts at any element offset); a
// micro-tile cut by the tile's valid extent moves element by element.
template <int U, int G, bool S>
RR_HD void write_umt(const TileArgs& a, const TileCtx& t, const uint8_t* lds, uint32_t tid) {
    constexpr int W = U * G;
    constexpr int NW = NWords<W>::value;
    for (uint32_t gi = tid; gi < a.nwork; gi += NT) {
        const uint32_t ma = mdiv(gi, a.mnmb);
        const uint32_t mb = gi - ma * a.nmb;
        const uint32_t ia0 = ma * G, ib0 = mb * G;
        if (ia0 >= t.TAv || ib0 >= t.TBv) continue;
        if (ia0 + G <= t.TAv && ib0 + G <= t.TBv) {
            uint32_t r[G][NW];
#pragma unroll
            for (int j = 0; j < G; ++j) sload<W>(lds + lds_pos<G>(a, ib0 + j, ia0 * U), r[j]);
            uint32_t o[G][NW];
            xpose<U, G>(r, o);
#pragma unroll
            for (int i = 0; i < G; ++i)
                gstore_u<W, S>(reinterpret_cast<uint8_t*>(t.bout + row_out(a, ia0 + i) + (uint64_t)ib0 * U), o[i]);
        } else {
            const uint32_t ni = umin(G, t.TAv - ia0), nj = umin(G, t.TBv - ib0);
            for (uint32_t i = 0; i < ni; ++i) {
                uint8_t* q = reinterpret_cast<uint8_t*>(t.bout + row_out(a, ia0 + i) + (uint64_t)ib0 * U);
                for (uint32_t j = 0; j < nj; ++j) {
                    uint32_t e[NWords<U>::value];
                    sload<U>(lds + lds_pos<G>(a, ib0 + j, (ia0 + i) * U), e);
                    gstore<U, S>(q + j * U, e);
                }
            }
        }
    }
}

template <int U, int G, bool S>
RR_HD void write_tile(const TileArgs& a, const TileCtx& t, const uint8_t* lds, uint32_t tid) {
    constexpr int W = U * G;
    constexpr int NW = NWords<W>::value;
    if constexpr (G == 1 && U < 16) {   // 16-byte units are always aligned vectors
        if (a.flags & TF_STACK) {
            write_stack<U, S>(a, t, lds, tid);
            return;
        }
        if (a.flags & TF_OUT_FLAT) {
            write_flat<U, S>(a, t, lds, tid);
            return;
        }
        if (a.flags & TF_RAGGED_OUT) {
            write_ragged<U, S>(a, t, lds, tid);
            return;
        }
    }
    if constexpr (G > 1 && U < 16) {
        if (a.flags & TF_UMT) {
            write_umt<U, G, S>(a, t, lds, tid);
            return;
        }
    }
    // Work items are taken WB per round: every item's LDS rows and store
    // addresses first, then all the round's stores back to back.  Computing an
    // address between stores made the compiler wait for every outstanding store
    // (the plane-table branch of the address can load, and the wait it needs
    // stayed in the shared path), so a thread's stores went out one at a time.
    if (G > 1 || a.k == 1) {
        constexpr int WB = G == 1 ? 4 : G == 2 ? 2 : 1;
        constexpr bool CAN_MERGE = W >= 4 && W * G >= 16;
        constexpr int NV = CAN_MERGE ? W * G / 16 : 1;   // 16-byte vectors of a merged micro-tile
        constexpr int PER = W >= 4 ? W / 4 : 1;
        const bool table = (a.flags & TF_OUT_TABLE) != 0;
        const bool merge = CAN_MERGE && !table && (a.flags & TF_OUT_MERGE);
        for (uint32_t g0 = tid; g0 < a.nwork; g0 += NT * WB) {
            uint32_t o[WB][G][NW];
            uint64_t dst[WB][G];
            bool ok[WB];
#pragma unroll
            for (int w = 0; w < WB; ++w) {
                const uint32_t gi = g0 + (uint32_t)w * NT;
                const uint32_t ma = mdiv(gi, a.mnmb);
                const uint32_t mb = gi - ma * a.nmb;
                const uint32_t ia0 = ma * G, ib0 = mb * G;
                ok[w] = gi < a.nwork && ia0 < t.TAv && ib0 < t.TBv;
                if (!ok[w]) continue;
                uint32_t r[G][NW];
#pragma unroll
                for (int j = 0; j < G; ++j) sload<W>(lds + lds_pos<rot_group<U, G>()>(a, ib0 + j, ia0 * U), r[j]);
                xpose<U, G>(r, o[w]);
                if (table) {
#pragma unroll
                    for (int i = 0; i < G; ++i) dst[w][i] = a.table[ia0 + i] + t.bout + (uint64_t)ib0 * U;
                } else {
                    const uint64_t q = t.bout + row_out(a, ia0) + (merge ? 0 : (uint64_t)ib0 * U);
#pragma unroll
                    for (int i = 0; i < G; ++i) dst[w][i] = merge ? q + (uint64_t)i * 16u : q + (uint64_t)i * a.soutA[0];
                }
            }
            sched_fence();
#pragma unroll
            for (int w = 0; w < WB; ++w) {
                if (!ok[w]) continue;
                if (merge) {
                    // the G output rows are back to back: store them as 16-byte vectors
                    uint32_t flat[NV * 4];
#pragma unroll
                    for (int i = 0; i < G; ++i)
#pragma unroll
                        for (int c = 0; c < PER; ++c)
                            if (i * PER + c < NV * 4) flat[i * PER + c] = o[w][i][c];
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        gstore<16, S>(reinterpret_cast<uint8_t*>(dst[w][v]), *reinterpret_cast<const uint32_t(*)[4]>(&flat[v * 4]));
                } else {
#pragma unroll
                    for (int i = 0; i < G; ++i) gstore<W, S>(reinterpret_cast<uint8_t*>(dst[w][i]), o[w][i]);
                }
            }
        }
    } else {
        constexpr int WB = U == 16 ? 1 : 4;
        for (uint32_t g0 = tid; g0 < a.nwork; g0 += NT * WB) {
            uint32_t v[WB][NWords<U>::value];
            uint64_t dst[WB];
            bool ok[WB];
#pragma unroll
            for (int w = 0; w < WB; ++w) {
                const uint32_t gi = g0 + (uint32_t)w * NT;
                const uint32_t ia = mdiv(gi, a.mnmb);
                const uint32_t m = gi - ia * a.nmb;
                const uint32_t ib = mdiv(m, a.mk);
                const uint32_t s = m - ib * a.k;
                ok[w] = gi < a.nwork && ia < t.TAv && ib < t.TBv;
                if (!ok[w]) continue;
                sload<U>(lds + lds_pos<rot_group<U, 1>()>(a, ib, (ia * a.k + s) * U), v[w]);
                dst[w] = t.bout + row_out(a, ia) + (uint64_t)m * U;
            }
            sched_fence();
#pragma unroll
            for (int w = 0; w < WB; ++w)
                if (ok[w]) gstore<U, S>(reinterpret_cast<uint8_t*>(dst[w]), v[w]);
        }
    }
}

template <int U, int G>
RR_HD void write_phase(const TileArgs& a, const TileCtx& t, const uint8_t* lds, uint32_t tid) {
    if (a.flags & TF_ST_CACHED) write_tile<U, G, false>(a, t, lds, tid);
    else write_tile<U, G, true>(a, t, lds, tid);
}

// ----------------------------------------------------------------- batches
// Job of workgroup b in a batch group: the largest j with prefix[j] <= b
// (prefix holds njobs+1 exclusive sums of the jobs' workgroup counts, then the
// bucket index).  The bucket bounds the search to the jobs between the ones
// holding workgroups k * BATCH_BUCKET and (k + 1) * BATCH_BUCKET: one or two
// dependent loads for most workgroups instead of log2(njobs).
RR_HD uint32_t find_job(const uint32_t* prefix, uint32_t njobs, uint32_t b) {
    const uint32_t* bucket = prefix + njobs + 1;
    const uint32_t k = b / BATCH_BUCKET;
    uint32_t lo = bucket[k], hi = bucket[k + 1] + 1;
    if (hi > njobs) hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Block (tile, or run-copy block) of workgroup b of entry r in a batch group,
// each XCD taking a contiguous run of the entry's blocks.  Workgroups reach the
// XCDs round-robin (workgroup b on XCD b % 8); this gives each XCD a contiguous
// run of the entry's blocks instead, as xcd_range does for a single launch.
// The entry's workgroups [start, start + n) map one to one onto its blocks
// [first, first + n): workgroup b is virtual index v = b - start + start % 8
// (so v % 8 is its XCD), and XCD x's runs are laid out in x order.
RR_HD uint32_t batch_xcd_block(const EntryRange& r, uint32_t b) {
    const uint32_t lb = b - r.start;
    const uint32_t n = r.count, q0 = r.start % NXCD;
    const uint32_t v = lb + q0, x = v % NXCD, k = v / NXCD;
    // tiles of the XCDs before x: the virtual indices in [q0, q0 + n) whose XCD is
    // below x, i.e. #{u < q0 + n : u % 8 < x} - #{u < q0 : u % 8 < x} (q0 < 8)
    const uint32_t m = q0 + n;
    const uint32_t start = (m / NXCD) * x + umin(m % NXCD, x) - umin(q0, x);
    return r.first + start + k - (x < q0 ? 1u : 0u);
}
// Tile of workgroup b of entry r: XCD ranges with TF_XCD, else in order.
RR_HD uint32_t batch_block_to_tile(uint32_t flags, const EntryRange& r, uint32_t b) {
    if (!(flags & TF_XCD)) return r.first + (b - r.start);
    return batch_xcd_block(r, b);
}

template <int W>
RR_HD void batch_copy_block(const CopyArgs* args, const uint32_t* prefix, const EntryRange* ranges,
                            uint32_t njobs, uint32_t b, uint32_t tid) {
    const uint32_t j = find_job(prefix, njobs, b);
    const EntryRange r = ranges[j];
    copy_thread<W>(args[j], b - r.start + r.first, r.job_blocks, tid);
}

template <int W>
RR_HD void batch_run_block(const RunArgs* args, const uint32_t* prefix, const EntryRange* ranges,
                           uint32_t njobs, uint32_t b, uint32_t tid) {
    const uint32_t j = find_job(prefix, njobs, b);
    const EntryRange r = ranges[j];
    const RunArgs& a = args[j];
    run_thread<W>(a, a.cached ? batch_xcd_block(r, b) : b - r.start + r.first, tid);
}

}  // namespace rr
