// rr_kernels.hip -- gfx950 kernels for N-D data rearrangement.
//
// Pure data movement, so no MFMA: every kernel is bound by HBM bandwidth and is
// shaped so that both its read side and its write side move whole 16-byte
// vectors along contiguous memory (the paper's requirement that "coalescing is
// maintained during both read and write", Sec. III.B).
//
//  * k_copy  -- identity after canonicalisation (the order [0 1 ... ] row of
//               Table 1, which the paper measures as a memcpy).
//  * k_run   -- permutes whose fastest axis stays fastest: every output run is
//               a contiguous input run, copied with vector loads and stores.
//  * k_select -- boxes that keep a strided fastest axis (one component of
//               interleaved records): whole records are read with 16-byte
//               vectors and the kept bytes packed in registers.
//  * k_weave -- interlace / de-interlace of 2-8 aligned sets of 1-8-byte
//               elements joined or split in registers, one 16-byte vector of
//               each set per thread; each wave swaps the joined vectors through
//               its own LDS region so both sides are read and written with
//               consecutive lanes at consecutive addresses.
//  * k_tile  -- a true transpose between the input's fastest axis (or axes) and
//               the output's fastest axis (or axes), staged through an LDS
//               tile (Sec. III.B's shared-memory tile; Sec. III.C's shared
//               buffer for interlace).  Each lane reads G rows of G elements
//               (G*U = up to 16 bytes) from LDS, transposes the GxG block in
//               registers, and writes G output vectors -- so LDS traffic is in
//               16-byte operations even for 1- and 2-byte elements.
#include <hip/hip_runtime.h>

#include "rr_device.hpp"
#include "rr_kernels.hpp"

namespace rr {

template <int W>
__global__ __launch_bounds__(NT) void k_copy(const CopyArgs a) {
    copy_thread<W>(a, blockIdx.x, gridDim.x, threadIdx.x);
}

// Each XCD takes a contiguous range of tiles (whole tile rows on large grids):
// a tile row's 16-byte side halos touch the 128-byte lines its neighbours load,
// and its halo rows the rows above and below, so neighbours share them in one L2
// instead of each XCD fetching them again.
template <int R, int SHAPE, int TH>
__global__ __launch_bounds__(NT) void k_stencil(const StencilArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[(TH + 2 * R) * ST_PITCH];
    const uint32_t tile = xcd_range(blockIdx.x, a.ntiles);
    stencil_load<R, TH>(a, tile, lds, threadIdx.x);
    __syncthreads();
    stencil_compute<R, SHAPE, TH>(a, tile, lds, threadIdx.x);
}

template <int W>
__global__ __launch_bounds__(NT) void k_gather(const GatherArgs a) {
    const uint32_t nbad = gather_thread<W>(a, blockIdx.x, gridDim.x, threadIdx.x);
    if (nbad && a.bad) atomicAdd(reinterpret_cast<unsigned long long*>(a.bad), (unsigned long long)nbad);
}

template <int W>
__global__ __launch_bounds__(NT) void k_run(const RunArgs a) {
    // runs that share input lines: each XCD takes a contiguous range of blocks,
    // so neighbouring runs meet in one L2
    run_thread<W>(a, a.cached ? xcd_range(blockIdx.x, gridDim.x) : blockIdx.x, threadIdx.x);
}

template <int R, int M>
__global__ __launch_bounds__(NT) void k_select(const SelectArgs a) {
    if (a.nax == 0) {   // one run: stage the workgroup's span through LDS
        __shared__ __attribute__((aligned(16))) uint8_t lds[NT * 16 * M];
        select_stage<R, M>(a, blockIdx.x, lds, threadIdx.x);
        __syncthreads();
        select_pack_store<R, M>(a, blockIdx.x, lds, threadIdx.x);
    } else {
        select_thread<R, M>(a, blockIdx.x, threadIdx.x);
    }
}

// Lanes of one wave exchange vectors through their own LDS region: LDS
// operations of a wave complete in issue order, so a wave-level barrier (which
// keeps the compiler from moving the reads above the writes) is enough.
template <int U, int N, bool DE, bool C, int R>
__device__ __forceinline__ void weave_block(const WeaveArgs& a, uint32_t block, uint64_t off, uint8_t* lds) {
    weave_stage<U, N, DE, C, R>(a, block, off, lds, threadIdx.x);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    weave_finish<U, N, DE, C, R>(a, block, off, lds, threadIdx.x);
}

// Workgroups [b * bpb, (b + 1) * bpb) cover batch b (one batch for rr_interlace).
template <int U, int N, bool DE, int R>
__global__ __launch_bounds__(NT) void k_weave(const WeaveArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[R * NT * N * 16];
    const uint32_t batch = blockIdx.x / a.bpb;
    const uint32_t block = blockIdx.x - batch * a.bpb;
    const uint64_t off = (uint64_t)batch * a.bstride;
    if (a.cached) weave_block<U, N, DE, true, R>(a, block, off, lds);
    else weave_block<U, N, DE, false, R>(a, block, off, lds);
}

template <int U, int G>
__global__ __launch_bounds__(NT) void k_tile(const TileArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const TileCtx t = tile_decode(a, block_to_tile(a, blockIdx.x));
    read_dispatch<U, G>(a, t, smem, threadIdx.x);
    __syncthreads();
    write_phase<U, G>(a, t, smem, threadIdx.x);
}

// ----------------------------------------------------------------- launch
template <int U, int G>
static hipError_t launch_tile_ug(const TileArgs& a, uint32_t grid, hipStream_t st) {
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tile<U, G>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    hipLaunchKernelGGL((k_tile<U, G>), dim3(grid), dim3(NT), a.lds_bytes, st, a);
    return hipGetLastError();
}

static hipError_t launch_tile(const TileArgs& a, uint32_t grid, hipStream_t st) {
    switch (a.unit * 100 + a.g) {
        case 101: return launch_tile_ug<1, 1>(a, grid, st);
        case 102: return launch_tile_ug<1, 2>(a, grid, st);
        case 104: return launch_tile_ug<1, 4>(a, grid, st);
        case 108: return launch_tile_ug<1, 8>(a, grid, st);
        case 116: return launch_tile_ug<1, 16>(a, grid, st);
        case 201: return launch_tile_ug<2, 1>(a, grid, st);
        case 202: return launch_tile_ug<2, 2>(a, grid, st);
        case 204: return launch_tile_ug<2, 4>(a, grid, st);
        case 208: return launch_tile_ug<2, 8>(a, grid, st);
        case 401: return launch_tile_ug<4, 1>(a, grid, st);
        case 402: return launch_tile_ug<4, 2>(a, grid, st);
        case 404: return launch_tile_ug<4, 4>(a, grid, st);
        case 801: return launch_tile_ug<8, 1>(a, grid, st);
        case 802: return launch_tile_ug<8, 2>(a, grid, st);
        case 1601: return launch_tile_ug<16, 1>(a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

template <int TH>
static hipError_t launch_stencil_th(const StencilArgs& a, hipStream_t st) {
    const dim3 g(a.ntiles), b(NT);
    switch (a.radius * 2 + a.shape) {
        case 2: hipLaunchKernelGGL((k_stencil<1, 0, TH>), g, b, 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_stencil<1, 1, TH>), g, b, 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_stencil<2, 0, TH>), g, b, 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_stencil<2, 1, TH>), g, b, 0, st, a); break;
        case 6: hipLaunchKernelGGL((k_stencil<3, 0, TH>), g, b, 0, st, a); break;
        case 7: hipLaunchKernelGGL((k_stencil<3, 1, TH>), g, b, 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_stencil<4, 0, TH>), g, b, 0, st, a); break;
        case 9: hipLaunchKernelGGL((k_stencil<4, 1, TH>), g, b, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stencil(const StencilArgs& a, hipStream_t st) {
    if (a.ntiles == 0) return hipSuccess;
    switch (a.th) {
        case 16: return launch_stencil_th<16>(a, st);
        case 32: return launch_stencil_th<32>(a, st);
        default: return hipErrorInvalidValue;
    }
}

template <int R>
static hipError_t launch_select_r(const SelectArgs& a, uint32_t grid, hipStream_t st) {
    switch (a.M) {
        case 2: hipLaunchKernelGGL((k_select<R, 2>), dim3(grid), dim3(NT), 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_select<R, 3>), dim3(grid), dim3(NT), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_select<R, 4>), dim3(grid), dim3(NT), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t launch_select(const SelectArgs& a, uint32_t grid, hipStream_t st) {
    switch (a.R) {
        case 1: return launch_select_r<1>(a, grid, st);
        case 2: return launch_select_r<2>(a, grid, st);
        case 4: return launch_select_r<4>(a, grid, st);
        case 8: return launch_select_r<8>(a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

// Two chunks per wave are built for up to four sets only (the planner's choice).
template <int U, int N>
static hipError_t launch_weave_un(const WeaveArgs& a, uint32_t grid, hipStream_t st) {
    if (a.chunks == 1) {
        if (a.de) hipLaunchKernelGGL((k_weave<U, N, true, 1>), dim3(grid), dim3(NT), 0, st, a);
        else hipLaunchKernelGGL((k_weave<U, N, false, 1>), dim3(grid), dim3(NT), 0, st, a);
        return hipGetLastError();
    }
    if constexpr (N <= 4) {
        if (a.chunks == 2) {
            if (a.de) hipLaunchKernelGGL((k_weave<U, N, true, 2>), dim3(grid), dim3(NT), 0, st, a);
            else hipLaunchKernelGGL((k_weave<U, N, false, 2>), dim3(grid), dim3(NT), 0, st, a);
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

template <int U>
static hipError_t launch_weave_u(const WeaveArgs& a, uint32_t grid, hipStream_t st) {
    switch (a.n) {
        case 2: return launch_weave_un<U, 2>(a, grid, st);
        case 3: return launch_weave_un<U, 3>(a, grid, st);
        case 4: return launch_weave_un<U, 4>(a, grid, st);
        case 5: return launch_weave_un<U, 5>(a, grid, st);
        case 6: return launch_weave_un<U, 6>(a, grid, st);
        case 7: return launch_weave_un<U, 7>(a, grid, st);
        case 8: return launch_weave_un<U, 8>(a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_weave(const WeaveArgs& a, uint32_t grid, hipStream_t st) {
    switch (a.unit) {
        case 1: return launch_weave_u<1>(a, grid, st);
        case 2: return launch_weave_u<2>(a, grid, st);
        case 4: return launch_weave_u<4>(a, grid, st);
        case 8: return launch_weave_u<8>(a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_plan(const Plan& p, hipStream_t st) {
    switch (p.kind) {
        case K_EMPTY:
            return hipSuccess;
        case K_COPY:
            switch (p.copy.wbytes) {
                case 16: hipLaunchKernelGGL(k_copy<16>, dim3(p.grid), dim3(NT), 0, st, p.copy); break;
                case 8: hipLaunchKernelGGL(k_copy<8>, dim3(p.grid), dim3(NT), 0, st, p.copy); break;
                case 4: hipLaunchKernelGGL(k_copy<4>, dim3(p.grid), dim3(NT), 0, st, p.copy); break;
                case 2: hipLaunchKernelGGL(k_copy<2>, dim3(p.grid), dim3(NT), 0, st, p.copy); break;
                default: hipLaunchKernelGGL(k_copy<1>, dim3(p.grid), dim3(NT), 0, st, p.copy); break;
            }
            return hipGetLastError();
        case K_RUN:
            switch (p.run.wbytes) {
                case 16: hipLaunchKernelGGL(k_run<16>, dim3(p.grid), dim3(NT), 0, st, p.run); break;
                case 8: hipLaunchKernelGGL(k_run<8>, dim3(p.grid), dim3(NT), 0, st, p.run); break;
                case 4: hipLaunchKernelGGL(k_run<4>, dim3(p.grid), dim3(NT), 0, st, p.run); break;
                case 2: hipLaunchKernelGGL(k_run<2>, dim3(p.grid), dim3(NT), 0, st, p.run); break;
                default: hipLaunchKernelGGL(k_run<1>, dim3(p.grid), dim3(NT), 0, st, p.run); break;
            }
            return hipGetLastError();
        case K_TILE:
            return launch_tile(p.tile, p.grid, st);
        case K_SELECT:
            return launch_select(p.select, p.grid, st);
        case K_WEAVE:
            return launch_weave(p.weave, p.grid, st);
        case K_GATHER:
            switch (p.gather.wbytes) {
                case 16: hipLaunchKernelGGL(k_gather<16>, dim3(p.grid), dim3(NT), 0, st, p.gather); break;
                case 8: hipLaunchKernelGGL(k_gather<8>, dim3(p.grid), dim3(NT), 0, st, p.gather); break;
                case 4: hipLaunchKernelGGL(k_gather<4>, dim3(p.grid), dim3(NT), 0, st, p.gather); break;
                case 2: hipLaunchKernelGGL(k_gather<2>, dim3(p.grid), dim3(NT), 0, st, p.gather); break;
                default: hipLaunchKernelGGL(k_gather<1>, dim3(p.grid), dim3(NT), 0, st, p.gather); break;
            }
            return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace rr
