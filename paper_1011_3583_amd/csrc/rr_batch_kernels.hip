// rr_batch_kernels.hip -- gfx950 kernels that run a whole batch group per launch.
//
// The same tile, run and copy bodies as the single-problem kernels
// (rr_device.hpp), reached through a per-group table of argument blocks: a
// workgroup finds its job by binary search over the prefix sums of the jobs'
// workgroup counts.  Kept in a file of its own so the two kernel sets compile
// in parallel.
#include <hip/hip_runtime.h>

#include "rr_device.hpp"
#include "rr_kernels.hpp"

namespace rr {

// Register budget of the batch tile kernels: eight waves per SIMD.  At the
// compiler's own choice the job lookups of a batch workgroup take these kernels
// a few scalar registers past the eight-wave limit (seven waves); held to eight
// they keep the excess in vector-register lanes, and the 4096-job batch ran
// 2-4 % faster.  The two largest micro-tiles and the 2-byte G = 1 kernel would
// spill vector registers to memory at that budget and keep the compiler's choice.
template <int U, int G>
constexpr int batch_tile_waves() { return (U == 1 && G == 16) || (U == 2 && (G == 8 || G == 1)) ? 1 : 8; }

// One launch per kernel family covers every job of a batch group; the
// workgroup index walks the concatenation of the jobs' own launch grids.

template <int U, int G>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(batch_tile_waves<U, G>(), 8)))
void k_batch_tile(const TileArgs* __restrict__ args, const uint32_t* __restrict__ prefix,
                  const EntryRange* __restrict__ ranges, uint32_t njobs, uint32_t total) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    for (uint32_t b = blockIdx.x; b < total; b += gridDim.x) {
        const uint32_t j = find_job(prefix, njobs, b);
        // the entry's record and the job's flags are loaded together: both
        // depend on j only
        const EntryRange r = ranges[j];
        const TileArgs& a = args[j];
        const TileCtx t = tile_decode(a, batch_block_to_tile(a.flags, r, b));
        read_dispatch<U, G>(a, t, smem, threadIdx.x);
        __syncthreads();
        write_phase<U, G>(a, t, smem, threadIdx.x);
        __syncthreads();
    }
}

template <int W>
__global__ __launch_bounds__(NT) void k_batch_run(const RunArgs* __restrict__ args,
                                                  const uint32_t* __restrict__ prefix,
                                                  const EntryRange* __restrict__ ranges, uint32_t njobs,
                                                  uint32_t total) {
    for (uint32_t b = blockIdx.x; b < total; b += gridDim.x)
        batch_run_block<W>(args, prefix, ranges, njobs, b, threadIdx.x);
}

template <int W>
__global__ __launch_bounds__(NT) void k_batch_copy(const CopyArgs* __restrict__ args,
                                                   const uint32_t* __restrict__ prefix,
                                                   const EntryRange* __restrict__ ranges, uint32_t njobs,
                                                   uint32_t total) {
    for (uint32_t b = blockIdx.x; b < total; b += gridDim.x)
        batch_copy_block<W>(args, prefix, ranges, njobs, b, threadIdx.x);
}

// ----------------------------------------------------------------- launch
template <int U, int G>
static hipError_t launch_batch_tile_ug(const BatchGroup& g, const uint8_t* table, uint32_t grid,
                                       hipStream_t st) {
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_tile<U, G>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    hipLaunchKernelGGL((k_batch_tile<U, G>), dim3(grid), dim3(NT), g.lds_bytes, st,
                       reinterpret_cast<const TileArgs*>(table + g.args_off),
                       reinterpret_cast<const uint32_t*>(table + g.prefix_off),
                       reinterpret_cast<const EntryRange*>(table + g.range_off), g.njobs, g.total_blocks);
    return hipGetLastError();
}

hipError_t launch_batch_group(const BatchGroup& g, const uint8_t* table, uint32_t grid, hipStream_t st) {
    if (g.total_blocks == 0) return hipSuccess;
    if (grid == 0 || grid > g.total_blocks) grid = g.total_blocks;
    const uint32_t* prefix = reinterpret_cast<const uint32_t*>(table + g.prefix_off);
    const EntryRange* ranges = reinterpret_cast<const EntryRange*>(table + g.range_off);
    if (g.kind == K_COPY) {
        const CopyArgs* args = reinterpret_cast<const CopyArgs*>(table + g.args_off);
        switch (g.variant) {
            case 16: hipLaunchKernelGGL(k_batch_copy<16>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
            case 8: hipLaunchKernelGGL(k_batch_copy<8>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
            case 4: hipLaunchKernelGGL(k_batch_copy<4>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
            case 2: hipLaunchKernelGGL(k_batch_copy<2>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
            default: hipLaunchKernelGGL(k_batch_copy<1>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
        }
        return hipGetLastError();
    }
    if (g.kind == K_RUN) {
        const RunArgs* args = reinterpret_cast<const RunArgs*>(table + g.args_off);
        switch (g.variant) {
            case 16: hipLaunchKernelGGL(k_batch_run<16>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
            case 8: hipLaunchKernelGGL(k_batch_run<8>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
            case 4: hipLaunchKernelGGL(k_batch_run<4>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
            case 2: hipLaunchKernelGGL(k_batch_run<2>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
            default: hipLaunchKernelGGL(k_batch_run<1>, dim3(grid), dim3(NT), 0, st, args, prefix, ranges, g.njobs, g.total_blocks); break;
        }
        return hipGetLastError();
    }
    switch (g.variant) {
        case 101: return launch_batch_tile_ug<1, 1>(g, table, grid, st);
        case 102: return launch_batch_tile_ug<1, 2>(g, table, grid, st);
        case 104: return launch_batch_tile_ug<1, 4>(g, table, grid, st);
        case 108: return launch_batch_tile_ug<1, 8>(g, table, grid, st);
        case 116: return launch_batch_tile_ug<1, 16>(g, table, grid, st);
        case 201: return launch_batch_tile_ug<2, 1>(g, table, grid, st);
        case 202: return launch_batch_tile_ug<2, 2>(g, table, grid, st);
        case 204: return launch_batch_tile_ug<2, 4>(g, table, grid, st);
        case 208: return launch_batch_tile_ug<2, 8>(g, table, grid, st);
        case 401: return launch_batch_tile_ug<4, 1>(g, table, grid, st);
        case 402: return launch_batch_tile_ug<4, 2>(g, table, grid, st);
        case 404: return launch_batch_tile_ug<4, 4>(g, table, grid, st);
        case 801: return launch_batch_tile_ug<8, 1>(g, table, grid, st);
        case 802: return launch_batch_tile_ug<8, 2>(g, table, grid, st);
        case 1601: return launch_batch_tile_ug<16, 1>(g, table, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rr
