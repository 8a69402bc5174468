// The direct-vertical wave kernel's tall form (vertical windows kDirectMax + 1 ..
// kDirectMaxTall, a longer ring of input rows kept as loaded): kernel templates,
// instantiated per element type in k_wave_tall_u8.hip and k_wave_tall_u16.hip.
#pragma once
#include "morph_device.h"

namespace morph {

// NTS: non-temporal destination stores (plain where a later launch reads the
// destination again: TileJob::keep)
template <typename T, bool MAXOP, bool AL, bool NTS>
__global__ __launch_bounds__(NT) void wave_tall_kernel(TileJob J)
{
    const int units = J.tiles_x * J.tiles_y;
    const int u = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (u >= units) return; // the whole wave leaves
    wave_body<T, MAXOP, AL, true, false, NTS>(J, u);
}

// Batch form: one wave per unit of the group's tile table, four per workgroup.
template <typename T, bool AL>
__global__ __launch_bounds__(NT) void batch_wave_tall_kernel(BatchTables bt)
{
    const int t = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (t >= bt.n_tiles) return; // the whole wave leaves
    const int jb = bt.tile_job[t];
    const TileJob J = bt.jobs[jb];
    const int u = (int)(t - bt.tile_start[jb]);
    if (J.op) wave_body<T, true, AL, true, false, false>(J, u);
    else wave_body<T, false, AL, true, false, false>(J, u);
}

template <typename T, bool NTS> static TileKernelFn pick_wave_tall(const TileJob &job)
{
    const bool al = rows_aligned(job);
    return job.op ? (al ? wave_tall_kernel<T, true, true, NTS> : wave_tall_kernel<T, true, false, NTS>)
                  : (al ? wave_tall_kernel<T, false, true, NTS> : wave_tall_kernel<T, false, false, NTS>);
}

template <typename T>
hipError_t launch_wave_tall_t(const TileJob &job, hipStream_t stream)
{
    const TileKernelFn fn = job.keep ? pick_wave_tall<T, false>(job) : pick_wave_tall<T, true>(job);
    const int units = job.tiles_x * job.tiles_y;
    hipLaunchKernelGGL(fn, dim3((units + 3) / 4), dim3(NT), 0, stream, job);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_wave_tall_t(const BatchTables &t, bool aligned, int grid,
                                    hipStream_t stream)
{
    typedef void (*BatchFn)(BatchTables);
    const BatchFn fn = aligned ? batch_wave_tall_kernel<T, true> : batch_wave_tall_kernel<T, false>;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), 0, stream, t);
    return hipGetLastError();
}

} // namespace morph
