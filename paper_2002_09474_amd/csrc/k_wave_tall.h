// The direct-vertical wave kernel's tall form (vertical windows kDirectMax + 1 ..
// kDirectMaxTall, a longer ring of input rows kept as loaded): kernel templates,
// instantiated per element type in k_wave_tall_u8.hip and k_wave_tall_u16.hip.
#pragma once
#include "morph_device.h"

namespace morph {

template <typename T, bool MAXOP, bool AL>
__global__ __launch_bounds__(NT) void wave_tall_kernel(TileJob J)
{
    const int units = J.tiles_x * J.tiles_y;
    const int u = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (u >= units) return; // the whole wave leaves
    wave_body<T, MAXOP, AL, true>(J, u);
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
    if (J.op) wave_body<T, true, AL, true>(J, u);
    else wave_body<T, false, AL, true>(J, u);
}

template <typename T>
hipError_t launch_wave_tall_t(const TileJob &job, hipStream_t stream)
{
    const bool al = rows_aligned(job);
    const TileKernelFn fn = job.op ? (al ? wave_tall_kernel<T, true, true> : wave_tall_kernel<T, true, false>)
                                   : (al ? wave_tall_kernel<T, false, true> : wave_tall_kernel<T, false, false>);
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
