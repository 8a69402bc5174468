// The wide-row kernel (vertical window 1, wide horizontal windows), one image and
// batch forms.
#include "morph_device.h"

namespace morph {

// NTS: non-temporal destination stores (plain where a later launch reads the
// destination again: TileJob::keep)
template <typename T, bool MAXOP, bool AL, bool NTS>
__global__ __launch_bounds__(NT) void rows_kernel(TileJob J)
{
    const int units = J.tiles_x * J.tiles_y;
    const int u = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (u >= units) return; // the whole wave leaves
    __shared__ __align__(16) uint32_t lds[4 * kRowsWaveLdsDwords];
    uint32_t *wl = lds + (threadIdx.x >> 6) * kRowsWaveLdsDwords;
    rows_body<T, MAXOP, AL, NTS>(J, u, wl);
}

template <bool NTS> static TileKernelFn pick_rows_kernel_n(const TileJob &j)
{
    const bool al = rows_aligned(j);
    if (j.dtype == 0) {
        if (j.op) return al ? rows_kernel<uint8_t, true, true, NTS> : rows_kernel<uint8_t, true, false, NTS>;
        return al ? rows_kernel<uint8_t, false, true, NTS> : rows_kernel<uint8_t, false, false, NTS>;
    }
    if (j.op) return al ? rows_kernel<uint16_t, true, true, NTS> : rows_kernel<uint16_t, true, false, NTS>;
    return al ? rows_kernel<uint16_t, false, true, NTS> : rows_kernel<uint16_t, false, false, NTS>;
}

static TileKernelFn pick_rows_kernel(const TileJob &j)
{
    return j.keep ? pick_rows_kernel_n<false>(j) : pick_rows_kernel_n<true>(j);
}

// The batch form of the wide-row kernel: one wave per unit, four per workgroup.
template <typename T, bool AL>
__global__ __launch_bounds__(NT) void batch_rows_kernel(BatchTables bt)
{
    const int t = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (t >= bt.n_tiles) return; // the whole wave leaves
    const int jb = bt.tile_job[t];
    const TileJob J = bt.jobs[jb];
    const int u = (int)(t - bt.tile_start[jb]);
    __shared__ __align__(16) uint32_t lds[4 * kRowsWaveLdsDwords];
    uint32_t *wl = lds + (threadIdx.x >> 6) * kRowsWaveLdsDwords;
    if (J.op) rows_body<T, true, AL, false>(J, u, wl);
    else rows_body<T, false, AL, false>(J, u, wl);
}


hipError_t launch_rows_kernel(const TileJob &job, hipStream_t stream)
{
    const int units = job.tiles_x * job.tiles_y;
    hipLaunchKernelGGL(pick_rows_kernel(job), dim3((units + 3) / 4), dim3(NT), 0, stream, job);
    return hipGetLastError();
}

hipError_t launch_batch_rows(const BatchTables &t, int dtype, bool aligned, int grid,
                             hipStream_t stream)
{
    typedef void (*BatchFn)(BatchTables);
    const BatchFn fn = dtype == 0 ? (aligned ? batch_rows_kernel<uint8_t, true> : batch_rows_kernel<uint8_t, false>)
                                  : (aligned ? batch_rows_kernel<uint16_t, true> : batch_rows_kernel<uint16_t, false>);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), 0, stream, t);
    return hipGetLastError();
}

} // namespace morph
