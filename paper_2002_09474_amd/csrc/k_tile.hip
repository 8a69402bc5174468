// The workgroup-tile kernel (the paper's two methods per pass through LDS), one
// image per launch and the persistent batch form.
#include "morph_device.h"

namespace morph {

template <typename T, bool MAXOP, bool AL>
__global__ __launch_bounds__(NT) void tile_kernel(TileJob J)
{
    extern __shared__ uint32_t lds[];
    tile_body<T, MAXOP, AL>(J, xcd_tile(blockIdx.x, gridDim.x), lds);
}

static TileKernelFn pick_kernel(const TileJob &j)
{
    const bool al = rows_aligned(j);
    if (j.dtype == 0) {
        if (j.op) return al ? tile_kernel<uint8_t, true, true> : tile_kernel<uint8_t, true, false>;
        return al ? tile_kernel<uint8_t, false, true> : tile_kernel<uint8_t, false, false>;
    }
    if (j.op) return al ? tile_kernel<uint16_t, true, true> : tile_kernel<uint16_t, true, false>;
    return al ? tile_kernel<uint16_t, false, true> : tile_kernel<uint16_t, false, false>;
}

// ---------------- persistent batch kernel ----------------
// One launch per group of jobs sharing the element type and row alignment; erosion
// and dilation jobs share it through the complement (tile_body's flip).  Every
// workgroup takes tile indices from one atomic counter (counter[0]) until the group
// is exhausted; a tile index is mapped to its image by binary search over the prefix
// sums of tiles per image.  Every wave leaves the loop once the counter passes the
// tile count, so the grid always drains.
template <typename T, bool AL>
__global__ __launch_bounds__(NT) void batch_kernel(BatchTables bt)
{
    extern __shared__ uint32_t lds[];
    __shared__ long long next_tile;
    constexpr uint32_t all_ones = Px<T>::maxv | (Px<T>::maxv << 16);
    if (threadIdx.x == 0) next_tile = (long long)atomicAdd(bt.counter, 1ull);
    __syncthreads();
    long long t = next_tile;
    while (t < bt.n_tiles) {
        __syncthreads(); // everyone has read next_tile
        // claim the following tile now, so the atomic's round trip overlaps this tile
        if (threadIdx.x == 0) next_tile = (long long)atomicAdd(bt.counter, 1ull);
        const int jb = bt.tile_job[t];
        const TileJob J = bt.jobs[jb];
        tile_body<T, false, AL>(J, (int)(t - bt.tile_start[jb]), lds, J.op ? all_ones : 0u);
        __syncthreads(); // LDS is reused by the next tile; next_tile is visible
        t = next_tile;
    }
    // The last workgroup to finish puts both counters back to zero for the next
    // launch (every other workgroup has left the loop by then), so a replayed graph
    // needs no separate reset.
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(bt.counter + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
            atomicExch(bt.counter, 0ull);
            atomicExch(bt.counter + 1, 0ull);
        }
    }
}


hipError_t launch_tile_kernel(const TileJob &job, hipStream_t stream)
{
    TileKernelFn fn = pick_kernel(job);
    const int lds = lds_bytes(job);
    hipError_t e = set_lds_limit((const void *)fn, lds);
    if (e != hipSuccess) return e;
    const int grid = job.tiles_x * job.tiles_y;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, stream, job);
    return hipGetLastError();
}

hipError_t launch_batch_tile(const BatchTables &t, int dtype, bool aligned, int grid, int lds,
                             hipStream_t stream)
{
    typedef void (*BatchFn)(BatchTables);
    const BatchFn fn = dtype == 0 ? (aligned ? batch_kernel<uint8_t, true> : batch_kernel<uint8_t, false>)
                                  : (aligned ? batch_kernel<uint16_t, true> : batch_kernel<uint16_t, false>);
    hipError_t e = set_lds_limit((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, stream, t);
    return hipGetLastError();
}

} // namespace morph
