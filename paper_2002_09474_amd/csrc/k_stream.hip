// The streaming kernel (vertical vHGW walking down the rows), one image and batch
// forms.
#include "morph_device.h"

namespace morph {

// XV: the horizontal pass is the cross-lane vHGW (a plan that asks for vHGW along x).
// NTS: non-temporal destination stores (plain where a later launch reads the
// destination again: TileJob::keep)
template <typename T, bool MAXOP, bool AL, bool RUNS, bool XV, bool NTS>
__global__ __launch_bounds__(64) void stream_kernel(TileJob J)
{
    extern __shared__ uint32_t lds[];
    stream_body<T, MAXOP, AL, RUNS, XV, NTS>(J, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <bool RUNS, bool XV, bool NTS>
static TileKernelFn pick_stream_kernel_v(const TileJob &j)
{
    const bool al = rows_aligned(j);
    if (j.dtype == 0) {
        if (j.op) return al ? stream_kernel<uint8_t, true, true, RUNS, XV, NTS> : stream_kernel<uint8_t, true, false, RUNS, XV, NTS>;
        return al ? stream_kernel<uint8_t, false, true, RUNS, XV, NTS> : stream_kernel<uint8_t, false, false, RUNS, XV, NTS>;
    }
    if (j.op) return al ? stream_kernel<uint16_t, true, true, RUNS, XV, NTS> : stream_kernel<uint16_t, true, false, RUNS, XV, NTS>;
    return al ? stream_kernel<uint16_t, false, true, RUNS, XV, NTS> : stream_kernel<uint16_t, false, false, RUNS, XV, NTS>;
}

static TileKernelFn pick_stream_kernel(const TileJob &j)
{
    const bool xv = j.hm == PASS_VHGW;
    if (j.keep) {
        if (stream_two_level(j.wy))
            return xv ? pick_stream_kernel_v<true, true, false>(j) : pick_stream_kernel_v<true, false, false>(j);
        return xv ? pick_stream_kernel_v<false, true, false>(j) : pick_stream_kernel_v<false, false, false>(j);
    }
    if (stream_two_level(j.wy))
        return xv ? pick_stream_kernel_v<true, true, true>(j) : pick_stream_kernel_v<true, false, true>(j);
    return xv ? pick_stream_kernel_v<false, true, true>(j) : pick_stream_kernel_v<false, false, true>(j);
}

// The batch form of the stream kernel: one single-wave workgroup per unit.
template <typename T, bool AL, bool RUNS>
__global__ __launch_bounds__(64) void batch_stream_kernel(BatchTables bt)
{
    extern __shared__ uint32_t lds[];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= bt.n_tiles) return;
    const int jb = bt.tile_job[t];
    const TileJob J = bt.jobs[jb];
    const int u = (int)(t - bt.tile_start[jb]);
    if (J.op) stream_body<T, true, AL, RUNS, false, false>(J, u, lds);
    else stream_body<T, false, AL, RUNS, false, false>(J, u, lds);
}


hipError_t launch_stream_kernel(const TileJob &job, hipStream_t stream)
{
    TileKernelFn fn = pick_stream_kernel(job);
    const int lds = lds_bytes(job);
    hipError_t e = set_lds_limit((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(job.tiles_x * job.tiles_y), dim3(64), lds, stream, job);
    return hipGetLastError();
}

hipError_t launch_batch_stream(const BatchTables &t, bool runs, int dtype, bool aligned, int grid,
                               int lds, hipStream_t stream)
{
    typedef void (*BatchFn)(BatchTables);
    BatchFn fn;
    if (runs)
        fn = dtype == 0 ? (aligned ? batch_stream_kernel<uint8_t, true, true> : batch_stream_kernel<uint8_t, false, true>)
                        : (aligned ? batch_stream_kernel<uint16_t, true, true> : batch_stream_kernel<uint16_t, false, true>);
    else
        fn = dtype == 0 ? (aligned ? batch_stream_kernel<uint8_t, true, false> : batch_stream_kernel<uint8_t, false, false>)
                        : (aligned ? batch_stream_kernel<uint16_t, true, false> : batch_stream_kernel<uint16_t, false, false>);
    hipError_t e = set_lds_limit((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(64), lds, stream, t);
    return hipGetLastError();
}

} // namespace morph
