// The direct-vertical wave kernel (registers only), its one-pass gradient and the
// clamped subtraction of the composed combinations, one image and batch forms.
#include "morph_device.h"

namespace morph {

// XV: the horizontal pass is the cross-lane vHGW (a plan that asks for vHGW along x).
// NTS: non-temporal destination stores (plain where a later launch reads the
// destination again: TileJob::keep)
template <typename T, bool MAXOP, bool AL, bool XV, bool NTS>
__global__ __launch_bounds__(NT) void wave_kernel(TileJob J)
{
    const int units = J.tiles_x * J.tiles_y;
    const int u = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (u >= units) return; // the whole wave leaves
    wave_body<T, MAXOP, AL, false, XV, NTS>(J, u);
}

template <bool XV, bool NTS>
static TileKernelFn pick_wave_kernel_x(const TileJob &j)
{
    const bool al = rows_aligned(j);
    if (j.dtype == 0) {
        if (j.op) return al ? wave_kernel<uint8_t, true, true, XV, NTS> : wave_kernel<uint8_t, true, false, XV, NTS>;
        return al ? wave_kernel<uint8_t, false, true, XV, NTS> : wave_kernel<uint8_t, false, false, XV, NTS>;
    }
    if (j.op) return al ? wave_kernel<uint16_t, true, true, XV, NTS> : wave_kernel<uint16_t, true, false, XV, NTS>;
    return al ? wave_kernel<uint16_t, false, true, XV, NTS> : wave_kernel<uint16_t, false, false, XV, NTS>;
}

static TileKernelFn pick_wave_kernel(const TileJob &j)
{
    if (j.hm == PASS_VHGW) return j.keep ? pick_wave_kernel_x<true, false>(j) : pick_wave_kernel_x<true, true>(j);
    return j.keep ? pick_wave_kernel_x<false, false>(j) : pick_wave_kernel_x<false, true>(j);
}

template <typename T>
__global__ __launch_bounds__(NT) void grad_kernel(TileJob J)
{
    const int units = J.tiles_x * J.tiles_y;
    const int u = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (u >= units) return; // the whole wave leaves
    grad_body<T>(J, u);
}

// p - q clamped at 0
template <typename T>
__device__ __forceinline__ T sub_clamped(T p, T q)
{
    return p > q ? (T)(p - q) : (T)0;
}

// dst = dst - a (REV false) or a - dst (REV true), clamped at 0, pixel by pixel,
// for the combinations composed from separate passes (gradient, top-hat,
// black-hat): block b covers 256 pixels of row b / nseg
template <typename T, bool REV>
__global__ __launch_bounds__(256) void sub_kernel(const uint8_t *a, uint8_t *dst, int W,
                                                  int64_t pitch, int nseg)
{
    const int y = blockIdx.x / nseg;
    const int x = (blockIdx.x - y * nseg) * 256 + (int)threadIdx.x;
    if (x >= W) return;
    const T v = *((const GLOBAL T *)(a + (int64_t)y * pitch) + x);
    GLOBAL T *d = (GLOBAL T *)(dst + (int64_t)y * pitch) + x;
    *d = REV ? sub_clamped<T>(v, *d) : sub_clamped<T>(*d, v);
}

hipError_t launch_gradient_job(const TileJob &job, hipStream_t stream)
{
    const int units = job.tiles_x * job.tiles_y;
    hipLaunchKernelGGL(job.dtype == 0 ? grad_kernel<uint8_t> : grad_kernel<uint16_t>,
                       dim3((units + 3) / 4), dim3(NT), 0, stream, job);
    return hipGetLastError();
}

// p - q clamped at 0 in each 16-bit half (v_pk_sub_u16 with clamp)
__device__ __forceinline__ uint32_t pk_sub_clamped(uint32_t p, uint32_t q)
{
    const u16x2 x = __builtin_bit_cast(u16x2, p), y = __builtin_bit_cast(u16x2, q);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(x, y));
}

// The same four bytes at a time, where a and dst have the same alignment: a thread
// takes one 4-byte-aligned dword of a dst row (four uint8 pixels, widened to two
// pairs, or two uint16 pixels) and subtracts with a clamp per pixel; dwords that
// reach past either end of the row go pixel by pixel.
template <typename T, bool REV>
__global__ __launch_bounds__(256) void sub4_kernel(const uint8_t *a, uint8_t *dst,
                                                   int64_t rowbytes, int64_t pitch, int nseg)
{
    const int y = blockIdx.x / nseg;
    const int64_t k = (int64_t)(blockIdx.x - y * nseg) * 256 + threadIdx.x;
    const uintptr_t rs = (uintptr_t)(dst + (int64_t)y * pitch), re = rs + (uintptr_t)rowbytes;
    const uintptr_t A = (rs & ~(uintptr_t)3) + 4 * (uintptr_t)k;
    if (A >= re) return;
    const intptr_t delta = (intptr_t)a - (intptr_t)dst;
    if (A >= rs && A + 4 <= re) {
        const uint32_t v = load_u32(A + delta);
        const uint32_t d = load_u32(A);
        const uint32_t p = REV ? v : d, q = REV ? d : v;
        if constexpr (sizeof(T) == 1) {
            const uint32_t lo = pk_sub_clamped(perm(0u, p, SEL_U8_01), perm(0u, q, SEL_U8_01));
            const uint32_t hi = pk_sub_clamped(perm(0u, p, SEL_U8_23), perm(0u, q, SEL_U8_23));
            store_u32(A, perm(hi, lo, SEL_NARROW));
        } else {
            store_u32(A, pk_sub_clamped(p, q));
        }
    } else {
        for (uintptr_t p = A > rs ? A : rs; p < A + 4 && p < re; p += sizeof(T)) {
            const T v = *(const GLOBAL T *)(p + delta);
            GLOBAL T *d = (GLOBAL T *)p;
            *d = REV ? sub_clamped<T>(v, *d) : sub_clamped<T>(*d, v);
        }
    }
}

hipError_t launch_subtract(const void *a, void *dst, int H, int W, size_t pitch, int dtype,
                           bool reverse, hipStream_t stream)
{
    if ((((uintptr_t)a - (uintptr_t)dst) & 3) == 0) {
        const int64_t rowbytes = (int64_t)W * (dtype ? 2 : 1);
        const int nseg = (int)(((rowbytes + 3) / 4 + 1 + 255) / 256);
        if ((int64_t)nseg * H > INT32_MAX) return hipErrorInvalidValue;
        typedef void (*Sub4Fn)(const uint8_t *, uint8_t *, int64_t, int64_t, int);
        const Sub4Fn fn = dtype == 0 ? (reverse ? sub4_kernel<uint8_t, true> : sub4_kernel<uint8_t, false>)
                                     : (reverse ? sub4_kernel<uint16_t, true> : sub4_kernel<uint16_t, false>);
        hipLaunchKernelGGL(fn, dim3(nseg * H), dim3(256), 0, stream, (const uint8_t *)a,
                           (uint8_t *)dst, rowbytes, (int64_t)pitch, nseg);
        return hipGetLastError();
    }
    const int nseg = (W + 255) / 256;
    if ((int64_t)nseg * H > INT32_MAX) return hipErrorInvalidValue;
    typedef void (*SubFn)(const uint8_t *, uint8_t *, int, int64_t, int);
    const SubFn fn = dtype == 0 ? (reverse ? sub_kernel<uint8_t, true> : sub_kernel<uint8_t, false>)
                                : (reverse ? sub_kernel<uint16_t, true> : sub_kernel<uint16_t, false>);
    hipLaunchKernelGGL(fn, dim3(nseg * H), dim3(256), 0, stream, (const uint8_t *)a,
                       (uint8_t *)dst, W, (int64_t)pitch, nseg);
    return hipGetLastError();
}


// The batch form of the wave kernel: one wave per unit of the group's tile table (four
// per workgroup), no persistence and no shared counter: units cost about the same,
// so the hardware's workgroup dispatch balances them, and a hundred thousand small
// units would serialise on one counter.
template <typename T, bool AL>
__global__ __launch_bounds__(NT) void batch_wave_kernel(BatchTables bt)
{
    const int t = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (t >= bt.n_tiles) return; // the whole wave leaves
    const int jb = bt.tile_job[t];
    const TileJob J = bt.jobs[jb];
    const int u = (int)(t - bt.tile_start[jb]);
    if (J.op) wave_body<T, true, AL, false, false, false>(J, u);
    else wave_body<T, false, AL, false, false, false>(J, u);
}


hipError_t launch_wave_kernel(const TileJob &job, hipStream_t stream)
{
    const int units = job.tiles_x * job.tiles_y;
    hipLaunchKernelGGL(pick_wave_kernel(job), dim3((units + 3) / 4), dim3(NT), 0, stream, job);
    return hipGetLastError();
}

hipError_t launch_batch_wave(const BatchTables &t, int dtype, bool aligned, int grid,
                             hipStream_t stream)
{
    typedef void (*BatchFn)(BatchTables);
    const BatchFn fn = dtype == 0 ? (aligned ? batch_wave_kernel<uint8_t, true> : batch_wave_kernel<uint8_t, false>)
                                  : (aligned ? batch_wave_kernel<uint16_t, true> : batch_wave_kernel<uint16_t, false>);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), 0, stream, t);
    return hipGetLastError();
}

} // namespace morph
