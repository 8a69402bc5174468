// Single-pass opening and closing (§2: an opening is a dilation of an erosion,
// a closing an erosion of a dilation, both with the same rectangle and anchor).
//
// One workgroup produces a kOcTileH x kOcTileW output tile.  It reads the input
// region the two passes need -- the tile grown by 2(w - 1) along each axis -- into
// LDS once, runs the first operation's horizontal and vertical direct passes over
// the region the second operation needs (the tile grown by w - 1), then the second
// operation's two passes, and stores the tile.  The intermediate image never goes
// to HBM: sizeof(T) bytes read and written per pixel plus halos, against four
// per pixel when the two operations run as separate launches through a workspace.
//
// Border rule (Eq. (1) reads only in-image pixels): input pixels outside the image
// enter the first operation as its identity, and intermediate pixels whose
// position lies outside the image enter the second operation as the second
// operation's identity -- the intermediate image has exactly the image's extent.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "morph_internal.h"

namespace morph {
namespace {

constexpr int kOcThreads = 256;
constexpr int kOcLdsW = kOcTileW + 2 * (kOcMaxW - 1); // row stride of both LDS buffers
constexpr int kOcLdsH = kOcTileH + 2 * (kOcMaxW - 1);

template <bool IsMin>
__device__ __forceinline__ uint32_t pick(uint32_t a, uint32_t b)
{
    return IsMin ? (a < b ? a : b) : (a > b ? a : b);
}

// Calls fn(std::integral_constant<int, w>) for 1 <= w <= kOcMaxW, so that a pass's
// per-tap loop has a compile-time trip count and unrolls (no loop control per pixel).
template <typename Fn>
__device__ __forceinline__ void with_window(int w, Fn &&fn)
{
    switch (w) {
#define OC_CASE(n)                                                                            \
    case n: fn(std::integral_constant<int, n>{}); break;
        OC_CASE(1) OC_CASE(2) OC_CASE(3) OC_CASE(4) OC_CASE(5) OC_CASE(6) OC_CASE(7) OC_CASE(8)
        OC_CASE(9) OC_CASE(10) OC_CASE(11) OC_CASE(12) OC_CASE(13) OC_CASE(14) OC_CASE(15)
        OC_CASE(16)
#undef OC_CASE
    default: break;
    }
}
static_assert(kOcMaxW == 16, "with_window covers windows 1..16");

// FirstMin: the first operation is an erosion (opening), else a dilation (closing).
template <typename T, bool FirstMin>
__global__ __launch_bounds__(kOcThreads) void openclose_kernel(const uint8_t *__restrict__ src,
                                                               uint8_t *__restrict__ dst, int H,
                                                               int W, int64_t pitch, int wx,
                                                               int wy, int ax, int ay, int tiles_x)
{
    __shared__ T A[kOcLdsH * kOcLdsW];
    __shared__ T B[kOcLdsH * kOcLdsW];
    constexpr uint32_t kMax = (uint32_t)(T)~(T)0;
    constexpr uint32_t id1 = FirstMin ? kMax : 0u; // identity of the first operation
    constexpr uint32_t id2 = FirstMin ? 0u : kMax; // identity of the second

    const int tile = blockIdx.x;
    const int y0 = (tile / tiles_x) * kOcTileH;
    const int x0 = (tile % tiles_x) * kOcTileW;
    const int cx = threadIdx.x % 128;
    const int ry = threadIdx.x / 128;
    constexpr int kRowStep = kOcThreads / 128;

    // 1. input region: rows y0 - 2ay .., columns x0 - 2ax .., identity outside.
    // Each thread loads kLoadRows rows of a column with no branch around the loads
    // (the address clamped into the image, the identity selected afterwards), so
    // that all of them are in flight before the first store to LDS.
    const int in_h = kOcTileH + 2 * (wy - 1), in_w = kOcTileW + 2 * (wx - 1);
    constexpr int kLoadRows = 8;
    for (int rb = ry; rb < in_h; rb += kRowStep * kLoadRows)
        for (int c = cx; c < in_w; c += 128) {
            const int gx = x0 - 2 * ax + c;
            const bool col_in = gx >= 0 && gx < W;
            const int gxc = min(max(gx, 0), W - 1);
            T v[kLoadRows];
#pragma unroll
            for (int k = 0; k < kLoadRows; ++k) {
                const int gy = y0 - 2 * ay + rb + k * kRowStep;
                const int gyc = min(max(gy, 0), H - 1);
                v[k] = ((const T *)(src + (int64_t)gyc * pitch))[gxc];
            }
#pragma unroll
            for (int k = 0; k < kLoadRows; ++k) {
                const int r = rb + k * kRowStep;
                const int gy = y0 - 2 * ay + r;
                if (r < in_h) A[r * kOcLdsW + c] = (col_in && gy >= 0 && gy < H) ? v[k] : (T)id1;
            }
        }
    __syncthreads();

    // 2. first operation, horizontal: B[r][c] = op1 of A[r][c .. c + wx - 1]
    const int h1_w = kOcTileW + wx - 1;
    with_window(wx, [&](auto n) {
        constexpr int N = decltype(n)::value;
        for (int r = ry; r < in_h; r += kRowStep)
            for (int c = cx; c < h1_w; c += 128) {
                const T *a = &A[r * kOcLdsW + c];
                uint32_t v = a[0];
#pragma unroll
                for (int j = 1; j < N; ++j) v = pick<FirstMin>(v, (uint32_t)a[j]);
                B[r * kOcLdsW + c] = (T)v;
            }
    });
    __syncthreads();

    // 3. first operation, vertical, into A: the intermediate image at rows
    // y0 - ay + r, columns x0 - ax + c; positions outside the image take the
    // second operation's identity
    const int mid_h = kOcTileH + wy - 1;
    with_window(wy, [&](auto n) {
        constexpr int N = decltype(n)::value;
        for (int r = ry; r < mid_h; r += kRowStep) {
            const int gy = y0 - ay + r;
            const bool row_in = gy >= 0 && gy < H;
            for (int c = cx; c < h1_w; c += 128) {
                const int gx = x0 - ax + c;
                const T *b = &B[r * kOcLdsW + c];
                uint32_t v = b[0];
#pragma unroll
                for (int i = 1; i < N; ++i) v = pick<FirstMin>(v, (uint32_t)b[i * kOcLdsW]);
                A[r * kOcLdsW + c] = (T)((row_in && gx >= 0 && gx < W) ? v : id2);
            }
        }
    });
    __syncthreads();

    // 4. second operation, horizontal: B[r][c] = op2 of A[r][c .. c + wx - 1]
    with_window(wx, [&](auto n) {
        constexpr int N = decltype(n)::value;
        for (int r = ry; r < mid_h; r += kRowStep) {
            const T *a = &A[r * kOcLdsW + cx];
            uint32_t v = a[0];
#pragma unroll
            for (int j = 1; j < N; ++j) v = pick<!FirstMin>(v, (uint32_t)a[j]);
            B[r * kOcLdsW + cx] = (T)v;
        }
    });
    __syncthreads();

    // 5. second operation, vertical, to the output tile
    const int gx = x0 + cx;
    if (gx >= W) return;
    with_window(wy, [&](auto n) {
        constexpr int N = decltype(n)::value;
        for (int r = ry; r < kOcTileH; r += kRowStep) {
            const int gy = y0 + r;
            if (gy >= H) break;
            const T *b = &B[r * kOcLdsW + cx];
            uint32_t v = b[0];
#pragma unroll
            for (int i = 1; i < N; ++i) v = pick<!FirstMin>(v, (uint32_t)b[i * kOcLdsW]);
            ((T *)(dst + (int64_t)gy * pitch))[gx] = (T)v;
        }
    });
}

static_assert(kOcTileW == 128, "one thread per output column of a tile row");

} // namespace

hipError_t launch_openclose(const void *src, void *dst, int H, int W, size_t pitch, int wx,
                            int wy, int ax, int ay, bool opening, int dtype, hipStream_t stream)
{
    if (wx < 1 || wy < 1 || wx > kOcMaxW || wy > kOcMaxW) return hipErrorInvalidValue;
    const int tiles_x = (W + kOcTileW - 1) / kOcTileW;
    const int tiles_y = (H + kOcTileH - 1) / kOcTileH;
    if ((int64_t)tiles_x * tiles_y > INT32_MAX) return hipErrorInvalidValue;
    typedef void (*Fn)(const uint8_t *, uint8_t *, int, int, int64_t, int, int, int, int, int);
    const Fn fn = dtype == 0 ? (opening ? openclose_kernel<uint8_t, true> : openclose_kernel<uint8_t, false>)
                             : (opening ? openclose_kernel<uint16_t, true> : openclose_kernel<uint16_t, false>);
    hipLaunchKernelGGL(fn, dim3(tiles_x * tiles_y), dim3(kOcThreads), 0, stream,
                       (const uint8_t *)src, (uint8_t *)dst, H, W, (int64_t)pitch, wx, wy, ax, ay,
                       tiles_x);
    return hipGetLastError();
}

} // namespace morph
