// Image transpose for gfx950 (the operation of §4, whose use §1 gives: the row
// pass of a separable filter as a transpose, a column pass and a second
// transpose).  The paper builds 8x8.16 and 16x16.8 transposes out of NEON VTRN
// steps; here a 4x4-byte (or 2x2-halfword) block is transposed in a lane's
// registers with shifts and masks, and the rest of the reordering goes through
// LDS (whole images) or straight to global memory (independent small blocks).
//
// Whole images: a workgroup of 256 threads transposes a tile of 128 input rows
// by 128 bytes.  Each thread loads 16 bytes from each of 4 consecutive rows,
// transposes the four 4x4-byte (u8) or eight 2x2-halfword (u16) sub-blocks in
// registers and writes them to the transposed position of an LDS tile; the tile
// is then stored as 16-byte row segments of the destination.  Tiles that lie
// entirely inside the image with 16-byte aligned pointers and pitches take
// vector loads and stores; the others move one element at a time with bounds
// checks.  One read and one write of every element, 2 sizeof(T) bytes a pixel.
#include "morph_internal.h"

// The destination is written once and not read again by the launch: non-temporal
// stores keep it from displacing the source rows other workgroups still read from L2.
typedef uint32_t tr_u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void tr_store16(uint8_t *q, uint32_t a, uint32_t b, uint32_t c,
                                           uint32_t d)
{
    const tr_u32x4 v = {a, b, c, d};
    __builtin_nontemporal_store(v, reinterpret_cast<tr_u32x4 *>(q));
}
__device__ __forceinline__ void tr_store4(uint8_t *q, uint32_t v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<uint32_t *>(q));
}

namespace morph {
namespace {

constexpr int kTrRows = 128;  // input rows per tile (output columns)
constexpr int kTrBytes = 128; // input bytes per tile row

// dwords of an LDS row (one output row of the tile) and its stride: 128 rows of
// es bytes, plus two dwords so that rows start on different banks
template <typename T> __device__ constexpr int tr_out_dwords() { return kTrRows * (int)sizeof(T) / 4; }
template <typename T> __device__ constexpr int tr_stride() { return tr_out_dwords<T>() + 2; }

// 4x4 bytes: in[k] holds row k (byte c = column c); out[c] holds column c (byte
// k = row k)
__device__ inline void transpose4x4_u8(const uint32_t in[4], uint32_t out[4])
{
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int s = 8 * c;
        out[c] = ((in[0] >> s) & 0xffu) | (((in[1] >> s) & 0xffu) << 8) |
                 (((in[2] >> s) & 0xffu) << 16) | (((in[3] >> s) & 0xffu) << 24);
    }
}

// element e of the 16-byte segment held as 4 dwords
template <typename T> __device__ inline uint32_t seg_get(const uint32_t d[4], int e)
{
    const int b = e * (int)sizeof(T);
    return (d[b >> 2] >> (8 * (b & 3))) & (sizeof(T) == 1 ? 0xffu : 0xffffu);
}

template <typename T> __device__ inline void seg_put(uint32_t d[4], int e, uint32_t v)
{
    const int b = e * (int)sizeof(T);
    d[b >> 2] |= v << (8 * (b & 3));
}

template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const uint8_t *__restrict__ src,
                                                        uint8_t *__restrict__ dst, int H, int W,
                                                        int64_t spitch, int64_t dpitch,
                                                        int tiles_y, bool vec)
{
    constexpr int es = (int)sizeof(T);
    constexpr int R = kTrBytes / es;       // input columns per tile = output rows
    constexpr int S = tr_stride<T>();      // LDS row stride (dwords)
    constexpr int SEGS = tr_out_dwords<T>() / 4; // 16-byte segments per output row
    __shared__ uint32_t lds[R * S];

    const int t = threadIdx.x;
    const int tile_y = (int)(blockIdx.x % (unsigned)tiles_y);
    const int tile_x = (int)(blockIdx.x / (unsigned)tiles_y);
    const int y0 = tile_y * kTrRows; // first input row
    const int x0 = tile_x * R;       // first input column (element)
    const bool full = vec && y0 + kTrRows <= H && x0 + R <= W;

    // phase 1: rows 4 ty .. 4 ty + 3, bytes 16 tx .. 16 tx + 15 of the tile
    const int ty = t & 31, tx = t >> 5;
    uint32_t r[4][4];
    if (full) {
        const uint8_t *p = src + (int64_t)(y0 + 4 * ty) * spitch + (int64_t)x0 * es + 16 * tx;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint4 v = *reinterpret_cast<const uint4 *>(p + (int64_t)k * spitch);
            r[k][0] = v.x;
            r[k][1] = v.y;
            r[k][2] = v.z;
            r[k][3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            r[k][0] = r[k][1] = r[k][2] = r[k][3] = 0;
            const int y = y0 + 4 * ty + k;
            if (y >= H) continue;
            const T *row = reinterpret_cast<const T *>(src + (int64_t)y * spitch);
            for (int e = 0; e < 16 / es; e++) {
                const int x = x0 + tx * (16 / es) + e;
                if (x < W) seg_put<T>(r[k], e, (uint32_t)row[x]);
            }
        }
    }
    if constexpr (es == 1) {
        // dword j of the four rows: output rows 16 tx + 4 j + c, output dword ty
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t in[4] = {r[0][j], r[1][j], r[2][j], r[3][j]};
            uint32_t o[4];
            transpose4x4_u8(in, o);
#pragma unroll
            for (int c = 0; c < 4; c++) lds[(16 * tx + 4 * j + c) * S + ty] = o[c];
        }
    } else {
        // dword j holds columns 8 tx + 2 j (low half) and 8 tx + 2 j + 1 (high half);
        // output row gets the four rows' halfwords, two dwords at 2 ty
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint2 lo = make_uint2((r[0][j] & 0xffffu) | (r[1][j] << 16),
                                        (r[2][j] & 0xffffu) | (r[3][j] << 16));
            const uint2 hi = make_uint2((r[0][j] >> 16) | (r[1][j] & 0xffff0000u),
                                        (r[2][j] >> 16) | (r[3][j] & 0xffff0000u));
            *reinterpret_cast<uint2 *>(&lds[(8 * tx + 2 * j) * S + 2 * ty]) = lo;
            *reinterpret_cast<uint2 *>(&lds[(8 * tx + 2 * j + 1) * S + 2 * ty]) = hi;
        }
    }
    __syncthreads();

    // phase 2: R output rows of SEGS 16-byte segments, four per thread
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int g = t + 256 * i;
        const int row = g / SEGS, s = g % SEGS;
        const uint2 a = *reinterpret_cast<const uint2 *>(&lds[row * S + 4 * s]);
        const uint2 b = *reinterpret_cast<const uint2 *>(&lds[row * S + 4 * s + 2]);
        const int orow = x0 + row;
        if (full) {
            uint8_t *q = dst + (int64_t)orow * dpitch + (int64_t)y0 * es + 16 * s;
            tr_store16(q, a.x, a.y, b.x, b.y);
        } else if (orow < W) {
            const uint32_t d[4] = {a.x, a.y, b.x, b.y};
            T *q = reinterpret_cast<T *>(dst + (int64_t)orow * dpitch);
            for (int e = 0; e < 16 / es; e++) {
                const int y = y0 + s * (16 / es) + e;
                if (y < H) q[y] = (T)seg_get<T>(d, e);
            }
        }
    }
}

// n independent k x k blocks stored one after another, each row-major: 16x16 u8
// (256 bytes) or 8x8 u16 (128 bytes).  16 lanes a block, each lane moving one
// 4x4-byte (u8) or 2x2-halfword (u16) sub-block straight from and to global
// memory; all of a block's bytes are read and written by the same 16 lanes.
__global__ __launch_bounds__(256) void transpose_blocks_u8_kernel(const uint8_t *__restrict__ src,
                                                                  uint8_t *__restrict__ dst,
                                                                  int64_t n)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t blk = gid >> 4;
    if (blk >= n) return;
    const int l = (int)(gid & 15), qy = l >> 2, qx = l & 3;
    const uint8_t *p = src + blk * 256;
    uint8_t *q = dst + blk * 256;
    uint32_t in[4], o[4];
#pragma unroll
    for (int k = 0; k < 4; k++) in[k] = *reinterpret_cast<const uint32_t *>(p + (4 * qy + k) * 16 + 4 * qx);
    transpose4x4_u8(in, o);
#pragma unroll
    for (int c = 0; c < 4; c++) tr_store4(q + (4 * qx + c) * 16 + 4 * qy, o[c]);
}

__global__ __launch_bounds__(256) void transpose_blocks_u16_kernel(const uint8_t *__restrict__ src,
                                                                   uint8_t *__restrict__ dst,
                                                                   int64_t n)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t blk = gid >> 4;
    if (blk >= n) return;
    // rows 2 qy, 2 qy + 1; dword qx = columns 2 qx, 2 qx + 1
    const int l = (int)(gid & 15), qy = l >> 2, qx = l & 3;
    const uint8_t *p = src + blk * 128;
    uint8_t *q = dst + blk * 128;
    const uint32_t a = *reinterpret_cast<const uint32_t *>(p + (2 * qy) * 16 + 4 * qx);
    const uint32_t b = *reinterpret_cast<const uint32_t *>(p + (2 * qy + 1) * 16 + 4 * qx);
    tr_store4(q + (2 * qx) * 16 + 4 * qy, (a & 0xffffu) | (b << 16));
    tr_store4(q + (2 * qx + 1) * 16 + 4 * qy, (a >> 16) | (b & 0xffff0000u));
}

} // namespace

hipError_t launch_transpose(const void *src, void *dst, int H, int W, size_t spitch,
                            size_t dpitch, int dtype, hipStream_t stream)
{
    const int es = dtype ? 2 : 1;
    const int R = kTrBytes / es;
    const int64_t tiles_y = (H + kTrRows - 1) / kTrRows;
    const int64_t tiles_x = (W + R - 1) / R;
    const int64_t grid = tiles_y * tiles_x;
    if (grid <= 0) return hipSuccess;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    const bool vec = (((uintptr_t)src | (uintptr_t)dst | spitch | dpitch) & 15) == 0;
    const uint8_t *s = static_cast<const uint8_t *>(src);
    uint8_t *d = static_cast<uint8_t *>(dst);
    if (dtype)
        hipLaunchKernelGGL(transpose_kernel<uint16_t>, dim3((unsigned)grid), dim3(256), 0, stream,
                           s, d, H, W, (int64_t)spitch, (int64_t)dpitch, (int)tiles_y, vec);
    else
        hipLaunchKernelGGL(transpose_kernel<uint8_t>, dim3((unsigned)grid), dim3(256), 0, stream,
                           s, d, H, W, (int64_t)spitch, (int64_t)dpitch, (int)tiles_y, vec);
    return hipGetLastError();
}

hipError_t launch_transpose_blocks(const void *src, void *dst, int64_t n, int dtype,
                                   hipStream_t stream)
{
    const int64_t grid = (n * 16 + 255) / 256;
    if (grid <= 0) return hipSuccess;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    const uint8_t *s = static_cast<const uint8_t *>(src);
    uint8_t *d = static_cast<uint8_t *>(dst);
    if (dtype)
        hipLaunchKernelGGL(transpose_blocks_u16_kernel, dim3((unsigned)grid), dim3(256), 0, stream,
                           s, d, n);
    else
        hipLaunchKernelGGL(transpose_blocks_u8_kernel, dim3((unsigned)grid), dim3(256), 0, stream,
                           s, d, n);
    return hipGetLastError();
}

} // namespace morph
