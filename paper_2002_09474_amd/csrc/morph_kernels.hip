// Fused separable erosion / dilation kernels for gfx950 (CDNA4).
//
// The method (Limonova et al., arXiv:2002.09474): a rectangle is separable, so the
// w_x-by-w_y min/max is a vertical 1-D pass of w_y followed by a horizontal 1-D pass
// of w_x (§1, §5).  Each pass is either a direct sliding window ("linear", §5.1.2 and
// §5.2.2) or van Herk/Gil-Werman (vHGW) prefix/suffix extrema over blocks of w
// (§5.1.1, §5.2.1).  The paper runs each pass over the whole image with NEON and
// turns the row-direction pass into a column pass by transposing (§4, §5.2.1);
// here both passes run inside one workgroup on one output tile:
//
//   1. vertical pass: each work unit owns four adjacent columns and reads the
//      image rows straight from global memory (coalesced across the wave, with the
//      out-of-image identity applied while loading), and writes the tile's
//      intermediate rows into LDS;
//   2. horizontal pass: each work unit owns a pair of tile rows and walks along
//      them in LDS;
//   3. store: coalesced row stores of the finished tile.
//
// Arithmetic is on packed pairs of 16-bit lanes (v_pk_min_u16 / v_pk_max_u16) for
// both element types: uint8 pixels are widened on load and narrowed on store.  The
// LDS intermediate is kept in "row-pair" layout: dword (p, c) holds rows 2p (low
// half) and 2p+1 (high half) of column c, so the horizontal pass also works on two
// rows per instruction.  Converting between the vertical pass's column pairs and
// this layout is a 2x2 transpose of 16-bit elements (one v_perm_b32 per dword),
// the role the paper gives to VTRN (§4).
//
// vHGW in a pass of window w over a line of L = n + w - 1 inputs (n outputs): blocks
// of w start at input 0; g is the running extremum from each block start, h the
// running extremum to each block end, and output s = op(h[s], g[s + w - 1]).  Work
// units are (line group, block): phase F writes g shifted by w - 1 into the output
// slot it pairs with; phase B walks each block backwards, forms h on the fly and
// combines it in place.  Per pixel that is three min/max ops whatever w is.
#include "morph_internal.h"

namespace morph {

constexpr int NT = kThreads;
constexpr int DMAX = kDirectMax;
constexpr int KV = 8; // output rows per direct vertical work unit
constexpr int KH = 8; // output columns per direct horizontal work unit

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

template <bool MAXOP>
__device__ __forceinline__ uint32_t pk(uint32_t a, uint32_t b)
{
    u16x2 x = __builtin_bit_cast(u16x2, a), y = __builtin_bit_cast(u16x2, b);
    u16x2 r = MAXOP ? __builtin_elementwise_max(x, y) : __builtin_elementwise_min(x, y);
    return __builtin_bit_cast(uint32_t, r);
}

// v_perm_b32 selectors.  perm(hi, lo, sel) picks bytes of the 64-bit value {hi, lo}
// (lo = bytes 0-3, hi = bytes 4-7); selector byte 0x0c yields 0.
#define SEL_LO16_PAIR 0x05040100u // (lo.lo16, hi.lo16)
#define SEL_HI16_PAIR 0x07060302u // (lo.hi16, hi.hi16)
#define SEL_U8_01 0x0c010c00u     // widen bytes 0,1 of lo to two u16
#define SEL_U8_23 0x0c030c02u     // widen bytes 2,3 of lo to two u16
#define SEL_NARROW 0x06040200u    // low bytes of lo's and hi's u16 lanes -> 4 bytes

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ uint32_t load_u32(uintptr_t a) { return *(const uint32_t *)a; }

// Replace the 16-bit lanes of pixels outside [0, W) by the identity.
__device__ __forceinline__ void mask_quad(int gx, int W, uint32_t id, uint32_t &p01,
                                          uint32_t &p23)
{
    uint32_t m01 = ((unsigned)gx < (unsigned)W ? 0x0000ffffu : 0u) |
                   ((unsigned)(gx + 1) < (unsigned)W ? 0xffff0000u : 0u);
    uint32_t m23 = ((unsigned)(gx + 2) < (unsigned)W ? 0x0000ffffu : 0u) |
                   ((unsigned)(gx + 3) < (unsigned)W ? 0xffff0000u : 0u);
    p01 = (p01 & m01) | (id & ~m01);
    p23 = (p23 & m23) | (id & ~m23);
}

// Four consecutive pixels of one image row (row = address of its first pixel),
// starting at column gx (which may be negative or past the end), as two packed
// u16 pairs.  Only dwords that hold at least one byte of the row are read, so no
// read leaves the 4-byte granules the row occupies.
template <typename T> struct Px;

template <> struct Px<uint8_t> {
    static constexpr uint32_t maxv = 255u;
    static __device__ __forceinline__ void load(const uint8_t *row, int gx, int W, uint32_t id,
                                                uint32_t &p01, uint32_t &p23)
    {
        const uintptr_t lo = (uintptr_t)row, hi = lo + (uintptr_t)W;
        const uintptr_t ba = lo + (intptr_t)gx;
        const bool inside = gx >= 0 && gx + 4 <= W;
        uint32_t d;
        if (inside && (ba & 3u) == 0) {
            d = load_u32(ba);
        } else {
            const uintptr_t a0 = ba & ~(uintptr_t)3;
            uint32_t d0 = (a0 + 4 > lo && a0 < hi) ? load_u32(a0) : 0u;
            uint32_t d1 = (a0 + 8 > lo && a0 + 4 < hi) ? load_u32(a0 + 4) : 0u;
            d = __builtin_amdgcn_alignbyte(d1, d0, (uint32_t)(ba & 3u));
        }
        p01 = perm(0u, d, SEL_U8_01);
        p23 = perm(0u, d, SEL_U8_23);
        if (!inside) mask_quad(gx, W, id, p01, p23);
    }
    // Store pixels gx .. gx+3 (gx >= 0) of which those < W are written.
    static __device__ __forceinline__ void store(uint8_t *row, int gx, int W, uint32_t p01,
                                                 uint32_t p23)
    {
        const uintptr_t ba = (uintptr_t)row + gx;
        const uint32_t d = perm(p23, p01, SEL_NARROW);
        if (gx + 4 <= W && (ba & 3u) == 0) {
            *(uint32_t *)ba = d;
        } else {
            uint8_t *b = (uint8_t *)ba;
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (gx + j < W) b[j] = (uint8_t)(d >> (8 * j));
        }
    }
};

template <> struct Px<uint16_t> {
    static constexpr uint32_t maxv = 65535u;
    static __device__ __forceinline__ void load(const uint8_t *row, int gx, int W, uint32_t id,
                                                uint32_t &p01, uint32_t &p23)
    {
        const uintptr_t lo = (uintptr_t)row, hi = lo + 2 * (uintptr_t)W;
        const uintptr_t ba = lo + 2 * (intptr_t)gx;
        const bool inside = gx >= 0 && gx + 4 <= W;
        if (inside && (ba & 3u) == 0) {
            p01 = load_u32(ba);
            p23 = load_u32(ba + 4);
        } else {
            const uintptr_t a0 = ba & ~(uintptr_t)3;
            uint32_t d0 = (a0 + 4 > lo && a0 < hi) ? load_u32(a0) : 0u;
            uint32_t d1 = (a0 + 8 > lo && a0 + 4 < hi) ? load_u32(a0 + 4) : 0u;
            uint32_t d2 = (a0 + 12 > lo && a0 + 8 < hi) ? load_u32(a0 + 8) : 0u;
            const uint32_t sh = (uint32_t)(ba & 3u);
            p01 = __builtin_amdgcn_alignbyte(d1, d0, sh);
            p23 = __builtin_amdgcn_alignbyte(d2, d1, sh);
        }
        if (!inside) mask_quad(gx, W, id, p01, p23);
    }
    static __device__ __forceinline__ void store(uint8_t *row, int gx, int W, uint32_t p01,
                                                 uint32_t p23)
    {
        const uintptr_t ba = (uintptr_t)row + 2 * (uintptr_t)gx;
        if (gx + 4 <= W && (ba & 3u) == 0) {
            *(uint32_t *)ba = p01;
            *(uint32_t *)(ba + 4) = p23;
        } else {
            uint16_t *b = (uint16_t *)ba;
            const uint32_t v[2] = {p01, p23};
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (gx + j < W) b[j] = (uint16_t)(v[j >> 1] >> (16 * (j & 1)));
        }
    }
};

// One tile row of four columns into the row-pair LDS layout (16-bit stores, so two
// work units may fill the two halves of the same dwords).
__device__ __forceinline__ void put_row(uint32_t *L, int S, int s, int c, uint32_t x01,
                                        uint32_t x23)
{
    uint16_t *b = (uint16_t *)(L + (s >> 1) * S + c) + (s & 1);
    b[0] = (uint16_t)x01;
    b[2] = (uint16_t)(x01 >> 16);
    b[4] = (uint16_t)x23;
    b[6] = (uint16_t)(x23 >> 16);
}

__device__ __forceinline__ void get_row(const uint32_t *L, int S, int s, int c, uint32_t &x01,
                                        uint32_t &x23)
{
    const uint16_t *b = (const uint16_t *)(L + (s >> 1) * S + c) + (s & 1);
    x01 = (uint32_t)b[0] | ((uint32_t)b[2] << 16);
    x23 = (uint32_t)b[4] | ((uint32_t)b[6] << 16);
}

template <typename T, bool MAXOP, int VM, int HM>
__device__ __forceinline__ void tile_body(const TileJob &J, int tile, uint32_t *lds)
{
    const int tid = threadIdx.x;
    const int tx = tile % J.tiles_x, ty = tile / J.tiles_x;
    const int x0 = tx * J.TW, y0 = ty * J.TB;
    const int out_w = min(J.TW, J.W - x0), out_h = min(J.TB, J.H - y0);
    const int wx = J.wx, wy = J.wy;
    const int IW = out_w + wx - 1; // tile input columns
    const int cx0 = x0 - J.ax, cy0 = y0 - J.ay;
    const int SA = J.SA, SB = J.SB;
    uint32_t *A = lds;                    // [TB/2][SA]: vertical-pass output (row pairs)
    uint32_t *B = lds + (J.TB >> 1) * SA; // [TB/2][SB]: g of the horizontal pass / its output
    const uint32_t id = MAXOP ? 0u : (Px<T>::maxv | (Px<T>::maxv << 16));
    const uint8_t *src = J.src;
    const int H = J.H, W = J.W;
    const int64_t pitch = J.pitch;
    const int NQ = (IW + 3) >> 2; // column quads of the tile input

    // input row `pos` of the tile (image row cy0 + pos), quad q
    auto ld = [&](int pos, int q, uint32_t &a, uint32_t &b) {
        const int gy = cy0 + pos;
        if (gy >= 0 && gy < H)
            Px<T>::load(src + (int64_t)gy * pitch, cx0 + 4 * q, W, id, a, b);
        else {
            a = id;
            b = id;
        }
    };

    // ---------------- vertical pass: A[rows 0..out_h) x [cols 0..IW) ----------------
    if constexpr (VM == PASS_DIRECT) {
        // Sliding window over KV + wy - 1 rows held in registers (direct method);
        // wy == 1 is a plain load.
        const int NKV = (out_h + KV - 1) / KV;
        for (int u = tid; u < NQ * NKV; u += NT) {
            const int q = u % NQ, s0 = (u / NQ) * KV;
            uint32_t r01[KV + DMAX - 1], r23[KV + DMAX - 1];
#pragma unroll
            for (int j = 0; j < KV + DMAX - 1; j++) {
                if (j < KV + wy - 1)
                    ld(s0 + j, q, r01[j], r23[j]);
                else
                    r01[j] = r23[j] = id;
            }
#pragma unroll
            for (int m = 0; m < KV; m += 2) {
                if (s0 + m >= out_h) break;
                uint32_t a01 = r01[m], a23 = r23[m], b01 = r01[m + 1], b23 = r23[m + 1];
#pragma unroll
                for (int j = 1; j < DMAX; j++) {
                    if (j < wy) {
                        a01 = pk<MAXOP>(a01, r01[m + j]);
                        a23 = pk<MAXOP>(a23, r23[m + j]);
                        b01 = pk<MAXOP>(b01, r01[m + 1 + j]);
                        b23 = pk<MAXOP>(b23, r23[m + 1 + j]);
                    }
                }
                uint32_t *d = A + ((s0 + m) >> 1) * SA + 4 * q;
                d[0] = perm(b01, a01, SEL_LO16_PAIR);
                d[1] = perm(b01, a01, SEL_HI16_PAIR);
                d[2] = perm(b23, a23, SEL_LO16_PAIR);
                d[3] = perm(b23, a23, SEL_HI16_PAIR);
            }
        }
    } else {
        // vHGW along y.  Phase F: g over each block of wy input rows, stored in the
        // output row it pairs with (s = i - wy + 1).
        const int NBF = (out_h + wy - 1 + wy - 1) / wy;
        for (int u = tid; u < NQ * NBF; u += NT) {
            const int q = u % NQ, i0 = (u / NQ) * wy;
            const int i1 = min(i0 + wy, out_h + wy - 1);
            uint32_t g01 = id, g23 = id;
            for (int i = i0; i < i1; i++) {
                uint32_t v01, v23;
                ld(i, q, v01, v23);
                g01 = pk<MAXOP>(g01, v01);
                g23 = pk<MAXOP>(g23, v23);
                const int s = i - wy + 1;
                if (s >= 0) put_row(A, SA, s, 4 * q, g01, g23);
            }
        }
        __syncthreads();
        // Phase B: walk each block backwards; h[s] = op of rows s .. block end,
        // out[s] = op(h[s], g[s + wy - 1]).
        const int NBB = (out_h + wy - 1) / wy;
        for (int u = tid; u < NQ * NBB; u += NT) {
            const int q = u % NQ, i0 = (u / NQ) * wy;
            uint32_t h01 = id, h23 = id;
            for (int i = i0 + wy - 1; i >= i0; i--) {
                uint32_t v01, v23;
                ld(i, q, v01, v23);
                h01 = pk<MAXOP>(h01, v01);
                h23 = pk<MAXOP>(h23, v23);
                if (i < out_h) {
                    uint32_t g01, g23;
                    get_row(A, SA, i, 4 * q, g01, g23);
                    put_row(A, SA, i, 4 * q, pk<MAXOP>(h01, g01), pk<MAXOP>(h23, g23));
                }
            }
        }
    }
    __syncthreads();

    // ---------------- horizontal pass over row pairs ----------------
    const int NP = (out_h + 1) >> 1;
    if constexpr (HM == PASS_DIRECT) {
        const int NKH = (out_w + KH - 1) / KH;
        for (int u = tid; u < NP * NKH; u += NT) {
            const int p = u % NP, c0 = (u / NP) * KH;
            const uint32_t *a = A + p * SA;
            uint32_t r[KH + DMAX - 1];
#pragma unroll
            for (int j = 0; j < KH + DMAX - 1; j++)
                r[j] = (j < KH + wx - 1 && c0 + j < IW) ? a[c0 + j] : id;
#pragma unroll
            for (int m = 0; m < KH; m++) {
                uint32_t acc = r[m];
#pragma unroll
                for (int j = 1; j < DMAX; j++)
                    if (j < wx) acc = pk<MAXOP>(acc, r[m + j]);
                if (c0 + m < out_w) B[p * SB + c0 + m] = acc;
            }
        }
        __syncthreads();
    } else if constexpr (HM == PASS_VHGW) {
        const int NBF = (IW + wx - 1) / wx;
        for (int u = tid; u < NP * NBF; u += NT) {
            const int p = u % NP, i0 = (u / NP) * wx;
            const int i1 = min(i0 + wx, IW);
            const uint32_t *a = A + p * SA;
            uint32_t *g = B + p * SB;
            uint32_t acc = id;
            for (int i = i0; i < i1; i++) {
                acc = pk<MAXOP>(acc, a[i]);
                const int s = i - wx + 1;
                if (s >= 0) g[s] = acc;
            }
        }
        __syncthreads();
        const int NBB = (out_w + wx - 1) / wx;
        for (int u = tid; u < NP * NBB; u += NT) {
            const int p = u % NP, i0 = (u / NP) * wx;
            uint32_t *a = A + p * SA;
            const uint32_t *g = B + p * SB;
            uint32_t h = id;
            for (int i = i0 + wx - 1; i >= i0; i--) {
                h = pk<MAXOP>(h, a[i]);
                if (i < out_w) a[i] = pk<MAXOP>(h, g[i]);
            }
        }
        __syncthreads();
    }

    // ---------------- store: row pairs back to rows ----------------
    const uint32_t *O = (HM == PASS_DIRECT) ? B : A;
    const int SO = (HM == PASS_DIRECT) ? SB : SA;
    const int NQo = (out_w + 3) >> 2;
    for (int u = tid; u < NQo * NP; u += NT) {
        const int q = u % NQo, p = u / NQo;
        const uint32_t *o = O + p * SO + 4 * q;
        const uint32_t c0 = o[0], c1 = o[1], c2 = o[2], c3 = o[3];
        const int y = y0 + 2 * p, x = x0 + 4 * q;
        uint8_t *row = J.dst + (int64_t)y * pitch;
        Px<T>::store(row, x, W, perm(c1, c0, SEL_LO16_PAIR), perm(c3, c2, SEL_LO16_PAIR));
        if (2 * p + 1 < out_h)
            Px<T>::store(row + pitch, x, W, perm(c1, c0, SEL_HI16_PAIR),
                         perm(c3, c2, SEL_HI16_PAIR));
    }
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  Give each
// XCD a contiguous run of tiles so that neighbouring tiles, whose halos overlap,
// share an L2.  A bijection on [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <typename T, bool MAXOP, int VM, int HM>
__global__ __launch_bounds__(NT) void tile_kernel(TileJob J)
{
    extern __shared__ uint32_t lds[];
    tile_body<T, MAXOP, VM, HM>(J, xcd_tile(blockIdx.x, gridDim.x), lds);
}

typedef void (*TileKernelFn)(TileJob);

template <typename T, bool MAXOP>
static TileKernelFn pick(int vm, int hm)
{
    if (vm == PASS_DIRECT) {
        if (hm == PASS_NONE) return tile_kernel<T, MAXOP, PASS_DIRECT, PASS_NONE>;
        if (hm == PASS_DIRECT) return tile_kernel<T, MAXOP, PASS_DIRECT, PASS_DIRECT>;
        return tile_kernel<T, MAXOP, PASS_DIRECT, PASS_VHGW>;
    }
    if (hm == PASS_NONE) return tile_kernel<T, MAXOP, PASS_VHGW, PASS_NONE>;
    if (hm == PASS_DIRECT) return tile_kernel<T, MAXOP, PASS_VHGW, PASS_DIRECT>;
    return tile_kernel<T, MAXOP, PASS_VHGW, PASS_VHGW>;
}

static TileKernelFn pick_kernel(const TileJob &j)
{
    if (j.dtype == 0)
        return j.op ? pick<uint8_t, true>(j.vm, j.hm) : pick<uint8_t, false>(j.vm, j.hm);
    return j.op ? pick<uint16_t, true>(j.vm, j.hm) : pick<uint16_t, false>(j.vm, j.hm);
}

hipError_t launch_tile_job(const TileJob &job, hipStream_t stream)
{
    TileKernelFn fn = pick_kernel(job);
    const int lds = lds_bytes(job);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)fn,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    const int grid = job.tiles_x * job.tiles_y;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, stream, job);
    return hipGetLastError();
}

// ---------------- persistent batch kernel ----------------
// Every workgroup takes tile indices from one atomic counter until the batch is
// exhausted; a tile index is mapped to its image by binary search over the prefix
// sums of tiles per image.  Every wave leaves the loop once the counter passes the
// tile count, so the grid always drains.
template <typename T, bool MAXOP>
__device__ void run_job_tile(const TileJob &J, int t, uint32_t *lds)
{
    if (J.vm == PASS_DIRECT) {
        if (J.hm == PASS_NONE) tile_body<T, MAXOP, PASS_DIRECT, PASS_NONE>(J, t, lds);
        else if (J.hm == PASS_DIRECT) tile_body<T, MAXOP, PASS_DIRECT, PASS_DIRECT>(J, t, lds);
        else tile_body<T, MAXOP, PASS_DIRECT, PASS_VHGW>(J, t, lds);
    } else {
        if (J.hm == PASS_NONE) tile_body<T, MAXOP, PASS_VHGW, PASS_NONE>(J, t, lds);
        else if (J.hm == PASS_DIRECT) tile_body<T, MAXOP, PASS_VHGW, PASS_DIRECT>(J, t, lds);
        else tile_body<T, MAXOP, PASS_VHGW, PASS_VHGW>(J, t, lds);
    }
}

__global__ __launch_bounds__(NT) void batch_kernel(BatchTables bt)
{
    extern __shared__ uint32_t lds[];
    __shared__ long long next_tile;
    for (;;) {
        if (threadIdx.x == 0) next_tile = (long long)atomicAdd(bt.counter, 1ull);
        __syncthreads();
        const long long t = next_tile;
        __syncthreads(); // everyone has read next_tile before thread 0 overwrites it
        if (t >= bt.n_tiles) break;
        int lo = 0, hi = bt.n_jobs - 1; // last job with tile_start <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (bt.tile_start[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const TileJob J = bt.jobs[lo];
        const int lt = (int)(t - bt.tile_start[lo]);
        if (J.dtype == 0) {
            if (J.op) run_job_tile<uint8_t, true>(J, lt, lds);
            else run_job_tile<uint8_t, false>(J, lt, lds);
        } else {
            if (J.op) run_job_tile<uint16_t, true>(J, lt, lds);
            else run_job_tile<uint16_t, false>(J, lt, lds);
        }
        __syncthreads(); // LDS is reused by the next tile
    }
}

int batch_kernel_max_lds() { return kMaxLdsBytes - 64; }

hipError_t launch_batch(const BatchTables &t, int grid, int lds, hipStream_t stream)
{
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)batch_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(NT), lds, stream, t);
    return hipGetLastError();
}

} // namespace morph
