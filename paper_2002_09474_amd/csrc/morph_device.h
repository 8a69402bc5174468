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
#pragma once
#include "morph_internal.h"

#include <type_traits>
#include <utility>

namespace morph {

constexpr int NT = kThreads;
constexpr int DMAX = kDirectMax;
constexpr int KV = 8; // output rows per direct vertical work unit
constexpr int KH = kDirectChunkX; // output columns per direct horizontal work unit

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

// Image memory is always device (global) memory: address it as such, so that the
// compiler emits global_* rather than flat_* accesses also where the pointer comes
// from a table in memory (the batch kernels).
#define GLOBAL __attribute__((address_space(1)))
// Word 3 of a raw (untyped, unswizzled) buffer resource on gfx9-family GPUs.
constexpr int kBufferWord3 = 0x00020000;
__device__ __forceinline__ uint32_t load_u32(uintptr_t a) { return *(const GLOBAL uint32_t *)a; }
// Single images' output pixels are written once and not read again by the launch:
// their stores are non-temporal (NTS), which leaves L2 to the input rows (4096x4096
// uint8 3x3 11.8 -> 9.6 us).  Batches keep plain stores (non-temporal ones made the
// 512-image batch 6% slower).  kStoreCpol: the non-temporal bit of a buffer store's
// cache-policy operand.
constexpr int kStoreCpol = 2;
template <bool NTS = true> __device__ __forceinline__ void store_u32(uintptr_t a, uint32_t v)
{
    if constexpr (NTS) __builtin_nontemporal_store(v, (GLOBAL uint32_t *)a);
    else *(GLOBAL uint32_t *)a = v;
}
template <bool NTS = true> __device__ __forceinline__ void store_u8(uintptr_t a, uint8_t v)
{
    if constexpr (NTS) __builtin_nontemporal_store(v, (GLOBAL uint8_t *)a);
    else *(GLOBAL uint8_t *)a = v;
}
template <bool NTS = true> __device__ __forceinline__ void store_u16(uintptr_t a, uint16_t v)
{
    if constexpr (NTS) __builtin_nontemporal_store(v, (GLOBAL uint16_t *)a);
    else *(GLOBAL uint16_t *)a = v;
}

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
    template <bool NTS = true>
    static __device__ __forceinline__ void store(uint8_t *row, int gx, int W, uint32_t p01,
                                                 uint32_t p23)
    {
        const uintptr_t ba = (uintptr_t)row + gx;
        const uint32_t d = perm(p23, p01, SEL_NARROW);
        if (gx + 4 <= W && (ba & 3u) == 0) {
            store_u32<NTS>(ba, d);
        } else {
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (gx + j < W) store_u8<NTS>(ba + j, (uint8_t)(d >> (8 * j)));
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
    template <bool NTS = true>
    static __device__ __forceinline__ void store(uint8_t *row, int gx, int W, uint32_t p01,
                                                 uint32_t p23)
    {
        const uintptr_t ba = (uintptr_t)row + 2 * (uintptr_t)gx;
        if (gx + 4 <= W && (ba & 3u) == 0) {
            store_u32<NTS>(ba, p01);
            store_u32<NTS>(ba + 4, p23);
        } else {
            const uint32_t v[2] = {p01, p23};
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (gx + j < W) store_u16<NTS>(ba + 2 * j, (uint16_t)(v[j >> 1] >> (16 * (j & 1))));
        }
    }
};

// A buffer store of the destination, non-temporal or plain (the cache-policy operand
// is an immediate).  (The policy is a template argument throughout: a run-time choice
// between two otherwise identical stores is merged by the compiler into one plain
// store.)
template <bool NTS>
__device__ __forceinline__ void buffer_store_nt(uint32_t v, __amdgpu_buffer_rsrc_t rs, int voff,
                                                int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(v, rs, voff, soff, NTS ? kStoreCpol : 0);
}

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

// Reads of one image row quad for the vertical pass.  The tile's input columns
// start at cxa, rounded down to a multiple of 4 pixels, so every quad starts at a
// multiple of 4.  With AL (rows 4-byte aligned for uint8, 8-byte for uint16) each
// quad is one naturally aligned load.  Loads are split in two steps so that a
// batch of them can be issued before any is waited on: issue() reads (a quad
// outside the image, or a slot not wanted, reads the image's first element
// instead) and finish() widens and replaces pixels outside the image by the
// identity with selects, never branches.
template <typename T> struct RawQuad;
template <> struct RawQuad<uint8_t> { uint32_t d; };
template <> struct RawQuad<uint16_t> { uint2 d; };

template <typename T, bool AL> struct RowLoader {
    const uint8_t *src;
    int64_t pitch;
    int H, W;
    uint32_t id;
    uint32_t flip; // XOR applied to every loaded pixel (complement for dilation-as-erosion)
    // AL: the pitch is a multiple of the quad size (4 bytes for uint8, 8 for uint16)
    // and the image spans less than 4 GiB.  Quads are then addressed as 32-bit
    // offsets from abase, src rounded down to the quad size, and mis is how many
    // pixels src lies past abase; quad columns gx are chosen with gx + mis a
    // multiple of 4, so every quad is one naturally aligned load.
    const uint8_t *abase;
    int mis;

    __device__ __forceinline__ RowLoader(const uint8_t *src_, int64_t pitch_, int H_, int W_,
                                         uint32_t id_, uint32_t flip_)
        : src(src_), pitch(pitch_), H(H_), W(W_), id(id_), flip(flip_)
    {
        const uintptr_t m = (uintptr_t)src_ & (4 * sizeof(T) - 1);
        abase = src_ - m;
        mis = (int)(m / sizeof(T));
    }
    __device__ __forceinline__ RawQuad<T> at(uint32_t off) const
    {
        RawQuad<T> r;
        if constexpr (sizeof(T) == 1) r.d = *(const GLOBAL uint32_t *)(abase + off);
        else r.d = __builtin_bit_cast(uint2, *(const GLOBAL uint64_t *)(abase + off));
        return r;
    }
    // offset of the quad at (gy, gx); gx + mis >= 0 for every quad that touches the
    // image, as gx > -4 and gx + mis is a multiple of 4
    __device__ __forceinline__ uint32_t offset(int gy, int gx) const
    {
        return (uint32_t)gy * (uint32_t)pitch + (uint32_t)(gx + mis) * (uint32_t)sizeof(T);
    }
    __device__ __forceinline__ static bool touches(int gx, int W) { return gx > -4 && gx < W; }
    __device__ __forceinline__ void widen(const RawQuad<T> &r, uint32_t &a, uint32_t &b) const
    {
        if constexpr (sizeof(T) == 1) {
            a = perm(0u, r.d, SEL_U8_01) ^ flip;
            b = perm(0u, r.d, SEL_U8_23) ^ flip;
        } else {
            a = r.d.x ^ flip;
            b = r.d.y ^ flip;
        }
    }
    // 16-bit lane masks of the quad at gx: lane j survives when 0 <= gx + j < W
    __device__ __forceinline__ void col_masks(int gx, uint32_t &m01, uint32_t &m23) const
    {
        const int lo = max(-gx, 0), hi = min(W - gx, 4); // surviving lanes [lo, hi)
        m01 = (lo <= 0 && hi > 0 ? 0x0000ffffu : 0u) | (lo <= 1 && hi > 1 ? 0xffff0000u : 0u);
        m23 = (lo <= 2 && hi > 2 ? 0x0000ffffu : 0u) | (lo <= 3 && hi > 3 ? 0xffff0000u : 0u);
    }
    __device__ __forceinline__ uint32_t sel(uint32_t m, uint32_t x) const
    {
        return (x & m) | (id & ~m);
    }
    // one quad, any alignment (slow path)
    __device__ __forceinline__ void load_any(int gy, int gx, bool want, uint32_t &a,
                                             uint32_t &b) const
    {
        if (want && (unsigned)gy < (unsigned)H) {
            // masked pixels come back as id ^ flip, so after the flip they are id
            Px<T>::load(src + (int64_t)gy * pitch, gx, W, id ^ flip, a, b);
            a ^= flip;
            b ^= flip;
        } else {
            a = b = id;
        }
    }
};

// NR rows gy0, gy0 + step, ... of the quad at column gx; rows k >= n are not wanted
// and come back as the identity.  Every load is issued before any is used.  Units
// whose rows and columns all lie inside the image skip every check.
template <int NR, typename T, bool AL>
__device__ __forceinline__ void load_rows(const RowLoader<T, AL> &L, int gy0, int step, int gx,
                                          int n, uint32_t *v01, uint32_t *v23)
{
    if constexpr (AL) {
        RawQuad<T> raw[NR];
        const int glast = gy0 + step * (min(n, NR) - 1);
        const bool interior = gx >= 0 && gx + 4 <= L.W && min(gy0, glast) >= 0 &&
                              max(gy0, glast) < L.H && n > 0;
        if (interior) {
            const uint32_t off = L.offset(gy0, gx);
            const int32_t d = step * (int32_t)L.pitch;
#pragma unroll
            for (int k = 0; k < NR; k++)
                if (k < n) raw[k] = L.at(off + (uint32_t)(k * d));
#pragma unroll
            for (int k = 0; k < NR; k++) {
                if (k < n) L.widen(raw[k], v01[k], v23[k]);
                else v01[k] = v23[k] = L.id;
            }
        } else {
            uint32_t m01, m23;
            L.col_masks(gx, m01, m23);
            bool ok[NR];
#pragma unroll
            for (int k = 0; k < NR; k++) {
                const int gy = gy0 + step * k;
                ok[k] = k < n && (unsigned)gy < (unsigned)L.H && L.touches(gx, L.W);
                raw[k] = L.at(ok[k] ? L.offset(gy, gx) : 0u);
            }
#pragma unroll
            for (int k = 0; k < NR; k++) {
                uint32_t a, b;
                L.widen(raw[k], a, b);
                v01[k] = L.sel(ok[k] ? m01 : 0u, a);
                v23[k] = L.sel(ok[k] ? m23 : 0u, b);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < NR; k++) L.load_any(gy0 + step * k, gx, k < n, v01[k], v23[k]);
    }
}

// A batch of NR rows of one quad, split so that the next batch's loads can be in
// flight while the current one is used: issue() sends every load without a branch
// (rows not wanted or outside the image read the image's first element), finish()
// widens and masks.  Used by the vHGW vertical pass, which walks long runs of rows.
template <int NR, typename T, bool AL> struct RowBatch {
    RawQuad<T> raw[NR];
    uint32_t ok; // bit k: row k wanted and inside the image (column validity aside)
    __device__ __forceinline__ void issue(const RowLoader<T, AL> &L, int gy0, int step, int gx,
                                          int n)
    {
        const bool colok = L.touches(gx, L.W);
        const uint32_t off0 = L.offset(gy0, gx); // unused (and possibly wrapped) when !ok
        const int32_t d = step * (int32_t)L.pitch;
        ok = 0u;
#pragma unroll
        for (int k = 0; k < NR; k++) {
            const int gy = gy0 + step * k;
            const bool o = colok && k < n && (unsigned)gy < (unsigned)L.H;
            ok |= (uint32_t)o << k;
            raw[k] = L.at(o ? off0 + (uint32_t)(k * d) : 0u);
        }
    }
    __device__ __forceinline__ void finish(const RowLoader<T, AL> &L, int gx, uint32_t *v01,
                                           uint32_t *v23) const
    {
        if (ok == (1u << NR) - 1u && gx >= 0 && gx + 4 <= L.W) { // all rows and pixels inside
#pragma unroll
            for (int k = 0; k < NR; k++) L.widen(raw[k], v01[k], v23[k]);
        } else {
            uint32_t m01, m23;
            L.col_masks(gx, m01, m23);
#pragma unroll
            for (int k = 0; k < NR; k++) {
                uint32_t a, b;
                L.widen(raw[k], a, b);
                const bool o = (ok >> k) & 1u;
                v01[k] = L.sel(o ? m01 : 0u, a);
                v23[k] = L.sel(o ? m23 : 0u, b);
            }
        }
    }
};

// Division of work-unit indices by a per-tile divisor d without an integer divide:
// with m = ceil(2^32 / d), floor(u / d) = mulhi(u, m) exactly whenever u * d < 2^32,
// which the host planner guarantees for every loop below.
struct FastDiv {
    uint32_t d, m;
    __device__ __forceinline__ explicit FastDiv(int d_)
        : d((uint32_t)d_), m(d_ > 1 ? (uint32_t)__builtin_ceil(4294967296.0 / (double)d_) : 0u)
    {
    }
    __device__ __forceinline__ uint32_t div(uint32_t u) const { return d > 1 ? __umulhi(u, m) : u; }
};

// Everything one tile's passes share.  LDS holds two arrays:
//   A  [TB rows][SA dwords]  vertical-pass output, row-major 16-bit pixels; LDS column
//                            c is image column cxa + c (cxa rounded down to a quad);
//   B  [TB/2][SB dwords]     horizontal pass, "row-pair" layout: dword (p, c) holds
//                            rows 2p (low half) and 2p+1 (high half) of column c.
// Both strides are odd, so the row-pair walks of the horizontal pass (one lane per
// row pair) spread over the banks.
template <typename T, bool AL> struct TileCtx {
    int tid, x0, y0, out_w, out_h, wx, wy, cy0, co, cxa, IWL, SA, SB, NQ, NP;
    uint32_t id, flip;
    uint32_t *A, *B;
    RowLoader<T, AL> L;
    FastDiv fq, fp;
    __device__ __forceinline__ TileCtx(const TileJob &J, int tile, uint32_t *lds, uint32_t id_,
                                       uint32_t flip_)
        : tid(threadIdx.x), id(id_), flip(flip_), L(J.src, J.pitch, J.H, J.W, id_, flip_), fq(1),
          fp(1)
    {
        const int tx = tile % J.tiles_x, ty = tile / J.tiles_x;
        x0 = tx * J.TW;
        y0 = ty * J.TB;
        out_w = min(J.TW, J.W - x0);
        out_h = min(J.TB, J.H - y0);
        wx = J.wx;
        wy = J.wy;
        const int cx0 = x0 - J.ax;
        cy0 = y0 - J.ay;
        co = (cx0 + (AL ? L.mis : 0)) & 3; // quads start where image column + mis is 4k
        cxa = cx0 - co;
        IWL = out_w + wx - 1 + co;
        SA = J.SA;
        SB = J.SB;
        NQ = (IWL + 3) >> 2;
        NP = (out_h + 1) >> 1;
        A = lds;
        B = lds + J.TB * SA;
        fq = FastDiv(NQ);
        fp = FastDiv(NP);
    }
    // row s, quad q of A (two dwords: pixels 0,1 and 2,3)
    __device__ __forceinline__ uint32_t *arow(int s, int q) const { return A + s * SA + 2 * q; }
};

// Outputs for window starts 0 and 1 over x[0 .. W]: the two windows share the W-1
// inputs x[1 .. W-1] (the paper's pairing of adjacent outputs in its direct pass).
template <int W, bool MAXOP>
__device__ __forceinline__ void pair_window(const uint32_t *x, uint32_t &o0, uint32_t &o1)
{
    if constexpr (W == 1) {
        o0 = x[0];
        o1 = x[1];
    } else {
        uint32_t core = x[1];
#pragma unroll
        for (int j = 2; j < W; j++) core = pk<MAXOP>(core, x[j]);
        o0 = pk<MAXOP>(core, x[0]);
        o1 = pk<MAXOP>(core, x[W]);
    }
}

// Outputs for the 8 window starts 0 .. 7 over x[0 .. W + 6], W >= 8, each the extremum
// of its W inputs.  The rows 7 .. W - 1 lie in all eight windows and are reduced once;
// window r adds the rows r .. 6 before them (a suffix, grown downwards from row 6) and
// the rows W .. W + r - 1 after them (a prefix, grown upwards from row W): W + 18
// operations for the eight outputs, where pairs of adjacent outputs take 4 W.  The
// same values as the definition (the extremum is associative and commutative).
template <int W, bool MAXOP>
__device__ __forceinline__ void chunk8_window(const uint32_t *x, uint32_t *o)
{
    static_assert(W >= 8, "the eight windows share rows 7 .. W - 1");
    uint32_t c = x[7];
#pragma unroll
    for (int j = 8; j < W; j++) c = pk<MAXOP>(c, x[j]);
    uint32_t b = x[W]; // rows W .. W + r - 1, for r = 1 .. 7
    o[1] = pk<MAXOP>(c, b);
#pragma unroll
    for (int r = 2; r < 8; r++) {
        b = pk<MAXOP>(b, x[W + r - 1]);
        o[r] = pk<MAXOP>(c, b);
    }
    uint32_t a = x[6]; // rows r .. 6, for r = 6 .. 0
    o[6] = pk<MAXOP>(o[6], a);
#pragma unroll
    for (int r = 5; r >= 1; r--) {
        a = pk<MAXOP>(a, x[r]);
        o[r] = pk<MAXOP>(o[r], a);
    }
    o[0] = pk<MAXOP>(c, pk<MAXOP>(a, x[0]));
}

// ---- vertical pass, direct, window W: A rows [0, out_h) ----
// Work unit: one quad of columns and KV output rows; its KV + W - 1 input rows are
// loaded at once.
template <int W, bool MAXOP, typename T, bool AL>
__device__ __forceinline__ void vpass_direct(const TileCtx<T, AL> &c)
{
    constexpr int NR = KV + W - 1;
    const int NKV = (c.out_h + KV - 1) / KV;
    for (int u = c.tid; u < c.NQ * NKV; u += NT) {
        const int k = c.fq.div(u), q = u - k * c.NQ, s0 = k * KV;
        uint32_t r01[NR], r23[NR];
        load_rows<NR>(c.L, c.cy0 + s0, 1, c.cxa + 4 * q, NR, r01, r23);
#pragma unroll
        for (int m = 0; m < KV; m += 2) {
            uint32_t a01, a23, b01, b23;
            pair_window<W, MAXOP>(r01 + m, a01, b01);
            pair_window<W, MAXOP>(r23 + m, a23, b23);
            if (s0 + m < c.out_h) {
                uint32_t *d = c.arow(s0 + m, q);
                d[0] = a01;
                d[1] = a23;
                d[c.SA] = b01; // row s0 + m + 1 (A has TB rows, TB even)
                d[c.SA + 1] = b23;
            }
        }
    }
}

// ---- vertical pass, direct, any window (w > DMAX) ----
// The definition with a loop over the taps: each of a unit's KV + w - 1 input rows
// (read KV at a time) enters the extremum of every output row whose window holds
// it, so a pixel costs O(w) operations, the direct pass's cost (§5.1.2) without its
// compiled sharing.  Work unit: one quad of columns and KV output rows.
template <bool MAXOP, typename T, bool AL>
__device__ __forceinline__ void vpass_direct_any(const TileCtx<T, AL> &c, int w)
{
    const int NKV = (c.out_h + KV - 1) / KV;
    const int nin = KV + w - 1;
    for (int u = c.tid; u < c.NQ * NKV; u += NT) {
        const int k = c.fq.div(u), q = u - k * c.NQ, s0 = k * KV;
        uint32_t o01[KV], o23[KV];
#pragma unroll
        for (int m = 0; m < KV; m++) o01[m] = o23[m] = c.id;
        for (int i0 = 0; i0 < nin; i0 += KV) {
            uint32_t x01[KV], x23[KV];
            load_rows<KV>(c.L, c.cy0 + s0 + i0, 1, c.cxa + 4 * q, nin - i0, x01, x23);
#pragma unroll
            for (int r = 0; r < KV; r++)
#pragma unroll
                for (int m = 0; m < KV; m++) {
                    const int i = i0 + r; // input row i is in output m's window
                    if (i >= m && i < m + w) {
                        o01[m] = pk<MAXOP>(o01[m], x01[r]);
                        o23[m] = pk<MAXOP>(o23[m], x23[r]);
                    }
                }
        }
#pragma unroll
        for (int m = 0; m < KV; m++)
            if (s0 + m < c.out_h) {
                uint32_t *d = c.arow(s0 + m, q);
                d[0] = o01[m];
                d[1] = o23[m];
            }
    }
}

// ---- vertical pass, vHGW ----
// Phase F: g over each block of wy input rows, stored in the output row it pairs with
// (s = i - wy + 1).  Phase B: walk each block backwards; h[s] = op of rows s .. block
// end; out[s] = op(h[s], g[s + wy - 1]), in place.  Rows are read VB at a time.
// Work unit: one quad of columns and one run of R = vrun rows of a block (a block is
// scanned as NS = ceil(wy / R) runs).  Phase F walks its run forward keeping the
// running extremum from the run start, stores it in the output row it pairs with
// (s = i - wy + 1) and records the run total.  Phase B walks a run of output rows
// backwards: h = (suffix within the run) op (totals of the later runs of the block),
// g = (stored prefix) op (totals of the earlier runs of its block), out = op(h, g).
// With NS = 1 this is the plain two-phase vHGW.  Rows are read VB at a time and the
// next batch's loads are in flight while the current one is used.
template <bool MAXOP, typename T, bool AL>
__device__ __forceinline__ void vpass_vhgw(const TileCtx<T, AL> &c, int R, int tt_quads)
{
    constexpr int VB = kVhgwBatch;
    const int wy = c.wy;
    const int IH = c.out_h + wy - 1;
    const int NS = (wy + R - 1) / R;
    const int NBF = (IH + wy - 1) / wy;
    const int NRF = NBF * NS; // runs over all blocks of the input rows
    uint32_t *TT = c.B;       // run totals: [(b * NS + j) * tt_quads + q] x 2 dwords
    for (int u = c.tid; u < c.NQ * NRF; u += NT) {
        const int r = c.fq.div(u), q = u - r * c.NQ;
        const int b = r / NS, j = r - b * NS; // NS is small; a plain divide here is rare
        const int gx = c.cxa + 4 * q;
        const int i0 = b * wy + j * R;
        const int i1 = min(min(i0 + R, (b + 1) * wy), IH);
        uint32_t g01 = c.id, g23 = c.id;
        RowBatch<VB, T, AL> nxt;
        if constexpr (AL) nxt.issue(c.L, c.cy0 + i0, 1, gx, i1 - i0);
        for (int i = i0; i < i1; i += VB) {
            uint32_t v01[VB], v23[VB];
            if constexpr (AL) {
                const RowBatch<VB, T, AL> cur = nxt;
                nxt.issue(c.L, c.cy0 + i + VB, 1, gx, i1 - i - VB); // in flight meanwhile
                cur.finish(c.L, gx, v01, v23);
            } else {
                load_rows<VB>(c.L, c.cy0 + i, 1, gx, i1 - i, v01, v23);
            }
#pragma unroll
            for (int k = 0; k < VB; k++) {
                g01 = pk<MAXOP>(g01, v01[k]);
                g23 = pk<MAXOP>(g23, v23[k]);
                const int s = i + k - wy + 1;
                if (i + k < i1 && s >= 0) {
                    uint32_t *d = c.arow(s, q);
                    d[0] = g01;
                    d[1] = g23;
                }
            }
        }
        if (NS > 1) {
            uint32_t *t = TT + 2 * (r * tt_quads + q);
            t[0] = g01;
            t[1] = g23;
        }
    }
    __syncthreads();
    const int NBB = (c.out_h + wy - 1) / wy;
    for (int u = c.tid; u < c.NQ * NBB * NS; u += NT) {
        const int r = c.fq.div(u), q = u - r * c.NQ;
        const int b = r / NS, j = r - b * NS;
        const int gx = c.cxa + 4 * q;
        const int s0 = b * wy + j * R;
        if (s0 >= c.out_h) continue;
        const int i_hi = min(min(s0 + R, (b + 1) * wy), IH); // rows of this run
        // totals of the later runs of block b
        uint32_t ch01 = c.id, ch23 = c.id;
        // g carries for the runs holding p = s + wy - 1 over this run's outputs s: the
        // first output's p is the last row of the run before run j of block b + 1 (rA);
        // every later p lies in run j of block b + 1 (rB)
        uint32_t cA01 = c.id, cA23 = c.id, cB01 = c.id, cB23 = c.id;
        int pB0 = 0x7fffffff; // first p of run rB
        if (NS > 1) {
            for (int jj = j + 1; jj < NS; jj++) {
                const uint32_t *t = TT + 2 * ((b * NS + jj) * tt_quads + q);
                ch01 = pk<MAXOP>(ch01, t[0]);
                ch23 = pk<MAXOP>(ch23, t[1]);
            }
            const int pA = s0 + wy - 1, pLast = min(i_hi, c.out_h) - 1 + wy - 1;
            const int bA = pA / wy, jA = (pA - bA * wy) / R;
            const int bB = pLast / wy, jB = (pLast - bB * wy) / R;
            for (int jj = 0; jj < jA; jj++) {
                const uint32_t *t = TT + 2 * ((bA * NS + jj) * tt_quads + q);
                cA01 = pk<MAXOP>(cA01, t[0]);
                cA23 = pk<MAXOP>(cA23, t[1]);
            }
            if (bB != bA || jB != jA) {
                for (int jj = 0; jj < jB; jj++) {
                    const uint32_t *t = TT + 2 * ((bB * NS + jj) * tt_quads + q);
                    cB01 = pk<MAXOP>(cB01, t[0]);
                    cB23 = pk<MAXOP>(cB23, t[1]);
                }
                pB0 = bB * wy + jB * R;
            }
        }
        uint32_t h01 = c.id, h23 = c.id;
        RowBatch<VB, T, AL> nxt;
        if constexpr (AL) nxt.issue(c.L, c.cy0 + i_hi - 1, -1, gx, i_hi - s0);
        for (int i = i_hi - 1; i >= s0; i -= VB) {
            uint32_t v01[VB], v23[VB];
            if constexpr (AL) {
                const RowBatch<VB, T, AL> cur = nxt;
                nxt.issue(c.L, c.cy0 + i - VB, -1, gx, i - VB - s0 + 1);
                cur.finish(c.L, gx, v01, v23);
            } else {
                load_rows<VB>(c.L, c.cy0 + i, -1, gx, i - s0 + 1, v01, v23);
            }
#pragma unroll
            for (int k = 0; k < VB; k++) {
                h01 = pk<MAXOP>(h01, v01[k]);
                h23 = pk<MAXOP>(h23, v23[k]);
                const int s = i - k;
                if (s >= s0 && s < c.out_h) {
                    const bool inB = s + wy - 1 >= pB0;
                    uint32_t *d = c.arow(s, q);
                    const uint32_t g01 = pk<MAXOP>(d[0], inB ? cB01 : cA01);
                    const uint32_t g23 = pk<MAXOP>(d[1], inB ? cB23 : cA23);
                    d[0] = pk<MAXOP>(pk<MAXOP>(h01, ch01), g01);
                    d[1] = pk<MAXOP>(pk<MAXOP>(h23, ch23), g23);
                }
            }
        }
    }
}

// Column `col` (LDS coordinates) of row pair p of A as one row-pair dword.
template <typename T, bool AL>
__device__ __forceinline__ uint32_t col_pair(const TileCtx<T, AL> &c, const uint32_t *r0, int col)
{
    const uint32_t x = r0[col >> 1], y = r0[(col >> 1) + c.SA];
    return (col & 1) ? perm(y, x, SEL_HI16_PAIR) : perm(y, x, SEL_LO16_PAIR);
}

// ---- horizontal pass, direct, window W: B (row pairs) columns [0, out_w) ----
// Work unit: one row pair and KH output columns.  The unit reads the dwords that
// cover its KH + W - 1 input columns from both rows and transposes them to row-pair
// form.  The parity of the first input column (co) is the same for every unit of a
// tile, so each parity has its own fully unrolled code.
template <int W, bool MAXOP, int PAR, typename T, bool AL>
__device__ __forceinline__ void hpass_direct_par(const TileCtx<T, AL> &c)
{
    constexpr int NC = KH + W - 1;        // input columns per unit
    constexpr int ND = (NC + PAR + 1) / 2; // dwords covering them
    const int NKH = (c.out_w + KH - 1) / KH;
    for (int u = c.tid; u < c.NP * NKH; u += NT) {
        const int k = c.fp.div(u), p = u - k * c.NP, c0 = k * KH;
        const uint32_t *r0 = c.A + 2 * p * c.SA + ((c.co + c0) >> 1);
        uint32_t x[NC + 1];
#pragma unroll
        for (int d = 0; d < ND; d++) {
            const uint32_t lo = r0[d], hi = r0[d + c.SA];
            const int e0 = 2 * d - PAR; // column (relative to c0) of the low half
            if (e0 >= 0 && e0 < NC + 1) x[e0] = perm(hi, lo, SEL_LO16_PAIR);
            if (e0 + 1 >= 0 && e0 + 1 < NC + 1) x[e0 + 1] = perm(hi, lo, SEL_HI16_PAIR);
        }
        uint32_t *o = c.B + p * c.SB + c0;
#pragma unroll
        for (int m = 0; m < KH; m += 2) {
            uint32_t o0, o1;
            pair_window<W, MAXOP>(x + m, o0, o1);
            if (c0 + m < c.out_w) o[m] = o0;
            if (c0 + m + 1 < c.out_w) o[m + 1] = o1;
        }
    }
}

template <int W, bool MAXOP, typename T, bool AL>
__device__ __forceinline__ void hpass_direct(const TileCtx<T, AL> &c)
{
    if (c.co & 1) hpass_direct_par<W, MAXOP, 1>(c);
    else hpass_direct_par<W, MAXOP, 0>(c);
}

// ---- horizontal pass, direct, any window (w > DMAX) ----
// As vpass_direct_any along the row pairs of A: work unit one row pair and KH
// output columns, a loop over its KH + w - 1 input columns.
template <bool MAXOP, typename T, bool AL>
__device__ __forceinline__ void hpass_direct_any(const TileCtx<T, AL> &c, int w)
{
    const int NKH = (c.out_w + KH - 1) / KH;
    const int nin = KH + w - 1;
    for (int u = c.tid; u < c.NP * NKH; u += NT) {
        const int k = c.fp.div(u), p = u - k * c.NP, c0 = k * KH;
        const uint32_t *r0 = c.A + 2 * p * c.SA;
        uint32_t o[KH];
#pragma unroll
        for (int m = 0; m < KH; m++) o[m] = c.id;
        for (int e = 0; e < nin; e++) {
            const uint32_t x = col_pair(c, r0, c.co + c0 + e);
#pragma unroll
            for (int m = 0; m < KH; m++)
                if (e >= m && e < m + w) o[m] = pk<MAXOP>(o[m], x);
        }
        uint32_t *d = c.B + p * c.SB + c0;
#pragma unroll
        for (int m = 0; m < KH; m++)
            if (c0 + m < c.out_w) d[m] = o[m];
    }
}

// ---- horizontal pass, vHGW ----
// Work unit: one row pair and one block of wx input columns.  Phase F writes g
// shifted by wx - 1 into B; phase B walks the block backwards and combines h with g
// in place in B.  Columns are read HB at a time.
template <bool MAXOP, typename T, bool AL>
__device__ __forceinline__ void hpass_vhgw(const TileCtx<T, AL> &c)
{
    constexpr int HB = 8;
    const int wx = c.wx;
    const int IW = c.out_w + wx - 1;
    const int NBF = (IW + wx - 1) / wx;
    for (int u = c.tid; u < c.NP * NBF; u += NT) {
        const int b = c.fp.div(u), p = u - b * c.NP, i0 = b * wx;
        const int i1 = min(i0 + wx, IW);
        const uint32_t *r0 = c.A + 2 * p * c.SA;
        uint32_t *g = c.B + p * c.SB;
        uint32_t acc = c.id;
        for (int i = i0; i < i1; i += HB) {
            uint32_t v[HB];
#pragma unroll
            for (int k = 0; k < HB; k++) {
                const bool ok = i + k < i1;
                const uint32_t x = col_pair(c, r0, c.co + (ok ? i + k : i0));
                v[k] = ok ? x : c.id;
            }
#pragma unroll
            for (int k = 0; k < HB; k++) {
                acc = pk<MAXOP>(acc, v[k]);
                const int s = i + k - wx + 1;
                if (i + k < i1 && s >= 0) g[s] = acc;
            }
        }
    }
    __syncthreads();
    const int NBB = (c.out_w + wx - 1) / wx;
    for (int u = c.tid; u < c.NP * NBB; u += NT) {
        const int b = c.fp.div(u), p = u - b * c.NP, i0 = b * wx;
        const uint32_t *r0 = c.A + 2 * p * c.SA;
        uint32_t *g = c.B + p * c.SB;
        uint32_t h = c.id;
        for (int i = i0 + wx - 1; i >= i0; i -= HB) {
            uint32_t v[HB], gg[HB];
#pragma unroll
            for (int k = 0; k < HB; k++) {
                const bool in = i - k >= i0;
                const bool og = in && i - k < c.out_w;
                const uint32_t x = col_pair(c, r0, c.co + (in ? i - k : i0));
                const uint32_t y = g[og ? i - k : 0];
                v[k] = in ? x : c.id;
                gg[k] = og ? y : c.id;
            }
#pragma unroll
            for (int k = 0; k < HB; k++) {
                h = pk<MAXOP>(h, v[k]);
                if (i - k >= i0 && i - k < c.out_w) g[i - k] = pk<MAXOP>(h, gg[k]);
            }
        }
    }
}

// ---- store ----
template <typename T, bool AL>
__device__ __forceinline__ void store_pairs(const TileCtx<T, AL> &c, const TileJob &J)
{
    // from B (row pairs): a quad of columns of two rows per unit
    const int NQo = (c.out_w + 3) >> 2;
    const FastDiv fo(NQo);
    for (int u = c.tid; u < NQo * c.NP; u += NT) {
        const int p = fo.div(u), q = u - p * NQo;
        const uint32_t *o = c.B + p * c.SB + 4 * q;
        const uint32_t c0 = o[0], c1 = o[1], c2 = o[2], c3 = o[3];
        const int y = c.y0 + 2 * p, x = c.x0 + 4 * q;
        uint8_t *row = J.dst + (int64_t)y * J.dpitch;
        Px<T>::store(row, x, J.W, perm(c1, c0, SEL_LO16_PAIR) ^ c.flip,
                     perm(c3, c2, SEL_LO16_PAIR) ^ c.flip);
        if (2 * p + 1 < c.out_h)
            Px<T>::store(row + J.dpitch, x, J.W, perm(c1, c0, SEL_HI16_PAIR) ^ c.flip,
                         perm(c3, c2, SEL_HI16_PAIR) ^ c.flip);
    }
}

template <typename T, bool AL>
__device__ __forceinline__ void store_rows(const TileCtx<T, AL> &c, const TileJob &J)
{
    // from A (rows), when there is no horizontal pass: output column x0 + k is LDS
    // column co + k, so odd co shifts every quad by half a dword
    const int NQo = (c.out_w + 3) >> 2;
    const FastDiv fo(NQo);
    for (int u = c.tid; u < NQo * c.out_h; u += NT) {
        const int s = fo.div(u), q = u - s * NQo;
        const uint32_t *a = c.A + s * c.SA + ((c.co + 4 * q) >> 1);
        uint32_t x = a[0], y = a[1];
        if (c.co & 1) {
            const uint32_t z = a[2];
            x = __builtin_amdgcn_alignbit(y, x, 16);
            y = __builtin_amdgcn_alignbit(z, y, 16);
        }
        Px<T>::store(J.dst + (int64_t)(c.y0 + s) * J.dpitch, c.x0 + 4 * q, J.W, x ^ c.flip,
                     y ^ c.flip);
    }
}

// One tile.  flip = 0 computes op MAXOP directly; the batch kernel instead runs every
// job as an erosion (MAXOP false) and passes flip = the type's all-ones value for
// dilations: max(x) = maxv - min(maxv - x), and maxv - x is x ^ maxv.
template <typename T, bool MAXOP, bool AL>
__device__ __forceinline__ void tile_body(const TileJob &J, int tile, uint32_t *lds,
                                          uint32_t flip = 0u)
{
    const uint32_t id = MAXOP ? 0u : (Px<T>::maxv | (Px<T>::maxv << 16));
    const TileCtx<T, AL> c(J, tile, lds, id, flip);
    switch (J.vcode) {
    case 1: vpass_direct<1, MAXOP>(c); break;
    case 2: vpass_direct<2, MAXOP>(c); break;
    case 3: vpass_direct<3, MAXOP>(c); break;
    case 4: vpass_direct<4, MAXOP>(c); break;
    case 5: vpass_direct<5, MAXOP>(c); break;
    case 6: vpass_direct<6, MAXOP>(c); break;
    case 7: vpass_direct<7, MAXOP>(c); break;
    case 8: vpass_direct<8, MAXOP>(c); break;
    case 9: vpass_direct<9, MAXOP>(c); break;
    default:
        if (J.vm == PASS_DIRECT) vpass_direct_any<MAXOP>(c, J.wy);
        else vpass_vhgw<MAXOP>(c, J.vrun, (J.TW + J.wx - 1 + 3 + 3) / 4);
        break;
    }
    __syncthreads();
    if (J.hcode == 1) {
        store_rows(c, J);
        return;
    }
    switch (J.hcode) {
    case 2: hpass_direct<2, MAXOP>(c); break;
    case 3: hpass_direct<3, MAXOP>(c); break;
    case 4: hpass_direct<4, MAXOP>(c); break;
    case 5: hpass_direct<5, MAXOP>(c); break;
    case 6: hpass_direct<6, MAXOP>(c); break;
    case 7: hpass_direct<7, MAXOP>(c); break;
    case 8: hpass_direct<8, MAXOP>(c); break;
    case 9: hpass_direct<9, MAXOP>(c); break;
    default:
        if (J.hm == PASS_DIRECT) hpass_direct_any<MAXOP>(c, J.wx);
        else hpass_vhgw<MAXOP>(c);
        break;
    }
    __syncthreads();
    store_pairs(c, J);
}

// ======================= lane moves and the doubling pass ==========================
// Used by the wave and streaming kernels for windows wider than the direct pass
// takes: min/max over a row held across the wave's lanes (a lane holds four
// consecutive pixels as two pair dwords) by log-step doubling,
// m_2L[k] = min(m_L[k], m_L[k + L]), then m_w[k] = min(m_L[k], m_L[k + w - L]) for the
// largest L <= w; shifts by one or two pixels are in-lane (alignbit) plus one DPP
// move, by one lane DPP, by more lanes ds_bpermute.
// Lane i gets x of lane i + 1 (DPP wave_shl:1; lane 63 gets 0 through bound_ctrl,
// which also spares the move that would give the destination an old value).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}

__device__ __forceinline__ uint32_t lane_fetch(uint32_t v, uint32_t byte_addr)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)byte_addr, (int)v);
}

// Per-unit constants of the doubling pass.
struct Doubling {
    int wx;
    int c0, c1;        // pixel offsets co and co + wx - L within their first quad (0..3)
    uint32_t ad0, ad1; // ds_bpermute addresses of lanes + q1 and + q1 + 1, q1 = (co + wx - L) / 4

    __device__ __forceinline__ Doubling(int wx_, int co)
    {
        wx = wx_;
        int L = 1;
        while (2 * L <= wx) L *= 2;
        const int d1 = co + wx - L;
        c0 = co;
        c1 = d1 & 3;
        const int lane = threadIdx.x & 63;
        ad0 = (uint32_t)(lane + (d1 >> 2)) << 2;
        ad1 = (uint32_t)(lane + (d1 >> 2) + 1) << 2;
    }
};

// The pixel pairs at offsets c and c + 2 from four consecutive pair dwords F
// (offsets 0, 2, 4, 6).
template <int C>
__device__ __forceinline__ void pairs_at(uint32_t f0, uint32_t f1, uint32_t f2, uint32_t f3,
                                         uint32_t &p, uint32_t &p2)
{
    const uint32_t lo = (C >> 1) ? f1 : f0, mid = (C >> 1) ? f2 : f1, hi = (C >> 1) ? f3 : f2;
    p = (C & 1) ? __builtin_amdgcn_alignbit(mid, lo, 16) : lo;
    p2 = (C & 1) ? __builtin_amdgcn_alignbit(hi, mid, 16) : mid;
}

// m_wx[k] = min(m_L[k], m_L[k + wx - L]) at k = co .. co + 3, from the level-L pairs.
template <int C0, int C1, int G, bool MAXOP>
__device__ __forceinline__ void doubling_final(const Doubling &S, uint32_t *e0, uint32_t *e1)
{
#pragma unroll
    for (int r = 0; r < G; r++) {
        const uint32_t a0 = e0[r], a1 = e1[r];
        const uint32_t n0 = from_next_lane(a0), n1 = (C0 >> 1) ? from_next_lane(a1) : 0u;
        uint32_t p0, p2, r0, r2;
        pairs_at<C0>(a0, a1, n0, n1, p0, p2);
        const uint32_t f0 = (C1 >> 1) ? 0u : lane_fetch(a0, S.ad0), f1 = lane_fetch(a1, S.ad0);
        const uint32_t f2 = lane_fetch(a0, S.ad1), f3 = (C1 >> 1) ? lane_fetch(a1, S.ad1) : 0u;
        pairs_at<C1>(f0, f1, f2, f3, r0, r2);
        e0[r] = pk<MAXOP>(p0, r0);
        e1[r] = pk<MAXOP>(p2, r2);
    }
}

// The horizontal passes below work on G rows at once, level by level, so that the
// rows' chains of lane moves and min/max interleave.
template <int G, bool MAXOP>
__device__ __forceinline__ void doubling_rows(const Doubling &S, uint32_t *e0, uint32_t *e1)
{
    // e0 = (m_L[0], m_L[1]), e1 = (m_L[2], m_L[3]) for the lane's quad
    const int lane = threadIdx.x & 63;
    if (S.wx >= 2) { // L = 1 -> 2: shift by one pixel
#pragma unroll
        for (int r = 0; r < G; r++) {
            const uint32_t n0 = from_next_lane(e0[r]);
            const uint32_t s1 = __builtin_amdgcn_alignbit(e1[r], e0[r], 16);
            const uint32_t s3 = __builtin_amdgcn_alignbit(n0, e1[r], 16);
            e0[r] = pk<MAXOP>(e0[r], s1);
            e1[r] = pk<MAXOP>(e1[r], s3);
        }
    }
    if (S.wx >= 4) { // 2 -> 4: two pixels
#pragma unroll
        for (int r = 0; r < G; r++) {
            const uint32_t n0 = from_next_lane(e0[r]);
            e0[r] = pk<MAXOP>(e0[r], e1[r]);
            e1[r] = pk<MAXOP>(e1[r], n0);
        }
    }
    if (S.wx >= 8) { // 4 -> 8: one lane
#pragma unroll
        for (int r = 0; r < G; r++) {
            const uint32_t n0 = from_next_lane(e0[r]), n1 = from_next_lane(e1[r]);
            e0[r] = pk<MAXOP>(e0[r], n0);
            e1[r] = pk<MAXOP>(e1[r], n1);
        }
    }
    for (int q = 2; 8 * q <= S.wx; q *= 2) { // 4q -> 8q: q lanes
        const uint32_t ad = (uint32_t)(lane + q) << 2;
#pragma unroll
        for (int r = 0; r < G; r++) {
            const uint32_t n0 = lane_fetch(e0[r], ad), n1 = lane_fetch(e1[r], ad);
            e0[r] = pk<MAXOP>(e0[r], n0);
            e1[r] = pk<MAXOP>(e1[r], n1);
        }
    }
#define MORPH_FIN1(A, B)                                                                     \
    case A * 4 + B: doubling_final<A, B, G, MAXOP>(S, e0, e1); break;
#define MORPH_FIN(A) MORPH_FIN1(A, 0) MORPH_FIN1(A, 1) MORPH_FIN1(A, 2) MORPH_FIN1(A, 3)
    switch (S.c0 * 4 + S.c1) {
        MORPH_FIN(0) MORPH_FIN(1) MORPH_FIN(2) MORPH_FIN(3)
    default: break;
    }
#undef MORPH_FIN
#undef MORPH_FIN1
}

// ======================= horizontal vHGW across the lanes ==========================
// The paper's van Herk/Gil-Werman pass (§5.1.1, along x as in §5.2.1) on a row held
// across the wave's lanes (lane L holds strip positions p = 4L .. 4L + 3 as two pair
// dwords).  Blocks of w positions start at p = 0.  g[p] is the extremum from p's
// block start to p, h[p] from p to its block end, both by segmented Hillis-Steele
// scans: K = ceil(log2 w) steps of shifts s = 1, 2, 4, ... (one or two pixels within
// the lane and the neighbouring lane by DPP, whole lanes by DPP or ds_bpermute), the
// shifted value taking part only where it lies in the same block (per-lane masks that
// substitute the identity).  Then m_w[k] = op(h[k], g[k + w - 1]) at k = co .. co + 3
// past the lane's first position, the output quad's window starts.
constexpr int kVhgwLaneSteps = 7; // w <= 128 = kStreamMaxWx

// Lane i gets x of lane i - 1 (DPP wave_shr:1; lane 0 gets 0).
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}

template <bool MAXOP> struct LaneVhgw {
    int K;                                   // steps: 2^K >= w
    uint32_t gm[kVhgwLaneSteps][2];          // per step and pair dword: identity where the
    uint32_t hm[kVhgwLaneSteps][2];          // shifted value lies in another block
    int c0, c1;                              // offsets co and co + w - 1 within their quads
    uint32_t ad0, ad1;                       // ds_bpermute addresses of lanes + q1, + q1 + 1

    __device__ __forceinline__ LaneVhgw(int w, int co)
    {
        const int lane = threadIdx.x & 63;
        K = 0;
        while ((1 << K) < w) K++;
        int r[4];
#pragma unroll
        for (int j = 0; j < 4; j++) r[j] = (4 * lane + j) % w; // position in its block
#pragma unroll
        for (int k = 0; k < kVhgwLaneSteps; k++) {
            const int st = 1 << k;
#pragma unroll
            for (int d = 0; d < 2; d++) {
                // 16-bit half of pixel 2d (low) and 2d + 1 (high): all ones where the
                // shifted value is outside the block, for an erosion's OR; the opposite
                // for a dilation's AND
                const uint32_t gi = (r[2 * d] < st ? 0xffffu : 0u) |
                                    (r[2 * d + 1] < st ? 0xffff0000u : 0u);
                const uint32_t hi = (r[2 * d] + st > w - 1 ? 0xffffu : 0u) |
                                    (r[2 * d + 1] + st > w - 1 ? 0xffff0000u : 0u);
                gm[k][d] = MAXOP ? ~gi : gi;
                hm[k][d] = MAXOP ? ~hi : hi;
            }
        }
        const int d1 = co + w - 1;
        c0 = co;
        c1 = d1 & 3;
        ad0 = (uint32_t)(lane + (d1 >> 2)) << 2;
        ad1 = (uint32_t)(lane + (d1 >> 2) + 1) << 2;
    }
    // the shifted value where it is in the block, else the identity
    static __device__ __forceinline__ uint32_t keep(uint32_t y, uint32_t m)
    {
        return MAXOP ? (y & m) : (y | m);
    }
};

// One scan step of shift 1 << k for G rows: g from lower positions, h from higher.
template <int k, int G, bool MAXOP>
__device__ __forceinline__ void lane_vhgw_step(const LaneVhgw<MAXOP> &V, uint32_t *g0, uint32_t *g1,
                                               uint32_t *h0, uint32_t *h1)
{
    const int lane = threadIdx.x & 63;
    constexpr int q = (1 << k) / 4; // whole lanes (k >= 2)
#pragma unroll
    for (int r = 0; r < G; r++) {
        uint32_t a0, a1, b0, b1; // g[p - s], h[p + s] as pair dwords
        if constexpr (k == 0) {
            const uint32_t pv = from_prev_lane(g1[r]);
            a0 = __builtin_amdgcn_alignbit(g0[r], pv, 16);
            a1 = __builtin_amdgcn_alignbit(g1[r], g0[r], 16);
            const uint32_t nx = from_next_lane(h0[r]);
            b0 = __builtin_amdgcn_alignbit(h1[r], h0[r], 16);
            b1 = __builtin_amdgcn_alignbit(nx, h1[r], 16);
        } else if constexpr (k == 1) {
            a0 = from_prev_lane(g1[r]);
            a1 = g0[r];
            b0 = h1[r];
            b1 = from_next_lane(h0[r]);
        } else if constexpr (q == 1) {
            a0 = from_prev_lane(g0[r]);
            a1 = from_prev_lane(g1[r]);
            b0 = from_next_lane(h0[r]);
            b1 = from_next_lane(h1[r]);
        } else {
            const uint32_t adp = (uint32_t)((lane - q) & 63) << 2, adn = (uint32_t)((lane + q) & 63) << 2;
            a0 = lane_fetch(g0[r], adp);
            a1 = lane_fetch(g1[r], adp);
            b0 = lane_fetch(h0[r], adn);
            b1 = lane_fetch(h1[r], adn);
        }
        g0[r] = pk<MAXOP>(g0[r], LaneVhgw<MAXOP>::keep(a0, V.gm[k][0]));
        g1[r] = pk<MAXOP>(g1[r], LaneVhgw<MAXOP>::keep(a1, V.gm[k][1]));
        h0[r] = pk<MAXOP>(h0[r], LaneVhgw<MAXOP>::keep(b0, V.hm[k][0]));
        h1[r] = pk<MAXOP>(h1[r], LaneVhgw<MAXOP>::keep(b1, V.hm[k][1]));
    }
}

// m_w[k] = op(h[k], g[k + w - 1]) at k = co .. co + 3: h's pairs from the lane and the
// next one, g's from lanes + q1 and + q1 + 1.
template <int C0, int C1, int G, bool MAXOP>
__device__ __forceinline__ void lane_vhgw_final(const LaneVhgw<MAXOP> &V, uint32_t *h0,
                                                uint32_t *h1, const uint32_t *g0,
                                                const uint32_t *g1)
{
#pragma unroll
    for (int r = 0; r < G; r++) {
        const uint32_t n0 = from_next_lane(h0[r]), n1 = (C0 >> 1) ? from_next_lane(h1[r]) : 0u;
        uint32_t p0, p2, r0, r2;
        pairs_at<C0>(h0[r], h1[r], n0, n1, p0, p2);
        const uint32_t f0 = (C1 >> 1) ? 0u : lane_fetch(g0[r], V.ad0), f1 = lane_fetch(g1[r], V.ad0);
        const uint32_t f2 = lane_fetch(g0[r], V.ad1), f3 = (C1 >> 1) ? lane_fetch(g1[r], V.ad1) : 0u;
        pairs_at<C1>(f0, f1, f2, f3, r0, r2);
        h0[r] = pk<MAXOP>(p0, r0);
        h1[r] = pk<MAXOP>(p2, r2);
    }
}

// The horizontal vHGW pass on G rows: e0, e1 hold the rows on entry and the outputs
// on return.  The rows go through each step together so their lane moves interleave.
template <int G, bool MAXOP>
__device__ __forceinline__ void lane_vhgw_rows(const LaneVhgw<MAXOP> &V, uint32_t *e0, uint32_t *e1)
{
    uint32_t g0[G], g1[G];
#pragma unroll
    for (int r = 0; r < G; r++) {
        g0[r] = e0[r];
        g1[r] = e1[r];
    }
    // (e0, e1 become h)
    if (V.K > 0) lane_vhgw_step<0, G, MAXOP>(V, g0, g1, e0, e1);
    if (V.K > 1) lane_vhgw_step<1, G, MAXOP>(V, g0, g1, e0, e1);
    if (V.K > 2) lane_vhgw_step<2, G, MAXOP>(V, g0, g1, e0, e1);
    if (V.K > 3) lane_vhgw_step<3, G, MAXOP>(V, g0, g1, e0, e1);
    if (V.K > 4) lane_vhgw_step<4, G, MAXOP>(V, g0, g1, e0, e1);
    if (V.K > 5) lane_vhgw_step<5, G, MAXOP>(V, g0, g1, e0, e1);
    if (V.K > 6) lane_vhgw_step<6, G, MAXOP>(V, g0, g1, e0, e1);
    static_assert(kVhgwLaneSteps == 7, "steps unrolled");
#define MORPH_VF1(A, B)                                                                      \
    case A * 4 + B: lane_vhgw_final<A, B, G, MAXOP>(V, e0, e1, g0, g1); break;
#define MORPH_VF(A) MORPH_VF1(A, 0) MORPH_VF1(A, 1) MORPH_VF1(A, 2) MORPH_VF1(A, 3)
    switch (V.c0 * 4 + V.c1) {
        MORPH_VF(0) MORPH_VF(1) MORPH_VF(2) MORPH_VF(3)
    default: break;
    }
#undef MORPH_VF
#undef MORPH_VF1
}

// ======================= direct vertical pass: one wave per strip ==================
// When the vertical window is at most kDirectMax, a wave works alone on a strip of
// 64 column quads and J.TB output rows, KR rows at a time: the vertical pass in
// registers, then the horizontal pass in registers too, taking the columns right
// of its own quad from the next lanes with wave-wide DPP shifts (v_mov_b32_dpp
// wave_shl:1): the direct pass, or for wider windows the doubling pass.  No LDS,
// no barrier.  The last lanes of the wave only supply those columns: a wave stores
// wq = J.TW / 4 = stream_quads(wx) quads, those whose input lies in its 64.
// Input quad Q starts at image column gxa + 4Q, gxa = 4 wq sx - ax - co, where co
// puts the quad grid on multiples of the load size; output quad Q (columns 4Q ..
// 4Q + 3 of the strip) reads input pixels 4Q + co .. 4Q + co + 3 + wx - 1.  The
// wy - 1 input rows that two chunks of KR rows share stay in registers: a ring of
// KR + wy - 1 rows moves down KR rows per chunk.
//
// Pixels outside the image are not replaced by the identity here but by the
// nearest image pixel (rows and columns clamped into the image).  For a flat
// window the two give the same result: the output pixel itself lies in its window
// and windows are contiguous, so every clamped-to row or column is already in the
// window, and a repeated value changes no minimum or maximum.  Clamping costs no
// per-pixel work: rows are clamped on the scalar unit, and a lane whose quad
// reaches outside loads the nearest quad inside and picks its pixels with the
// byte selectors of the widening v_perm (uint8) or of one v_perm per output row
// (uint16).
constexpr int KR = kWaveRows;
static_assert(KR == 8, "chunk8_window takes the vertical windows of a chunk");
// registers of the row ring: the short form (wy <= kDirectMax) and the tall one
template <bool TALL> constexpr int ring_rows() { return KR + (TALL ? kDirectMaxTall : kDirectMax) - 1; }

// Rows with 4-aligned (uint8) / 8-aligned (uint16) pitch: lane set-up for a unit.
// Loads go through a buffer resource on the image (it spans < 4 GiB): the row
// offset is a scalar operand and the lane's column offset a fixed vector operand,
// so a row costs no vector instruction to address.
template <typename T> struct WaveLoader {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t pitch;       // bytes
    int H;
    uint32_t voff;        // byte offset of the lane's (clamped) quad within a row
    uint32_t s01, s23;    // v_perm selectors that pick the lane's four pixels

    __device__ __forceinline__ WaveLoader(const TileJob &J, int mis, int gx)
    {
        const uint8_t *abase = J.src - mis * (int)sizeof(T);
        pitch = (uint32_t)J.pitch;
        H = J.H;
        const uint64_t span = (uint64_t)(J.H - 1) * J.pitch + (uint64_t)(J.W + mis + 3) * sizeof(T);
        rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)abase, (short)0,
                                                 (int)(uint32_t)min(span, (uint64_t)0xffffffffu),
                                                 kBufferWord3);
        // the lane's quad covers image columns gx .. gx + 3 (gx + mis a multiple of
        // 4); outside the image, take the quad holding column 0 or W - 1
        int gq = gx;
        if (gx + 3 < 0) gq = -mis;
        else if (gx > J.W - 1) gq = ((J.W - 1 + mis) & ~3) - mis;
        voff = (uint32_t)(gq + mis) * (uint32_t)sizeof(T);
        int b[4];
#pragma unroll
        for (int j = 0; j < 4; j++) b[j] = min(max(gx + j, 0), J.W - 1) - gq;
        if constexpr (sizeof(T) == 1) {
            // widen bytes b0, b1 (b2, b3) into the two u16 halves; 0x0c gives 0
            s01 = (uint32_t)b[0] | 0x0c00u | ((uint32_t)b[1] << 16) | 0x0c000000u;
            s23 = (uint32_t)b[2] | 0x0c00u | ((uint32_t)b[3] << 16) | 0x0c000000u;
        } else {
            // u16 halves of {p23, p01}: pixel b is bytes 2b, 2b + 1
            s01 = (uint32_t)(2 * b[0]) | (uint32_t)(2 * b[0] + 1) << 8 |
                  (uint32_t)(2 * b[1]) << 16 | (uint32_t)(2 * b[1] + 1) << 24;
            s23 = (uint32_t)(2 * b[2]) | (uint32_t)(2 * b[2] + 1) << 8 |
                  (uint32_t)(2 * b[3]) << 16 | (uint32_t)(2 * b[3] + 1) << 24;
        }
    }
    // input row gy (clamped into the image; gy is the same in every lane): the load,
    // then the lane's four pixels as two pair dwords
    using Raw = typename std::conditional<sizeof(T) == 1, uint32_t, uint64_t>::type;
    __device__ __forceinline__ Raw issue(int gy) const
    {
        return issue_at((uint32_t)min(max(gy, 0), H - 1) * pitch);
    }
    // the row at byte offset soff (a row inside the image)
    __device__ __forceinline__ Raw issue_at(uint32_t soff_) const
    {
        const int soff = (int)soff_;
        if constexpr (sizeof(T) == 1) {
            return __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)voff, soff, 0);
        } else {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, (int)voff, soff, 0);
            return (uint64_t)v[0] | ((uint64_t)v[1] << 32);
        }
    }
    __device__ __forceinline__ void widen(Raw d, uint32_t &v01, uint32_t &v23) const
    {
        if constexpr (sizeof(T) == 1) {
            v01 = perm(0u, d, s01);
            v23 = perm(0u, d, s23);
        } else {
            v01 = (uint32_t)d;
            v23 = (uint32_t)(d >> 32);
        }
    }
    __device__ __forceinline__ void row(int gy, uint32_t &v01, uint32_t &v23) const
    {
        widen(issue(gy), v01, v23);
    }
    template <int N>
    __device__ __forceinline__ void rows(int gy0, uint32_t *v01, uint32_t *v23) const
    {
#pragma unroll
        for (int k = 0; k < N; k++) row(gy0 + k, v01[k], v23[k]);
    }
    // uint16: pick the lane's pixels from an output row computed on the raw quad
    __device__ __forceinline__ void fix(uint32_t &v01, uint32_t &v23) const
    {
        const uint32_t a = perm(v23, v01, s01), b = perm(v23, v01, s23);
        v01 = a;
        v23 = b;
    }
};

// The unit's first WY - 1 input rows into the ring, and the loads of the first
// chunk's KR new rows (input row gy0 + WY - 1 onwards) into raw.
template <int WY, typename Ld>
__device__ __forceinline__ void wv_first(const Ld &L, int gy0, uint32_t *r01, uint32_t *r23,
                                         typename Ld::Raw *raw)
{
    L.template rows<WY - 1>(gy0, r01, r23);
#pragma unroll
    for (int m = 0; m < KR; m++) raw[m] = L.issue(gy0 + WY - 1 + m);
}

// One chunk's vertical pass: its KR new rows (the loads in cur, issued during the
// previous chunk) into the ring, its output rows, and the ring moved down for the
// next chunk.
template <int WY, bool MAXOP, typename Ld>
__device__ __forceinline__ void wv_vertical(const Ld &L, const typename Ld::Raw *cur,
                                            uint32_t *r01, uint32_t *r23, uint32_t *o01,
                                            uint32_t *o23)
{
#pragma unroll
    for (int m = 0; m < KR; m++) L.widen(cur[m], r01[WY - 1 + m], r23[WY - 1 + m]);
    if constexpr (WY >= KR) {
        chunk8_window<WY, MAXOP>(r01, o01);
        chunk8_window<WY, MAXOP>(r23, o23);
    } else {
#pragma unroll
        for (int m = 0; m < KR; m += 2) {
            pair_window<WY, MAXOP>(r01 + m, o01[m], o01[m + 1]);
            pair_window<WY, MAXOP>(r23 + m, o23[m], o23[m + 1]);
        }
    }
#pragma unroll
    for (int k = 0; k < WY - 1; k++) {
        r01[k] = r01[k + KR];
        r23[k] = r23[k + KR];
    }
}

// The tall form keeps its ring of input rows as loaded (one register a row for
// uint8 quads), widening each row where a chunk uses it: the same pairs of outputs
// share their WY - 1 middle rows as in pair_window, with the rows visited once each.
template <int WY, typename Ld>
__device__ __forceinline__ void wv_first_raw(const Ld &L, int gy0, typename Ld::Raw *ring,
                                             typename Ld::Raw *raw)
{
#pragma unroll
    for (int k = 0; k < WY - 1; k++) ring[k] = L.issue(gy0 + k);
#pragma unroll
    for (int m = 0; m < KR; m++) raw[m] = L.issue(gy0 + WY - 1 + m);
}

template <int WY, bool MAXOP, typename Ld>
__device__ __forceinline__ void wv_vertical_raw(const Ld &L, const typename Ld::Raw *cur,
                                                typename Ld::Raw *ring, uint32_t *o01,
                                                uint32_t *o23)
{
#pragma unroll
    for (int m = 0; m < KR; m++) ring[WY - 1 + m] = cur[m];
    if constexpr (WY <= 2) { // (no middle rows to share)
#pragma unroll
        for (int m = 0; m < KR; m++) {
            L.widen(ring[m], o01[m], o23[m]);
            if constexpr (WY == 2) {
                uint32_t x01, x23;
                L.widen(ring[m + 1], x01, x23);
                o01[m] = pk<MAXOP>(o01[m], x01);
                o23[m] = pk<MAXOP>(o23[m], x23);
            }
        }
#pragma unroll
        for (int k = 0; k < WY - 1; k++) ring[k] = ring[k + KR];
        return;
    }
    if constexpr (WY >= KR) { // (every row widened once, then the chunk's shared form)
        uint32_t x01[WY + KR - 1], x23[WY + KR - 1];
#pragma unroll
        for (int r = 0; r < WY + KR - 1; r++) L.widen(ring[r], x01[r], x23[r]);
        chunk8_window<WY, MAXOP>(x01, o01);
        chunk8_window<WY, MAXOP>(x23, o23);
#pragma unroll
        for (int k = 0; k < WY - 1; k++) ring[k] = ring[k + KR];
        return;
    }
    uint32_t c01[KR / 2], c23[KR / 2]; // output pair p: the extremum of rows 2p + 1 .. 2p + WY - 1
#pragma unroll
    for (int r = 0; r < WY + KR - 1; r++) {
        uint32_t x01, x23;
        L.widen(ring[r], x01, x23);
#pragma unroll
        for (int p = 0; p < KR / 2; p++) {
            const int a = 2 * p; // outputs a (rows a .. a + WY - 1) and a + 1
            if (r == a) {
                o01[a] = x01;
                o23[a] = x23;
            } else if (r == a + 1) {
                c01[p] = x01;
                c23[p] = x23;
            } else if (r < a + WY) {
                if (r > a + 1) {
                    c01[p] = pk<MAXOP>(c01[p], x01);
                    c23[p] = pk<MAXOP>(c23[p], x23);
                }
            } else if (r == a + WY) {
                o01[a + 1] = x01;
                o23[a + 1] = x23;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < KR / 2; p++) {
        o01[2 * p] = pk<MAXOP>(c01[p], o01[2 * p]);
        o23[2 * p] = pk<MAXOP>(c23[p], o23[2 * p]);
        o01[2 * p + 1] = pk<MAXOP>(c01[p], o01[2 * p + 1]);
        o23[2 * p + 1] = pk<MAXOP>(c23[p], o23[2 * p + 1]);
    }
#pragma unroll
    for (int k = 0; k < WY - 1; k++) ring[k] = ring[k + KR];
}

// Rows of any pitch: the general loader (identity outside the image).
template <typename T> struct WaveLoaderAny {
    RowLoader<T, false> L;
    int gx;
    __device__ __forceinline__ WaveLoaderAny(const TileJob &J, uint32_t id, int gx_)
        : L(J.src, J.pitch, J.H, J.W, id, 0u), gx(gx_)
    {
    }
    template <int N>
    __device__ __forceinline__ void rows(int gy0, uint32_t *v01, uint32_t *v23) const
    {
        load_rows<N>(L, gy0, 1, gx, N, v01, v23);
    }
    struct Raw {
        uint32_t a, b;
    };
    __device__ __forceinline__ Raw issue(int gy) const
    {
        Raw r;
        L.load_any(gy, gx, true, r.a, r.b);
        return r;
    }
    __device__ __forceinline__ void widen(Raw d, uint32_t &v01, uint32_t &v23) const
    {
        v01 = d.a;
        v23 = d.b;
    }
};

template <int WX, int CO, bool MAXOP>
__device__ __forceinline__ void wv_horizontal_row(uint32_t &v01, uint32_t &v23)
{
    constexpr int NPX = CO + WX + 3; // pixels 0 .. CO + WX + 2 of the span
    constexpr int NQ = (NPX + 3) / 4;
    uint32_t d[2 * NQ]; // d[k] = pixels (2k, 2k + 1)
    d[0] = v01;
    d[1] = v23;
#pragma unroll
    for (int q = 1; q < NQ; q++) {
        d[2 * q] = from_next_lane(d[2 * q - 2]);
        d[2 * q + 1] = from_next_lane(d[2 * q - 1]);
    }
    uint32_t p[NPX - 1]; // p[k] = pixels (k, k + 1)
#pragma unroll
    for (int k = 0; k < NPX - 1; k++)
        p[k] = (k & 1) ? __builtin_amdgcn_alignbit(d[(k + 1) / 2], d[(k - 1) / 2], 16) : d[k / 2];
    if constexpr (WX == 1) {
        v01 = p[CO];
        v23 = p[CO + 2];
    } else if constexpr (WX == 2) {
        v01 = pk<MAXOP>(p[CO], p[CO + 1]);
        v23 = pk<MAXOP>(p[CO + 2], p[CO + 3]);
    } else {
        // the two output pairs share the window starts CO + 2 .. CO + WX - 1
        uint32_t core = p[CO + 2];
#pragma unroll
        for (int t = CO + 3; t < CO + WX; t++) core = pk<MAXOP>(core, p[t]);
        v01 = pk<MAXOP>(pk<MAXOP>(core, p[CO]), p[CO + 1]);
        v23 = pk<MAXOP>(pk<MAXOP>(core, p[CO + WX]), p[CO + WX + 1]);
    }
}

template <int WX, int CO, bool MAXOP>
__device__ __forceinline__ void wv_horizontal(uint32_t *v01, uint32_t *v23)
{
#pragma unroll
    for (int m = 0; m < KR; m++) wv_horizontal_row<WX, CO, MAXOP>(v01[m], v23[m]);
}

template <bool MAXOP>
__device__ __forceinline__ void wv_horizontal_any(int wx, int co, uint32_t *v01, uint32_t *v23)
{
#define MORPH_WH(W)                                                                          \
    case W * 4 + 0: wv_horizontal<W, 0, MAXOP>(v01, v23); break;                             \
    case W * 4 + 1: wv_horizontal<W, 1, MAXOP>(v01, v23); break;                             \
    case W * 4 + 2: wv_horizontal<W, 2, MAXOP>(v01, v23); break;                             \
    case W * 4 + 3: wv_horizontal<W, 3, MAXOP>(v01, v23); break;
    switch (wx * 4 + co) {
        MORPH_WH(1) MORPH_WH(2) MORPH_WH(3) MORPH_WH(4) MORPH_WH(5) MORPH_WH(6) MORPH_WH(7)
        MORPH_WH(8) MORPH_WH(9) MORPH_WH(10) MORPH_WH(11) MORPH_WH(12) MORPH_WH(13)
        MORPH_WH(14) MORPH_WH(15) MORPH_WH(16)
    default: break;
    }
    static_assert(kDirectMaxX == 16, "horizontal direct windows compiled");
#undef MORPH_WH
}

#define MORPH_WY_SWITCH(WYV, CALL)                                                           \
    switch (WYV) {                                                                           \
    case 1: CALL(1); break;                                                                  \
    case 2: CALL(2); break;                                                                  \
    case 3: CALL(3); break;                                                                  \
    case 4: CALL(4); break;                                                                  \
    case 5: CALL(5); break;                                                                  \
    case 6: CALL(6); break;                                                                  \
    case 7: CALL(7); break;                                                                  \
    case 8: CALL(8); break;                                                                  \
    default: CALL(9); break;                                                                 \
    }

#define MORPH_WY_SWITCH_TALL(WYV, CALL)                                                      \
    switch (WYV) {                                                                           \
    case 10: CALL(10); break;                                                                \
    case 11: CALL(11); break;                                                                \
    case 12: CALL(12); break;                                                                \
    case 13: CALL(13); break;                                                                \
    case 14: CALL(14); break;                                                                \
    case 15: CALL(15); break;                                                                \
    case 16: CALL(16); break;                                                                \
    case 17: CALL(17); break;                                                                \
    case 18: CALL(18); break;                                                                \
    case 19: CALL(19); break;                                                                \
    case 20: CALL(20); break;                                                                \
    case 21: CALL(21); break;                                                                \
    case 22: CALL(22); break;                                                                \
    case 23: CALL(23); break;                                                                \
    case 24: CALL(24); break;                                                                \
    case 25: CALL(25); break;                                                                \
    case 26: CALL(26); break;                                                                \
    case 27: CALL(27); break;                                                                \
    case 28: CALL(28); break;                                                                \
    case 29: CALL(29); break;                                                                \
    case 30: CALL(30); break;                                                                \
    default: CALL(31); break;                                                                \
    }
static_assert(kDirectMaxTall == 31, "tall vertical windows compiled");

// TALL: the vertical window is kDirectMax + 1 .. kDirectMaxTall (a longer register ring,
// so fewer waves fit a SIMD; a kernel of its own); else 1 .. kDirectMax.
// XV: the horizontal pass is the cross-lane vHGW (wx <= kStreamMaxWx; a kernel of its
// own, for single images whose plan asks for it).
template <typename T, bool MAXOP, bool AL, bool TALL = false, bool XV = false, bool NTS = true>
__device__ __forceinline__ void wave_body(const TileJob &J, int unit)
{
    constexpr int RING = ring_rows<TALL>();
    const int lane = threadIdx.x & 63;
    const int sx = unit % J.tiles_x, sy = unit / J.tiles_x;
    const int mis = AL ? (int)(((uintptr_t)J.src & (4 * sizeof(T) - 1)) / sizeof(T)) : 0;
    const int co = (mis - J.ax) & 3;
    const int wq = J.TW >> 2; // output quads per strip
    const int gxa = 4 * wq * sx - J.ax - co; // lane 0's first input column
    const int gx = gxa + 4 * lane;
    const int y0 = sy * J.TB;
    const int y1 = min(y0 + J.TB, J.H);
    // uint16 lanes whose quad reaches outside the image pick their pixels per row
    const bool edge = gxa < 0 || gxa + 4 * 64 > J.W;
    using Ld = typename std::conditional<AL, WaveLoader<T>, WaveLoaderAny<T>>::type;
    const Ld L = [&]() {
        if constexpr (AL) return WaveLoader<T>(J, mis, gx);
        else return WaveLoaderAny<T>(J, MAXOP ? 0u : (Px<T>::maxv | (Px<T>::maxv << 16)), gx);
    }();
    using Raw = typename Ld::Raw;
    // the ring of input rows: widened (short form) or as loaded (tall form)
    uint32_t r01[TALL ? 1 : RING], r23[TALL ? 1 : RING];
    Raw rr[TALL ? RING : 1];
    Raw ra[KR], rb[KR];
    if constexpr (TALL) {
#define MORPH_FIRST(W) wv_first_raw<W>(L, y0 - J.ay, rr, ra)
        MORPH_WY_SWITCH_TALL(J.wy, MORPH_FIRST)
#undef MORPH_FIRST
    } else {
#define MORPH_FIRST(W) wv_first<W>(L, y0 - J.ay, r01, r23, ra)
        MORPH_WY_SWITCH(J.wy, MORPH_FIRST)
#undef MORPH_FIRST
    }
    // destination: 4-byte aligned rows and a strip wholly inside the image take
    // one plain store per row and lane (a choice the whole wave makes, outside the
    // row loop)
    const int Q = wq * sx + lane;
    const bool fast_store = (((uintptr_t)J.dst | (uintptr_t)J.dpitch) & 3) == 0 &&
                            4 * (wq * sx + wq) <= J.W;
    const bool doubling = J.hm == PASS_DOUBLING;
    const Doubling S(J.wx, co);
    const LaneVhgw<MAXOP> V(XV ? J.wx : 1, co);
    int y = y0;
    // rows y .. y + KR - 1 from the loads in cur, the next chunk's issued into nxt
    // (two buffers taking turns, so no load in flight is ever copied)
    auto chunk = [&](Raw (&cur)[KR], Raw (&nxt)[KR]) __attribute__((always_inline)) -> bool {
        uint32_t v01[KR], v23[KR];
        const bool more = y + KR < y1;
        // the next chunk's KR new rows (input row gn onwards) complete while this
        // chunk's passes and stores run; they are widened only by the next chunk
        if (more) {
            const int gn = y + KR - J.ay + J.wy - 1;
#pragma unroll
            for (int m = 0; m < KR; m++) nxt[m] = L.issue(gn + m);
        }
        if constexpr (TALL) {
#define MORPH_VERT(W) wv_vertical_raw<W, MAXOP>(L, cur, rr, v01, v23)
            MORPH_WY_SWITCH_TALL(J.wy, MORPH_VERT)
#undef MORPH_VERT
        } else {
#define MORPH_VERT(W) wv_vertical<W, MAXOP>(L, cur, r01, r23, v01, v23)
            MORPH_WY_SWITCH(J.wy, MORPH_VERT)
#undef MORPH_VERT
        }
        if constexpr (AL && sizeof(T) == 2) {
            if (edge) {
#pragma unroll
                for (int m = 0; m < KR; m++) L.fix(v01[m], v23[m]);
            }
        }
        // every lane takes part in the shifts
        if constexpr (XV) lane_vhgw_rows<KR, MAXOP>(V, v01, v23);
        else if (doubling) doubling_rows<KR, MAXOP>(S, v01, v23);
        else wv_horizontal_any<MAXOP>(J.wx, co, v01, v23);
        if (lane < wq) {
            uint8_t *drow = J.dst + (int64_t)y * J.dpitch;
            if (fast_store) {
                const uint32_t o = (uint32_t)Q * 4u * (uint32_t)sizeof(T);
#pragma unroll
                for (int m = 0; m < KR; m++) {
                    if (y + m < y1) {
                        if constexpr (sizeof(T) == 1) {
                            store_u32<NTS>((uintptr_t)(drow + o),
                                           perm(v23[m], v01[m], SEL_NARROW));
                        } else {
                            store_u32<NTS>((uintptr_t)(drow + o), v01[m]);
                            store_u32<NTS>((uintptr_t)(drow + o + 4), v23[m]);
                        }
                    }
                    drow += J.dpitch;
                }
            } else {
#pragma unroll
                for (int m = 0; m < KR; m++) {
                    if (y + m < y1) Px<T>::template store<NTS>(drow, 4 * Q, J.W, v01[m], v23[m]);
                    drow += J.dpitch;
                }
            }
        }
        y += KR;
        return more;
    };
    while (chunk(ra, rb) && chunk(rb, ra)) {
    }
}

// ======================= morphological gradient: both extrema from one read ========
// Dilation minus erosion with the same rectangle (one of §2's combinations of the
// two), on the wave kernel's path: a direct vertical window and rows of aligned
// pitch, whose loads clamp to the image, so that one loaded row serves the minimum
// and the maximum alike (with the identity border the two would need different
// fill values).  The vertical and horizontal passes run twice on the same
// registers, once per extremum, and the difference is stored: 2 sizeof(T) bytes a
// pixel instead of the 6 of erosion, dilation and a subtraction through memory.
template <int WY, typename Ld>
__device__ __forceinline__ void wv_vertical2(const Ld &L, const typename Ld::Raw *cur,
                                             uint32_t *r01, uint32_t *r23, uint32_t *lo01,
                                             uint32_t *lo23, uint32_t *hi01, uint32_t *hi23)
{
#pragma unroll
    for (int m = 0; m < KR; m++) L.widen(cur[m], r01[WY - 1 + m], r23[WY - 1 + m]);
    if constexpr (WY >= KR) {
        chunk8_window<WY, false>(r01, lo01);
        chunk8_window<WY, false>(r23, lo23);
        chunk8_window<WY, true>(r01, hi01);
        chunk8_window<WY, true>(r23, hi23);
    } else {
#pragma unroll
        for (int m = 0; m < KR; m += 2) {
            pair_window<WY, false>(r01 + m, lo01[m], lo01[m + 1]);
            pair_window<WY, false>(r23 + m, lo23[m], lo23[m + 1]);
            pair_window<WY, true>(r01 + m, hi01[m], hi01[m + 1]);
            pair_window<WY, true>(r23 + m, hi23[m], hi23[m + 1]);
        }
    }
#pragma unroll
    for (int k = 0; k < WY - 1; k++) {
        r01[k] = r01[k + KR];
        r23[k] = r23[k + KR];
    }
}

// a - b in each 16-bit half (b <= a in both)
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b)
{
    const u16x2 x = __builtin_bit_cast(u16x2, a), y = __builtin_bit_cast(u16x2, b);
    return __builtin_bit_cast(uint32_t, (u16x2)(x - y));
}

template <typename T>
__device__ __forceinline__ void grad_body(const TileJob &J, int unit)
{
    const int lane = threadIdx.x & 63;
    const int sx = unit % J.tiles_x, sy = unit / J.tiles_x;
    const int mis = (int)(((uintptr_t)J.src & (4 * sizeof(T) - 1)) / sizeof(T));
    const int co = (mis - J.ax) & 3;
    const int wq = J.TW >> 2; // output quads per strip
    const int gxa = 4 * wq * sx - J.ax - co; // lane 0's first input column
    const int gx = gxa + 4 * lane;
    const int y0 = sy * J.TB;
    const int y1 = min(y0 + J.TB, J.H);
    const bool edge = gxa < 0 || gxa + 4 * 64 > J.W;
    using Ld = WaveLoader<T>;
    const Ld L(J, mis, gx);
    constexpr int RING = ring_rows<false>(); // vertical windows up to kDirectMax
    uint32_t r01[RING], r23[RING];
    using Raw = typename Ld::Raw;
    Raw ra[KR], rb[KR];
#define MORPH_FIRST(W) wv_first<W>(L, y0 - J.ay, r01, r23, ra)
    MORPH_WY_SWITCH(J.wy, MORPH_FIRST)
#undef MORPH_FIRST
    const int Q = wq * sx + lane;
    const bool fast_store = (((uintptr_t)J.dst | (uintptr_t)J.dpitch) & 3) == 0 &&
                            4 * (wq * sx + wq) <= J.W;
    const bool doubling = J.hm == PASS_DOUBLING;
    const Doubling S(J.wx, co);
    int y = y0;
    auto chunk = [&](Raw (&cur)[KR], Raw (&nxt)[KR]) __attribute__((always_inline)) -> bool {
        uint32_t lo01[KR], lo23[KR], hi01[KR], hi23[KR];
        const bool more = y + KR < y1;
        if (more) {
            const int gn = y + KR - J.ay + J.wy - 1;
#pragma unroll
            for (int m = 0; m < KR; m++) nxt[m] = L.issue(gn + m);
        }
#define MORPH_VERT2(W) wv_vertical2<W>(L, cur, r01, r23, lo01, lo23, hi01, hi23)
        MORPH_WY_SWITCH(J.wy, MORPH_VERT2)
#undef MORPH_VERT2
        if constexpr (sizeof(T) == 2) {
            if (edge) {
#pragma unroll
                for (int m = 0; m < KR; m++) {
                    L.fix(lo01[m], lo23[m]);
                    L.fix(hi01[m], hi23[m]);
                }
            }
        }
        // every lane takes part in the shifts
        if (doubling) {
            doubling_rows<KR, false>(S, lo01, lo23);
            doubling_rows<KR, true>(S, hi01, hi23);
        } else {
            wv_horizontal_any<false>(J.wx, co, lo01, lo23);
            wv_horizontal_any<true>(J.wx, co, hi01, hi23);
        }
        if (lane < wq) {
            uint8_t *drow = J.dst + (int64_t)y * J.dpitch;
#pragma unroll
            for (int m = 0; m < KR; m++) {
                const uint32_t v01 = pk_sub(hi01[m], lo01[m]), v23 = pk_sub(hi23[m], lo23[m]);
                if (y + m < y1) {
                    if (fast_store) {
                        const uintptr_t o = (uintptr_t)(drow + (uint32_t)Q * 4u * (uint32_t)sizeof(T));
                        if constexpr (sizeof(T) == 1) {
                            store_u32(o, perm(v23, v01, SEL_NARROW));
                        } else {
                            store_u32(o, v01);
                            store_u32(o + 4, v23);
                        }
                    } else {
                        Px<T>::store(drow, 4 * Q, J.W, v01, v23);
                    }
                }
                drow += J.dpitch;
            }
        }
        y += KR;
        return more;
    };
    while (chunk(ra, rb) && chunk(rb, ra)) {
    }
}
#undef MORPH_WY_SWITCH

// ======================= wide rows: vertical window 1, 16 pixels per lane ===========
// A horizontal window too wide for a 64-quad strip (wx > 128) with a vertical window
// of 1: a lane holds four quads of a row (16 pixels as eight pair dwords), so a wave
// covers 1024 pixels and stores rows_lanes(wx) lanes' worth of them.  The doubling
// pass as above: shifts of up to 16 pixels take the lane and the next one (DPP),
// shifts of whole lanes ds_bpermute.  The final step, op(m_L[k], m_L[k + wx - L]) at
// k = co .. co + 15, reads m_L back from a copy of the row in LDS at offsets that are
// the same in every lane (uint8: as bytes, the first operand from the lane's own
// quads and the next lane's first; uint16: as pixel pairs, both operands from LDS);
// byte or half-dword shifts (alignbyte, alignbit) take the offsets at run time, so
// every row takes the same straight-line code and the rows of a group go through
// each step together.
constexpr int NP16 = 8; // pair dwords per lane
// rows of a group: 4 (uint8) or 2 (uint16), so that a wave's LDS is 6 KB either way
template <typename T> constexpr int rows_group() { return sizeof(T) == 1 ? 4 : 2; }
// LDS per row of a group: m_L (1024 bytes for uint8, 2048 for uint16), and reads of
// lanes that store nothing run on to byte 16 * 63 + 3 + (1000 - 512) + 20 < 1536
// (uint8) or dword 8 * 63 + (3 + 1000 - 512) / 2 + 9 <= 768 (uint16)
template <typename T> constexpr int rows_lds_dwords() { return sizeof(T) == 1 ? 384 : 768; }
constexpr int kRowsWaveLdsDwords = 1536; // per wave: rows_group<T>() * rows_lds_dwords<T>()
static_assert(kRowsMaxWx <= 1000 && 16 * 63 + 3 + (1000 - 512) + 20 <= 4 * 384 &&
                  8 * 63 + (3 + 1000 - 512) / 2 + 9 <= 768,
              "wide-row LDS reads must stay inside a row's region");
static_assert(4 * 384 == kRowsWaveLdsDwords && 2 * 768 == kRowsWaveLdsDwords, "");

// Pixel pair (D, D + 1) of the lane's 16 pixels followed by 16 more (n).
template <int D>
__device__ __forceinline__ uint32_t pair16(const uint32_t *e, const uint32_t *n)
{
    constexpr int i = D / 2;
    uint32_t lo, hi = 0;
    if constexpr (i < NP16) lo = e[i];
    else lo = n[i - NP16];
    if constexpr (D % 2 == 0) {
        return lo;
    } else {
        if constexpr (i + 1 < NP16) hi = e[i + 1];
        else hi = n[i + 1 - NP16];
        return __builtin_amdgcn_alignbit(hi, lo, 16);
    }
}

// e[i] = op(e[i], pair at 2i + S) for all eight pairs, S pixels (S <= 16) to the right.
template <int S, bool MAXOP, int... I>
__device__ __forceinline__ void level16_in(uint32_t *e, const uint32_t *n,
                                          std::integer_sequence<int, I...>)
{
    const uint32_t out[NP16] = {pk<MAXOP>(e[I], pair16<2 * I + S>(e, n))...};
    ((e[I] = out[I]), ...);
}

template <int S, bool MAXOP, int RG>
__device__ __forceinline__ void level16(uint32_t (&e)[RG][NP16])
{
    // next-lane pairs the shift reaches: pairs up to index (14 + S + 1) / 2
    constexpr int NN = (15 + S) / 2 + 1 - NP16;
#pragma unroll
    for (int m = 0; m < RG; m++) {
        uint32_t n[NP16];
#pragma unroll
        for (int k = 0; k < NP16; k++) n[k] = k < NN ? from_next_lane(e[m][k]) : 0u;
        level16_in<S, MAXOP>(e[m], n, std::make_integer_sequence<int, NP16>{});
    }
}

// Doubling across lanes: wx > 128, so L reaches 128 at least.
template <bool MAXOP, int RG>
__device__ __forceinline__ void doubling16(int wx, uint32_t (&e)[RG][NP16])
{
    const int lane = threadIdx.x & 63;
    level16<1, MAXOP, RG>(e);
    level16<2, MAXOP, RG>(e);
    level16<4, MAXOP, RG>(e);
    level16<8, MAXOP, RG>(e);
    level16<16, MAXOP, RG>(e);
    for (int q = 2; 32 * q <= wx; q *= 2) { // 16q -> 32q pixels: q lanes
        const uint32_t ad = (uint32_t)(lane + q) << 2;
#pragma unroll
        for (int m = 0; m < RG; m++)
#pragma unroll
            for (int i = 0; i < NP16; i++) e[m][i] = pk<MAXOP>(e[m][i], lane_fetch(e[m][i], ad));
    }
}

// The lane's 16 output pixels of one row, as four dwords of bytes: op of the pixels
// at byte offsets sh0 (0..3) and k1 (>= 0) past the lane's first, row = the row's
// LDS copy (its m_L bytes are written here).
template <bool MAXOP>
__device__ __forceinline__ void final16(const uint32_t *e, uint32_t *row, uint32_t sh0,
                                        uint32_t k1, uint4 &out)
{
    const int lane = threadIdx.x & 63;
    uint32_t w[5];
#pragma unroll
    for (int j = 0; j < 4; j++) w[j] = perm(e[2 * j + 1], e[2 * j], SEL_NARROW);
    w[4] = from_next_lane(w[0]);
    *(uint4 *)(row + 4 * lane) = uint4{w[0], w[1], w[2], w[3]};
    const uint32_t *r1 = row + 4 * lane + (k1 >> 2);
    uint32_t v[5];
#pragma unroll
    for (int j = 0; j < 5; j++) v[j] = r1[j];
    const uint32_t sh1 = k1 & 3;
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t a = __builtin_amdgcn_alignbyte(w[j + 1], w[j], sh0);
        const uint32_t b = __builtin_amdgcn_alignbyte(v[j + 1], v[j], sh1);
        const uint32_t lo = pk<MAXOP>(perm(0u, a, SEL_U8_01), perm(0u, b, SEL_U8_01));
        const uint32_t hi = pk<MAXOP>(perm(0u, a, SEL_U8_23), perm(0u, b, SEL_U8_23));
        o[j] = perm(hi, lo, SEL_NARROW);
    }
    out = uint4{o[0], o[1], o[2], o[3]};
}

// uint16: the lane's 16 output pixels as eight pair dwords, op of the pixels at
// offsets co (0..3) and k1 (>= 0) past the lane's first, both read back from the
// row's LDS copy (its m_L pairs are written here) and shifted by half a dword when
// the offset is odd.
template <bool MAXOP>
__device__ __forceinline__ void final16_u16(const uint32_t *e, uint32_t *row, uint32_t co,
                                            uint32_t k1, uint32_t *out)
{
    const int lane = threadIdx.x & 63;
    *(uint4 *)(row + 8 * lane) = uint4{e[0], e[1], e[2], e[3]};
    *(uint4 *)(row + 8 * lane + 4) = uint4{e[4], e[5], e[6], e[7]};
    const uint32_t *r0 = row + 8 * lane + (co >> 1);
    const uint32_t *r1 = row + 8 * lane + (k1 >> 1);
    uint32_t a[NP16 + 1], b[NP16 + 1];
#pragma unroll
    for (int j = 0; j <= NP16; j++) {
        a[j] = r0[j];
        b[j] = r1[j];
    }
    const uint32_t sh0 = (co & 1) * 16, sh1 = (k1 & 1) * 16;
#pragma unroll
    for (int j = 0; j < NP16; j++)
        out[j] = pk<MAXOP>(__builtin_amdgcn_alignbit(a[j + 1], a[j], sh0),
                           __builtin_amdgcn_alignbit(b[j + 1], b[j], sh1));
}

template <typename T, bool MAXOP, bool AL, bool NTS = true>
__device__ __forceinline__ void rows_body(const TileJob &J, int unit, uint32_t *lds)
{
    constexpr int RG = rows_group<T>();
    constexpr int LD = rows_lds_dwords<T>();
    const int lane = threadIdx.x & 63;
    const int sx = unit % J.tiles_x, sy = unit / J.tiles_x;
    const int mis = AL ? (int)(((uintptr_t)J.src & (4 * sizeof(T) - 1)) / sizeof(T)) : 0;
    const int co = (mis - J.ax) & 3;
    const int nl = J.TW >> 4;              // lanes that store
    const int gx = J.TW * sx - J.ax - co + 16 * lane; // the lane's first input column
    const int y0 = sy * J.TB;
    const int y1 = min(y0 + J.TB, J.H);
    using Ld = typename std::conditional<AL, WaveLoader<T>, WaveLoaderAny<T>>::type;
    auto mk = [&](int q) {
        if constexpr (AL) return WaveLoader<T>(J, mis, gx + 4 * q);
        else return WaveLoaderAny<T>(J, MAXOP ? 0u : (Px<T>::maxv | (Px<T>::maxv << 16)),
                                     gx + 4 * q);
    };
    const Ld L0 = mk(0), L1 = mk(1), L2 = mk(2), L3 = mk(3);
    // uint16 lanes whose quads reach outside the image pick their pixels per row
    const bool edge = gx - 16 * lane < 0 || gx - 16 * lane + 1024 > J.W;
    int L = 1;
    while (2 * L <= J.wx) L *= 2;
    const uint32_t k1 = (uint32_t)(co + J.wx - L); // byte offset of the second operand
    const int xo = J.TW * sx + 16 * lane;          // the lane's first output column
    const bool store_lane = lane < nl && xo < J.W;
    const bool fast_store = ((uintptr_t)J.dst & 3) == 0 && (J.dpitch & 3) == 0 && xo + 16 <= J.W;
    constexpr int ES = (int)sizeof(T);
    using Raw = typename Ld::Raw;
    auto issue = [&](Raw (&r)[RG][4], int y) {
#pragma unroll
        for (int m = 0; m < RG; m++) {
            const int gy = min(y + m, y1 - 1);
            r[m][0] = L0.issue(gy);
            r[m][1] = L1.issue(gy);
            r[m][2] = L2.issue(gy);
            r[m][3] = L3.issue(gy);
        }
    };
    int y = y0;
    // rows y .. y + RG - 1 (those past the unit repeat its last row and store
    // nothing) from cur, with the next group's loads in flight in nxt
    auto group = [&](Raw (&cur)[RG][4], Raw (&nxt)[RG][4]) -> bool {
        const bool more = y + RG < y1;
        if (more) issue(nxt, y + RG);
        uint32_t e[RG][NP16];
#pragma unroll
        for (int m = 0; m < RG; m++) {
            L0.widen(cur[m][0], e[m][0], e[m][1]);
            L1.widen(cur[m][1], e[m][2], e[m][3]);
            L2.widen(cur[m][2], e[m][4], e[m][5]);
            L3.widen(cur[m][3], e[m][6], e[m][7]);
            if constexpr (AL && sizeof(T) == 2) {
                if (edge) {
                    L0.fix(e[m][0], e[m][1]);
                    L1.fix(e[m][2], e[m][3]);
                    L2.fix(e[m][4], e[m][5]);
                    L3.fix(e[m][6], e[m][7]);
                }
            }
        }
        doubling16<MAXOP, RG>(J.wx, e); // every lane takes part in the lane moves
#pragma unroll
        for (int m = 0; m < RG; m++) {
            // the lane's 16 output pixels: four dwords of bytes (uint8) or eight
            // pair dwords (uint16)
            uint32_t o[4 * ES];
            if constexpr (sizeof(T) == 1) {
                uint4 q;
                final16<MAXOP>(e[m], lds + m * LD, (uint32_t)co, k1, q);
                o[0] = q.x;
                o[1] = q.y;
                o[2] = q.z;
                o[3] = q.w;
            } else {
                final16_u16<MAXOP>(e[m], lds + m * LD, (uint32_t)co, k1, o);
            }
            if (store_lane && y + m < y1) {
                uint8_t *drow = J.dst + (int64_t)(y + m) * J.dpitch;
                if (fast_store) {
                    const uintptr_t a = (uintptr_t)(drow + ES * xo);
#pragma unroll
                    for (int j = 0; j < 4 * ES; j++) store_u32<NTS>(a + 4 * j, o[j]);
                } else if constexpr (sizeof(T) == 1) {
#pragma unroll
                    for (int j = 0; j < 16; j++)
                        if (xo + j < J.W)
                            store_u8<NTS>((uintptr_t)(drow + xo + j),
                                          (uint8_t)(o[j >> 2] >> (8 * (j & 3))));
                } else {
#pragma unroll
                    for (int q = 0; q < 4; q++)
                        if (xo + 4 * q < J.W)
                            Px<T>::template store<NTS>(drow, xo + 4 * q, J.W, o[2 * q], o[2 * q + 1]);
                }
            }
        }
        y += RG;
        return more;
    };
    Raw ra[RG][4], rb[RG][4];
    issue(ra, y0);
    while (group(ra, rb) && group(rb, ra)) {
    }
}

// ======================= larger windows: one wave per strip, streaming down =======
// One wave per strip of 64 column quads and J.TB output rows, walking down the
// input rows once (no LDS shared between waves, no barrier):
//  - vertical pass, van Herk/Gil-Werman over blocks of wy input rows (the paper's
//    vHGW, Section 3.2) with a ring of wy rows in LDS per wave: while block b + 1
//    streams in, its prefix g runs in registers and output row s = b wy + j is
//    min(h_b[j], g over the first j rows of block b + 1), h_b read from the ring,
//    where the incoming row then takes its place; at the end of a block a backward
//    walk over the ring turns it into that block's suffixes h.
//  - horizontal pass on each output row as it is produced, across the lanes: the
//    direct pass (wx <= kDirectMax) or, for wider windows, a log-step doubling
//    (m_2L[k] = min(m_L[k], m_L[k + L]), then m_w[k] = min(m_L[k], m_L[k + w - L])
//    for the largest L <= w), whose shifts are lane moves (DPP, ds_bpermute).
// The wave stores the output quads whose input lies inside its 64 quads: J.TW / 4 of
// them.  Pixels outside the image are the nearest image pixels, as in the direct
// wave kernel.
constexpr int SD = kStreamChunk; // input rows per chunk (and rows in flight) per wave

template <int G, bool MAXOP>
__device__ __forceinline__ void direct_rows_any(int wx, int co, uint32_t *v01, uint32_t *v23)
{
#define MORPH_WH1(W, C)                                                                      \
    case W * 4 + C:                                                                          \
        _Pragma("unroll") for (int r = 0; r < G; r++)                                        \
            wv_horizontal_row<W, C, MAXOP>(v01[r], v23[r]);                                  \
        break;
#define MORPH_WH(W) MORPH_WH1(W, 0) MORPH_WH1(W, 1) MORPH_WH1(W, 2) MORPH_WH1(W, 3)
    // (the streaming kernel's direct windows stop at kDirectMax: more cases make the
    // chunk too large to keep its arrays in registers)
    switch (wx * 4 + co) {
        MORPH_WH(1) MORPH_WH(2) MORPH_WH(3) MORPH_WH(4) MORPH_WH(5) MORPH_WH(6) MORPH_WH(7)
        MORPH_WH(8) MORPH_WH(9)
    default: break;
    }
#undef MORPH_WH
#undef MORPH_WH1
}

// The per-wave ring of the vertical vHGW pass in LDS: stream_ring_entries(wy) entries
// (wy of them used; the rest let a chunk read SD entries from any position) of 64
// lanes.  uint8: an entry is a lane's raw quad (4 bytes), written as loaded and,
// once a block's suffixes replace it, as the narrowed suffix; uint16: the two pair
// dwords.
template <typename T> struct Ring;
template <> struct Ring<uint8_t> {
    uint32_t *e; // lane's entry 0; entry j at e[64 j]
    __device__ __forceinline__ explicit Ring(uint32_t *lds) : e(lds + (threadIdx.x & 63)) {}
    template <typename R>
    __device__ __forceinline__ void put(int j, R raw, uint32_t x01, uint32_t x23) const
    {
        // a raw quad as loaded, or (rows of any pitch, loaded widened) narrowed back
        if constexpr (std::is_same<R, uint32_t>::value) e[64 * j] = raw;
        else e[64 * j] = perm(x23, x01, SEL_NARROW);
    }
    __device__ __forceinline__ void get(int j, uint32_t &h01, uint32_t &h23) const
    {
        const uint32_t d = e[64 * j];
        h01 = perm(0u, d, SEL_U8_01);
        h23 = perm(0u, d, SEL_U8_23);
    }
    // entries wy - 1 .. 0 become suffix minima (raw quads widened with the lane's
    // selectors s01 / s23)
    template <bool MAXOP>
    __device__ __forceinline__ void suffixes(int wy, uint32_t s01, uint32_t s23) const
    {
        uint32_t h01 = MAXOP ? 0u : 0xffffffffu, h23 = h01;
        int j = wy - 1;
        for (; j >= 7; j -= 8) { // whole batches of 8 entries
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; k++) v[k] = e[64 * (j - k)];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                h01 = pk<MAXOP>(h01, perm(0u, v[k], s01));
                h23 = pk<MAXOP>(h23, perm(0u, v[k], s23));
                e[64 * (j - k)] = perm(h23, h01, SEL_NARROW);
            }
        }
        for (; j >= 0; j--) {
            const uint32_t v = e[64 * j];
            h01 = pk<MAXOP>(h01, perm(0u, v, s01));
            h23 = pk<MAXOP>(h23, perm(0u, v, s23));
            e[64 * j] = perm(h23, h01, SEL_NARROW);
        }
    }
};
template <> struct Ring<uint16_t> {
    uint2 *e;
    __device__ __forceinline__ explicit Ring(uint32_t *lds) : e((uint2 *)lds + (threadIdx.x & 63)) {}
    template <typename R>
    __device__ __forceinline__ void put(int j, R, uint32_t x01, uint32_t x23) const
    {
        e[64 * j] = make_uint2(x01, x23);
    }
    __device__ __forceinline__ void get(int j, uint32_t &h01, uint32_t &h23) const
    {
        const uint2 d = e[64 * j];
        h01 = d.x;
        h23 = d.y;
    }
    template <bool MAXOP>
    __device__ __forceinline__ void suffixes(int wy, uint32_t, uint32_t) const
    {
        uint32_t h01 = MAXOP ? 0u : 0xffffffffu, h23 = h01;
        int j = wy - 1;
        for (; j >= 7; j -= 8) { // whole batches of 8 entries
            uint2 v[8];
#pragma unroll
            for (int k = 0; k < 8; k++) v[k] = e[64 * (j - k)];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                h01 = pk<MAXOP>(h01, v[k].x);
                h23 = pk<MAXOP>(h23, v[k].y);
                e[64 * (j - k)] = make_uint2(h01, h23);
            }
        }
        for (; j >= 0; j--) {
            const uint2 v = e[64 * j];
            h01 = pk<MAXOP>(h01, v.x);
            h23 = pk<MAXOP>(h23, v.y);
            e[64 * j] = make_uint2(h01, h23);
        }
    }
};

// Per-wave LDS of the vertical pass: the run totals of the block being streamed (T,
// stream_runs(wy) entries) and the suffix minima over the runs of the previous
// block (S, one more entry, the last the identity), 64 lanes each.  uint8: an entry
// is a lane's four pixels narrowed to bytes; uint16: the two pair dwords.
template <typename T> struct RunTable;
template <> struct RunTable<uint8_t> {
    uint32_t *e;
    __device__ __forceinline__ explicit RunTable(uint32_t *lds) : e(lds + (threadIdx.x & 63)) {}
    __device__ __forceinline__ void put(int i, uint32_t v01, uint32_t v23) const
    {
        e[64 * i] = perm(v23, v01, SEL_NARROW);
    }
    __device__ __forceinline__ void get(int i, uint32_t &v01, uint32_t &v23) const
    {
        const uint32_t d = e[64 * i];
        v01 = perm(0u, d, SEL_U8_01);
        v23 = perm(0u, d, SEL_U8_23);
    }
};
template <> struct RunTable<uint16_t> {
    uint2 *e;
    __device__ __forceinline__ explicit RunTable(uint32_t *lds)
        : e((uint2 *)lds + (threadIdx.x & 63)) {}
    __device__ __forceinline__ void put(int i, uint32_t v01, uint32_t v23) const
    {
        e[64 * i] = make_uint2(v01, v23);
    }
    __device__ __forceinline__ void get(int i, uint32_t &v01, uint32_t &v23) const
    {
        const uint2 d = e[64 * i];
        v01 = d.x;
        v23 = d.y;
    }
};

// The vertical pass is vHGW over blocks of wy input rows (§5.1.1), in one of two
// forms (RUNS, chosen by stream_two_level(wy)):
//  - ring (small wy): block b's suffixes h_b sit in a per-wave LDS ring of wy rows;
//    while block b + 1 streams in, output row b wy + j is op(h_b[j], prefix of block
//    b + 1 over its first j rows) and the incoming row takes h_b[j]'s slot; at the
//    end of a block a backward walk over the ring turns it into that block's h.
//  - runs (larger wy): each block is split into runs of SD rows: output row
//    s = b wy + j (j in run r of block b) is
//     op( suffix of run r of block b from row s,  S_b[r + 1],  prefix of block b + 1
//         over its first j rows )
// where S_b[r + 1] is the extremum of block b's runs after r.  Streaming down, the
// chunk of block b + 1 that emits rows s .. s + SD - 1 also re-reads block b's rows
// at the same offsets (from cache: they streamed past wy rows earlier) and forms the
// in-run suffixes in registers; the run totals of each block go to LDS as the block
// streams past, and at its end a backward walk over them gives S.  Per wave this
// keeps 2 stream_runs(wy) + 1 small LDS entries instead of a ring of wy rows, at the
// price of a second (cached) load of every row: a win where the ring's LDS would
// limit the waves resident per CU.
template <typename T, bool MAXOP, bool AL, bool RUNS, bool XV = false, bool NTS = true>
__device__ __forceinline__ void stream_body(const TileJob &J, int unit, uint32_t *lds)
{
    const int lane = threadIdx.x & 63;
    const int sx = unit % J.tiles_x, sy = unit / J.tiles_x;
    const int mis = AL ? (int)(((uintptr_t)J.src & (4 * sizeof(T) - 1)) / sizeof(T)) : 0;
    const int co = (mis - J.ax) & 3;
    const int gxa = J.TW * sx - J.ax - co; // lane 0's first input column
    const int gx = gxa + 4 * lane;
    const int y0 = sy * J.TB;
    const int rows = min(J.TB, J.H - y0);
    const int wy = J.wy;
    // input rows 0 .. last - 1 feed the outputs; input row t >= wy emits output row
    // t - wy, so steps run up to t = last
    const int last = rows + wy - 1;
    const int gy0 = y0 - J.ay;
    const bool edge = gxa < 0 || gxa + 4 * 64 > J.W;
    using Ld = typename std::conditional<AL, WaveLoader<T>, WaveLoaderAny<T>>::type;
    const Ld L = [&]() {
        if constexpr (AL) return WaveLoader<T>(J, mis, gx);
        else return WaveLoaderAny<T>(J, MAXOP ? 0u : (Px<T>::maxv | (Px<T>::maxv << 16)), gx);
    }();
    const Doubling S(J.wx, co);
    const LaneVhgw<MAXOP> V(XV ? J.wx : 1, co); // XV: the horizontal pass is vHGW
    const bool hdirect = J.hm != PASS_DOUBLING; // direct (wx <= kDirectMax) or none
    const int nruns = stream_runs(wy);
    const RunTable<T> tot(lds);                  // runs: T, entries 0 .. nruns - 1
    const RunTable<T> suf(lds + nruns * 64 * (sizeof(T) == 1 ? 1 : 2)); // S: 0 .. nruns
    const Ring<T> ring(lds);                     // ring: wy (+ SD - 1) entries
    // uint8 rings hold raw quads, widened with the loader's selectors (identity ones
    // for rows of any pitch, which the loader returns widened already)
    uint32_t rs01 = SEL_U8_01, rs23 = SEL_U8_23;
    if constexpr (AL) {
        rs01 = L.s01;
        rs23 = L.s23;
    }
    // destination: rows 4-byte aligned, the strip wholly inside the image and the
    // image spanning < 4 GiB take buffer stores (row offset scalar)
    const int Q = (J.TW >> 2) * sx + lane;
    const bool store_lane = lane < (J.TW >> 2);
    const uint64_t dspan = (uint64_t)(J.H - 1) * J.dpitch + (uint64_t)J.W * sizeof(T);
    const bool fast_store = (((uintptr_t)J.dst | (uintptr_t)J.dpitch) & 3) == 0 &&
                            J.TW * (sx + 1) <= J.W && dspan < 0xffffffffull;
    const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)J.dst, (short)0, (int)(uint32_t)min(dspan, (uint64_t)0xffffffffu), kBufferWord3);
    const uint32_t dvoff = (uint32_t)Q * 4u * (uint32_t)sizeof(T);
    const uint32_t id = MAXOP ? 0u : 0xffffffffu;

    // units clear of the image's top and bottom rows load without clamping
    const bool rows_in = AL && gy0 >= 0 && gy0 + last + 2 * SD <= J.H;
    const uint32_t pitch = (uint32_t)J.pitch;
    auto issue8 = [&](typename Ld::Raw(&buf)[SD], int r0) {
        if constexpr (AL) {
            // row offsets first (scalar), then the loads in one straight run
            uint32_t so[SD];
            if (rows_in) {
#pragma unroll
                for (int k = 0; k < SD; k++) so[k] = (uint32_t)(r0 + k) * pitch;
            } else {
#pragma unroll
                for (int k = 0; k < SD; k++)
                    so[k] = (uint32_t)min(max(r0 + k, 0), J.H - 1) * pitch;
            }
#pragma unroll
            for (int k = 0; k < SD; k++) buf[k] = L.issue_at(__builtin_amdgcn_readfirstlane(so[k]));
        } else {
#pragma unroll
            for (int k = 0; k < SD; k++) buf[k] = L.issue(r0 + k);
        }
    };

    uint32_t g01 = id, g23 = id;
    int t = 0, j = 0;
    bool fill = true;
    // One chunk: rows t .. t + cnt - 1 of the current block from `cur` and, once
    // outputs are due, the previous block's rows at the same offsets from `hcur`; the
    // next chunk's rows are loaded into `nxt` / `hnxt`.  The loop alternates the
    // buffers so that no loaded register is copied (a copy would wait for its load).
    auto chunk = [&](typename Ld::Raw(&cur)[SD], typename Ld::Raw(&nxt)[SD],
                     typename Ld::Raw(&hcur)[SD], typename Ld::Raw(&hnxt)[SD]) -> bool {
        const int runlen = min(SD, wy - j);       // rows of this run of the block
        const int cnt = min(runlen, last - t + 1); // of which this unit still needs
        const bool full = cnt == SD;
        uint32_t x01[SD], x23[SD];
#pragma unroll
        for (int k = 0; k < SD; k++) L.widen(cur[k], x01[k], x23[k]);
        issue8(nxt, gy0 + t + cnt);
        if constexpr (RUNS) {
            if (t + cnt >= wy) issue8(hnxt, gy0 + t + cnt - wy);
            // this run's total, for the block's S
            // (full chunks, the common case, fold without a test per row)
            uint32_t r01 = x01[0], r23 = x23[0];
            if (full) {
#pragma unroll
                for (int k = 1; k < SD; k++) {
                    r01 = pk<MAXOP>(r01, x01[k]);
                    r23 = pk<MAXOP>(r23, x23[k]);
                }
            } else {
#pragma unroll
                for (int k = 1; k < SD; k++)
                    if (k < cnt) {
                        r01 = pk<MAXOP>(r01, x01[k]);
                        r23 = pk<MAXOP>(r23, x23[k]);
                    }
            }
            tot.put(j / SD, r01, r23);
        } else if (fill) {
            if (full) {
#pragma unroll
                for (int k = 0; k < SD; k++) ring.put(j + k, cur[k], x01[k], x23[k]);
            } else {
#pragma unroll
                for (int k = 0; k < SD; k++)
                    if (k < cnt) ring.put(j + k, cur[k], x01[k], x23[k]);
            }
        }
        if (!fill) {
            uint32_t o01[SD], o23[SD];
            if constexpr (RUNS) {
                // previous block's rows at these offsets: suffixes over the whole run
                // (even where this unit stops early), then the later runs' extremum
                // S_b[r + 1]
                uint32_t s01, s23;
                suf.get(j / SD + 1, s01, s23);
#pragma unroll
                for (int k = 0; k < SD; k++) L.widen(hcur[k], o01[k], o23[k]);
                if (runlen == SD) {
#pragma unroll
                    for (int k = SD - 1; k >= 0; k--) {
                        s01 = o01[k] = pk<MAXOP>(s01, o01[k]);
                        s23 = o23[k] = pk<MAXOP>(s23, o23[k]);
                    }
                } else {
#pragma unroll
                    for (int k = SD - 1; k >= 0; k--) {
                        if (k < runlen) {
                            s01 = pk<MAXOP>(s01, o01[k]);
                            s23 = pk<MAXOP>(s23, o23[k]);
                        }
                        o01[k] = s01;
                        o23[k] = s23;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < SD; k++) ring.get(j + k, o01[k], o23[k]);
            }
#pragma unroll
            for (int k = 0; k < SD; k++) {
                // h_b[j + k] against the prefix of this block's first j + k rows
                o01[k] = pk<MAXOP>(o01[k], g01);
                o23[k] = pk<MAXOP>(o23[k], g23);
                g01 = pk<MAXOP>(g01, x01[k]);
                g23 = pk<MAXOP>(g23, x23[k]);
            }
            if constexpr (!RUNS) {
                if (full) {
#pragma unroll
                    for (int k = 0; k < SD; k++) ring.put(j + k, cur[k], x01[k], x23[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < SD; k++)
                        if (k < cnt) ring.put(j + k, cur[k], x01[k], x23[k]);
                }
            }
            // output rows t - wy .. t - wy + cnt - 1: horizontal pass, then store
            if constexpr (AL && sizeof(T) == 2)
                if (edge) {
#pragma unroll
                    for (int k = 0; k < SD; k++) L.fix(o01[k], o23[k]);
                }
            if constexpr (XV) lane_vhgw_rows<SD, MAXOP>(V, o01, o23);
            else if (hdirect) direct_rows_any<SD, MAXOP>(J.wx, co, o01, o23);
            else doubling_rows<SD, MAXOP>(S, o01, o23);
            if (store_lane) {
                const int y = y0 + t - wy;
                if (fast_store) {
                    uint32_t so = (uint32_t)y * (uint32_t)J.dpitch;
#pragma unroll
                    for (int k = 0; k < SD; k++, so += (uint32_t)J.dpitch) {
                        if (full || k < cnt) {
                            if constexpr (sizeof(T) == 1) {
                                buffer_store_nt<NTS>(perm(o23[k], o01[k], SEL_NARROW), drs,
                                                (int)dvoff, (int)so);
                            } else {
                                buffer_store_nt<NTS>(o01[k], drs, (int)dvoff, (int)so);
                                buffer_store_nt<NTS>(o23[k], drs, (int)dvoff + 4, (int)so);
                            }
                        }
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < SD; k++)
                        if (k < cnt)
                            Px<T>::template store<NTS>(J.dst + (int64_t)(y + k) * J.dpitch, 4 * Q, J.W, o01[k],
                                         o23[k]);
                }
            }
        }
        t += cnt;
        j += cnt;
        if (j == wy) { // block complete
            if constexpr (RUNS) { // S over its runs, from the last one back
                uint32_t a01 = id, a23 = id;
                suf.put(nruns, id, id);
                for (int r = nruns - 1; r >= 0; r--) {
                    uint32_t v01, v23;
                    tot.get(r, v01, v23);
                    a01 = pk<MAXOP>(a01, v01);
                    a23 = pk<MAXOP>(a23, v23);
                    suf.put(r, a01, a23);
                }
            } else { // its suffixes replace it in the ring
                ring.template suffixes<MAXOP>(wy, rs01, rs23);
            }
            j = 0;
            fill = false;
            g01 = g23 = id;
        }
        return t <= last;
    };
    typename Ld::Raw bufa[SD], bufb[SD], hbufa[SD], hbufb[SD];
    issue8(bufa, gy0);
    while (chunk(bufa, bufb, hbufa, hbufb) && chunk(bufb, bufa, hbufb, hbufa)) {
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

typedef void (*TileKernelFn)(TileJob);


static inline hipError_t set_lds_limit(const void *fn, int lds)
{
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

// Batches are launched per group of jobs with the same kernel kind, element type and
// row alignment.
// The wave and streaming groups of a batch in one dispatch: the dispatcher deals the
// run-total streaming units out first, then the ring ones, then the wave units, so
// the short units fill in behind the long ones instead of each group filling and
// draining the GPU on its own.
template <typename T, bool AL>
__global__ __launch_bounds__(64) void batch_fused_kernel(FusedTables ft)
{
    extern __shared__ uint32_t lds[];
    const int b = blockIdx.x;
    const int c = b < ft.b0[1] ? 0 : (b < ft.b0[2] ? 1 : 2);
    const BatchTables &bt = c == 0 ? ft.g[0] : (c == 1 ? ft.g[1] : ft.g[2]);
    const int t = xcd_tile(b - ft.b0[c], ft.b0[c + 1] - ft.b0[c]);
    if (t >= bt.n_tiles) return;
    const int jb = bt.tile_job[t];
    const TileJob J = bt.jobs[jb];
    const int u = (int)(t - bt.tile_start[jb]);
    if (c == 0) {
        if (J.op) stream_body<T, true, AL, true, false, false>(J, u, lds);
        else stream_body<T, false, AL, true, false, false>(J, u, lds);
    } else if (c == 1) {
        if (J.op) stream_body<T, true, AL, false, false, false>(J, u, lds);
        else stream_body<T, false, AL, false, false, false>(J, u, lds);
    } else {
        if (J.op) wave_body<T, true, AL, false, false, false>(J, u);
        else wave_body<T, false, AL, false, false, false>(J, u);
    }
}

} // namespace morph
