// Opening and closing in one pass on the wave kernel's form (templates; instantiated per
// element type in k_oc_u8.hip and k_oc_u16.hip) (§2: an opening is the
// dilation of the erosion, a closing the erosion of the dilation, both with the
// same rectangle and anchor).
//
// One wave per strip of output quads and TB output rows, registers only.  Input rows
// stream down through the first operation as in the wave kernel (vertical direct
// pass over a ring of rows, then the horizontal pass across the lanes), giving the
// intermediate rows E a chunk of 8 at a time; they enter a queue of 8k rows, and the
// second operation's vertical direct pass reads its window from the queue's head,
// then its horizontal pass, then the store.  The intermediate image never reaches
// memory: sizeof(T) bytes read and written a pixel, as for one erosion.
//
// Border rule (Eq. (1) takes in-image pixels only): input rows and columns outside
// the image are clamped into it, exact for the first operation as in the wave kernel
// (its windows hold the output pixel, so a repeated edge pixel changes nothing);
// intermediate pixels whose row or column lies outside the image must not enter the
// second operation, so they are replaced by its identity.
//
// Geometry.  Lane L's input quad starts at image column gxa + 4L with
// gxa = 4 wq sx - 2 ax - co1 (co1 puts the quads on the load alignment); the first
// operation's output at strip position p = 4L + j is the intermediate pixel of image
// column 4 wq sx - ax + p (its window starts at input position p + co1); the second
// operation's output quad Q reads intermediate positions 4Q .. 4Q + 3 + wx - 1 and is
// image columns 4 wq sx + 4Q .. + 3.  A strip stores the quads whose inputs lie in
// its 64 lanes: 4Q + 3 + (wx - 1) + co1 + (wx - 1) <= 255.
#pragma once
#include "morph_device.h"

namespace morph {

// windows the one-pass form compiles: vertical up to kOcWaveMaxWy, horizontal up to
// kOcWaveMaxWx (direct up to kDirectMax, doubling beyond)
static_assert(kOcWaveMaxWy == 15, "vertical windows compiled below");

template <int WY> constexpr int oc_queue_rows() { return 8 * ((WY + 7 + 7) / 8); }

// The horizontal direct pass with the window starts at offset CO, windows 1..9.
template <bool MAXOP, int CO>
__device__ __forceinline__ void oc_direct_rows(int wx, uint32_t *v01, uint32_t *v23)
{
    switch (wx) {
#define OC_WH(W)                                                                             \
    case W: wv_horizontal<W, CO, MAXOP>(v01, v23); break;
        OC_WH(1) OC_WH(2) OC_WH(3) OC_WH(4) OC_WH(5) OC_WH(6) OC_WH(7) OC_WH(8) OC_WH(9)
#undef OC_WH
    default: break;
    }
}

template <bool MAXOP>
__device__ __forceinline__ void oc_direct_rows_co(int wx, int co, uint32_t *v01, uint32_t *v23)
{
    switch (co) {
    case 0: oc_direct_rows<MAXOP, 0>(wx, v01, v23); break;
    case 1: oc_direct_rows<MAXOP, 1>(wx, v01, v23); break;
    case 2: oc_direct_rows<MAXOP, 2>(wx, v01, v23); break;
    default: oc_direct_rows<MAXOP, 3>(wx, v01, v23); break;
    }
}

// OPENING: erosion then dilation, else dilation then erosion.
template <typename T, bool OPENING, int WY, bool NTS>
__device__ __forceinline__ void oc_wave_body(const TileJob &J, int unit)
{
    constexpr bool MAX1 = !OPENING, MAX2 = OPENING; // op of each stage
    constexpr int QN = oc_queue_rows<WY>();          // intermediate queue rows
    constexpr int RING = KR + WY - 1;
    const int lane = threadIdx.x & 63;
    const int sx = unit % J.tiles_x, sy = unit / J.tiles_x;
    const int mis = (int)(((uintptr_t)J.src & (4 * sizeof(T) - 1)) / sizeof(T));
    const int co1 = (mis - 2 * J.ax) & 3;
    const int wq = J.TW >> 2;
    const int gxa = 4 * wq * sx - 2 * J.ax - co1;
    const int gx = gxa + 4 * lane;
    const int y0 = sy * J.TB;
    const int y1 = min(y0 + J.TB, J.H);
    const bool edge = gxa < 0 || gxa + 4 * 64 > J.W; // (uint16: per-row pixel picks)
    using Ld = WaveLoader<T>;
    const Ld L(J, mis, gx);
    using Raw = typename Ld::Raw;
    const uint32_t id2 = MAX2 ? 0u : 0xffffffffu;

    // intermediate columns outside the image: the second operation's identity
    const int ec = 4 * wq * sx - J.ax + 4 * lane; // image column of the lane's first one
    const bool cols_out = 4 * wq * sx - J.ax < 0 || 4 * wq * sx - J.ax + 4 * 64 > J.W;
    uint32_t cm01 = 0, cm23 = 0; // 16-bit halves to replace
    if (cols_out) {
        cm01 = ((ec < 0 || ec >= J.W) ? 0xffffu : 0u) | ((ec + 1 < 0 || ec + 1 >= J.W) ? 0xffff0000u : 0u);
        cm23 = ((ec + 2 < 0 || ec + 2 >= J.W) ? 0xffffu : 0u) | ((ec + 3 < 0 || ec + 3 >= J.W) ? 0xffff0000u : 0u);
    }

    // intermediate rows: chunk c holds rows eb + 8c .. + 7; output chunk o needs chunks
    // o .. o + QN/8 - 1, so the queue runs QN/8 - 1 chunks ahead
    const int eb = y0 - J.ay;
    const int n_out = (y1 - y0 + KR - 1) / KR;
    const int n_e = n_out + QN / KR - 1;
    const int gi0 = eb - J.ay; // first input row of the ring
    const bool rows_out = eb < 0 || eb + KR * n_e > J.H;

    Raw rr[RING];
    Raw ra[KR], rb[KR];
    wv_first_raw<WY>(L, gi0, rr, ra);
    uint32_t q01[QN], q23[QN];
#pragma unroll
    for (int i = 0; i < QN; i++) q01[i] = q23[i] = id2;

    const Doubling S1(J.wx, co1), S2(J.wx, 0);
    const bool doubling = J.hm == PASS_DOUBLING; // (else direct, wx <= kDirectMax)
    const int Q = wq * sx + lane;
    const bool fast_store = (((uintptr_t)J.dst | (uintptr_t)J.dpitch) & 3) == 0 &&
                            4 * (wq * sx + wq) <= J.W;
    int c = 0;
    // one intermediate chunk (from the loads in cur; the next chunk's issued into
    // nxt), then, once the queue is full, one output chunk
    auto step = [&](Raw (&cur)[KR], Raw (&nxt)[KR]) __attribute__((always_inline)) -> bool {
        uint32_t v01[KR], v23[KR];
        if (c + 1 < n_e) {
            const int gn = gi0 + WY - 1 + KR * (c + 1);
#pragma unroll
            for (int m = 0; m < KR; m++) nxt[m] = L.issue(gn + m);
        }
        wv_vertical_raw<WY, MAX1>(L, cur, rr, v01, v23);
        if constexpr (sizeof(T) == 2) {
            if (edge) {
#pragma unroll
                for (int m = 0; m < KR; m++) L.fix(v01[m], v23[m]);
            }
        }
        if (doubling) doubling_rows<KR, MAX1>(S1, v01, v23);
        else oc_direct_rows_co<MAX1>(J.wx, co1, v01, v23);
        // the queue moves down a chunk; the new rows go to its tail
#pragma unroll
        for (int i = 0; i < QN - KR; i++) {
            q01[i] = q01[i + KR];
            q23[i] = q23[i + KR];
        }
#pragma unroll
        for (int m = 0; m < KR; m++) {
            uint32_t a = v01[m] | (MAX2 ? 0u : cm01), b = v23[m] | (MAX2 ? 0u : cm23);
            if (MAX2) {
                a &= ~cm01;
                b &= ~cm23;
            }
            const int e = eb + KR * c + m;
            if (rows_out && (e < 0 || e >= J.H)) a = b = id2;
            q01[QN - KR + m] = a;
            q23[QN - KR + m] = b;
        }
        const int o = c - (QN / KR - 1);
        c++;
        if (o < 0) return true;
        // the second operation on output rows y0 + 8 o ..: vertical from the queue head
        uint32_t w01[KR], w23[KR];
        if constexpr (WY >= KR) {
            chunk8_window<WY, MAX2>(q01, w01);
            chunk8_window<WY, MAX2>(q23, w23);
        } else {
#pragma unroll
            for (int m = 0; m < KR; m += 2) {
                pair_window<WY, MAX2>(q01 + m, w01[m], w01[m + 1]);
                pair_window<WY, MAX2>(q23 + m, w23[m], w23[m + 1]);
            }
        }
        if (doubling) doubling_rows<KR, MAX2>(S2, w01, w23);
        else oc_direct_rows<MAX2, 0>(J.wx, w01, w23);
        const int y = y0 + KR * o;
        if (lane < wq) {
            uint8_t *drow = J.dst + (int64_t)y * J.dpitch;
            if (fast_store) {
                const uint32_t off = (uint32_t)Q * 4u * (uint32_t)sizeof(T);
#pragma unroll
                for (int m = 0; m < KR; m++) {
                    if (y + m < y1) {
                        if constexpr (sizeof(T) == 1) {
                            store_u32<NTS>((uintptr_t)(drow + off),
                                           perm(w23[m], w01[m], SEL_NARROW));
                        } else {
                            store_u32<NTS>((uintptr_t)(drow + off), w01[m]);
                            store_u32<NTS>((uintptr_t)(drow + off + 4), w23[m]);
                        }
                    }
                    drow += J.dpitch;
                }
            } else {
#pragma unroll
                for (int m = 0; m < KR; m++) {
                    if (y + m < y1) Px<T>::template store<NTS>(drow, 4 * Q, J.W, w01[m], w23[m]);
                    drow += J.dpitch;
                }
            }
        }
        return c < n_e;
    };
    while (step(ra, rb) && step(rb, ra)) {
    }
}

template <typename T, bool OPENING, bool TALL, bool NTS>
__device__ __forceinline__ void oc_wave_dispatch(const TileJob &J, int u)
{
    if constexpr (TALL) {
        switch (J.wy) {
#define OC_WY(W)                                                                             \
    case W: oc_wave_body<T, OPENING, W, NTS>(J, u); break;
            OC_WY(10) OC_WY(11) OC_WY(12) OC_WY(13) OC_WY(14)
#undef OC_WY
        default: oc_wave_body<T, OPENING, 15, NTS>(J, u); break;
        }
    } else {
        switch (J.wy) {
#define OC_WY(W)                                                                             \
    case W: oc_wave_body<T, OPENING, W, NTS>(J, u); break;
            OC_WY(1) OC_WY(2) OC_WY(3) OC_WY(4) OC_WY(5) OC_WY(6) OC_WY(7) OC_WY(8)
#undef OC_WY
        default: oc_wave_body<T, OPENING, 9, NTS>(J, u); break;
        }
    }
}

// TALL: vertical windows kDirectMax + 1 .. kOcWaveMaxWy (a longer queue and ring, a
// kernel of its own so that the short windows keep their occupancy)
// NTS: non-temporal destination stores (plain where a later launch reads the
// destination again: TileJob::keep)
template <typename T, bool OPENING, bool TALL, bool NTS>
__global__ __launch_bounds__(NT) void oc_wave_kernel(TileJob J)
{
    const int units = J.tiles_x * J.tiles_y;
    const int u = __builtin_amdgcn_readfirstlane(4 * xcd_tile(blockIdx.x, gridDim.x) +
                                                 (int)(threadIdx.x >> 6));
    if (u >= units) return; // the whole wave leaves
    oc_wave_dispatch<T, OPENING, TALL, NTS>(J, u);
}

template <typename T>
hipError_t launch_openclose_wave_t(const TileJob &job, hipStream_t stream)
{
    typedef void (*Fn)(TileJob);
    const bool tall = job.wy > kDirectMax;
    const Fn fn = job.keep
        ? (job.op ? (tall ? oc_wave_kernel<T, true, true, false> : oc_wave_kernel<T, true, false, false>)
                  : (tall ? oc_wave_kernel<T, false, true, false> : oc_wave_kernel<T, false, false, false>))
        : (job.op ? (tall ? oc_wave_kernel<T, true, true, true> : oc_wave_kernel<T, true, false, true>)
                  : (tall ? oc_wave_kernel<T, false, true, true> : oc_wave_kernel<T, false, false, true>));
    const int units = job.tiles_x * job.tiles_y;
    hipLaunchKernelGGL(fn, dim3((units + 3) / 4), dim3(NT), 0, stream, job);
    return hipGetLastError();
}

} // namespace morph
