// The streaming kernel's cooperative form: vertical vHGW (§5.1.1) for single images
// with large vertical windows, the NW waves of one workgroup (4, 8 or 16) sharing a unit of
// TB output rows of one strip.
//
// With the input rows of the unit numbered from its first one (gy0 = y0 - ay) and cut
// into blocks of wy rows, each block into runs of kStreamChunk rows, output row i
// (block b = i / wy, offset j = i mod wy, run r = j / 8, k = j mod 8) is
//   op( rows j .. wy - 1 of block b,  rows 0 .. j - 1 of block b + 1 )
// = op( in-run suffix of block b's run r from k,  S_b[r + 1],
//       P_{b+1}[r],  in-run prefix of block b + 1's run r before k )
// with S_b[r] the extremum of block b's runs r .. and P_b[r] that of its runs before r.
// The streaming kernel walks a unit's rows one chunk after another, so a wave's
// chain of loads is TB + wy - 1 rows long and short units re-read many halo rows.
// Here the three steps run side by side over the workgroup's waves:
//   1. every run's extremum (its total) into LDS, the runs dealt out over the waves;
//   2. S and P of every block by scans over its run totals (one scan a wave);
//   3. the output runs (b, r), dealt out over the waves: the run's rows of blocks b
//      and b + 1 again (from cache), the in-run suffix and prefix, the combination
//      above, then the horizontal pass and the store as in the streaming kernel.
// Borders, loads, the horizontal pass and the store are the streaming kernel's.
#include "morph_device.h"

namespace morph {

static_assert(kStreamChunk == SD && SD == 8, "runs of 8 rows");

template <typename T, bool MAXOP, int NW, bool NTS = true>
__device__ __forceinline__ void stream_coop_body(const TileJob &J, int unit, uint32_t *lds)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int sx = unit % J.tiles_x, sy = unit / J.tiles_x;
    const int mis = (int)(((uintptr_t)J.src & (4 * sizeof(T) - 1)) / sizeof(T));
    const int co = (mis - J.ax) & 3;
    const int gxa = J.TW * sx - J.ax - co; // lane 0's first input column
    const int gx = gxa + 4 * lane;
    const int y0 = sy * J.TB;
    const int rows = min(J.TB, J.H - y0);
    const int wy = J.wy;
    const int gy0 = y0 - J.ay;
    const bool edge = gxa < 0 || gxa + 4 * 64 > J.W;
    const WaveLoader<T> L(J, mis, gx);
    const uint32_t id = MAXOP ? 0u : 0xffffffffu;

    // runs and blocks of the unit (the same numbers on the host: coop_lds_bytes)
    const int nr = stream_runs(wy);
    const int bmax = (rows - 1) / wy; // last block holding an output's window start
    const int ni = rows + wy - 1;     // input rows the outputs read
    const int tail = ni - (bmax + 1) * wy; // rows of block bmax + 1 they read (>= 0)
    const int n_runs = (bmax + 1) * nr + min(nr, (tail + SD - 1) / SD);
    const RunTable<T> tot(lds);                                  // n_runs totals
    const int ent = 64 * (sizeof(T) == 1 ? 1 : 2);               // dwords an entry
    // S_b[r] (b <= bmax) and P_{b+1}[r] after the totals.  With one block of outputs
    // (bmax 0) block 0 needs only S and block 1 only P, so for uint16, whose LDS limits
    // the workgroups a CU holds at the largest windows, both scans overwrite the totals
    // they read: S_0[r] at entry r (r < nr), P_1[r] at entry nr + r - 1 (r >= 1), and
    // S_0[nr], P_1[0] (the identity) are not stored (uint8, held back by its registers
    // instead, measured 1-3% slower so)
    const bool inplace = sizeof(T) == 2 && bmax == 0;
    const RunTable<T> suf(lds + (inplace ? 0 : n_runs * ent));
    const RunTable<T> pre(lds + (inplace ? (nr - 1) * ent : (n_runs + (bmax + 1) * (nr + 1)) * ent));

    const uint32_t pitch = (uint32_t)J.pitch;
    using Raw = typename WaveLoader<T>::Raw;
    // rows r0 .. r0 + len - 1 of the unit (clamped into the image) into buf[0 .. len - 1].
    // For uint8 buf[len ..] repeat row r0 + len - 1, which leaves every min / max over
    // the buffer and every suffix and prefix up to len unchanged, so that the folds
    // below take all SD rows without a test per row (measured faster for uint8, slower
    // at large windows for uint16, which keeps the tests).
    constexpr bool kDup = sizeof(T) == 1;
    auto issue8 = [&](Raw(&buf)[SD], int r0, int len) __attribute__((always_inline)) {
        uint32_t so[SD];
#pragma unroll
        for (int k = 0; k < SD; k++)
            so[k] = (uint32_t)min(max(gy0 + r0 + (kDup ? min(k, len - 1) : k), 0), J.H - 1) * pitch;
#pragma unroll
        for (int k = 0; k < SD; k++) buf[k] = L.issue_at(__builtin_amdgcn_readfirstlane(so[k]));
    };
    auto run_rows = [&](int g) { return min(SD, wy - SD * (g % nr)); };
    auto run_start = [&](int g) { return (g / nr) * wy + SD * (g % nr); };

    // 1. run totals: the wave's runs w, w + NW, ..., the next one's loads in flight
    // while one is reduced
    {
        constexpr int D = 2; // (deeper measured slower: the registers cost occupancy)
        Raw buf[D][SD];
#pragma unroll
        for (int d = 0; d < D - 1; d++) {
            const int gd = wave + d * NW;
            if (gd < n_runs) issue8(buf[d], run_start(gd), run_rows(gd));
        }
        for (int g = wave; g < n_runs; g += D * NW) {
#pragma unroll
            for (int d = 0; d < D; d++) {
                const int gc = g + d * NW;
                if (gc >= n_runs) break;
                const int gn = gc + (D - 1) * NW;
                if (gn < n_runs) issue8(buf[(d + D - 1) % D], run_start(gn), run_rows(gn));
                const int len = run_rows(gc);
                uint32_t a01, a23;
                L.widen(buf[d][0], a01, a23);
#pragma unroll
                for (int k = 1; k < SD; k++) {
                    uint32_t x01, x23;
                    L.widen(buf[d][k], x01, x23);
                    if (kDup || k < len) {
                        a01 = pk<MAXOP>(a01, x01);
                        a23 = pk<MAXOP>(a23, x23);
                    }
                }
                tot.put(gc, a01, a23);
            }
        }
    }
    __syncthreads();

    // 2. scans: S_b for b = 0 .. bmax, then P_{b+1} for b = 0 .. bmax, one a wave; the
    // run totals read SD at a time (independent LDS reads in flight together), then
    // folded in order
    for (int q = wave; q < 2 * (bmax + 1); q += NW) {
        uint32_t a01 = id, a23 = id;
        if (q <= bmax) { // S_q[r] = op of runs r .. nr - 1 of block q
            const int b = q;
            if (!inplace) suf.put(b * (nr + 1) + nr, id, id);
            for (int r1 = nr; r1 > 0; r1 -= SD) { // runs r1 - 1 down to max(r1 - SD, 0)
                uint32_t v01[SD], v23[SD];
#pragma unroll
                for (int k = 0; k < SD; k++)
                    if (r1 - 1 - k >= 0) tot.get(b * nr + r1 - 1 - k, v01[k], v23[k]);
#pragma unroll
                for (int k = 0; k < SD; k++)
                    if (r1 - 1 - k >= 0) {
                        a01 = pk<MAXOP>(a01, v01[k]);
                        a23 = pk<MAXOP>(a23, v23[k]);
                        suf.put(b * (nr + 1) + r1 - 1 - k, a01, a23);
                    }
            }
        } else { // P_{b+1}[r] = op of runs 0 .. r - 1 of block b + 1, for the runs it has
            const int b = q - (bmax + 1);
            const int have = min(nr, n_runs - (b + 1) * nr); // runs of block b + 1 held
            if (!inplace) pre.put(b * (nr + 1), id, id);
            for (int r0 = 0; r0 < have; r0 += SD) { // runs r0 .. r0 + SD - 1
                uint32_t v01[SD], v23[SD];
#pragma unroll
                for (int k = 0; k < SD; k++)
                    if (r0 + k < have) tot.get((b + 1) * nr + r0 + k, v01[k], v23[k]);
#pragma unroll
                for (int k = 0; k < SD; k++)
                    if (r0 + k < have) {
                        a01 = pk<MAXOP>(a01, v01[k]);
                        a23 = pk<MAXOP>(a23, v23[k]);
                        pre.put(b * (nr + 1) + r0 + k + 1, a01, a23);
                    }
            }
        }
    }
    __syncthreads();

    // 3. output runs (b, r) whose first row is an output: the wave's runs g = wave,
    // wave + NW, ... (increasing first rows, so the first one past the unit ends them),
    // each reading its rows of blocks b and b + 1
    const Doubling S(J.wx, co);
    const bool hdirect = J.hm != PASS_DOUBLING; // direct (wx <= kDirectMax) or none
    const int Q = (J.TW >> 2) * sx + lane;
    const bool store_lane = lane < (J.TW >> 2);
    const uint64_t dspan = (uint64_t)(J.H - 1) * J.dpitch + (uint64_t)J.W * sizeof(T);
    const bool fast_store = (((uintptr_t)J.dst | (uintptr_t)J.dpitch) & 3) == 0 &&
                            J.TW * (sx + 1) <= J.W && dspan < 0xffffffffull;
    const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)J.dst, (short)0, (int)(uint32_t)min(dspan, (uint64_t)0xffffffffu), kBufferWord3);
    const uint32_t dvoff = (uint32_t)Q * 4u * (uint32_t)sizeof(T);
    auto out_run = [&](Raw(&xb)[SD], Raw(&zb)[SD], int g) __attribute__((always_inline)) {
        const int i0 = run_start(g); // first output row of the run
        const int b = g / nr, r = g % nr;
        const int len = run_rows(g);
        uint32_t s01 = id, s23 = id, p01 = id, p23 = id;
        if (!inplace || r + 1 < nr) suf.get(b * (nr + 1) + r + 1, s01, s23);
        if (!inplace || r > 0) pre.get(b * (nr + 1) + r, p01, p23);
        uint32_t o01[SD], o23[SD];
#pragma unroll
        for (int k = SD - 1; k >= 0; k--) {
            uint32_t x01, x23;
            L.widen(xb[k], x01, x23);
            if (kDup || k < len) {
                s01 = pk<MAXOP>(s01, x01);
                s23 = pk<MAXOP>(s23, x23);
            }
            o01[k] = s01;
            o23[k] = s23;
        }
#pragma unroll
        for (int k = 0; k < SD; k++) {
            o01[k] = pk<MAXOP>(o01[k], p01);
            o23[k] = pk<MAXOP>(o23[k], p23);
            uint32_t z01, z23;
            L.widen(zb[k], z01, z23);
            p01 = pk<MAXOP>(p01, z01);
            p23 = pk<MAXOP>(p23, z23);
        }
        if constexpr (sizeof(T) == 2)
            if (edge) {
#pragma unroll
                for (int k = 0; k < SD; k++) L.fix(o01[k], o23[k]);
            }
        if (hdirect) direct_rows_any<SD, MAXOP>(J.wx, co, o01, o23);
        else doubling_rows<SD, MAXOP>(S, o01, o23);
        if (store_lane) {
            const int y = y0 + i0;
            const int cnt = min(len, rows - i0);
            if (fast_store) {
                uint32_t so = (uint32_t)y * (uint32_t)J.dpitch;
#pragma unroll
                for (int k = 0; k < SD; k++, so += (uint32_t)J.dpitch) {
                    if (k < cnt) {
                        if constexpr (sizeof(T) == 1) {
                            buffer_store_nt<NTS>(perm(o23[k], o01[k], SEL_NARROW), drs, (int)dvoff,
                                            (int)so);
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
                        Px<T>::template store<NTS>(J.dst + (int64_t)(y + k) * J.dpitch, 4 * Q, J.W,
                                                   o01[k], o23[k]);
            }
        }
    };
    const int n_out = (bmax + 1) * nr;
    for (int g = wave; g < n_out && run_start(g) < rows; g += NW) {
        Raw xb[SD], zb[SD];
        issue8(xb, run_start(g), run_rows(g));      // block b's run r: the suffix side
        issue8(zb, run_start(g) + wy, run_rows(g)); // block b + 1's run r: the prefix side
        out_run(xb, zb, g);
    }
}

// NTS: non-temporal destination stores (plain where a later launch reads the
// destination again: TileJob::keep)
template <typename T, bool MAXOP, int NW, bool NTS>
__global__ __launch_bounds__(64 * NW) void stream_coop_kernel(TileJob J)
{
    extern __shared__ uint32_t lds[];
    stream_coop_body<T, MAXOP, NW, NTS>(J, xcd_tile(blockIdx.x, gridDim.x), lds);
}

// The batch form: one workgroup of NW waves per unit of the group's jobs.
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void batch_coop_kernel(BatchTables bt)
{
    extern __shared__ uint32_t lds[];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= bt.n_tiles) return; // (the whole workgroup leaves)
    const int jb = bt.tile_job[t];
    const TileJob J = bt.jobs[jb];
    const int u = (int)(t - bt.tile_start[jb]);
    if (J.op) stream_coop_body<T, true, NW, false>(J, u, lds);
    else stream_coop_body<T, false, NW, false>(J, u, lds);
}

template <int NW, bool NTS> static TileKernelFn pick_coop_n(const TileJob &job)
{
    return job.dtype == 0 ? (job.op ? stream_coop_kernel<uint8_t, true, NW, NTS>
                                    : stream_coop_kernel<uint8_t, false, NW, NTS>)
                          : (job.op ? stream_coop_kernel<uint16_t, true, NW, NTS>
                                    : stream_coop_kernel<uint16_t, false, NW, NTS>);
}
template <int NW> static TileKernelFn pick_coop(const TileJob &job)
{
    return job.keep ? pick_coop_n<NW, false>(job) : pick_coop_n<NW, true>(job);
}

hipError_t launch_stream_coop(const TileJob &job, hipStream_t stream)
{
    if (job.coop != 4 && job.coop != 8 && job.coop != 16) return hipErrorInvalidValue;
    const TileKernelFn fn = job.coop == 16 ? pick_coop<16>(job)
                          : job.coop == 8  ? pick_coop<8>(job)
                                           : pick_coop<4>(job);
    const int lds = coop_lds_bytes(job);
    hipError_t e = set_lds_limit((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(job.tiles_x * job.tiles_y), dim3(64 * job.coop), lds, stream, job);
    return hipGetLastError();
}

hipError_t launch_batch_coop(const BatchTables &t, int dtype, int waves, int grid, int lds,
                             hipStream_t stream)
{
    typedef void (*BatchFn)(BatchTables);
    BatchFn fn;
    if (waves == 16) fn = dtype == 0 ? batch_coop_kernel<uint8_t, 16> : batch_coop_kernel<uint16_t, 16>;
    else if (waves == 8) fn = dtype == 0 ? batch_coop_kernel<uint8_t, 8> : batch_coop_kernel<uint16_t, 8>;
    else if (waves == 4) fn = dtype == 0 ? batch_coop_kernel<uint8_t, 4> : batch_coop_kernel<uint16_t, 4>;
    else return hipErrorInvalidValue;
    hipError_t e = set_lds_limit((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * waves), lds, stream, t);
    return hipGetLastError();
}

} // namespace morph
