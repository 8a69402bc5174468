// Internal declarations shared by the host planner and the kernels of the HIP
// morphology library.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace morph {

constexpr int kThreads = 256;  // threads per workgroup of every kernel
// Direct (sliding) passes: compiled per window up to kDirectMax on every kernel; the
// wave kernel's tall form compiles vertical windows kDirectMax + 1 .. kDirectMaxTall,
// and the wave and streaming kernels' horizontal direct pass windows up to
// kDirectMaxX; the tile kernel runs larger direct windows with a loop over the taps.
constexpr int kDirectMax = 9;
constexpr int kDirectMaxTall = 31;
constexpr int kDirectMaxX = 16;
constexpr int kDirectChunkX = 8; // output columns per direct horizontal work unit
constexpr int kVhgwBatch = 8;    // rows the vertical vHGW pass loads at a time
constexpr int kMaxLdsBytes = 160 * 1024;

enum PassMode { PASS_NONE = 0, PASS_DIRECT = 1, PASS_VHGW = 2, PASS_DOUBLING = 3 };
// KIND_TILE: a workgroup per tile through LDS (any windows).  KIND_WAVE: vertical pass
// direct, a wave per strip of stream_quads(wx) output quads and TB rows (a multiple of
// kWaveRows, done kWaveRows at a time), in registers.  KIND_STREAM: a wave per strip
// of TW / 4 output quads and TB rows, walking down the rows once: vertical vHGW
// through a ring of wy rows in LDS, horizontal direct or log-step doubling across
// the lanes.
enum KernelKind { KIND_TILE = 0, KIND_WAVE = 1, KIND_STREAM = 2, KIND_ROWS = 3 };
constexpr int kKinds = 4;
// KIND_ROWS: vertical window 1, horizontal window kStreamMaxWx < wx <=
// kRowsMaxWx: a wave per strip of rows_lanes(wx) lanes x 16 pixels and kWaveRows rows.
constexpr int kRowsMaxWx = 1000;
// lanes of a wide-row strip that store: the last one's input, 16 l + 3 + wx + 14,
// must lie in the 1024 pixels of 64 lanes
inline int rows_lanes(int wx) { return (1006 - wx) / 16 + 1; }
constexpr int kStreamMaxWx = 128; // wider windows leave a 64-quad strip too few outputs
constexpr int kStreamMaxWy = 256; // run tables grow with wy / 8
constexpr int kStreamChunk = 8; // rows a streaming wave takes at a time (one run of a block)
// runs of kStreamChunk rows in a block of wy rows (the last may be shorter)
__host__ __device__ inline int stream_runs(int wy) { return (wy + kStreamChunk - 1) / kStreamChunk; }
// vertical vHGW form of the streaming kernel: a ring of the block's wy suffixes in LDS
// up to kStreamRingMaxWy, above it run totals in LDS and a second read of the rows
constexpr int kStreamRingMaxWy = 16;
__host__ __device__ inline bool stream_two_level(int wy) { return wy > kStreamRingMaxWy; }
// ring entries: wy, plus slack so that a chunk may read kStreamChunk entries from any
// position
__host__ __device__ inline int stream_ring_entries(int wy) { return wy + kStreamChunk - 1; }
constexpr int kWaveRows = 8;

// One image as the tile kernels see it.  Windows and anchors are the effective
// ones: both extents of the rectangle are clipped to the image size, which does
// not change any result (pixels beyond the far edge never take part).
struct TileJob {
    const uint8_t *src;
    uint8_t *dst;
    int32_t H, W;
    int64_t pitch;   // bytes between source rows
    int64_t dpitch;  // bytes between destination rows
    int32_t wx, wy;  // effective window
    int32_t ax, ay;  // effective anchors
    int32_t TW, TB;  // output tile: TW columns (multiple of 4), TB rows (even)
    int32_t tiles_x, tiles_y;
    int32_t SA, SB;  // LDS row-pair strides in dwords (odd)
    int32_t vm, hm;  // PassMode of the vertical / horizontal pass
    int32_t vcode;   // vertical pass: w >= 1 direct with that window, 0 vHGW
    int32_t hcode;   // horizontal pass: 1 none, w >= 2 direct with that window, 0 vHGW
                     // or doubling
    int32_t vrun;    // vertical vHGW: rows per run (a multiple of kVhgwBatch); a block of wy
                     // rows is scanned as ceil(wy / vrun) runs joined by their totals
    int32_t vtt;     // dwords of LDS for the run totals (shares B's space)
    int32_t kind;    // KernelKind
    int32_t op;      // 0 erode, 1 dilate
    int32_t dtype;   // 0 u8, 1 u16
    int32_t coop;    // KIND_STREAM: 0, or the cooperative form's waves a unit (4, 8, 16)
    int32_t keep;    // 1: a later launch of the same call reads dst (an intermediate), so
                     // single-image kernels store it plainly, else non-temporally
};

// the streaming kernel's cooperative form (k_stream_coop.hip): rows
// aligned, vertical vHGW in run totals; a workgroup of j.coop waves (4, 8, 16) per unit
// of TB output rows builds the unit's run totals, their scans and the output runs
// side by side.  LDS: the unit's run totals, then S and P of each block (entries of 64
// lanes x 4 bytes for uint8, 8 for uint16); a uint16 unit with one block of outputs
// (bmax 0) writes its two scans over the totals and needs the totals' entries only.
constexpr int kCoopMaxLds = 64 * 1024;
inline int coop_lds_bytes(const TileJob &j)
{
    const int rows = j.TB < j.H ? j.TB : j.H;
    const int nr = stream_runs(j.wy), bmax = (rows - 1) / j.wy;
    const int tail = rows + j.wy - 1 - (bmax + 1) * j.wy;
    const int n_runs = (bmax + 1) * nr + (nr < (tail + 7) / 8 ? nr : (tail + 7) / 8);
    const bool inplace = j.dtype == 1 && bmax == 0;
    return (n_runs + (inplace ? 0 : 2 * (bmax + 1) * (nr + 1))) * 64 * (j.dtype ? 8 : 4);
}
inline int lds_bytes(const TileJob &j)
{
    if (j.kind == KIND_WAVE || j.kind == KIND_ROWS) return 0;
    if (j.kind == KIND_STREAM && j.coop) return coop_lds_bytes(j);
    if (j.kind == KIND_STREAM) // per single-wave workgroup, 64 lanes x 4 (u8) / 8 (u16)
                               // bytes per entry: run totals and suffixes, or the ring
        return (stream_two_level(j.wy) ? 2 * stream_runs(j.wy) + 1 : stream_ring_entries(j.wy)) *
               64 * (j.dtype ? 8 : 4);
    const int b = (j.TB / 2) * j.SB;
    return (j.TB * j.SA + (b > j.vtt ? b : j.vtt)) * 4;
}

// Keep e as the calling thread's last HIP error (morph_last_hip_error) and return
// MORPH_EHIP (-4).
int record_hip_error(hipError_t e);

// kernels (morph_kernels.hip)
hipError_t launch_tile_job(const TileJob &job, hipStream_t stream);
// one launcher per kernel family (each family is a translation unit of its own)
hipError_t launch_tile_kernel(const TileJob &job, hipStream_t stream);
hipError_t launch_wave_kernel(const TileJob &job, hipStream_t stream);
// the wave kernel's tall form: vertical windows kDirectMax + 1 .. kDirectMaxTall
hipError_t launch_wave_tall_kernel(const TileJob &job, hipStream_t stream);
inline bool wave_tall(const TileJob &j) { return j.kind == KIND_WAVE && j.wy > kDirectMax; }
hipError_t launch_stream_kernel(const TileJob &job, hipStream_t stream);
hipError_t launch_stream_coop(const TileJob &job, hipStream_t stream);
hipError_t launch_rows_kernel(const TileJob &job, hipStream_t stream);
// the morphological gradient of a wave-kernel job (kind KIND_WAVE, rows aligned):
// both extrema from one read, their difference stored
hipError_t launch_gradient_job(const TileJob &job, hipStream_t stream);
// dst = dst - a (reverse false) or a - dst (reverse true) over an H x W image of
// the given pitch (bytes) and dtype
hipError_t launch_subtract(const void *a, void *dst, int H, int W, size_t pitch, int dtype,
                           bool reverse, hipStream_t stream);

// transposes (morph_transpose.hip): an H x W image of dtype (0 u8, 1 u16) into a
// W x H one, pitches in bytes; n independent 16x16 u8 / 8x8 u16 row-major blocks
hipError_t launch_transpose(const void *src, void *dst, int H, int W, size_t spitch,
                            size_t dpitch, int dtype, hipStream_t stream);
hipError_t launch_transpose_blocks(const void *src, void *dst, int64_t n, int dtype,
                                   hipStream_t stream);
// opening / closing in one pass on the wave kernel's form (k_openclose_wave.hip):
// job.op 1 = opening, 0 = closing; rows aligned; wy <= kOcWaveMaxWy, wx <= kOcWaveMaxWx;
// a strip stores oc_quads(wx) output quads at most (both operations' inputs within the
// wave's 64 quads: 4Q + 3 + 2 (wx - 1) + 3 <= 255)
constexpr int kOcWaveMaxWy = 15; // MORPH_OPENCLOSE_ONE_PASS_MAX_WY
constexpr int kOcWaveMaxWx = 64; // MORPH_OPENCLOSE_ONE_PASS_MAX_WX
inline int oc_quads(int wx) { return (251 - 2 * wx) / 4 + 1; }
hipError_t launch_openclose_wave(const TileJob &job, hipStream_t stream);
hipError_t launch_openclose_wave_u8(const TileJob &job, hipStream_t stream);
hipError_t launch_openclose_wave_u16(const TileJob &job, hipStream_t stream);
// fused opening / closing (morph_openclose.hip): both operations' direct passes on
// one LDS tile of kOcTileH x kOcTileW output pixels, windows up to kOcMaxW per axis
constexpr int kOcTileH = 32;
constexpr int kOcTileW = 128;
constexpr int kOcMaxW = 16; // MORPH_OPENCLOSE_FUSED_MAX_W
hipError_t launch_openclose(const void *src, void *dst, int H, int W, size_t pitch, int wx,
                            int wy, int ax, int ay, bool opening, int dtype, hipStream_t stream);
// persistent batch kernel
struct BatchTables {
    const TileJob *jobs;       // device array of jobs
    const int64_t *tile_start; // device prefix sums of tiles per job (n + 1 entries)
    const int32_t *tile_job;   // device: job of every tile (n_tiles entries)
    int32_t n_jobs;
    int64_t n_tiles;
    unsigned long long *counter; // device: [0] next tile, [1] workgroups finished (both 0
                                 // between launches); not used by wave groups
};
hipError_t launch_batch(const BatchTables &t, int kind, int variant, int waves, int dtype, bool aligned,
                        int grid, int lds, hipStream_t stream);
// One dispatch for the wave and streaming groups of one element type and row
// alignment: classes 0 (streaming, run totals), 1 (streaming, LDS ring) and 2
// (wave), one single-wave workgroup per unit, class c taking blocks
// [b0[c], b0[c + 1]) (b0[c] a multiple of 8, so each class keeps its units
// contiguous per XCD).
struct FusedTables {
    BatchTables g[3];
    int32_t b0[4];
};
constexpr int kFusedClasses = 3;
hipError_t launch_fused(const FusedTables &t, int dtype, bool aligned, int lds, hipStream_t stream);
hipError_t launch_fused_u8(const FusedTables &t, bool aligned, int lds, hipStream_t stream);
hipError_t launch_fused_u16(const FusedTables &t, bool aligned, int lds, hipStream_t stream);
hipError_t launch_batch_tile(const BatchTables &t, int dtype, bool aligned, int grid, int lds,
                             hipStream_t stream);
hipError_t launch_batch_wave(const BatchTables &t, int dtype, bool aligned, int grid,
                             hipStream_t stream);
hipError_t launch_batch_wave_tall(const BatchTables &t, int dtype, bool aligned, int grid,
                                  hipStream_t stream);
hipError_t launch_wave_tall_u8(const TileJob &job, hipStream_t stream);
hipError_t launch_wave_tall_u16(const TileJob &job, hipStream_t stream);
hipError_t launch_batch_wave_tall_u8(const BatchTables &t, bool aligned, int grid,
                                     hipStream_t stream);
hipError_t launch_batch_wave_tall_u16(const BatchTables &t, bool aligned, int grid,
                                      hipStream_t stream);
hipError_t launch_batch_rows(const BatchTables &t, int dtype, bool aligned, int grid,
                             hipStream_t stream);
hipError_t launch_batch_stream(const BatchTables &t, bool runs, int dtype, bool aligned, int grid,
                               int lds, hipStream_t stream);
// the cooperative form's batch kernel: one workgroup of `waves` waves per unit
hipError_t launch_batch_coop(const BatchTables &t, int dtype, int waves, int grid, int lds,
                             hipStream_t stream);
// output quads of a stream-kernel strip for a horizontal window wx (worst-case
// origin offset 3): the last one's input, 4Q + 3 + wx + 2, must lie in 64 quads
inline int stream_quads(int wx) { return (250 - wx) / 4 + 1; }
// Rows are "aligned" when the pitch is a multiple of 4 bytes (uint8) or 8 bytes
// (uint16): with the tile origin placed where the address is a multiple of the quad
// size, each quad of 4 pixels in every row is then one natural load.  The image
// must also span less than 4 GiB, so 32-bit offsets address it.
__host__ __device__ inline bool rows_aligned(const TileJob &j)
{
    const uintptr_t m = j.dtype == 0 ? 3u : 7u;
    const uint64_t span = (uint64_t)(j.H - 1) * (uint64_t)j.pitch + (uint64_t)j.W * (j.dtype ? 2 : 1);
    return ((uintptr_t)j.pitch & m) == 0 && span + 8 < (1ull << 32);
}
inline bool job_rows_aligned(const TileJob &j) { return rows_aligned(j); }

} // namespace morph
