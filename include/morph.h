/*
 * morph.h - C ABI of the MI355X (gfx950) grayscale morphology library.
 *
 * Erosion and dilation of a 2-D image by a rectangular w_x-by-w_y structuring
 * element (Limonova et al., arXiv:2002.09474, §2 Eq. (1) and the sentence after
 * it), computed separably as a vertical 1-D pass and a horizontal 1-D pass
 * (§1, §5).  Each pass runs either a direct sliding min/max (the paper's
 * "linear" pass, §5.1.2 and §5.2.2) or van Herk/Gil-Werman prefix/suffix
 * extrema (§5.1.1, §5.2.1); a per-pass window threshold picks between them
 * (§5.3).  Both passes run in one kernel through an LDS tile.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Layout: row-major, H rows of W elements, `pitch` BYTES between the starts of
 *   consecutive rows, the same pitch for src and dst.  x is the column (contiguous
 *   in memory), y the row.  Elements are uint8 (unsuffixed names, the paper's
 *   8-bit type) or uint16 (`_u16` names).
 * Window: w_x columns by w_y rows, w >= 1, no upper bound.  The rectangle for
 *   output (x, y) covers columns x - anchor_x .. x - anchor_x + w_x - 1 and rows
 *   y - anchor_y .. y - anchor_y + w_y - 1.  anchor in [0, w-1], or -1 for the
 *   placement of Eq. (1): anchor = w - 1 - floor(w / 2) (the centre for odd w).
 * Border: MORPH_BORDER_NEUTRAL only: pixels outside the image count as the
 *   identity of the operation (the type's maximum for erosion, 0 for dilation),
 *   i.e. the extremum is taken over the in-image part of the rectangle.
 * Pointers: device pointers (hipMalloc / torch allocations) on the current
 *   device.  src and dst byte ranges must not overlap (MORPH_EALIAS).  uint16
 *   pointers and pitch must be 2-byte aligned.  Any other alignment is accepted;
 *   4-byte aligned rows take the faster load/store path.
 * Ownership: the caller owns src, dst and workspace and keeps them alive until
 *   the stream has passed the enqueued work.  The library keeps no pointer after
 *   a call returns, and the single-image entry points allocate nothing.
 * Streams and errors: arguments are checked before anything is enqueued; on an
 *   error nothing is enqueued.  Kernels are enqueued on `stream` (0 = the null
 *   stream) and the call returns without synchronizing.  A failed launch returns
 *   MORPH_EHIP and morph_last_hip_error() gives the hipError_t (per thread).
 *   Device faults surface at the caller's next synchronization.  Calls on
 *   distinct streams may run concurrently from different threads.
 * Empty images (H == 0 or W == 0) are a no-op returning MORPH_OK.
 */
#ifndef MORPH_H
#define MORPH_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MORPH_OK 0
#define MORPH_EINVAL (-1)       /* bad size, pitch, window, anchor or null pointer */
#define MORPH_EALIAS (-2)       /* src and dst byte ranges overlap */
#define MORPH_EUNSUPPORTED (-3) /* border rule or dtype not supported */
#define MORPH_EHIP (-4)         /* a HIP call failed; see morph_last_hip_error() */
#define MORPH_ENOMEM (-5)       /* workspace too small / device table too small */

/* border rules */
#define MORPH_BORDER_NEUTRAL 0

/* operations (morph_apply, batch descriptors) */
#define MORPH_OP_ERODE 0
#define MORPH_OP_DILATE 1
#define MORPH_OP_OPEN 2  /* dilate(erode(src)), same rectangle and anchor (§2) */
#define MORPH_OP_CLOSE 3 /* erode(dilate(src)), same rectangle and anchor (§2) */
#define MORPH_OP_GRADIENT 4 /* dilate(src) - erode(src), same rectangle and anchor (§2) */
#define MORPH_OP_TOPHAT 5   /* max(src - open(src), 0) (§2: erosion, dilation, arithmetic) */
#define MORPH_OP_BLACKHAT 6 /* max(close(src) - src, 0) */

/* element types */
#define MORPH_U8 0
#define MORPH_U16 1

/* per-pass method (morph_plan) */
#define MORPH_METHOD_AUTO 0
#define MORPH_METHOD_DIRECT 1 /* sliding min/max, O(w) per pixel (§5.1.2, §5.2.2) */
#define MORPH_METHOD_VHGW 2   /* van Herk/Gil-Werman, O(1) per pixel (§5.1.1, §5.2.1) */
#define MORPH_METHOD_DOUBLING 3 /* horizontal only, not in the paper: log-step doubling
                                 * min/max across a wave's lanes, O(log w) per pixel */

/* Optional launch plan.  Fields left 0 are filled from the tuning table.
 * method_x / method_y force the horizontal / vertical pass algorithm (a window of
 * 1 always skips its pass); tile_w / tile_h set the output tile of one workgroup
 * (tile_w a multiple of 4, tile_h a multiple of 2).  A plan never changes the
 * result, only how it is computed.
 * Kernels: a direct vertical pass (wy <= 31; a kernel of its own past 9) runs one
 * wave per strip in registers, its horizontal pass direct (wx <= 16) or (wider
 * windows, up to 128) doubling; with both methods AUTO and no tile, larger
 * vertical windows (wx <= 128, wy <= 256) run one wave per strip that streams down
 * the rows (vertical vHGW through LDS, horizontal direct up to 9 or doubling);
 * wy = 1 with 128 < wx <= 1000 runs one wave per strip of rows with 16 pixels a
 * lane (horizontal doubling); anything else -- a forced vHGW pass, a tile, a
 * forced direct pass past those windows, larger windows -- runs the workgroup-tile
 * kernel, which implements exactly the paper's two methods (direct windows past 9
 * as a loop over the taps).
 * method_x = DOUBLING takes the wave, streaming or wide-row kernel by the
 * windows (MORPH_EUNSUPPORTED where none fits); DOUBLING for method_y, or with a
 * tile, is MORPH_EINVAL.
 * morph_resolve_plan reports the kernel's passes and its unit (tile_w x tile_h
 * output pixels). */
typedef struct morph_plan {
    int32_t method_x;
    int32_t method_y;
    int32_t tile_w;
    int32_t tile_h;
    int32_t kernel; /* out (morph_resolve_plan): MORPH_KERNEL_*; ignored on input */
    int32_t batch;  /* in (morph_resolve_plan only): nonzero = plan the image as one of a
                     * batch (its thresholds and unit heights); ignored elsewhere */
} morph_plan;

/* kernels (morph_plan.kernel) */
#define MORPH_KERNEL_TILE 0   /* workgroup tile through LDS, the paper's two methods */
#define MORPH_KERNEL_WAVE 1   /* both passes direct, one wave per strip, registers only */
#define MORPH_KERNEL_STREAM 2 /* one wave per strip streaming down the rows */
#define MORPH_KERNEL_ROWS 3   /* wy = 1, wide wx: one wave per strip, 16 pixels a lane */
#define MORPH_KERNEL_STREAM_COOP 4 /* the streaming kernel's cooperative form: 4 to 16
                                      waves share a unit (tall vertical windows;
                                      reported by morph_resolve_plan) */

/* Erosion, uint8 (§2 Eq. (1)).  See the conventions above for every argument. */
int morph_erode(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                int anchor_x, int anchor_y, int border, hipStream_t stream);
/* Dilation, uint8: Eq. (1) with max in place of min (§2). */
int morph_dilate(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                 int anchor_x, int anchor_y, int border, hipStream_t stream);
/* uint16 siblings (the paper covers 8-bit only; the definition is unchanged). */
int morph_erode_u16(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                    int anchor_x, int anchor_y, int border, hipStream_t stream);
int morph_dilate_u16(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                     int anchor_x, int anchor_y, int border, hipStream_t stream);

/* Bytes of device workspace that morph_open / morph_close need for an image of
 * this shape: one intermediate image with the same pitch (H * pitch bytes).
 * Returns 0 for an empty image. */
size_t morph_workspace_bytes(int H, int W, size_t pitch, int elem_bytes);

/* Opening and closing (§2: compositions of erosion and dilation).  Where the one-pass
 * form applies -- rows aligned (pitch a multiple of 4 bytes for uint8, 8 for uint16),
 * windows (clipped to the image) up to MORPH_OPENCLOSE_ONE_PASS_MAX_WX by
 * MORPH_OPENCLOSE_ONE_PASS_MAX_WY -- both operations run in one kernel that keeps the
 * intermediate rows in registers and workspace may be NULL.  Elsewhere the
 * intermediate image goes to `workspace` (at least morph_workspace_bytes(), else
 * MORPH_ENOMEM), which must not overlap src or dst (MORPH_EALIAS), and the two
 * operations run as two launches.  (A tuning table with "oc_one_pass": 0 takes the
 * two launches everywhere.) */
#define MORPH_OPENCLOSE_ONE_PASS_MAX_WX 64
#define MORPH_OPENCLOSE_ONE_PASS_MAX_WY 15
int morph_open(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
               int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
               hipStream_t stream);
int morph_close(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                hipStream_t stream);
int morph_open_u16(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                   int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                   hipStream_t stream);
int morph_close_u16(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                    int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                    hipStream_t stream);

/* Opening (opening != 0) or closing in one launch with no workspace (§2: an
 * opening is the dilation of the erosion, a closing the erosion of the dilation,
 * same rectangle and anchor).  dtype MORPH_U8 or MORPH_U16; every other argument
 * as for morph_open.  Where the one-pass form of morph_open applies (see there) it
 * runs; elsewhere a workgroup reads its output tile grown by 2(w - 1) per axis into
 * LDS once, runs both operations' direct passes there (intermediate pixels outside
 * the image enter the second operation as its identity) and stores the tile,
 * windows up to MORPH_OPENCLOSE_FUSED_MAX_W on each axis, else MORPH_EUNSUPPORTED.
 * Either way the intermediate image never reaches HBM.  src and dst must not
 * overlap (MORPH_EALIAS). */
#define MORPH_OPENCLOSE_FUSED_MAX_W 16
int morph_openclose_fused(int dtype, int opening, const void *src, void *dst, int H, int W,
                          size_t pitch, int wx, int wy, int anchor_x, int anchor_y, int border,
                          hipStream_t stream);

/* Morphological gradient (§2 names the arithmetic combinations of erosion and
 * dilation): dst = dilation - erosion with the same rectangle and anchor, never
 * negative.  Where the wave kernel takes the job (vertical window <= 9, horizontal
 * <= 128, automatic or direct methods) and the rows are aligned (pitch a multiple
 * of 4 bytes for uint8, 8 for uint16), one pass computes both extrema from a single
 * read and workspace may be NULL; otherwise dilation goes to dst, erosion to
 * `workspace` (at least morph_workspace_bytes(), else MORPH_ENOMEM; it must not
 * overlap src or dst, MORPH_EALIAS) and a third launch subtracts. */
int morph_gradient(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                   int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                   hipStream_t stream);
int morph_gradient_u16(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                       int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                       hipStream_t stream);

/* Top-hat (src minus its opening) and black-hat (closing minus src), clamped at 0:
 * with the same rectangle and anchor in both passes, an even window or an
 * off-centre anchor can put the opening above src (the closing below it), and
 * there the result is 0.  The opening or closing as above (in one pass where that
 * applies, workspace NULL allowed; else through the workspace, same rules), then
 * one subtraction kernel on dst. */
int morph_tophat(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                 int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                 hipStream_t stream);
int morph_blackhat(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                   int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                   hipStream_t stream);
int morph_tophat_u16(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                     int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                     hipStream_t stream);
int morph_blackhat_u16(const void *src, void *dst, int H, int W, size_t pitch, int wx, int wy,
                       int anchor_x, int anchor_y, int border, void *workspace, size_t ws_bytes,
                       hipStream_t stream);

/* General entry: any op (MORPH_OP_*) and dtype (MORPH_U8 / MORPH_U16) with an
 * optional plan (NULL = tuned defaults).  workspace is needed only for OPEN, CLOSE,
 * TOPHAT and BLACKHAT where the one-pass opening/closing does not apply (see
 * morph_open; with a plan given they always take two launches through it), and for
 * GRADIENT where its one-pass form does not apply (see morph_gradient).  The named
 * entry points above are this call with plan = NULL.  Batch descriptors take ERODE,
 * DILATE, OPEN and CLOSE. */
int morph_apply(int op, int dtype, const void *src, void *dst, int H, int W, size_t pitch,
                int wx, int wy, int anchor_x, int anchor_y, int border,
                const morph_plan *plan, void *workspace, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): morph_apply with the
 * workspace taken from a fixed device array of MORPH_STATIC_SCRATCH_BYTES bytes
 * that the library holds on each GPU it runs on until the process ends, so that
 * nothing is allocated on any call.  Every argument as for morph_apply.  The calls
 * that need a workspace there (OPEN, CLOSE, TOPHAT, BLACKHAT where the one-pass
 * form does not apply, GRADIENT where its one-pass form does not apply) need
 * H * pitch <= MORPH_STATIC_SCRATCH_BYTES, else MORPH_ENOMEM and nothing is
 * enqueued; the others use no workspace.
 * All calls on one GPU share its array: calls whose work overlaps on the device
 * (other streams, other threads) race on it, so the caller serializes them, e.g.
 * on one stream.  The array's contents after a call are unspecified (every call
 * writes the intermediate before reading it).  The first call on a device looks
 * the array's address up (hipGetSymbolAddress) and may return MORPH_EHIP. */
#define MORPH_STATIC_SCRATCH_BYTES (64u << 20)
int morph_apply_static(int op, int dtype, const void *src, void *dst, int H, int W,
                       size_t pitch, int wx, int wy, int anchor_x, int anchor_y, int border,
                       const morph_plan *plan, hipStream_t stream);

/* ---- batched launch ---------------------------------------------------------
 * Many images of uneven sizes, windows and ops in a few kernel launches, one per
 * group of images sharing a kernel kind, element type and row alignment.  Images
 * whose two passes are both direct go to a kernel with one wave per strip unit
 * (a unit table, no shared state); the others to a persistent kernel whose
 * workgroups take tiles from an atomic work queue.  Not in the paper (which
 * handles one image at a time); it applies the same per-image computation, so
 * every image's result equals its single-image call.
 * Openings and closings (§2: an opening is the dilation of the erosion, a closing
 * the erosion of the dilation, same rectangle and anchor) run as two phases of the
 * same launch: every first operation (into an intermediate image in the caller's
 * workspace) with the batch's erosions and dilations, then every second operation
 * (from the intermediate into dst). */
typedef struct morph_desc {
    const void *src;
    void *dst;
    int32_t H, W;
    int64_t pitch;     /* bytes between source rows */
    int32_t wx, wy;
    int32_t ax, ay;    /* -1 = Eq. (1) placement */
    int32_t op;        /* MORPH_OP_ERODE, _DILATE, _OPEN or _CLOSE */
    int32_t dtype;     /* MORPH_U8 or MORPH_U16 */
    int64_t dst_pitch; /* bytes between destination rows; 0 = pitch */
} morph_desc;

typedef struct morph_batch *morph_batch_t;

/* Create a batch object able to hold up to max_images descriptors and max_tiles
 * tiles (work units) in total (an opening or closing counts its tiles twice),
 * 1 <= max_tiles < 2^31 - 4, else MORPH_EINVAL.  It owns device tables (two jobs
 * per descriptor, tile prefix sums, a job index per tile: 4 bytes per tile, queue
 * counters) and pinned staging copies of them, allocated here, once; nothing is
 * allocated per launch. */
int morph_batch_create(int max_images, int64_t max_tiles, morph_batch_t *out);
/* Validate n descriptors (as the single-image calls do; an op other than ERODE,
 * DILATE, OPEN, CLOSE -> MORPH_EINVAL; overlapping src/dst of one descriptor ->
 * MORPH_EALIAS), plan their tiles and copy the tables to the device on `stream`,
 * staged through pinned memory owned by the batch (a later set first waits, on the
 * host, for that copy to finish).  Launches enqueued before a set on the same
 * stream read the old tables; launch the batch on the stream of its set (or
 * synchronize first).  Too many images or tiles -> MORPH_ENOMEM.  An invalid
 * descriptor leaves the previous batch in place; a failure after the tables
 * started to change (MORPH_ENOMEM for tiles, MORPH_EHIP) leaves the batch without
 * work: enqueue and launch return MORPH_EINVAL until a set succeeds. */
int morph_batch_set(morph_batch_t b, const morph_desc *descs, int n, hipStream_t stream);
/* Enqueue the whole batch on `stream`: per phase, one kernel dispatch for the
 * wave and streaming units of each element type and row alignment (long streaming
 * units dealt out first), then the tile and wide-row groups' kernels (the last
 * workgroup of a persistent one leaves its queue counter at zero for the next
 * launch).  When that is more than one dispatch, the first call on a stream
 * captures the launch into a hipGraph that later calls replay (the graph is
 * re-captured when the stream or the batch's shape changes); a batch of one
 * dispatch, and any batch on the legacy null stream (which cannot be captured), is
 * dispatched directly.  Launches of one batch object must not overlap (they share
 * the counter and the job table).
 * workspace / ws_bytes: device memory for the intermediates of the batch's
 * openings and closings, at least morph_batch_workspace_bytes(b) bytes (else
 * MORPH_ENOMEM; NULL, 0 when the batch has none).  It must not overlap any
 * image of the batch (MORPH_EALIAS) and is in use until the stream has passed the
 * launch.  When it differs from the previous launch's, the job table is rewritten
 * (pinned staging, an asynchronous copy on `stream` ahead of the launch; the host
 * first waits for the previous such copy). */
int morph_batch_enqueue(morph_batch_t b, void *workspace, size_t ws_bytes, hipStream_t stream);
/* Enqueue the batch on `stream` as plain kernel launches, without a graph: for
 * callers whose batch changes on every launch (a serving loop).  workspace /
 * ws_bytes as for morph_batch_enqueue. */
int morph_batch_launch(morph_batch_t b, void *workspace, size_t ws_bytes, hipStream_t stream);
/* Bytes of workspace the current batch's openings and closings need (0 if none):
 * one intermediate per such image, rows of W elements padded to 64 bytes, each
 * image starting on a 256-byte boundary. */
size_t morph_batch_workspace_bytes(morph_batch_t b);
/* Number of tiles of the current batch (after morph_batch_set), or -1. */
int64_t morph_batch_tiles(morph_batch_t b);
/* Free the device tables and graphs.  The caller must have synchronized. */
int morph_batch_destroy(morph_batch_t b);

/* ---- transposes -------------------------------------------------------------- */
/* Image transpose (§4; §1 gives its use: a filter along rows as a transpose, a
 * filter along columns and a second transpose).  dst(x, y) = src(y, x): src is H
 * rows of W elements with src_pitch bytes between rows, dst is W rows of H
 * elements with dst_pitch bytes between rows.  uint8 (morph_transpose) or uint16
 * (morph_transpose_u16).  Requirements: H, W >= 0 (H == 0 or W == 0 is a no-op
 * returning MORPH_OK); src_pitch >= W * sizeof(T), dst_pitch >= H * sizeof(T),
 * both multiples of sizeof(T) (else MORPH_EINVAL); uint16 pointers 2-byte
 * aligned (else MORPH_EINVAL); the byte ranges of src and dst must not overlap
 * (MORPH_EALIAS).  Any alignment is correct; 16-byte aligned pointers and pitches
 * take vector loads and stores.  Device pointers, caller-owned; asynchronous on
 * `stream`; launch failures return MORPH_EHIP. */
int morph_transpose(const void *src, void *dst, int H, int W, size_t src_pitch,
                    size_t dst_pitch, hipStream_t stream);
int morph_transpose_u16(const void *src, void *dst, int H, int W, size_t src_pitch,
                        size_t dst_pitch, hipStream_t stream);
/* Transpose of n_blocks independent square blocks, the two sizes §4 builds and
 * times in Table 1: dtype MORPH_U8 takes 16x16 uint8 blocks (256 bytes each),
 * MORPH_U16 8x8 uint16 blocks (128 bytes each).  Blocks are stored one after
 * another, each row-major with no padding; block b of dst is the transpose of
 * block b of src.  n_blocks in [0, 2^34] (0 is a no-op), src and dst 4-byte
 * aligned (else MORPH_EINVAL), other dtypes MORPH_EUNSUPPORTED, overlapping
 * ranges MORPH_EALIAS.  Device pointers, caller-owned; asynchronous on `stream`. */
int morph_transpose_blocks(const void *src, void *dst, int64_t n_blocks, int dtype,
                           hipStream_t stream);

/* ---- misc ------------------------------------------------------------------ */
/* Load a tuning table (JSON written by the autotuner) replacing the current one.
 * Per dtype ("u8", "u16"), every key optional:
 *   t_x, t_y            direct/large-window thresholds of single images' passes
 *                       (direct when w <= t; the compiled direct windows cap them:
 *                       16 along x, 31 along y)
 *   batch_t_x, batch_t_y  the same for the images of a batch
 *   tiles               tile kernel shapes per window bucket: [{"wmax", "tq" (input
 *                       quads of a tile row), "tb" (output rows)}, ...]
 *   wave_rows           output rows of a direct wave unit (a multiple of 8, <= 64)
 *   wave_rows_tall      the same for the wave kernel's tall form (vertical windows
 *                       10..31)
 *   stream_rows, stream_rows_runs  output rows of a streaming unit (1 .. 4096), for
 *                       vertical windows up to 16 and above
 *   wide_rows           rows of a wide-row unit (1 .. 4096; taken in groups of 4 for
 *                       uint8, 2 for uint16)
 *   batch_wave_rows, batch_stream_rows, batch_stream_rows_runs  the same three for
 *                       the images of a batch
 *   fuse                0 / 1: a batch runs its wave and streaming units of one dtype
 *                       and row alignment as one kernel dispatch
 *   oc_one_pass         0 / 1: openings and closings take the one-pass form where it
 *                       applies
 *   oc_rows, oc_rows_tall  output rows of a one-pass unit (multiples of 8, <= 64), for
 *                       vertical windows up to 9 and above
 *   oc_t_x              largest horizontal window the one-pass form takes direct
 *                       (doubling above; at most 9)
 *   h_vhgw              0 / 1: single images' automatic large horizontal windows take
 *                       the paper's vHGW across the lanes instead of doubling (where
 *                       the kernel has that form)
 *   coop_min_wy         single images on aligned rows whose vertical pass is vHGW in
 *                       run totals (wy > 16) with wy >= coop_min_wy take the streaming
 *                       kernel's cooperative form (0: never)
 *   coop_rows           output rows of its units (a multiple of 8, 8 .. 1024)
 *   coop_waves          waves sharing one of its units (4, 8 or 16)
 *   batch_coop_min_wy, batch_coop_rows, batch_coop_waves  the same three for the
 *                       images of a batch (their cooperative units run as a dispatch
 *                       of their own; 0: never)
 *   fit_units           0 / 1: a single image, or a batch, whose wave and streaming
 *                       units would number under about 2048 gets shorter ones (in
 *                       steps of 8 rows, no fewer than 8; a batch only while its tile
 *                       table holds them)
 * e.g. {"u8": {"t_x": 5, "t_y": 5, "wave_rows": 16, "stream_rows": 64,
 *              "tiles": [{"wmax": 16, "tq": 32, "tb": 64}, ...]}}
 * The built-in values are the autotuner's measurement on MI355X (the table shipped
 * beside the Python package).  A dtype missing from the file keeps its table; a key
 * missing keeps its value.  NULL restores the built-in table.  A malformed file, or
 * a unit height, flag or tile shape outside its range, returns MORPH_EINVAL and
 * changes nothing. */
int morph_load_tuning(const char *json_path);
/* Current per-pass direct->vHGW thresholds of single images for a dtype (direct
 * when w <= t). */
int morph_get_thresholds(int dtype, int *t_x, int *t_y);
/* Override the single-image thresholds (for sweeps); t <= 0 leaves a value
 * unchanged.  The batch thresholds come from the tuning table. */
int morph_set_thresholds(int dtype, int t_x, int t_y);
/* Resolve the plan the library would use for these arguments (after threshold
 * and tuning lookup); fills *plan with concrete methods and tile shape. */
int morph_resolve_plan(int dtype, int H, int W, int wx, int wy, morph_plan *plan);
const char *morph_strerror(int status);
int morph_last_hip_error(void);
/* Library version string. */
const char *morph_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MORPH_H */
