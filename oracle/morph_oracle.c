/*
 * CPU oracle for grayscale erosion and dilation with a rectangular structuring
 * element (Limonova et al., "Fast Implementation of Morphological Filtering
 * Using ARM NEON Extension", arXiv:2002.09474).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  It shares no code, header, table or helper
 * with the HIP library, and the HIP library never calls it.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What is computed (paper §2, Eq. (1) and the sentence after it):
 *   erosion  D(x,y) = min of S over the w_x-by-w_y rectangle placed on (x,y)
 *   dilation D(x,y) = max of S over the same rectangle.
 * Eq. (1) places the rectangle so that its columns run from
 * x - (w_x - 1) + floor(w_x/2) to x + floor(w_x/2); in terms of an anchor a_x
 * (the offset of x from the rectangle's first column) that is
 * a_x = w_x - 1 - floor(w_x/2), and likewise for y.  Callers may pass any
 * other anchor in [0, w-1]; -1 selects the Eq. (1) placement.
 *
 * Border: the paper processes image edges "separately" without stating the
 * rule (§5.1.2, §5.2.2).  This oracle takes pixels outside the image as the
 * identity of the operation (the largest value for erosion, 0 for dilation),
 * which is the same as taking the min/max over the in-image part of the
 * rectangle only.  The rectangle always contains (x,y) itself, so that part
 * is never empty.
 *
 * Four ways of computing the same result are provided:
 *   1. oracle_brute2d_*     the definition, a quadruple loop;
 *   2. oracle_separable_*   with both methods DIRECT: a row pass of width w_x
 *                           then a column pass of height w_y, each an O(w)
 *                           loop per pixel (separability, §1 and §5);
 *   3. the same entry with method VHGW: each 1-D pass by van Herk/Gil-Werman
 *      prefix/suffix extrema over blocks of w (§5.1.1, §5.2.1), the column
 *      pass keeping whole-image prefix and suffix buffers as the paper
 *      describes (extra memory of twice the image);
 *   4. per-pass choice between 2 and 3 by a window threshold (§5.3).
 * Element types: uint8 (the paper's) and uint16.  Images are row-major with
 * a pitch given in elements.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_ERODE 0
#define ORACLE_DILATE 1
#define ORACLE_DIRECT 0
#define ORACLE_VHGW 1

/* Eq. (1): D(x) reads S(x - n + floor(w/2)) for n in [0, w-1], so the
 * rectangle's first element is x - (w - 1 - floor(w/2)). */
int oracle_default_anchor(int w) { return w - 1 - w / 2; }

static int resolve_anchor(int w, int a) { return a < 0 ? oracle_default_anchor(w) : a; }

static int check_args(int H, int W, int wx, int wy, int ax, int ay, int op)
{
    if (H < 0 || W < 0 || wx < 1 || wy < 1) return -1;
    if (ax < -1 || ax >= wx || ay < -1 || ay >= wy) return -1;
    if (op != ORACLE_ERODE && op != ORACLE_DILATE) return -1;
    return 0;
}

int oracle_get_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define DEFINE_ORACLE(T, SUF, MAXV)                                                        \
                                                                                           \
static inline T better_##SUF(T a, T b, int op)                                             \
{                                                                                          \
    if (op == ORACLE_ERODE) return a < b ? a : b;                                          \
    return a > b ? a : b;                                                                  \
}                                                                                          \
                                                                                           \
/* 1. The definition: min/max over the in-image part of the rectangle. */                 \
int oracle_brute2d_##SUF(const T *src, T *dst, int H, int W, long pitch,                  \
                         int wx, int wy, int ax, int ay, int op)                          \
{                                                                                          \
    if (check_args(H, W, wx, wy, ax, ay, op)) return -1;                                  \
    ax = resolve_anchor(wx, ax);                                                           \
    ay = resolve_anchor(wy, ay);                                                           \
    T ident = (op == ORACLE_ERODE) ? (T)(MAXV) : (T)0;                                     \
    for (int y = 0; y < H; y++)                                                            \
        for (int x = 0; x < W; x++) {                                                      \
            T acc = ident;                                                                 \
            for (int m = 0; m < wy; m++) {                                                 \
                int yy = y - ay + m;                                                       \
                if (yy < 0 || yy >= H) continue;                                           \
                for (int n = 0; n < wx; n++) {                                             \
                    int xx = x - ax + n;                                                   \
                    if (xx < 0 || xx >= W) continue;                                       \
                    acc = better_##SUF(acc, src[(long)yy * pitch + xx], op);               \
                }                                                                          \
            }                                                                              \
            dst[(long)y * pitch + x] = acc;                                                \
        }                                                                                  \
    return 0;                                                                              \
}                                                                                          \
                                                                                           \
/* One 1-D line, direct: out[i] = op of in[i-a .. i-a+w-1] within [0, n-1]. */             \
void oracle_line_direct_##SUF(const T *in, long sin, T *out, long sout,                   \
                              int n, int w, int a, int op)                                \
{                                                                                          \
    a = resolve_anchor(w, a);                                                              \
    T ident = (op == ORACLE_ERODE) ? (T)(MAXV) : (T)0;                                     \
    for (int i = 0; i < n; i++) {                                                          \
        T acc = ident;                                                                     \
        for (int j = 0; j < w; j++) {                                                      \
            int k = i - a + j;                                                             \
            if (k >= 0 && k < n) acc = better_##SUF(acc, in[(long)k * sin], op);           \
        }                                                                                  \
        out[(long)i * sout] = acc;                                                         \
    }                                                                                      \
}                                                                                          \
                                                                                           \
/* One 1-D line by van Herk/Gil-Werman.  The line is padded with the identity,           \
 * a elements in front and w-1-a behind, then up to a multiple of w.  Blocks of w        \
 * start at padded index 0.  g is the running op from the start of each block (prefix), \
 * h the running op to the end of each block (suffix).  The window of output i starts   \
 * at padded index i and ends at i+w-1; it spans at most two blocks, so                  \
 * out[i] = op(h[i], g[i+w-1]).  pad must hold 3 * (n + 2w) elements.                    \
 */                                                                                        \
void oracle_line_vhgw_##SUF(const T *in, long sin, T *out, long sout,                     \
                            int n, int w, int a, int op, T *pad)                          \
{                                                                                          \
    a = resolve_anchor(w, a);                                                              \
    T ident = (op == ORACLE_ERODE) ? (T)(MAXV) : (T)0;                                     \
    long len = (long)n + w - 1;                                                            \
    long nblk = (len + w - 1) / w;                                                         \
    long plen = nblk * w;                                                                  \
    T *p = pad, *g = pad + plen, *h = pad + 2 * plen;                                      \
    for (long i = 0; i < plen; i++) {                                                      \
        long k = i - a;                                                                    \
        p[i] = (k >= 0 && k < n) ? in[k * sin] : ident;                                    \
    }                                                                                      \
    for (long i = 0; i < plen; i++)                                                        \
        g[i] = (i % w == 0) ? p[i] : better_##SUF(g[i - 1], p[i], op);                     \
    for (long i = plen - 1; i >= 0; i--)                                                   \
        h[i] = ((i + 1) % w == 0) ? p[i] : better_##SUF(h[i + 1], p[i], op);               \
    for (long i = 0; i < n; i++)                                                           \
        out[i * sout] = better_##SUF(h[i], g[i + w - 1], op);                              \
}                                                                                          \
                                                                                           \
/* Column pass by vHGW over whole rows: blocks of wy rows, prefix and suffix kept as       \
 * two image-sized buffers (the paper's vertical-window vHGW runs every column of a row   \
 * in the same way, with 2x image of extra memory).  Rows outside the image are the       \
 * identity.  dst may not alias src. */                                                    \
static int column_vhgw_##SUF(const T *src, T *dst, int H, int W, long pitch,              \
                             int w, int a, int op, int nthreads)                          \
{                                                                                          \
    T ident = (op == ORACLE_ERODE) ? (T)(MAXV) : (T)0;                                     \
    long len = (long)H + w - 1;                                                            \
    long plen = ((len + w - 1) / w) * w;                                                   \
    T *g = (T *)malloc(sizeof(T) * plen * (size_t)W);                                      \
    T *h = (T *)malloc(sizeof(T) * plen * (size_t)W);                                      \
    if (!g || !h) { free(g); free(h); return -2; }                                         \
    /* padded row i is image row i - a; columns are split into strips across threads */    \
    _Pragma("omp parallel for schedule(static) num_threads(nthreads)")                     \
    for (int x0 = 0; x0 < W; x0 += 256) {                                                  \
        int x1 = x0 + 256 < W ? x0 + 256 : W;                                              \
        for (long i = 0; i < plen; i++) {                                                  \
            long r = i - a;                                                                \
            const T *srow = (r >= 0 && r < H) ? src + r * pitch : NULL;                    \
            T *grow = g + i * W;                                                           \
            for (int x = x0; x < x1; x++) {                                                \
                T v = srow ? srow[x] : ident;                                              \
                grow[x] = (i % w == 0) ? v : better_##SUF(grow[x - W], v, op);             \
            }                                                                              \
        }                                                                                  \
        for (long i = plen - 1; i >= 0; i--) {                                             \
            long r = i - a;                                                                \
            const T *srow = (r >= 0 && r < H) ? src + r * pitch : NULL;                    \
            T *hrow = h + i * W;                                                           \
            for (int x = x0; x < x1; x++) {                                                \
                T v = srow ? srow[x] : ident;                                              \
                hrow[x] = ((i + 1) % w == 0) ? v : better_##SUF(hrow[x + W], v, op);       \
            }                                                                              \
        }                                                                                  \
    }                                                                                      \
    for (long y = 0; y < H; y++) {                                                         \
        const T *hrow = h + y * W, *grow = g + (y + w - 1) * W;                            \
        T *drow = dst + y * pitch;                                                         \
        for (int x = 0; x < W; x++) drow[x] = better_##SUF(hrow[x], grow[x], op);          \
    }                                                                                      \
    free(g);                                                                               \
    free(h);                                                                               \
    return 0;                                                                              \
}                                                                                          \
                                                                                           \
/* Column pass, direct, row-major order: dst row y = op of src rows y-a .. y-a+w-1. */    \
static void column_direct_##SUF(const T *src, T *dst, int H, int W, long pitch,           \
                                int w, int a, int op, int nthreads)                       \
{                                                                                          \
    T ident = (op == ORACLE_ERODE) ? (T)(MAXV) : (T)0;                                     \
    (void)nthreads;                                                                        \
    _Pragma("omp parallel for schedule(static) num_threads(nthreads)")                     \
    for (int y = 0; y < H; y++) {                                                          \
        T *drow = dst + (long)y * pitch;                                                   \
        for (int x = 0; x < W; x++) drow[x] = ident;                                       \
        for (int m = 0; m < w; m++) {                                                      \
            int yy = y - a + m;                                                            \
            if (yy < 0 || yy >= H) continue;                                               \
            const T *srow = src + (long)yy * pitch;                                        \
            for (int x = 0; x < W; x++) drow[x] = better_##SUF(drow[x], srow[x], op);      \
        }                                                                                  \
    }                                                                                      \
}                                                                                          \
                                                                                           \
/* 2-4. Separable: a row pass (w_x) into a temporary image, then a column pass (w_y)      \
 * into dst.  method_x / method_y pick DIRECT or VHGW for each pass. */                    \
int oracle_separable_##SUF(const T *src, T *dst, int H, int W, long pitch,                \
                           int wx, int wy, int ax, int ay, int op,                        \
                           int method_x, int method_y, int nthreads)                      \
{                                                                                          \
    if (check_args(H, W, wx, wy, ax, ay, op)) return -1;                                  \
    if (nthreads < 1) nthreads = 1;                                                        \
    ax = resolve_anchor(wx, ax);                                                           \
    ay = resolve_anchor(wy, ay);                                                           \
    if (H == 0 || W == 0) return 0;                                                        \
    T *tmp = (T *)malloc(sizeof(T) * (size_t)H * (size_t)W);                               \
    if (!tmp) return -2;                                                                   \
    int bad = 0;                                                                           \
    _Pragma("omp parallel num_threads(nthreads)")                                          \
    {                                                                                      \
        T *pad = (T *)malloc(sizeof(T) * 3 * ((size_t)W + 2 * (size_t)wx));                \
        if (!pad) {                                                                        \
            _Pragma("omp atomic write")                                                    \
            bad = 1;                                                                       \
        } else {                                                                           \
            _Pragma("omp for schedule(static)")                                            \
            for (int y = 0; y < H; y++) {                                                  \
                if (method_x == ORACLE_VHGW)                                               \
                    oracle_line_vhgw_##SUF(src + (long)y * pitch, 1, tmp + (long)y * W, 1,\
                                           W, wx, ax, op, pad);                            \
                else                                                                       \
                    oracle_line_direct_##SUF(src + (long)y * pitch, 1, tmp + (long)y * W, \
                                             1, W, wx, ax, op);                            \
            }                                                                              \
            free(pad);                                                                     \
        }                                                                                  \
    }                                                                                      \
    if (bad) { free(tmp); return -2; }                                                     \
    int rc = 0;                                                                            \
    if (method_y == ORACLE_VHGW) {                                                         \
        /* the tmp image has pitch W; write dst rows with the caller's pitch */             \
        T *tmp2 = (T *)malloc(sizeof(T) * (size_t)H * (size_t)W);                          \
        if (!tmp2) { free(tmp); return -2; }                                               \
        rc = column_vhgw_##SUF(tmp, tmp2, H, W, W, wy, ay, op, nthreads);                  \
        for (int y = 0; y < H && rc == 0; y++)                                             \
            memcpy(dst + (long)y * pitch, tmp2 + (long)y * W, sizeof(T) * (size_t)W);      \
        free(tmp2);                                                                        \
    } else {                                                                               \
        T *tmp2 = (T *)malloc(sizeof(T) * (size_t)H * (size_t)W);                          \
        if (!tmp2) { free(tmp); return -2; }                                               \
        column_direct_##SUF(tmp, tmp2, H, W, W, wy, ay, op, nthreads);                     \
        for (int y = 0; y < H; y++)                                                        \
            memcpy(dst + (long)y * pitch, tmp2 + (long)y * W, sizeof(T) * (size_t)W);      \
        free(tmp2);                                                                        \
    }                                                                                      \
    free(tmp);                                                                             \
    return rc;                                                                             \
}                                                                                          \
                                                                                           \
/* 4. Per-pass choice (§5.3): direct when w <= threshold, vHGW otherwise. */               \
int oracle_hybrid_##SUF(const T *src, T *dst, int H, int W, long pitch,                   \
                        int wx, int wy, int ax, int ay, int op,                           \
                        int tx, int ty, int nthreads)                                     \
{                                                                                          \
    return oracle_separable_##SUF(src, dst, H, W, pitch, wx, wy, ax, ay, op,              \
                                  wx <= tx ? ORACLE_DIRECT : ORACLE_VHGW,                  \
                                  wy <= ty ? ORACLE_DIRECT : ORACLE_VHGW, nthreads);       \
}

DEFINE_ORACLE(uint8_t, u8, 255)
DEFINE_ORACLE(uint16_t, u16, 65535)

/*
 * Transpose (§4; §1 states its use: a filter along rows run as a transpose, a
 * filter along columns and a second transpose).  The definition, element by
 * element: dst row x, column y takes src row y, column x.  Elements are es bytes
 * (1 or 2); pitches are in bytes.
 */
int oracle_transpose(const void *src, void *dst, int H, int W, long spitch, long dpitch, int es)
{
    if (H < 0 || W < 0 || (es != 1 && es != 2)) return -1;
    const unsigned char *s = (const unsigned char *)src;
    unsigned char *d = (unsigned char *)dst;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
            memcpy(d + (long)x * dpitch + (long)y * es, s + (long)y * spitch + (long)x * es,
                   (size_t)es);
    return 0;
}

/*
 * n independent k-by-k blocks stored one after another, each row-major with no
 * padding (§4 builds these for 8x8 16-bit and 16x16 8-bit blocks): block b of dst
 * is the transpose of block b of src.
 */
int oracle_transpose_blocks(const void *src, void *dst, long n, int k, int es)
{
    if (n < 0 || k < 1 || (es != 1 && es != 2)) return -1;
    const long bb = (long)k * k * es;
    for (long b = 0; b < n; b++)
        if (oracle_transpose((const unsigned char *)src + b * bb, (unsigned char *)dst + b * bb,
                             k, k, (long)k * es, (long)k * es, es))
            return -1;
    return 0;
}
