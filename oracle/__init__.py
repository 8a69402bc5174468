"""CPU oracle for rectangular grayscale erosion / dilation (arXiv:2002.09474).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library under ``paper_2002_09474_amd/`` and never imports it.

The arithmetic lives in ``morph_oracle.c`` (plain C loops, compiled with gcc);
this module only marshals NumPy arrays into it.  ``npref`` holds a second, NumPy
statement of the definition for cross-checks on tiny images.

Semantics (paper §2, Eq. (1) and the sentence after it): erosion is the minimum
and dilation the maximum of the source over a ``wx``-by-``wy`` rectangle whose
first column is ``x - ax`` and first row ``y - ay``.  ``ax = -1`` (the default)
means the Eq. (1) placement ``ax = wx - 1 - wx // 2`` (likewise for y).  Pixels
outside the image count as the identity of the operation (the type's largest
value for erosion, 0 for dilation).  Opening is dilation after erosion and
closing erosion after dilation, with the same rectangle (§2); the morphological
gradient is dilation minus erosion, again with the same rectangle; the top-hat is
the image minus its opening and the black-hat the closing minus the image.
The transpose (§4, used as §1 describes) takes element (y, x) to (x, y), for a
whole image or for each of a stack of square blocks.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "morph_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

ERODE, DILATE = 0, 1
DIRECT, VHGW = 0, 1
_METHODS = ("brute2d", "direct", "vhgw", "hybrid")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP for the separable passes)."""
    if force or not os.path.exists(_LIB_PATH):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-shared",
                               "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    L = ctypes.c_long
    for suf in ("u8", "u16"):
        f = getattr(lib, "oracle_brute2d_" + suf)
        f.argtypes = [P, P, I, I, L, I, I, I, I, I]
        f.restype = I
        f = getattr(lib, "oracle_separable_" + suf)
        f.argtypes = [P, P, I, I, L, I, I, I, I, I, I, I, I]
        f.restype = I
        f = getattr(lib, "oracle_hybrid_" + suf)
        f.argtypes = [P, P, I, I, L, I, I, I, I, I, I, I, I]
        f.restype = I
        f = getattr(lib, "oracle_line_direct_" + suf)
        f.argtypes = [P, L, P, L, I, I, I, I]
        f.restype = None
        f = getattr(lib, "oracle_line_vhgw_" + suf)
        f.argtypes = [P, L, P, L, I, I, I, I, P]
        f.restype = None
    lib.oracle_transpose.argtypes = [P, P, I, I, L, L, I]
    lib.oracle_transpose.restype = I
    lib.oracle_transpose_blocks.argtypes = [P, P, L, I, I]
    lib.oracle_transpose_blocks.restype = I
    lib.oracle_default_anchor.argtypes = [I]
    lib.oracle_default_anchor.restype = I
    lib.oracle_get_max_threads.restype = I
    _lib = lib
    return lib


def default_anchor(w: int) -> int:
    """Eq. (1) anchor: the rectangle starts ``w - 1 - w // 2`` before x."""
    return int(_load().oracle_default_anchor(int(w)))


def max_threads() -> int:
    return int(_load().oracle_get_max_threads())


def _suffix(a: np.ndarray) -> str:
    if a.dtype == np.uint8:
        return "u8"
    if a.dtype == np.uint16:
        return "u16"
    raise TypeError("oracle supports uint8 and uint16 images, got %s" % a.dtype)


def morph(img: np.ndarray, op: int, wx: int, wy: int, ax: int = -1, ay: int = -1,
          method: str = "direct", thresholds=(9, 9), nthreads: int = 1) -> np.ndarray:
    """Erosion (op=ERODE) or dilation (op=DILATE) of a 2-D uint8/uint16 image.

    method: "brute2d" (the definition), "direct" (separable, O(w) per pixel per
    pass), "vhgw" (separable, van Herk/Gil-Werman per pass), "hybrid" (per pass:
    direct when w <= threshold, else vHGW; thresholds = (t_x, t_y)).
    """
    if method not in _METHODS:
        raise ValueError("unknown method %r" % method)
    img = np.ascontiguousarray(img)
    if img.ndim != 2:
        raise ValueError("expected a 2-D image")
    lib = _load()
    suf = _suffix(img)
    H, W = img.shape
    out = np.empty_like(img)
    if H == 0 or W == 0:
        return out
    src, dst = img.ctypes.data, out.ctypes.data
    if method == "brute2d":
        rc = getattr(lib, "oracle_brute2d_" + suf)(src, dst, H, W, W, wx, wy, ax, ay, op)
    elif method == "hybrid":
        rc = getattr(lib, "oracle_hybrid_" + suf)(src, dst, H, W, W, wx, wy, ax, ay, op,
                                                  int(thresholds[0]), int(thresholds[1]),
                                                  int(nthreads))
    else:
        m = DIRECT if method == "direct" else VHGW
        rc = getattr(lib, "oracle_separable_" + suf)(src, dst, H, W, W, wx, wy, ax, ay, op,
                                                     m, m, int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected arguments (rc=%d): H=%d W=%d wx=%d wy=%d ax=%d ay=%d"
                         % (rc, H, W, wx, wy, ax, ay))
    return out


def erode(img, wx, wy, ax=-1, ay=-1, **kw):
    return morph(img, ERODE, wx, wy, ax, ay, **kw)


def dilate(img, wx, wy, ax=-1, ay=-1, **kw):
    return morph(img, DILATE, wx, wy, ax, ay, **kw)


def opening(img, wx, wy, ax=-1, ay=-1, **kw):
    """Opening: dilation of the erosion, same rectangle and anchor (§2)."""
    return dilate(erode(img, wx, wy, ax, ay, **kw), wx, wy, ax, ay, **kw)


def closing(img, wx, wy, ax=-1, ay=-1, **kw):
    """Closing: erosion of the dilation, same rectangle and anchor (§2)."""
    return erode(dilate(img, wx, wy, ax, ay, **kw), wx, wy, ax, ay, **kw)


def gradient(img, wx, wy, ax=-1, ay=-1, **kw):
    """Morphological gradient: dilation minus erosion with the same rectangle and
    anchor, one of the arithmetic combinations of erosion and dilation §2 names.
    Never negative (a window's maximum is at least its minimum), so it keeps the
    input's type."""
    d = dilate(img, wx, wy, ax, ay, **kw).astype(np.int64)
    e = erode(img, wx, wy, ax, ay, **kw).astype(np.int64)
    return (d - e).astype(img.dtype)


def tophat(img, wx, wy, ax=-1, ay=-1, **kw):
    """White top-hat: the image minus its opening (§2's combinations of erosion and
    dilation), clamped at 0.  The opening uses the same rectangle and anchor in both
    passes, so with an even window or an off-centre anchor it can exceed the image
    (it stays below it only when the anchor is the centre, 2 a = w - 1); there the
    difference is 0 rather than negative."""
    o = opening(img, wx, wy, ax, ay, **kw).astype(np.int64)
    return np.maximum(img.astype(np.int64) - o, 0).astype(img.dtype)


def blackhat(img, wx, wy, ax=-1, ay=-1, **kw):
    """Black top-hat: the closing minus the image, clamped at 0 (as for the top-hat,
    a closing with an off-centre anchor can fall below the image)."""
    c = closing(img, wx, wy, ax, ay, **kw).astype(np.int64)
    return np.maximum(c - img.astype(np.int64), 0).astype(img.dtype)


OPS = {"erode": erode, "dilate": dilate, "open": opening, "close": closing,
       "gradient": gradient, "tophat": tophat, "blackhat": blackhat}


def apply(op_name: str, img, wx, wy, ax=-1, ay=-1, **kw):
    return OPS[op_name](img, wx, wy, ax, ay, **kw)


def line(x: np.ndarray, w: int, a: int = -1, op: int = ERODE, method: str = "direct"):
    """One 1-D line (1-D erosion/dilation), direct or vHGW."""
    x = np.ascontiguousarray(x)
    if x.ndim != 1:
        raise ValueError("expected a 1-D line")
    lib = _load()
    suf = _suffix(x)
    n = x.shape[0]
    out = np.empty_like(x)
    if method == "direct":
        getattr(lib, "oracle_line_direct_" + suf)(x.ctypes.data, 1, out.ctypes.data, 1,
                                                  n, w, a, op)
    elif method == "vhgw":
        pad = np.empty(3 * (n + 2 * w), dtype=x.dtype)
        getattr(lib, "oracle_line_vhgw_" + suf)(x.ctypes.data, 1, out.ctypes.data, 1,
                                                n, w, a, op, pad.ctypes.data)
    else:
        raise ValueError("unknown method %r" % method)
    return out


def transpose(img: np.ndarray) -> np.ndarray:
    """Image transpose by its definition (§4): out[x, y] = img[y, x]."""
    _suffix(img)
    if img.ndim != 2:
        raise ValueError("expected a 2-D image")
    img = np.ascontiguousarray(img)
    H, W = img.shape
    out = np.empty((W, H), dtype=img.dtype)
    es = img.itemsize
    rc = _load().oracle_transpose(img.ctypes.data, out.ctypes.data, H, W, W * es, H * es, es)
    if rc:
        raise ValueError("oracle_transpose failed (%d)" % rc)
    return out


def transpose_blocks(blocks: np.ndarray) -> np.ndarray:
    """Each k x k block of an (n, k, k) stack transposed (§4: 16x16 8-bit and
    8x8 16-bit blocks)."""
    _suffix(blocks)
    if blocks.ndim != 3 or blocks.shape[1] != blocks.shape[2]:
        raise ValueError("expected an (n, k, k) stack of blocks")
    blocks = np.ascontiguousarray(blocks)
    out = np.empty_like(blocks)
    n, k = blocks.shape[0], blocks.shape[1]
    rc = _load().oracle_transpose_blocks(blocks.ctypes.data, out.ctypes.data, n, k,
                                         blocks.itemsize)
    if rc:
        raise ValueError("oracle_transpose_blocks failed (%d)" % rc)
    return out
