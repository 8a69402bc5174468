"""Grayscale erosion, dilation, opening and closing with a rectangular structuring
element on AMD MI355X (gfx950), after Limonova et al., "Fast Implementation of
Morphological Filtering Using ARM NEON Extension" (arXiv:2002.09474).

Every operation runs in the hand-written HIP kernels of ``libmorph_hip.so``
(C ABI in ``include/morph.h``); this module only passes torch tensors' device
pointers, shapes and streams to it.  Images are 2-D torch tensors of dtype
uint8 or uint16 on a ROCm device whose last dimension is contiguous (any row
pitch).  Semantics (§2, Eq. (1)): erosion = min and dilation = max over the
``wx``-by-``wy`` rectangle whose first column is ``x - ax`` and first row
``y - ay`` (``-1`` = Eq. (1) placement ``w - 1 - w // 2``); pixels outside the
image count as the identity (max for erosion, 0 for dilation).
"""
from __future__ import annotations

import ctypes
import os

from . import _lib
from ._lib import MorphError, Plan  # noqa: F401

__all__ = ["erode", "dilate", "opening", "closing", "gradient", "tophat", "blackhat", "apply",
           "apply_static", "Batch", "workspace_bytes",
           "openclose_fused", "transpose", "transpose_blocks",
           "load_tuning", "get_thresholds", "set_thresholds", "resolve_plan", "MorphError",
           "version"]


def _torch():
    import torch
    return torch


def dtype_code(dtype) -> int:
    torch = _torch()
    if dtype == torch.uint8:
        return _lib.U8
    if dtype == getattr(torch, "uint16", None):
        return _lib.U16
    raise TypeError("morphology supports uint8 and uint16 images, got %s" % (dtype,))


def _geom(t):
    if t.dim() != 2:
        raise ValueError("expected a 2-D image tensor, got shape %s" % (tuple(t.shape),))
    if not t.is_cuda:
        raise ValueError("image tensors must live on the GPU (device %s)" % t.device)
    H, W = t.shape
    if H > 0 and W > 0 and t.stride(1) != 1:
        raise ValueError("the last dimension must be contiguous")
    es = t.element_size()
    pitch = (t.stride(0) if H > 1 else max(t.stride(0), W)) * es
    return int(H), int(W), int(pitch)


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _plan(method_x, method_y, tile):
    if method_x is None and method_y is None and tile is None:
        return None
    tw, th = (0, 0) if tile is None else (int(tile[0]), int(tile[1]))
    return Plan(_lib.METHOD_CODES[method_x], _lib.METHOD_CODES[method_y], tw, th, 0, 0)


def workspace_bytes(H: int, W: int, pitch: int, elem_bytes: int) -> int:
    return int(_lib.lib().morph_workspace_bytes(H, W, pitch, elem_bytes))


def apply(op: str, src, wx: int, wy: int | None = None, ax: int = -1, ay: int = -1, out=None,
          workspace=None, method_x: str | None = None, method_y: str | None = None,
          tile=None, stream=None):
    """Run ``op`` in {"erode", "dilate", "open", "close", "gradient", "tophat",
    "blackhat"} on ``src``; returns ``out``.

    ``method_x`` / ``method_y`` force "direct" or "vhgw" for a pass (and
    ``method_x="doubling"`` the streaming kernel's lane doubling) and ``tile`` =
    (tile_w, tile_h) sets the workgroup tile; neither changes the result.
    ``out`` must have the same shape, dtype and row pitch as ``src``.
    """
    torch = _torch()
    wy = wx if wy is None else wy
    code = _lib.OP_CODES[op]
    dt = dtype_code(src.dtype)
    H, W, pitch = _geom(src)
    if out is None:
        out = torch.empty_strided(src.shape, src.stride(), dtype=src.dtype, device=src.device)
    if out.shape != src.shape or out.dtype != src.dtype or _geom(out)[2] != pitch:
        raise ValueError("out must match src in shape, dtype and row pitch")
    ws_ptr, ws_bytes = None, 0
    if code not in (_lib.OP_ERODE, _lib.OP_DILATE):
        if workspace is None:
            workspace = torch.empty(workspace_bytes(H, W, pitch, src.element_size()),
                                    dtype=torch.uint8, device=src.device)
        ws_ptr = workspace.data_ptr()
        ws_bytes = workspace.numel() * workspace.element_size()
    plan = _plan(method_x, method_y, tile)
    rc = _lib.lib().morph_apply(code, dt, src.data_ptr(), out.data_ptr(), H, W, pitch, wx, wy,
                                ax, ay, 0, ctypes.byref(plan) if plan is not None else None,
                                ws_ptr, ws_bytes, _stream_ptr(stream))
    _lib.check(rc, "morph_apply(%s, %dx%d)" % (op, wx, wy))
    return out


def apply_static(op: str, src, wx: int, wy: int | None = None, ax: int = -1, ay: int = -1,
                 out=None, method_x: str | None = None, method_y: str | None = None, tile=None,
                 stream=None):
    """``apply`` without a workspace argument: ops that need one take it from the
    library's fixed per-GPU array (``morph_apply_static``; images of up to
    ``STATIC_SCRATCH_BYTES`` bytes of rows), so that the call allocates nothing.
    Calls whose work overlaps on one GPU share that array and must be serialized."""
    torch = _torch()
    wy = wx if wy is None else wy
    code = _lib.OP_CODES[op]
    dt = dtype_code(src.dtype)
    H, W, pitch = _geom(src)
    if out is None:
        out = torch.empty_strided(src.shape, src.stride(), dtype=src.dtype, device=src.device)
    if out.shape != src.shape or out.dtype != src.dtype or _geom(out)[2] != pitch:
        raise ValueError("out must match src in shape, dtype and row pitch")
    plan = _plan(method_x, method_y, tile)
    rc = _lib.lib().morph_apply_static(code, dt, src.data_ptr(), out.data_ptr(), H, W, pitch,
                                       wx, wy, ax, ay, 0,
                                       ctypes.byref(plan) if plan is not None else None,
                                       _stream_ptr(stream))
    _lib.check(rc, "morph_apply_static(%s, %dx%d)" % (op, wx, wy))
    return out


STATIC_SCRATCH_BYTES = 64 << 20  # MORPH_STATIC_SCRATCH_BYTES


def openclose_fused(op: str, src, wx: int, wy: int | None = None, ax: int = -1, ay: int = -1,
                    out=None, stream=None):
    """Opening (``op="open"``) or closing (``"close"``) in one launch with no
    workspace: both operations' direct passes on one LDS tile (windows up to 16 per
    axis).  Same result as ``apply(op, ...)``, which stays the faster path;
    returns ``out``."""
    torch = _torch()
    if op not in ("open", "close"):
        raise ValueError("op must be 'open' or 'close'")
    wy = wx if wy is None else wy
    dt = dtype_code(src.dtype)
    H, W, pitch = _geom(src)
    if out is None:
        out = torch.empty_strided(src.shape, src.stride(), dtype=src.dtype, device=src.device)
    if out.shape != src.shape or out.dtype != src.dtype or _geom(out)[2] != pitch:
        raise ValueError("out must match src in shape, dtype and row pitch")
    rc = _lib.lib().morph_openclose_fused(dt, 1 if op == "open" else 0, src.data_ptr(),
                                          out.data_ptr(), H, W, pitch, wx, wy, ax, ay, 0,
                                          _stream_ptr(stream))
    _lib.check(rc, "morph_openclose_fused(%s, %dx%d)" % (op, wx, wy))
    return out


def transpose(src, out=None, stream=None):
    """Transpose a 2-D uint8 or uint16 image: ``out[x, y] = src[y, x]`` (§4).

    ``out`` (W x H, same dtype, any row pitch with a contiguous last dimension)
    is allocated contiguous when not given; returns ``out``."""
    torch = _torch()
    dt = dtype_code(src.dtype)
    H, W, spitch = _geom(src)
    if out is None:
        out = torch.empty((W, H), dtype=src.dtype, device=src.device)
    if tuple(out.shape) != (W, H) or out.dtype != src.dtype:
        raise ValueError("out must be W x H with the dtype of src")
    _, _, dpitch = _geom(out)
    f = _lib.lib().morph_transpose_u16 if dt == _lib.U16 else _lib.lib().morph_transpose
    rc = f(src.data_ptr(), out.data_ptr(), H, W, spitch, dpitch, _stream_ptr(stream))
    _lib.check(rc, "morph_transpose(%dx%d)" % (H, W))
    return out


def transpose_blocks(src, out=None, stream=None):
    """Transpose every block of an (n, 16, 16) uint8 or (n, 8, 8) uint16 tensor
    (the 16x16.8 and 8x8.16 blocks of §4, Table 1); returns ``out``."""
    torch = _torch()
    dt = dtype_code(src.dtype)
    k = 16 if dt == _lib.U8 else 8
    if src.dim() != 3 or tuple(src.shape[1:]) != (k, k) or not src.is_contiguous():
        raise ValueError("expected a contiguous (n, %d, %d) tensor" % (k, k))
    if not src.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if out is None:
        out = torch.empty_like(src)
    if out.shape != src.shape or out.dtype != src.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor like src")
    rc = _lib.lib().morph_transpose_blocks(src.data_ptr(), out.data_ptr(), src.shape[0], dt,
                                           _stream_ptr(stream))
    _lib.check(rc, "morph_transpose_blocks(%d)" % src.shape[0])
    return out


def erode(src, wx, wy=None, ax=-1, ay=-1, **kw):
    return apply("erode", src, wx, wy, ax, ay, **kw)


def dilate(src, wx, wy=None, ax=-1, ay=-1, **kw):
    return apply("dilate", src, wx, wy, ax, ay, **kw)


def opening(src, wx, wy=None, ax=-1, ay=-1, **kw):
    return apply("open", src, wx, wy, ax, ay, **kw)


def closing(src, wx, wy=None, ax=-1, ay=-1, **kw):
    return apply("close", src, wx, wy, ax, ay, **kw)


def gradient(src, wx, wy=None, ax=-1, ay=-1, **kw):
    """Morphological gradient: dilation minus erosion, same rectangle and anchor."""
    return apply("gradient", src, wx, wy, ax, ay, **kw)


def tophat(src, wx, wy=None, ax=-1, ay=-1, **kw):
    """Top-hat: the image minus its opening."""
    return apply("tophat", src, wx, wy, ax, ay, **kw)


def blackhat(src, wx, wy=None, ax=-1, ay=-1, **kw):
    """Black-hat: the closing minus the image."""
    return apply("blackhat", src, wx, wy, ax, ay, **kw)


class Batch:
    """Many (src, dst, window, op) items in one persistent, graph-replayed launch."""

    def __init__(self, max_images: int, max_tiles: int):
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().morph_batch_create(max_images, max_tiles, ctypes.byref(h)),
                   "morph_batch_create")
        self._h = h
        self._keep = []

    def set(self, items, stream=None) -> int:
        """items: iterable of dicts with src, dst (tensors of the same shape and dtype;
        each may have its own row pitch), wx, wy, op ("erode", "dilate", "open",
        "close") and optional ax, ay.  Returns the number of tiles."""
        items = list(items)
        arr = (_lib.Desc * max(1, len(items)))()
        keep = []
        for i, it in enumerate(items):
            s, d = it["src"], it["dst"]
            H, W, pitch = _geom(s)
            if d.shape != s.shape or d.dtype != s.dtype:
                raise ValueError("dst must match src in shape and dtype")
            wx = int(it["wx"])
            wy = int(it.get("wy", wx))
            arr[i] = _lib.Desc(s.data_ptr(), d.data_ptr(), H, W, pitch, wx, wy,
                               int(it.get("ax", -1)), int(it.get("ay", -1)),
                               _lib.OP_CODES[it["op"]], dtype_code(s.dtype), _geom(d)[2])
            keep.append((s, d))
        _lib.check(_lib.lib().morph_batch_set(self._h, arr, len(items), _stream_ptr(stream)),
                   "morph_batch_set")
        self._keep = keep
        return self.tiles

    @property
    def tiles(self) -> int:
        return int(_lib.lib().morph_batch_tiles(self._h))

    @property
    def workspace_bytes(self) -> int:
        """Device bytes the current batch's openings and closings need."""
        return int(_lib.lib().morph_batch_workspace_bytes(self._h))

    def _workspace(self, workspace, stream=None):
        """(pointer, bytes) of the workspace to pass: the caller's, else one kept by
        this object and grown as the batch needs (torch device memory)."""
        need = self.workspace_bytes
        if need == 0:
            return None, 0
        if workspace is None:
            ws = getattr(self, "_ws", None)
            if ws is None or ws.numel() < need:
                torch = _torch()
                dev = self._keep[0][0].device if self._keep else torch.device("cuda")
                if ws is not None and stream is not None:
                    ws.record_stream(stream)  # the last launch may still use it
                self._ws = torch.empty(need, dtype=torch.uint8, device=dev)
            workspace = self._ws
        return workspace.data_ptr(), workspace.numel() * workspace.element_size()

    def enqueue(self, stream=None, workspace=None) -> None:
        """Graph-replayed launch (captured on first use per stream and layout).
        ``workspace``: a device tensor for the openings' and closings'
        intermediates (``workspace_bytes`` bytes); by default one kept here."""
        ptr, nb = self._workspace(workspace, stream)
        _lib.check(_lib.lib().morph_batch_enqueue(self._h, ptr, nb, _stream_ptr(stream)),
                   "morph_batch_enqueue")

    def launch(self, stream=None, workspace=None) -> None:
        """Plain launch without a graph, for batches that change every time."""
        ptr, nb = self._workspace(workspace, stream)
        _lib.check(_lib.lib().morph_batch_launch(self._h, ptr, nb, _stream_ptr(stream)),
                   "morph_batch_launch")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().morph_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def load_tuning(path=None) -> None:
    """Load a tuning table (JSON, as the autotuner writes it).  ``None`` restores the
    package default: the built-in table, then ``tuning_gfx950.json`` if it exists."""
    L = _lib.lib()
    if path is None:
        _lib.check(L.morph_load_tuning(None), "morph_load_tuning(NULL)")
        if os.path.exists(_lib.TUNING_PATH):
            path = _lib.TUNING_PATH
        else:
            return
    _lib.check(L.morph_load_tuning(path.encode()), "morph_load_tuning(%s)" % path)


def get_thresholds(dtype_name: str = "u8"):
    tx, ty = ctypes.c_int(), ctypes.c_int()
    _lib.check(_lib.lib().morph_get_thresholds(_lib.U8 if dtype_name == "u8" else _lib.U16,
                                               ctypes.byref(tx), ctypes.byref(ty)))
    return tx.value, ty.value


def set_thresholds(dtype_name: str, t_x: int, t_y: int) -> None:
    _lib.check(_lib.lib().morph_set_thresholds(_lib.U8 if dtype_name == "u8" else _lib.U16,
                                               t_x, t_y))


def resolve_plan(dtype_name: str, H: int, W: int, wx: int, wy: int, method_x=None,
                 method_y=None, tile=None, batch=False):
    """The plan the library takes for these arguments (``batch``: as an image of a
    batch, whose thresholds and unit heights are keys of their own)."""
    p = _plan(method_x, method_y, tile) or Plan(0, 0, 0, 0, 0, 0)
    p.batch = 1 if batch else 0
    _lib.check(_lib.lib().morph_resolve_plan(_lib.U8 if dtype_name == "u8" else _lib.U16,
                                             H, W, wx, wy, ctypes.byref(p)), "resolve_plan")
    names = {0: None, 1: "direct", 2: "vhgw", 3: "doubling"}
    return dict(method_x=names[p.method_x], method_y=names[p.method_y], tile_w=p.tile_w,
                tile_h=p.tile_h, kernel=_lib.KERNEL_NAMES[p.kernel])


def version() -> str:
    return _lib.lib().morph_version().decode()
