"""ctypes binding of the HIP morphology library (``include/morph.h``).

Argument marshalling only: every step of erosion/dilation runs in the HIP
kernels of ``libmorph_hip.so``.  Torch supplies device memory and streams.  If
the built library is missing, loading fails with an error; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libmorph_hip.so")
TUNING_PATH = os.path.join(HERE, "tuning_gfx950.json")

MORPH_OK = 0
MORPH_EINVAL = -1
MORPH_EALIAS = -2
MORPH_EUNSUPPORTED = -3
MORPH_EHIP = -4
MORPH_ENOMEM = -5

OP_ERODE, OP_DILATE, OP_OPEN, OP_CLOSE, OP_GRADIENT, OP_TOPHAT, OP_BLACKHAT = range(7)
OP_CODES = {"erode": OP_ERODE, "dilate": OP_DILATE, "open": OP_OPEN, "close": OP_CLOSE,
            "gradient": OP_GRADIENT, "tophat": OP_TOPHAT, "blackhat": OP_BLACKHAT}
U8, U16 = 0, 1
METHOD_AUTO, METHOD_DIRECT, METHOD_VHGW = 0, 1, 2
METHOD_CODES = {None: 0, "auto": 0, "direct": 1, "vhgw": 2, "doubling": 3}

# every symbol include/morph.h declares
EXPORTS = (
    "morph_erode", "morph_dilate", "morph_erode_u16", "morph_dilate_u16",
    "morph_workspace_bytes", "morph_open", "morph_close", "morph_open_u16", "morph_close_u16",
    "morph_gradient", "morph_gradient_u16", "morph_tophat", "morph_blackhat",
    "morph_tophat_u16", "morph_blackhat_u16",
    "morph_transpose", "morph_transpose_u16", "morph_transpose_blocks",
    "morph_openclose_fused", "morph_apply", "morph_batch_create", "morph_batch_set", "morph_batch_enqueue",
    "morph_batch_launch", "morph_batch_workspace_bytes",
    "morph_batch_tiles", "morph_batch_destroy", "morph_load_tuning", "morph_get_thresholds",
    "morph_set_thresholds", "morph_resolve_plan", "morph_strerror", "morph_last_hip_error",
    "morph_version", "morph_apply_static",
)


class MorphError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _strerror(status)
        if status == MORPH_EHIP:
            try:
                msg += " (hipError %d)" % lib().morph_last_hip_error()
            except Exception:  # pragma: no cover
                pass
        super().__init__("%s: %s (status %d)" % (what or "morph", msg, status))


class Plan(ctypes.Structure):
    _fields_ = [("method_x", ctypes.c_int32), ("method_y", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("batch", ctypes.c_int32)]


KERNEL_NAMES = {0: "tile", 1: "wave", 2: "stream", 3: "rows", 4: "stream_coop"}


class Desc(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("pitch", ctypes.c_int64),
                ("wx", ctypes.c_int32), ("wy", ctypes.c_int32),
                ("ax", ctypes.c_int32), ("ay", ctypes.c_int32),
                ("op", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("dst_pitch", ctypes.c_int64)]


_lib = None


def lib():
    """Load libmorph_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP morphology library not built: %s is missing "
                          "(run __graft_entry__.build() or paper_2002_09474_amd/build.py)"
                          % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I, Z, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_int64
    single = [P, P, I, I, Z, I, I, I, I, I, P]
    for n in ("morph_erode", "morph_dilate", "morph_erode_u16", "morph_dilate_u16"):
        f = getattr(L, n)
        f.argtypes = single
        f.restype = I
    composed = [P, P, I, I, Z, I, I, I, I, I, P, Z, P]
    for n in ("morph_open", "morph_close", "morph_open_u16", "morph_close_u16",
              "morph_gradient", "morph_gradient_u16", "morph_tophat", "morph_blackhat",
              "morph_tophat_u16", "morph_blackhat_u16"):
        f = getattr(L, n)
        f.argtypes = composed
        f.restype = I
    for n in ("morph_transpose", "morph_transpose_u16"):
        f = getattr(L, n)
        f.argtypes = [P, P, I, I, Z, Z, P]
        f.restype = I
    L.morph_transpose_blocks.argtypes = [P, P, I64, I, P]
    L.morph_transpose_blocks.restype = I
    L.morph_openclose_fused.argtypes = [I, I, P, P, I, I, Z, I, I, I, I, I, P]
    L.morph_openclose_fused.restype = I
    L.morph_workspace_bytes.argtypes = [I, I, Z, I]
    L.morph_workspace_bytes.restype = Z
    L.morph_apply.argtypes = [I, I, P, P, I, I, Z, I, I, I, I, I, ctypes.POINTER(Plan), P, Z, P]
    L.morph_apply.restype = I
    L.morph_apply_static.argtypes = [I, I, P, P, I, I, Z, I, I, I, I, I, ctypes.POINTER(Plan), P]
    L.morph_apply_static.restype = I
    L.morph_batch_create.argtypes = [I, I64, ctypes.POINTER(P)]
    L.morph_batch_create.restype = I
    L.morph_batch_set.argtypes = [P, ctypes.POINTER(Desc), I, P]
    L.morph_batch_set.restype = I
    L.morph_batch_enqueue.argtypes = [P, P, Z, P]
    L.morph_batch_enqueue.restype = I
    L.morph_batch_launch.argtypes = [P, P, Z, P]
    L.morph_batch_launch.restype = I
    L.morph_batch_workspace_bytes.argtypes = [P]
    L.morph_batch_workspace_bytes.restype = Z
    L.morph_batch_tiles.argtypes = [P]
    L.morph_batch_tiles.restype = I64
    L.morph_batch_destroy.argtypes = [P]
    L.morph_batch_destroy.restype = I
    L.morph_load_tuning.argtypes = [ctypes.c_char_p]
    L.morph_load_tuning.restype = I
    L.morph_get_thresholds.argtypes = [I, ctypes.POINTER(I), ctypes.POINTER(I)]
    L.morph_get_thresholds.restype = I
    L.morph_set_thresholds.argtypes = [I, I, I]
    L.morph_set_thresholds.restype = I
    L.morph_resolve_plan.argtypes = [I, I, I, I, I, ctypes.POINTER(Plan)]
    L.morph_resolve_plan.restype = I
    L.morph_strerror.argtypes = [I]
    L.morph_strerror.restype = ctypes.c_char_p
    L.morph_last_hip_error.argtypes = []
    L.morph_last_hip_error.restype = I
    L.morph_version.argtypes = []
    L.morph_version.restype = ctypes.c_char_p
    _lib = L
    if os.path.exists(TUNING_PATH):  # the autotuner's table for this GPU, if committed
        L.morph_load_tuning(TUNING_PATH.encode())
    return L


def _strerror(status: int) -> str:
    try:
        return lib().morph_strerror(status).decode()
    except Exception:  # pragma: no cover
        return "status %d" % status


def check(status: int, what: str = "") -> None:
    if status != MORPH_OK:
        raise MorphError(status, what)
