"""Helpers for GPU tests: host <-> device copies of uint8/uint16 images."""
import numpy as np


def to_dev(a: np.ndarray, pitch_elems: int | None = None, offset_elems: int = 0):
    """Copy a 2-D uint8/uint16 array to the GPU.  With pitch_elems / offset_elems
    the image is a strided view into a larger buffer (to exercise pitch and
    alignment); returns (view, backing buffer)."""
    import torch
    H, W = a.shape
    p = W if pitch_elems is None else pitch_elems
    if a.dtype == np.uint16:
        host = np.full(offset_elems + max(H, 1) * p + 64, 0x5a5a, np.uint16)
        host[offset_elems:offset_elems + H * p].reshape(H, p)[:, :W] = a
        buf = torch.from_numpy(host.view(np.int16)).cuda().view(torch.uint16)
    else:
        host = np.full(offset_elems + max(H, 1) * p + 64, 0x5a, np.uint8)
        host[offset_elems:offset_elems + H * p].reshape(H, p)[:, :W] = a
        buf = torch.from_numpy(host).cuda()
    view = buf[offset_elems:offset_elems + H * p].view(H, p)[:, :W]
    return view, buf


def empty_like_dev(view, fill: int = 0x5a):
    """A device buffer with the same geometry as `view` (a strided view made by
    to_dev), pre-filled with a sentinel so untouched bytes can be checked."""
    import torch
    H, W = view.shape
    p = view.stride(0)
    base_off = view.storage_offset()
    n = base_off + max(H, 1) * p + 64
    if view.dtype == torch.uint8:
        buf = torch.full((n,), fill, dtype=torch.uint8, device=view.device)
    else:
        buf = torch.full((n,), fill | (fill << 8), dtype=torch.int16,
                         device=view.device).view(torch.uint16)
    out = buf[base_off:base_off + H * p].view(H, p)[:, :W]
    return out, buf


def to_host(t) -> np.ndarray:
    import torch
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()
