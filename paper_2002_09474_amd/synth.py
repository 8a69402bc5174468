"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws inputs (pixel values, image sizes, windows, arrival
times).  It holds none of the erosion/dilation arithmetic and imports neither
the oracle nor the HIP library, so both sides can be fed the same bytes.

The paper's own test image (an 800x600 8-bit gray image, §5.1.3) is not
available; these generators stand in for it with the workload shapes named in
the project's benchmark configurations:

* ``uniform``     i.i.d. uniform pixels over the type's full range.
* ``document``    a document-like page: white background, black rectangles with
                  sides uniform in [2, 40] placed fully inside the image (2000 of
                  them on 1920x1080, scaled with the area elsewhere), then
                  Gaussian noise (sigma 12) rounded half-to-even and clipped.
* ``batch_specs`` per-image (H, W, window, op) for the mixed-size batch.
* ``request_stream`` Poisson arrivals with per-request crop size, window and op.
"""
from __future__ import annotations

import math

import numpy as np

MAXV = {np.dtype(np.uint8): 255, np.dtype(np.uint16): 65535}


def uniform(H: int, W: int, dtype=np.uint8, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    dt = np.dtype(dtype)
    return rng.integers(0, MAXV[dt] + 1, size=(H, W), dtype=dt)


def document(H: int, W: int, seed: int = 2, n_rect: int | None = None,
             sigma: float = 12.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    img = np.full((H, W), 255.0, dtype=np.float64)
    if n_rect is None:
        n_rect = max(1, int(round(2000.0 * H * W / (1920.0 * 1080.0))))
    for _ in range(n_rect):
        rh = min(int(rng.integers(2, 41)), H)
        rw = min(int(rng.integers(2, 41)), W)
        y = int(rng.integers(0, H - rh + 1))
        x = int(rng.integers(0, W - rw + 1))
        img[y:y + rh, x:x + rw] = 0.0
    img += rng.normal(0.0, sigma, size=(H, W))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def log_uniform_int(rng, lo: int, hi: int, size=None):
    """floor(exp(U(ln lo, ln hi))), clipped to [lo, hi]."""
    v = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)
    return np.clip(v, lo, hi)


BATCH_WINDOWS = (3, 5, 9, 15, 31, 63)


def batch_specs(n: int = 512, seed: int = 5, lo: int = 64, hi: int = 2048,
                windows=BATCH_WINDOWS):
    """Per-image sizes, square windows and ops of the mixed-size batch."""
    rng = np.random.default_rng(seed)
    Hs = log_uniform_int(rng, lo, hi, size=n)
    Ws = log_uniform_int(rng, lo, hi, size=n)
    ws = rng.choice(np.asarray(windows), size=n)
    ops = rng.choice(np.array(["erode", "dilate"]), size=n)
    return [dict(H=int(Hs[i]), W=int(Ws[i]), w=int(ws[i]), op=str(ops[i])) for i in range(n)]


def batch_images(specs, seed: int = 5, content: str = "document"):
    """Pixel content for each batch image (document-like per default)."""
    out = []
    for i, s in enumerate(specs):
        if content == "document":
            out.append(document(s["H"], s["W"], seed=seed * 100003 + i))
        else:
            out.append(uniform(s["H"], s["W"], np.uint8, seed=seed * 100003 + i))
    return out


REQUEST_OPS = ("erode", "dilate", "open", "close")


def request_stream(rate: float, duration: float, seed: int = 6, lo: int = 128, hi: int = 4096,
                   wmin: int = 3, wmax: int = 101, pool_h: int = 4096, pool_w: int = 4096,
                   pool_n: int = 32):
    """Poisson request stream: arrival time, crop (pool image, y, x, H, W), window, op.

    Windows are square and odd, uniform over {wmin, wmin+2, ..., wmax}.
    """
    rng = np.random.default_rng(seed)
    n_expect = rate * duration
    gaps = rng.exponential(1.0 / rate, size=int(n_expect * 1.2 + 100))
    t = np.cumsum(gaps)
    t = t[t < duration]
    n = t.shape[0]
    Hs = log_uniform_int(rng, lo, hi, size=n)
    Ws = log_uniform_int(rng, lo, hi, size=n)
    ys = (rng.uniform(size=n) * (pool_h - Hs + 1)).astype(np.int64)
    xs = (rng.uniform(size=n) * (pool_w - Ws + 1)).astype(np.int64)
    pool = rng.integers(0, pool_n, size=n)
    odd = np.arange(wmin, wmax + 1, 2)
    ws = rng.choice(odd, size=n)
    ops = rng.choice(np.array(REQUEST_OPS), size=n)
    return [dict(t=float(t[i]), img=int(pool[i]), y=int(ys[i]), x=int(xs[i]), H=int(Hs[i]),
                 W=int(Ws[i]), w=int(ws[i]), op=str(ops[i])) for i in range(n)]
