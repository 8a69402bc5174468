"""NumPy statement of the erosion/dilation definition (paper §2, Eq. (1)).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Used to cross-check the
C oracle on tiny images: the image is padded with the identity of the operation
(``ay`` rows above, ``wy-1-ay`` below, ``ax`` columns left, ``wx-1-ax`` right) and
the min/max is taken over every ``wy``-by-``wx`` window of the padded array.
"""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def morph(img, op, wx, wy, ax=-1, ay=-1):
    img = np.asarray(img)
    maxv = np.iinfo(img.dtype).max
    if ax < 0:
        ax = wx - 1 - wx // 2
    if ay < 0:
        ay = wy - 1 - wy // 2
    ident = maxv if op == 0 else 0
    padded = np.pad(img, ((ay, wy - 1 - ay), (ax, wx - 1 - ax)), mode="constant",
                    constant_values=ident)
    win = sliding_window_view(padded, (wy, wx))
    return (win.min(axis=(2, 3)) if op == 0 else win.max(axis=(2, 3))).astype(img.dtype)
