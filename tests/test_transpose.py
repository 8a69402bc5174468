"""Transposes (§4; §1 gives their use in separable filtering).

CPU part: the oracle's transpose pinned by hand-worked examples, closed forms,
NumPy's own transpose, the involution, and the identity §1 relies on (a filter
along rows equals transpose, the same filter along columns, transpose back); the
C-ABI argument checks of the HIP entry points (fake pointers, nothing launched).

GPU part: the HIP transposes through the C ABI against the oracle, bit for bit,
on sizes that span several 128-row tiles with ragged edges, odd pitches and
unaligned rows (the element-wise path), the full 4096 x 4096 images the
benchmark times, and stacks of 16x16 uint8 / 8x8 uint16 blocks."""
import numpy as np
import pytest

import oracle
from paper_2002_09474_amd import _lib

# ---------------------------------------------------------------- oracle pins


def test_hand_worked_u8():
    # rows [1 2 3], [4 5 6] -> columns become rows
    a = np.array([[1, 2, 3], [4, 5, 6]], np.uint8)
    assert oracle.transpose(a).tolist() == [[1, 4], [2, 5], [3, 6]]


def test_hand_worked_u16_keeps_both_bytes():
    # values above 255 catch a transpose that moves bytes instead of elements
    a = np.array([[0x0102, 0x0304], [0x0506, 0x0708], [0xfffe, 0x0001]], np.uint16)
    assert oracle.transpose(a).tolist() == [[0x0102, 0x0506, 0xfffe], [0x0304, 0x0708, 0x0001]]


@pytest.mark.parametrize("dt", [np.uint8, np.uint16])
@pytest.mark.parametrize("H,W", [(1, 1), (1, 7), (7, 1), (5, 9), (16, 16), (33, 130)])
def test_matches_numpy_and_closed_form(dt, H, W):
    rng = np.random.default_rng(H * 1000 + W)
    hi = 256 if dt == np.uint8 else 65536
    a = rng.integers(0, hi, (H, W)).astype(dt)
    t = oracle.transpose(a)
    assert t.shape == (W, H)
    assert np.array_equal(t, a.T)
    assert np.array_equal(oracle.transpose(t), a)  # involution
    # element (y, x) = y * W + x lands at (x, y)
    if H * W < 65536:
        enc = (np.arange(H)[:, None] * W + np.arange(W)[None, :]).astype(np.uint16)
        te = oracle.transpose(enc)
        x, y = np.meshgrid(np.arange(W), np.arange(H), indexing="ij")
        assert np.array_equal(te, (y * W + x).astype(np.uint16))


def test_empty_image():
    assert oracle.transpose(np.zeros((0, 5), np.uint8)).shape == (5, 0)


@pytest.mark.parametrize("wx,ax", [(5, -1), (4, 0), (7, 6)])
def test_row_filter_through_transposes(wx, ax):
    """§1: a filter along rows = transpose, the filter along columns, transpose;
    and for a rectangle, E_{wx x wy}(I)^T = E_{wy x wx}(I^T) with the anchors
    swapped."""
    rng = np.random.default_rng(wx)
    a = rng.integers(0, 256, (23, 31)).astype(np.uint8)
    rows = oracle.erode(a, wx, 1, ax, -1, method="brute2d")
    via = oracle.transpose(oracle.erode(oracle.transpose(a), 1, wx, -1, ax, method="brute2d"))
    assert np.array_equal(rows, via)
    r = oracle.dilate(a, wx, 3, ax, 1, method="brute2d")
    s = oracle.dilate(oracle.transpose(a), 3, wx, 1, ax, method="brute2d")
    assert np.array_equal(oracle.transpose(r), s)


@pytest.mark.parametrize("dt,k", [(np.uint8, 16), (np.uint16, 8)])
def test_blocks_closed_form(dt, k):
    # element (b, r, c) encodes (b, r, c); after the transpose (b, r, c) holds (b, c, r)
    n = 5
    b, r, c = np.meshgrid(np.arange(n), np.arange(k), np.arange(k), indexing="ij")
    if dt == np.uint8:
        src = (16 * r + c).astype(np.uint8)  # one block's worth of distinct values
        src[1] = 255 - src[1]                # blocks differ
        want = (16 * c + r).astype(np.uint8)
        want[1] = 255 - want[1]
    else:
        src = (b * 64 + 8 * r + c).astype(np.uint16)
        want = (b * 64 + 8 * c + r).astype(np.uint16)
    got = oracle.transpose_blocks(src)
    assert np.array_equal(got, want)
    # one block is the image transpose of that block
    assert np.array_equal(got[3], oracle.transpose(src[3]))
    assert oracle.transpose_blocks(src[:0]).shape == (0, k, k)


# ---------------------------------------------------------------- C-ABI checks

FAKE_SRC = 0x10000
FAKE_DST = 0x20000000


def test_transpose_validation():
    L = _lib.lib()
    E = _lib
    T = L.morph_transpose
    assert T(FAKE_SRC, FAKE_DST, -1, 8, 8, 8, None) == E.MORPH_EINVAL
    assert T(FAKE_SRC, FAKE_DST, 8, -1, 8, 8, None) == E.MORPH_EINVAL
    assert T(0, 0, 0, 8, 8, 8, None) == E.MORPH_OK        # empty: no-op
    assert T(FAKE_SRC, FAKE_DST, 8, 0, 8, 8, None) == E.MORPH_OK
    assert T(0, FAKE_DST, 8, 8, 8, 8, None) == E.MORPH_EINVAL
    assert T(FAKE_SRC, FAKE_DST, 8, 9, 8, 8, None) == E.MORPH_EINVAL   # src pitch < W
    assert T(FAKE_SRC, FAKE_DST, 9, 8, 8, 8, None) == E.MORPH_EINVAL   # dst pitch < H
    # dst's first row starts inside src's last row
    assert T(FAKE_SRC, FAKE_SRC + 7 * 16, 8, 8, 16, 8, None) == E.MORPH_EALIAS
    U = L.morph_transpose_u16
    assert U(FAKE_SRC + 1, FAKE_DST, 4, 4, 8, 8, None) == E.MORPH_EINVAL  # odd pointer
    assert U(FAKE_SRC, FAKE_DST, 4, 4, 9, 8, None) == E.MORPH_EINVAL      # odd pitch
    assert U(FAKE_SRC, FAKE_DST, 4, 4, 8, 6, None) == E.MORPH_EINVAL      # dst pitch < 2H
    B = L.morph_transpose_blocks
    assert B(FAKE_SRC, FAKE_DST, -1, 0, None) == E.MORPH_EINVAL
    assert B(FAKE_SRC, FAKE_DST, 0, 0, None) == E.MORPH_OK
    assert B(FAKE_SRC, FAKE_DST, 4, 2, None) == E.MORPH_EUNSUPPORTED
    assert B(FAKE_SRC + 2, FAKE_DST, 4, 0, None) == E.MORPH_EINVAL
    assert B(FAKE_SRC, FAKE_SRC + 1020, 4, 0, None) == E.MORPH_EALIAS
    assert B(FAKE_SRC, FAKE_SRC + 508, 4, 1, None) == E.MORPH_EALIAS   # 4 x 128 bytes


# ---------------------------------------------------------------- GPU parity


def _gpu_mods():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_09474_amd as morph
    from gpuutil import to_dev, to_host
    return torch, morph, to_dev, to_host


def _rand(H, W, dt, seed):
    rng = np.random.default_rng(seed)
    hi = 256 if dt == np.uint8 else 65536
    return rng.integers(0, hi, (H, W)).astype(dt)


@pytest.mark.gpu
@pytest.mark.parametrize("dt", [np.uint8, np.uint16])
@pytest.mark.parametrize("H,W", [(1, 1), (3, 200), (200, 3), (128, 128), (128, 64),
                                 (129, 129), (300, 517), (517, 300), (256, 384), (1000, 77),
                                 (272, 400), (1040, 336)])
def test_gpu_transpose_matches_oracle(dt, H, W):
    torch, morph, to_dev, to_host = _gpu_mods()
    a = _rand(H, W, dt, H * 7 + W)
    d, _ = to_dev(a)
    out = morph.transpose(d)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out), oracle.transpose(a))


@pytest.mark.gpu
@pytest.mark.parametrize("dt", [np.uint8, np.uint16])
@pytest.mark.parametrize("spitch_pad,dpitch_pad,off", [(10, 13, 0), (3, 5, 1), (0, 7, 3)])
def test_gpu_transpose_pitches_and_offsets(dt, spitch_pad, dpitch_pad, off):
    """Padded pitches (aligned: vector tiles), odd pitches and unaligned rows
    (element-wise tiles); bytes outside the destination view stay untouched."""
    torch, morph, to_dev, to_host = _gpu_mods()
    H, W = 259, 390
    a = _rand(H, W, dt, 11 + spitch_pad)
    d, _ = to_dev(a, pitch_elems=W + spitch_pad, offset_elems=off)
    dp = H + dpitch_pad
    tdt = torch.uint8 if dt == np.uint8 else torch.uint16
    fill = 0x5a if dt == np.uint8 else 0x5a5a
    buf = torch.full((off + W * dp + 64,), fill, dtype=torch.int32, device="cuda").to(
        torch.uint8 if dt == np.uint8 else torch.int16)
    if dt == np.uint16:
        buf = buf.view(torch.uint16)
    out = buf[off:off + W * dp].view(W, dp)[:, :H]
    assert out.dtype == tdt
    morph.transpose(d, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out), oracle.transpose(a))
    hb = buf.cpu().numpy() if dt == np.uint8 else buf.view(torch.int16).cpu().numpy().view(np.uint16)
    grid = hb[off:off + W * dp].reshape(W, dp)
    assert (grid[:, H:] == fill).all()
    assert (hb[:off] == fill).all() and (hb[off + W * dp:] == fill).all()


@pytest.mark.gpu
@pytest.mark.parametrize("dt", [np.uint8, np.uint16])
def test_gpu_transpose_full_size(dt):
    """The 4096 x 4096 images the benchmark times, in full."""
    torch, morph, to_dev, to_host = _gpu_mods()
    a = _rand(4096, 4096, dt, 3 if dt == np.uint8 else 4)
    d, _ = to_dev(a)
    out = morph.transpose(d)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out), oracle.transpose(a))


@pytest.mark.gpu
@pytest.mark.parametrize("dt,k", [(np.uint8, 16), (np.uint16, 8)])
@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000, 65537])
def test_gpu_transpose_blocks_matches_oracle(dt, k, n):
    torch, morph, _, _ = _gpu_mods()
    rng = np.random.default_rng(n + k)
    hi = 256 if dt == np.uint8 else 65536
    a = rng.integers(0, hi, (n, k, k)).astype(dt)
    if dt == np.uint8:
        d = torch.from_numpy(a).cuda()
    else:
        d = torch.from_numpy(a.view(np.int16)).cuda().view(torch.uint16)
    out = morph.transpose_blocks(d)
    torch.cuda.synchronize()
    got = out.cpu().numpy() if dt == np.uint8 else out.view(torch.int16).cpu().numpy().view(np.uint16)
    assert np.array_equal(got, oracle.transpose_blocks(a))


@pytest.mark.gpu
def test_gpu_row_erosion_through_transposes():
    """§1's use end to end on the GPU: transpose, a vertical erosion, transpose back
    equals the horizontal erosion of the image (and the oracle's)."""
    torch, morph, to_dev, to_host = _gpu_mods()
    a = _rand(300, 517, np.uint8, 99)
    d, _ = to_dev(a)
    direct = morph.erode(d, 31, 1)
    via = morph.transpose(morph.erode(morph.transpose(d), 1, 31))
    torch.cuda.synchronize()
    want = oracle.erode(a, 31, 1, method="direct")
    assert np.array_equal(to_host(direct), want)
    assert np.array_equal(to_host(via), want)
