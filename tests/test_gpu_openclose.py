"""GPU parity of the single-pass opening and closing (§2) against the CPU oracle, bit
for bit.  Two kernels: the one-pass form on the wave kernel (rows aligned, windows
up to 64 x 15; also what morph_open / morph_close run where it applies) and the
workgroup-tile kernel (both operations on one LDS tile, windows up to 16 on each
axis) that morph_openclose_fused runs elsewhere.  Every window pair of a grid over 1..16 with
default and extreme anchors, images spanning several 32 x 128 tiles with ragged
edges, values 0 and max, windows larger than the image, odd pitches and unaligned
rows (bytes outside the image untouched), agreement with the two-launch
composition, argument errors, and the full 4096 x 4096 and 1920 x 1080 images."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2002_09474_amd as morph  # noqa: E402
from paper_2002_09474_amd import synth  # noqa: E402
from gpuutil import empty_like_dev, to_dev, to_host  # noqa: E402

REF = {"open": oracle.opening, "close": oracle.closing}
FUSED_MAX = 16  # largest window per axis the fused kernel takes


def _want(img, op, wx, wy, ax=-1, ay=-1):
    return REF[op](img, wx, wy, ax, ay, method="hybrid", thresholds=(16, 16), nthreads=8)


def _run(d, op, wx, wy, ax=-1, ay=-1, **kw):
    out = morph.openclose_fused(op, d, wx, wy, ax, ay, **kw)
    torch.cuda.synchronize()
    return to_host(out)


def _img(H, W, dtype, seed):
    img = synth.document(H, W, seed=seed, n_rect=12)
    if dtype == np.uint16:
        noise = np.random.default_rng(seed).integers(0, 256, (H, W), dtype=np.uint16)
        img = img.astype(np.uint16) * 257 - noise * (img > 0)
    return img


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_window_grid_and_anchors(dtype):
    img = _img(75, 301, dtype, seed=41)
    d, _ = to_dev(img)
    ws = (1, 2, 3, 4, 7, 8, 15, 16)
    for wx in ws:
        for wy in ws:
            anchors = {(-1, -1), (0, 0), (wx - 1, wy - 1), (wx - 1, 0)}
            for ax, ay in sorted(anchors):
                for op in ("open", "close"):
                    got = _run(d, op, wx, wy, ax, ay)
                    assert np.array_equal(got, _want(img, op, wx, wy, ax, ay)), \
                        (op, wx, wy, ax, ay, dtype)


def test_values_zero_and_max():
    """Pixels at 0 and at the maximum, where identities and image values meet."""
    rng = np.random.default_rng(42)
    for dtype in (np.uint8, np.uint16):
        top = np.iinfo(dtype).max
        img = np.where(rng.random((67, 140)) < 0.5, 0, top).astype(dtype)
        d, _ = to_dev(img)
        for wx, wy, ax, ay in ((3, 3, -1, -1), (16, 5, 15, 0), (2, 16, 0, 15)):
            for op in ("open", "close"):
                assert np.array_equal(_run(d, op, wx, wy, ax, ay),
                                      _want(img, op, wx, wy, ax, ay)), (op, wx, wy, dtype)


def test_windows_larger_than_image():
    for H, W in ((1, 1), (1, 9), (7, 1), (5, 7), (3, 130)):
        img = synth.uniform(H, W, np.uint8, seed=H * 100 + W)
        d, _ = to_dev(img)
        for wx, wy, ax, ay in ((16, 16, -1, -1), (9, 13, 8, 0), (16, 2, 0, 1)):
            for op in ("open", "close"):
                assert np.array_equal(_run(d, op, wx, wy, ax, ay),
                                      _want(img, op, wx, wy, ax, ay)), (H, W, op, wx, wy)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_pitches_offsets_and_untouched_bytes(dtype):
    H, W = 45, 161
    img = _img(H, W, dtype, seed=43)
    for pitch, off in ((161, 0), (176, 0), (167, 1), (200, 3)):
        src, _ = to_dev(img, pitch_elems=pitch, offset_elems=off)
        for wx, wy in ((3, 3), (16, 1), (1, 16), (5, 11)):
            for op in ("open", "close"):
                out, buf = empty_like_dev(src)
                before = to_host(buf).copy()
                morph.openclose_fused(op, src, wx, wy, out=out)
                torch.cuda.synchronize()
                assert np.array_equal(to_host(out), _want(img, op, wx, wy)), \
                    (pitch, off, wx, wy, op)
                after = to_host(buf)
                mask = np.ones(after.shape, bool)
                rows = off + np.arange(H)[:, None] * pitch + np.arange(W)[None, :]
                mask[rows.ravel()] = False
                assert np.array_equal(after[mask], before[mask]), "bytes outside the image"


def test_matches_composition_and_errors():
    """Same bytes as the two-launch opening/closing (automatic and tile kernels);
    windows above 16, overlapping buffers and bad anchors are rejected."""
    img = _img(130, 170, np.uint8, seed=44)
    d, _ = to_dev(img)
    for wx, wy in ((3, 3), (9, 4), (16, 16)):
        for op in ("open", "close"):
            fused = _run(d, op, wx, wy)
            auto = to_host(morph.apply(op, d, wx, wy))
            tile = to_host(morph.apply(op, d, wx, wy, method_x="vhgw", method_y="vhgw"))
            torch.cuda.synchronize()
            assert np.array_equal(fused, auto) and np.array_equal(fused, tile), (op, wx, wy)
            assert np.array_equal(fused, _want(img, op, wx, wy)), (op, wx, wy)
    # (170-byte rows are not aligned: the tile kernel, windows up to 16)
    for wx, wy, status in ((FUSED_MAX + 1, 3, -3), (3, FUSED_MAX + 1, -3)):
        with pytest.raises(morph.MorphError) as ei:
            morph.openclose_fused("open", d, wx, wy)
        assert ei.value.status == status
    # aligned rows: the one-pass form takes wx up to 64 (wy up to 15)
    da, _ = to_dev(img, pitch_elems=176)
    for wx, wy in ((17, 3), (64, 15), (3, 16)):
        assert np.array_equal(_run(da, "open", wx, wy), _want(img, "open", wx, wy)), (wx, wy)
    with pytest.raises(morph.MorphError) as ei:
        morph.openclose_fused("open", da, 3, FUSED_MAX + 1)
    assert ei.value.status == -3
    with pytest.raises(morph.MorphError) as ei:
        morph.openclose_fused("close", d, 3, 3, out=d)
    assert ei.value.status == -2
    with pytest.raises(morph.MorphError) as ei:
        morph.openclose_fused("open", d, 3, 3, ax=3)
    assert ei.value.status == -1


def test_full_size_images():
    for (H, W, dtype, seed) in ((1080, 1920, np.uint8, 46), (4096, 4096, np.uint8, 47),
                                (4096, 4096, np.uint16, 48)):
        img = synth.uniform(H, W, dtype, seed=seed)
        d, _ = to_dev(img)
        for w in (3, 15):
            for op in ("open", "close"):
                assert np.array_equal(_run(d, op, w, w), _want(img, op, w, w)), (H, W, op, w)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_one_pass_form(dtype):
    """The one-pass opening/closing on the wave kernel's form, as morph_open /
    morph_close run it: horizontal windows direct (1..9) and doubling (10..64),
    vertical 1..15 (the short and tall kernels), anchors at both ends, images of
    several strips and units with ragged edges, thin images, even and odd pitches
    (aligned rows), against the oracle and against the two-launch composition."""
    rng = np.random.default_rng(61)
    for H, W in ((1, 37), (5, 3), (123, 611), (301, 257), (64, 1000)):
        img = _img(H, W, dtype, seed=H + W)
        d, _ = to_dev(img, pitch_elems=(W + 7) // 8 * 8)
        for wx, wy in ((1, 1), (2, 9), (3, 3), (9, 10), (10, 2), (15, 15), (33, 7), (64, 12),
                       (5, 14), (9, 1)):
            ax = int(rng.integers(-1, wx))
            ay = int(rng.integers(-1, wy))
            for op in ("open", "close", "tophat", "blackhat"):
                got = morph.apply(op, d, wx, wy, ax, ay)  # one pass (no plan)
                two = morph.apply(op, d, wx, wy, ax, ay, method_x="direct" if wx <= 9 else "doubling")
                torch.cuda.synchronize()
                ref = oracle.apply(op, img, wx, wy, ax, ay, method="vhgw", nthreads=8)
                assert np.array_equal(to_host(got), ref), (H, W, op, wx, wy, ax, ay, dtype)
                assert np.array_equal(to_host(two), ref), (H, W, op, wx, wy, "two launches")
