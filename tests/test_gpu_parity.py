"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for
bit (min/max of integers has exactly one correct result), on seeded inputs at
sizes that span several tiles with ragged edges, with each pass method forced so
the threshold cannot hide a bug, at the full benchmark sizes, and on the edge
cases (tiny and empty images, windows larger than the image, off-centre and
even-window anchors, odd pitches and unaligned rows, values 0 and max)."""
import os

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

OPN = {"erode": oracle.ERODE, "dilate": oracle.DILATE}
DMAX = 9  # largest window of the short wave kernel's vertical pass
TALL = 31  # the tall wave kernel's vertical windows: DMAX + 1 .. TALL
XMAX = 16  # the wave and streaming kernels' horizontal direct windows


def _ref(img, op, wx, wy, ax=-1, ay=-1):
    return oracle.morph(img, OPN[op], wx, wy, ax, ay, method="hybrid", thresholds=(16, 16),
                        nthreads=8)


def _gpu(img, op, wx, wy, ax=-1, ay=-1, **kw):
    d, _ = to_dev(img)
    out = morph.apply(op, d, wx, wy, ax, ay, **kw)
    torch.cuda.synchronize()
    return to_host(out)


def _check(img, op, wx, wy, ax=-1, ay=-1, **kw):
    got = _gpu(img, op, wx, wy, ax, ay, **kw)
    want = _ref(img, op, wx, wy, ax, ay)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("mismatch %s %dx%d a=(%d,%d) %s shape=%s at (%d,%d): got %d want %d "
                             "(%d bad)" % (op, wx, wy, ax, ay, kw, img.shape, y, x, got[y, x],
                                           want[y, x], len(bad)))


SHAPES = [(1, 1), (1, 7), (7, 1), (2, 3), (3, 2), (15, 17), (16, 16), (17, 15), (63, 65),
          (64, 64), (65, 63), (129, 257), (200, 131)]


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_small_shapes_all_methods(dtype):
    rng = np.random.default_rng(100)
    for i, (H, W) in enumerate(SHAPES):
        img = synth.uniform(H, W, dtype, seed=200 + i)
        img.flat[0] = 0
        img.flat[-1] = np.iinfo(dtype).max
        for wx, wy in ((1, 1), (3, 3), (2, 5), (7, 4), (9, 1), (1, 9), (16, 2), (5, 13)):
            ax = int(rng.integers(-1, wx))
            ay = int(rng.integers(-1, wy))
            for op in ("erode", "dilate"):
                for mx, my in (("direct", "direct"), ("vhgw", "vhgw"), ("direct", "vhgw"),
                               ("vhgw", "direct")):
                    _check(img, op, wx, wy, ax, ay, method_x=mx, method_y=my)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_every_window_1_to_64_both_methods(axis):
    img = synth.document(150, 333, seed=21, n_rect=60)
    for w in range(1, 65):
        wx, wy = (w, 1) if axis == "x" else (1, w)
        for op in ("erode", "dilate"):
            # direct: the wave kernel up to 16 along x and 31 along y, the tile
            # kernel's tap loops beyond
            for m in ("direct", "vhgw"):
                kw = {"method_x": m} if axis == "x" else {"method_y": m}
                _check(img, op, wx, wy, **kw)


def test_all_anchors_and_even_windows():
    img = synth.uniform(70, 90, np.uint8, seed=22)
    for w in (2, 4, 6, 9, 12, 16, 20, 21, 30):
        for a in sorted({0, 1, w // 2, w - 1}):
            for m in ("direct", "vhgw"):
                _check(img, "erode", w, 3, a, 1, method_x=m)
                _check(img, "dilate", 3, w, 0, a, method_y=m)


def test_windows_larger_than_image():
    img = synth.uniform(40, 50, np.uint16, seed=23)
    for wx, wy, ax, ay in ((101, 101, -1, -1), (255, 1, -1, -1), (1, 255, -1, -1),
                           (99, 97, 0, 96), (120, 3, 119, 0), (3, 300, 1, 0)):
        for op in ("erode", "dilate"):
            _check(img, op, wx, wy, ax, ay)
    # the whole image under every window: a constant
    g = _gpu(img, "erode", 99, 79)
    assert (g == img.min()).all()


@pytest.mark.parametrize("tile", [(4, 2), (8, 6), (128, 64), (256, 32), (64, 128)])
def test_tile_shapes_do_not_change_results(tile):
    img = synth.document(157, 203, seed=24, n_rect=40)
    for wx, wy in ((3, 3), (15, 9), (31, 31), (2, 40)):
        for op in ("erode", "dilate"):
            _check(img, op, wx, wy, tile=tile)


@pytest.mark.parametrize("rows", [8, 16, 64])
def test_wave_units_of_several_row_chunks(rows, tmp_path):
    """Both passes direct run one wave per strip unit of `rows` output rows, taken
    8 at a time with the shared input rows carried in registers: every unit height
    gives the oracle's result, with ragged last units and any anchor."""
    import json
    f = tmp_path / "t.json"
    # (fit_units 0: small images keep the given height instead of shortening units)
    t = {"wave_rows": rows, "fit_units": 0}
    f.write_text(json.dumps({"u8": t, "u16": t}))
    morph.load_tuning(str(f))
    try:
        rng = np.random.default_rng(rows)
        for dtype in (np.uint8, np.uint16):
            for i, (H, W) in enumerate([(1, 1), (7, 300), (63, 65), (129, 257), (517, 1000)]):
                img = synth.uniform(H, W, dtype, seed=900 + i)
                assert morph.resolve_plan("u8" if dtype == np.uint8 else "u16", H, W, 3, 3)[
                    "tile_h"] == min(rows, (H + 7) // 8 * 8)
                for wx, wy in ((3, 3), (9, 9), (1, 5), (5, 1), (2, 8), (8, 2)):
                    ax = int(rng.integers(-1, wx))
                    ay = int(rng.integers(-1, wy))
                    for op in ("erode", "dilate"):
                        _check(img, op, wx, wy, ax, ay)
    finally:
        morph.load_tuning(None)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_streaming_kernel_every_window(dtype):
    """The streaming kernel (vertical vHGW through the per-wave ring, horizontal
    direct or doubling across lanes) for every horizontal window 1..128 (doubling
    forced, so small windows take it too) and vertical windows up to 256, random
    anchors, on an image of two strips and two row bands with ragged edges."""
    rng = np.random.default_rng(31)
    img = synth.document(181, 333, seed=41, n_rect=50).astype(dtype)
    if dtype == np.uint16:
        img = img * 257 - rng.integers(0, 200, img.shape).astype(np.uint16)
    for wx in range(1, 129):
        wy = int(rng.integers(1, 257))
        ax = int(rng.integers(-1, wx))
        ay = int(rng.integers(-1, wy))
        op = ("erode", "dilate")[wx % 2]
        _check(img, op, wx, wy, ax, ay, method_x="doubling")
        if wx <= 64:
            _check(img, op, wy, wx, ay, ax)  # automatic: wave or streaming kernel


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_wide_short_windows_on_the_wave_kernel(dtype):
    """Horizontal windows wider than the direct pass with a direct-size vertical
    window run the wave kernel's doubling pass: strips of stream_quads(wx) quads,
    ragged edges, any anchor, aligned and unaligned rows, both ops."""
    rng = np.random.default_rng(77)
    for i, (H, W) in enumerate([(5, 700), (61, 333), (130, 1000)]):
        img = synth.uniform(H, W, dtype, seed=1300 + i)
        for wx, wy in ((10, 1), (63, 1), (31, 3), (128, 9), (17, 2), (100, 5)):
            ax = int(rng.integers(-1, wx))
            ay = int(rng.integers(-1, wy))
            assert morph.resolve_plan("u8" if dtype == np.uint8 else "u16", H, W, wx, wy)[
                "kernel"] == "wave"
            for op in ("erode", "dilate"):
                _check(img, op, wx, wy, ax, ay)
        d, _ = to_dev(img, pitch_elems=W + 5, offset_elems=3)
        out = empty_like_dev(d)[0]
        morph.apply("dilate", d, 45, 7, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out), _ref(img, "dilate", 45, 7))


@pytest.mark.parametrize("dtype,rows", [(np.uint8, 1), (np.uint8, 3), (np.uint8, 16),
                                        (np.uint8, 64), (np.uint16, 1), (np.uint16, 5),
                                        (np.uint16, 16)])
def test_wide_row_kernel(dtype, rows, tmp_path):
    """Rows with a vertical window of 1 and a horizontal window of 129 .. 1000 run the
    wide-row kernel (16 pixels a lane, doubling across lanes): windows on both sides
    of every power of two up to 512 and the largest, any anchor, images narrower than
    a strip and several strips wide with a ragged right edge, units of `rows` rows
    (shorter and longer than a row group: 4 for uint8, 2 for uint16), aligned and
    unaligned rows."""
    import json
    dn = "u8" if dtype == np.uint8 else "u16"
    f = tmp_path / "t.json"
    f.write_text(json.dumps({dn: {"wide_rows": rows}}))
    morph.load_tuning(str(f))
    try:
        rng = np.random.default_rng(500 + rows)
        for i, (H, W) in enumerate([(1, 130), (3, 1023), (37, 1500), (9, 4097), (6, 200)]):
            img = synth.uniform(H, W, dtype, seed=1400 + i)
            for wx in (129, 130, 200, 255, 256, 257, 383, 511, 512, 777, 1000):
                ax = int(rng.integers(-1, wx))
                if W >= wx:  # (a window clipped to a narrow image may take another kernel)
                    assert morph.resolve_plan(dn, H, W, wx, 1)["kernel"] == "rows"
                for op in ("erode", "dilate"):
                    _check(img, op, wx, 1, ax, -1)
            pitch = W + 3
            d, _ = to_dev(img, pitch_elems=pitch, offset_elems=1)
            out = empty_like_dev(d)[0]
            morph.apply("dilate", d, 300, 1, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(out), _ref(img, "dilate", 300, 1))
            d, _ = to_dev(img, pitch_elems=W + 8, offset_elems=2)
            out = empty_like_dev(d)[0]
            morph.apply("erode", d, 641, 1, out=out, method_x="doubling")
            torch.cuda.synchronize()
            assert np.array_equal(to_host(out), _ref(img, "erode", 641, 1))
    finally:
        morph.load_tuning(None)


@pytest.mark.parametrize("rows", [1, 5, 16, 40])
def test_streaming_units_of_any_height(rows, tmp_path):
    """Streaming units of `rows` output rows, shorter and longer than the vertical
    window (the vHGW blocks then span several units or one unit holds several
    blocks), in both vertical forms (LDS ring for wy <= 16, run totals above), for
    both element types, aligned and unaligned rows, and images a fraction of a strip
    wide."""
    import json
    f = tmp_path / "t.json"
    t = {"stream_rows": rows, "stream_rows_runs": rows, "fit_units": 0}
    f.write_text(json.dumps({"u8": t, "u16": t}))
    morph.load_tuning(str(f))
    try:
        rng = np.random.default_rng(rows)
        for dtype in (np.uint8, np.uint16):
            for i, (H, W) in enumerate([(1, 1), (3, 70), (64, 65), (97, 500)]):
                img = synth.uniform(H, W, dtype, seed=950 + i)
                for wx, wy in ((15, 15), (31, 3), (4, 63), (64, 64), (2, 17), (40, 120)):
                    ax = int(rng.integers(-1, wx))
                    ay = int(rng.integers(-1, wy))
                    for op in ("erode", "dilate"):
                        _check(img, op, wx, wy, ax, ay)
                # unaligned rows and a source that is not quad-aligned
                pitch = W + 3
                d, _ = to_dev(img, pitch_elems=pitch, offset_elems=1)
                out = empty_like_dev(d)[0]
                morph.apply("erode", d, 33, 21, out=out)
                torch.cuda.synchronize()
                assert np.array_equal(to_host(out), _ref(img, "erode", 33, 21))
    finally:
        morph.load_tuning(None)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_gradient(dtype):
    """Morphological gradient against the oracle: the one-pass form (wave kernel,
    aligned rows: every direct window pair, doubling horizontal windows, any anchor,
    ragged strips) and the composed form (unaligned rows, vertical windows over 9,
    wide rows, forced vHGW), on images from one pixel to several strips; bytes
    outside the image untouched."""
    rng = np.random.default_rng(88)
    dn = "u8" if dtype == np.uint8 else "u16"
    wins = [(1, 1), (3, 3), (2, 5), (9, 9), (5, 1), (1, 7), (4, 8), (31, 3), (128, 9),
            (15, 15), (63, 63), (300, 1), (1, 255)]
    for i, (H, W) in enumerate([(1, 1), (5, 7), (37, 300), (130, 517)]):
        img = synth.uniform(H, W, dtype, seed=1500 + i)
        for wx, wy in wins:
            ax = int(rng.integers(-1, wx))
            ay = int(rng.integers(-1, wy))
            want = oracle.gradient(img, wx, wy, ax, ay)
            for pitch, off in ((W + (-W) % 4, 0), (W + 3, 1)):
                d, _ = to_dev(img, pitch_elems=pitch, offset_elems=off)
                out, obuf = empty_like_dev(d)
                morph.gradient(d, wx, wy, ax, ay, out=out)
                torch.cuda.synchronize()
                got = to_host(out)
                if not np.array_equal(got, want):
                    bad = np.argwhere(got != want)
                    raise AssertionError("gradient %dx%d a=(%d,%d) %s pitch %d off %d: %d bad, "
                                         "first at %s" % (wx, wy, ax, ay, img.shape, pitch, off,
                                                          len(bad), bad[0]))
                # the padding between rows is untouched
                full = to_host(obuf)
                rows = full[off:off + H * pitch].reshape(H, pitch)
                assert (rows[:, W:] == (0x5a if dtype == np.uint8 else 0x5a5a)).all()
            if wy <= 9 and wx <= 128:  # the one-pass form on the aligned rows
                assert morph.resolve_plan(dn, H, W, wx, wy)["kernel"] == "wave"
    # forced vHGW: the composed form through the tile kernel
    img = synth.uniform(40, 90, dtype, seed=1600)
    d, _ = to_dev(img, pitch_elems=92)
    out = morph.gradient(d, 7, 5, method_x="vhgw", method_y="vhgw")
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out), oracle.gradient(img, 7, 5))


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_pitch_offset_and_guard_bytes(dtype):
    """Strided rows, a base pointer off by one element, and sentinel bytes around
    the image and in the pitch gap that must stay untouched."""
    img = synth.uniform(45, 61, dtype, seed=25)
    for pitch, off in ((61, 0), (64, 0), (67, 1), (80, 3), (61, 1)):
        src, _ = to_dev(img, pitch_elems=pitch, offset_elems=off)
        for wx, wy in ((3, 3), (9, 1), (1, 21), (33, 5)):
            for op in ("erode", "dilate"):
                out, buf = empty_like_dev(src)
                before = to_host(buf).copy()
                morph.apply(op, src, wx, wy, out=out)
                torch.cuda.synchronize()
                got = to_host(out)
                assert np.array_equal(got, _ref(img, op, wx, wy)), (pitch, off, wx, wy, op)
                after = to_host(buf)
                mask = np.ones(after.shape, bool)
                rows = off + np.arange(45)[:, None] * pitch + np.arange(61)[None, :]
                mask[rows.ravel()] = False
                assert np.array_equal(after[mask], before[mask]), "bytes outside the image changed"


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_open_close(dtype):
    img = synth.document(130, 170, seed=26, n_rect=30)
    if dtype == np.uint16:
        img = img.astype(np.uint16) * 257
    for w in (3, 5, 15, 31):
        for op, f in (("open", oracle.opening), ("close", oracle.closing)):
            got = _gpu(img, op, w, w)
            want = f(img, w, w, method="hybrid", thresholds=(16, 16), nthreads=8)
            assert np.array_equal(got, want), (op, w)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_tophat_blackhat(dtype):
    """Top-hat (image minus opening) and black-hat (closing minus image) against the
    oracle: small and large windows, off-centre anchors, aligned and unaligned rows."""
    img = synth.document(130, 170, seed=27, n_rect=30)
    if dtype == np.uint16:
        img = img.astype(np.uint16) * 257
    for (wx, wy, ax, ay) in ((3, 3, -1, -1), (5, 2, 0, 1), (15, 15, 3, 9), (31, 7, -1, 6)):
        for op, f in (("tophat", oracle.tophat), ("blackhat", oracle.blackhat)):
            want = f(img, wx, wy, ax, ay)
            assert np.array_equal(_gpu(img, op, wx, wy, ax, ay), want), (op, wx, wy)
            d, _ = to_dev(img, pitch_elems=173, offset_elems=1)
            out = morph.apply(op, d, wx, wy, ax, ay)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(out), want), (op, wx, wy, "unaligned")


def test_empty_images_and_errors():
    e = torch.empty((0, 5), dtype=torch.uint8, device="cuda")
    assert morph.erode(e, 3).shape == (0, 5)
    img = to_dev(synth.uniform(8, 8, np.uint8, seed=1))[0]
    with pytest.raises(morph.MorphError) as ei:
        morph.erode(img, 3, 3, ax=3)
    assert ei.value.status == -1
    with pytest.raises(morph.MorphError) as ei:
        morph.apply("erode", img, 3, 3, out=img)
    assert ei.value.status == -2


# ---------------- full benchmark sizes ----------------
def test_config_640x480_uniform():
    img = synth.uniform(480, 640, np.uint8, seed=1)
    for wx, wy in ((3, 3), (15, 15), (1, 31)):
        for op in ("erode", "dilate"):
            _check(img, op, wx, wy)


def test_config_1920x1080_document_sweep():
    img = synth.document(1080, 1920, seed=2)
    for w in (3, 5, 7, 9, 15, 21, 31, 45, 63):
        for op in ("erode", "dilate"):
            _check(img, op, w, w)  # wave kernel up to 9, streaming kernel beyond
            _check(img, op, w, w, method_x="vhgw", method_y="vhgw")  # tile kernel
            # direct: the wave kernel (tall form past 9) while both windows fit it,
            # the tile kernel's tap loops beyond
            _check(img, op, w, w, method_x="direct", method_y="direct")


@pytest.mark.parametrize("dtype,seed", [(np.uint8, 3), (np.uint16, 4)])
def test_config_4096_square_all_ops(dtype, seed):
    img = synth.uniform(4096, 4096, dtype, seed=seed)
    d, _ = to_dev(img)
    ws = None
    for wx, wy in ((101, 101), (1, 255), (255, 1), (7, 63)):
        for op in ("erode", "dilate", "open", "close"):
            out = morph.apply(op, d, wx, wy, workspace=ws)
            torch.cuda.synchronize()
            got = to_host(out)
            kw = dict(method="hybrid", thresholds=(16, 16), nthreads=8)
            want = oracle.apply(op, img, wx, wy, **kw)
            assert np.array_equal(got, want), (op, wx, wy, dtype)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_direct_windows_past_nine(dtype):
    """The direct passes past the short wave kernel: the tall wave kernel's vertical
    windows 10..31 and the horizontal direct windows 10..16 (both with every
    anchor class, on aligned and unaligned rows, with ragged strips and units), and
    the tile kernel's tap loops for windows past those (a tile forces it)."""
    img = synth.uniform(203, 517, dtype, seed=31)
    rng = np.random.default_rng(31)
    for wy in range(DMAX + 1, TALL + 1):
        wx = int(rng.choice([1, 3, 9, 12, 16, 40]))
        for ay in sorted({-1, 0, wy - 1}):
            for op in ("erode", "dilate"):
                mx = "direct" if wx <= XMAX else None
                plan = morph.resolve_plan("u8" if dtype == np.uint8 else "u16", 203, 517, wx, wy,
                                          method_x=mx, method_y="direct")
                assert plan["kernel"] == "wave", (wx, wy, plan)
                _check(img, op, wx, wy, -1, ay, method_x=mx, method_y="direct")
    for wx in range(DMAX + 1, XMAX + 1):
        for ax in sorted({-1, 0, wx - 1}):
            _check(img, "erode", wx, 3, ax, -1, method_x="direct")
            _check(img, "dilate", wx, 31, ax, -1, method_x="direct")  # streaming kernel
    # unaligned rows (odd pitch, odd offset)
    d, _ = to_dev(img, pitch_elems=517 + 1, offset_elems=1)
    for wx, wy in ((13, 17), (16, 31), (1, 11)):
        out = morph.apply("erode", d, wx, wy, method_x="direct", method_y="direct")
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out), _ref(img, "erode", wx, wy)), (wx, wy)
    # the tile kernel's direct tap loops, for windows past the compiled ones
    for wx, wy in ((10, 1), (1, 10), (23, 22), (40, 3), (3, 57), (70, 70)):
        for tile in ((64, 32), (128, 64)):
            _check(img, "dilate", wx, wy, -1, -1, method_x="direct", method_y="direct",
                   tile=tile)


def test_thresholds_route_windows_to_the_direct_passes():
    """With the thresholds raised, the automatic plan sends windows up to 16 (x) and
    31 (y) to the wave kernel's direct passes; results are unchanged."""
    img = synth.document(300, 700, seed=32, n_rect=80)
    t0 = morph.get_thresholds("u8")
    try:
        morph.set_thresholds("u8", 16, 31)
        for wx, wy in ((16, 31), (11, 15), (3, 19), (15, 1), (9, 27)):
            plan = morph.resolve_plan("u8", 300, 700, wx, wy)
            assert plan["kernel"] == "wave" and plan["method_y"] in ("direct", None), plan
            for op in ("erode", "dilate"):
                _check(img, op, wx, wy)
        # beyond the compiled windows the automatic plan takes the large-window passes
        morph.set_thresholds("u8", 40, 40)
        for wx, wy in ((17, 3), (3, 32), (31, 33)):
            assert morph.resolve_plan("u8", 300, 700, wx, wy)["kernel"] in ("stream", "stream_coop", "wave")
            _check(img, "erode", wx, wy)
    finally:
        morph.set_thresholds("u8", *t0)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_horizontal_vhgw_across_lanes(dtype):
    """The paper's vHGW along x run across the lanes of the wave kernel (vertical
    window direct) and of the streaming kernel (vertical vHGW), when a plan asks for
    vHGW without a tile: every horizontal window 1..128 against the oracle, with
    several anchors, both operations, aligned and unaligned rows and ragged strips."""
    img = synth.uniform(77, 1031, dtype, seed=51)
    dn = "u8" if dtype == np.uint8 else "u16"
    for wx in list(range(1, 40)) + [45, 63, 64, 65, 100, 101, 127, 128]:
        ax = (-1, 0, wx - 1)[wx % 3]
        for wy, my in ((1, None), (3, "direct"), (13, "vhgw")):
            k = morph.resolve_plan(dn, 77, 1031, wx, wy, method_x="vhgw", method_y=my)["kernel"]
            if wx > 1:  # (a window of 1 has no horizontal pass to run)
                assert k == ("wave" if my != "vhgw" else "stream"), (wx, wy, k)
            _check(img, "erode" if wx % 2 else "dilate", wx, wy, ax, -1, method_x="vhgw",
                   method_y=my)
    d, _ = to_dev(img, pitch_elems=1031 + 3, offset_elems=1)  # unaligned rows
    for wx in (5, 31, 128):
        out = morph.apply("dilate", d, wx, 5, method_x="vhgw", method_y="vhgw")
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out), _ref(img, "dilate", wx, 5)), wx


def test_automatic_horizontal_vhgw_by_tuning_table(tmp_path):
    """With "h_vhgw": 1 in the tuning table, single images' automatic large horizontal
    windows run the paper's vHGW across the lanes (the wave kernel's short form and the
    streaming kernel) and the tall wave form keeps doubling: plans and results against
    the oracle; batches keep doubling."""
    import json
    f = tmp_path / "t.json"
    f.write_text(json.dumps({"u8": {"h_vhgw": 1}, "u16": {"h_vhgw": 1}}))
    morph.load_tuning(str(f))
    try:
        for dtype in (np.uint8, np.uint16):
            dn = "u8" if dtype == np.uint8 else "u16"
            img = synth.uniform(150, 777, dtype, seed=52)
            for wx, wy, kernel, mx in ((33, 3, "wave", "vhgw"), (101, 1, "wave", "vhgw"),
                                       (45, 20, "wave", "doubling"), (63, 63, "stream", "vhgw"),
                                       (5, 5, "wave", "direct")):
                p = morph.resolve_plan(dn, 150, 777, wx, wy)
                assert (p["kernel"], p["method_x"]) == (kernel, mx), (dn, wx, wy, p)
                _check(img, "erode" if wx % 2 else "dilate", wx, wy)
                _check(img, "dilate", wx, wy, 0, -1)
            assert morph.resolve_plan(dn, 150, 777, 33, 3, batch=True)["method_x"] == "doubling"
    finally:
        morph.load_tuning(None)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_streaming_cooperative_form(dtype, tmp_path):
    """The streaming kernel's cooperative form (4 to 16 waves share a unit: run totals,
    their scans and the output runs side by side), routed by the tuning table from
    vertical window 17: every vertical window form it meets (several blocks a unit, a
    block longer than the unit, windows not a multiple of 8, windows larger than the
    image), units of 8 to 256 rows, horizontal windows none / direct / doubling,
    anchors at both ends, ragged images; against the oracle.  (Vertical windows past
    16 take vHGW here, so that 17..31 reach it too.)"""
    import json
    dn = "u8" if dtype == np.uint8 else "u16"
    f = tmp_path / "t.json"
    rng = np.random.default_rng(71)
    try:
        for rows, waves in ((8, 4), (64, 8), (256, 4), (96, 8), (192, 16)):
            f.write_text(json.dumps({dn: {"coop_min_wy": 17, "coop_rows": rows,
                                          "coop_waves": waves, "fit_units": 0, "t_y": 16}}))
            morph.load_tuning(str(f))
            for H, W in ((301, 776), (1000, 332), (40, 1032)):  # (rows aligned)
                img = synth.uniform(H, W, dtype, seed=H + W + rows)
                for wy in (17, 24, 31, 33, 64, 101, 200, 256):
                    wx = int(rng.choice([1, 3, 9, 15, 31, 101]))
                    p = morph.resolve_plan(dn, H, W, wx, wy)
                    # (uint16 units of 256 rows can need more than the form's 64 KB of
                    # LDS: those keep the streaming kernel)
                    if wy <= H and (dn == "u8" or rows <= 96):
                        assert p["kernel"] == "stream_coop", (H, W, wx, wy, p)
                    ay = int(rng.choice([-1, 0, wy - 1]))
                    _check(img, "erode" if wy % 2 else "dilate", wx, wy, -1, ay)
        # sources and destinations starting 1..3 pixels past a 4-pixel boundary (row
        # pitch still aligned, so the form is taken), at the table's shape
        morph.load_tuning(None)
        H, W = 150, 520
        for off in (1, 2, 3):
            img = synth.uniform(H, W, dtype, seed=80 + off)
            d, _ = to_dev(img, pitch_elems=W + 4 * off, offset_elems=off)
            for wx, wy, ax in ((1, 101, -1), (31, 63, 0), (9, 40, 8), (101, 101, -1)):
                assert morph.resolve_plan(dn, H, W, wx, wy)["kernel"] == "stream_coop"
                out = empty_like_dev(d)[0]
                morph.apply("dilate", d, wx, wy, ax, -1, out=out)
                torch.cuda.synchronize()
                assert np.array_equal(to_host(out), _ref(img, "dilate", wx, wy, ax, -1)), (
                    off, wx, wy)
    finally:
        morph.load_tuning(None)
