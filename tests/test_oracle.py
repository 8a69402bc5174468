"""Pins for the CPU oracle: values fixed by the paper's definition (§2, Eq. (1))
worked by hand, a library routine (scipy.ndimage) on the cases it covers,
closed forms, and invariants of erosion/dilation.  None of these re-types the
oracle's own code; each would fail on a dropped term, a wrong sign or index, a
swapped axis or a wrong border."""
import itertools
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle import npref
from paper_2002_09474_amd import synth

METHODS = ("brute2d", "direct", "vhgw", "hybrid")
OPN = {"erode": oracle.ERODE, "dilate": oracle.DILATE}
ROW = np.array([5, 3, 8, 1, 9, 2, 7], dtype=np.uint8)


def _read_row_cases(golden_dir):
    cases = []
    for ln in open(os.path.join(golden_dir, "row_1d.txt")):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        lhs, rhs = ln.split(":")
        op, w, a = lhs.split()
        cases.append((op, int(w), int(a), [int(v) for v in rhs.split()]))
    return cases


def test_default_anchor_matches_eq1():
    # Eq. (1): D(x) = op S(x - n + w/2), n in [0, w-1] (integer w/2): window [x-(w-1)+w//2, x+w//2]
    for w in range(1, 40):
        a = oracle.default_anchor(w)
        assert x_window(w, a) == (-(w - 1) + w // 2, w // 2)
    assert [oracle.default_anchor(w) for w in (1, 2, 3, 4, 5)] == [0, 0, 1, 1, 2]


def x_window(w, a):
    return (-a, -a + w - 1)


def test_golden_row_all_methods(golden_dir):
    cases = _read_row_cases(golden_dir)
    assert len(cases) >= 10
    for op, w, a, want in cases:
        want = np.array(want, dtype=np.uint8)
        for m in ("direct", "vhgw"):
            got = oracle.line(ROW, w, a, OPN[op], method=m)
            assert np.array_equal(got, want), (op, w, a, m, got)
        img = ROW[None, :]
        for m in METHODS:
            got = oracle.morph(img, OPN[op], w, 1, a, 0, method=m)[0]
            assert np.array_equal(got, want), (op, w, a, m, got)
            # the same row as a column exercises the y pass
            got = oracle.morph(img.T.copy(), OPN[op], 1, w, 0, a, method=m)[:, 0]
            assert np.array_equal(got, want), (op, w, a, m, "col", got)


def test_golden_vhgw_trace(golden_dir):
    vals = {}
    for ln in open(os.path.join(golden_dir, "vhgw_trace.txt")):
        if ln.startswith("#") or ":" not in ln:
            continue
        k, v = ln.split(":")
        vals[k.strip()] = [int(t) for t in v.split()]
    got = oracle.line(ROW, 3, 1, oracle.ERODE, method="vhgw")
    assert got.tolist() == vals["out"]
    # the trace is internally consistent with out[x] = min(h[x], g[x+w-1])
    g, h = vals["g"], vals["h"]
    assert [min(h[x], g[x + 2]) for x in range(7)] == vals["out"]


def _read_image_cases(golden_dir):
    lines = [ln.strip() for ln in open(os.path.join(golden_dir, "image_5x5.txt"))
             if ln.strip() and not ln.startswith("#")]
    i = lines.index("input")
    img = np.array([[int(v) for v in lines[i + 1 + r].split()] for r in range(5)], np.uint8)
    cases = []
    j = i + 6
    while j < len(lines):
        _, op, wx, wy = lines[j].split()
        want = np.array([[int(v) for v in lines[j + 1 + r].split()] for r in range(5)], np.uint8)
        cases.append((op, int(wx), int(wy), want))
        j += 6
    return img, cases


def test_golden_image_5x5(golden_dir):
    img, cases = _read_image_cases(golden_dir)
    assert len(cases) == 3
    for op, wx, wy, want in cases:
        for m in METHODS:
            got = oracle.morph(img, OPN[op], wx, wy, method=m)
            assert np.array_equal(got, want), (op, wx, wy, m, got)
        # transposing the image swaps the roles of wx and wy (and keeps anchors)
        got = oracle.morph(img.T.copy(), OPN[op], wy, wx, method="direct").T
        assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_scipy_cross_check_all_anchors(dtype):
    """scipy's rank filters with a constant border of the identity and the
    origin shifted so its window is [x - a, x - a + w - 1]."""
    rng = np.random.default_rng(11)
    maxv = np.iinfo(dtype).max
    for trial in range(40):
        H, W = int(rng.integers(1, 14)), int(rng.integers(1, 14))
        img = rng.integers(0, maxv + 1, size=(H, W), dtype=dtype)
        wx, wy = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        ax, ay = int(rng.integers(0, wx)), int(rng.integers(0, wy))
        origin = (ay - wy // 2, ax - wx // 2)
        ref_e = ndimage.minimum_filter(img, size=(wy, wx), mode="constant", cval=maxv,
                                       origin=origin)
        ref_d = ndimage.maximum_filter(img, size=(wy, wx), mode="constant", cval=0,
                                       origin=origin)
        for m in METHODS:
            assert np.array_equal(oracle.erode(img, wx, wy, ax, ay, method=m), ref_e), (trial, m)
            assert np.array_equal(oracle.dilate(img, wx, wy, ax, ay, method=m), ref_d), (trial, m)


def test_numpy_statement_cross_check():
    rng = np.random.default_rng(3)
    for trial in range(30):
        H, W = int(rng.integers(1, 10)), int(rng.integers(1, 10))
        img = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        wx, wy = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        ax, ay = int(rng.integers(-1, wx)), int(rng.integers(-1, wy))
        for op in (0, 1):
            ref = npref.morph(img, op, wx, wy, ax, ay)
            assert np.array_equal(oracle.morph(img, op, wx, wy, ax, ay, method="brute2d"), ref)


def test_vhgw_equals_brute_force_every_window_and_anchor():
    rng = np.random.default_rng(7)
    for n in (1, 2, 5, 17, 64, 131):
        x8 = rng.integers(0, 256, size=n, dtype=np.uint8)
        x16 = rng.integers(0, 65536, size=n, dtype=np.uint16)
        for w in range(1, 65):
            for a in range(w):
                for x in (x8, x16):
                    for op in (0, 1):
                        d = oracle.line(x, w, a, op, method="direct")
                        v = oracle.line(x, w, a, op, method="vhgw")
                        assert np.array_equal(d, v), (n, w, a, op)


def test_vhgw_2d_against_definition_large_windows():
    img = synth.uniform(37, 53, np.uint8, seed=9)
    for wx, wy in ((64, 1), (1, 64), (33, 20), (70, 75), (105, 3)):
        for op in (0, 1):
            ref = oracle.morph(img, op, wx, wy, method="brute2d")
            assert np.array_equal(oracle.morph(img, op, wx, wy, method="vhgw"), ref)
            assert np.array_equal(oracle.morph(img, op, wx, wy, method="direct"), ref)


def test_identity_window():
    img = synth.uniform(9, 11, np.uint16, seed=1)
    for m in METHODS:
        assert np.array_equal(oracle.erode(img, 1, 1, method=m), img)
        assert np.array_equal(oracle.dilate(img, 1, 1, method=m), img)


def test_window_covering_image_gives_global_extremum():
    img = synth.uniform(13, 17, np.uint8, seed=2)
    for m in METHODS:
        e = oracle.erode(img, 2 * 17 - 1, 2 * 13 - 1, method=m)
        d = oracle.dilate(img, 2 * 17 - 1, 2 * 13 - 1, method=m)
        assert (e == img.min()).all() and (d == img.max()).all()


def test_constant_image_unchanged():
    img = np.full((8, 12), 77, np.uint8)
    for m in METHODS:
        for w in (2, 5, 30):
            assert np.array_equal(oracle.erode(img, w, w + 1, method=m), img)
            assert np.array_equal(oracle.dilate(img, w + 1, w, method=m), img)


def test_checkerboard_closed_form():
    # 0/255 checkerboard, wx=2, wy=1, ax=0: window {x, x+1} holds both colours
    # except in the last column, whose clipped window is the pixel itself.
    H, W = 6, 9
    img = (((np.arange(H)[:, None] + np.arange(W)[None, :]) % 2) * 255).astype(np.uint8)
    for m in METHODS:
        e = oracle.erode(img, 2, 1, 0, 0, method=m)
        d = oracle.dilate(img, 2, 1, 0, 0, method=m)
        assert (e[:, :-1] == 0).all() and (d[:, :-1] == 255).all()
        assert np.array_equal(e[:, -1], img[:, -1]) and np.array_equal(d[:, -1], img[:, -1])


def test_duality():
    for dtype in (np.uint8, np.uint16):
        maxv = np.iinfo(dtype).max
        img = synth.uniform(21, 19, dtype, seed=4)
        for wx, wy, ax, ay in ((3, 3, -1, -1), (4, 7, 0, 6), (11, 2, 10, 1)):
            d = oracle.dilate(img, wx, wy, ax, ay, method="vhgw")
            e = oracle.erode((maxv - img).astype(dtype), wx, wy, ax, ay, method="direct")
            assert np.array_equal(d, (maxv - e).astype(dtype))


def test_separable_order_and_2d():
    img = synth.document(40, 50, seed=5, n_rect=12)
    for wx, wy in ((5, 9), (12, 3), (1, 17)):
        for op in (0, 1):
            hv = oracle.morph(oracle.morph(img, op, wx, 1, method="direct"), op, 1, wy, method="direct")
            vh = oracle.morph(oracle.morph(img, op, 1, wy, method="direct"), op, wx, 1, method="direct")
            ref = oracle.morph(img, op, wx, wy, method="brute2d")
            assert np.array_equal(hv, ref) and np.array_equal(vh, ref)


def test_erosion_below_image_below_dilation_and_monotone():
    rng = np.random.default_rng(8)
    img = synth.uniform(25, 31, np.uint8, seed=8)
    bump = rng.integers(0, 2, size=img.shape).astype(np.uint8)
    img2 = np.minimum(img.astype(np.int32) + bump * 40, 255).astype(np.uint8)
    for wx, wy, ax, ay in ((3, 5, -1, -1), (6, 6, 0, 5), (9, 1, 4, 0)):
        e = oracle.erode(img, wx, wy, ax, ay, method="vhgw")
        d = oracle.dilate(img, wx, wy, ax, ay, method="vhgw")
        assert (e <= img).all() and (img <= d).all()
        assert (e <= oracle.erode(img2, wx, wy, ax, ay, method="vhgw")).all()
        assert (d <= oracle.dilate(img2, wx, wy, ax, ay, method="vhgw")).all()


def test_decomposition_along_one_axis():
    # erosion by w1 then by w2 (anchors a1, a2) = erosion by w1+w2-1 with anchor a1+a2
    img = synth.uniform(15, 40, np.uint8, seed=12)
    for (w1, a1), (w2, a2) in itertools.product(((3, 1), (4, 0), (7, 6)), ((3, 1), (2, 1), (5, 0))):
        two = oracle.erode(oracle.erode(img, w1, 1, a1, 0, method="direct"), w2, 1, a2, 0, method="direct")
        one = oracle.erode(img, w1 + w2 - 1, 1, a1 + a2, 0, method="brute2d")
        assert np.array_equal(two, one), (w1, a1, w2, a2)


def test_open_close_properties():
    img = synth.document(48, 64, seed=13, n_rect=20)
    for w in (3, 5, 9):
        o = oracle.opening(img, w, w, method="vhgw")
        c = oracle.closing(img, w, w, method="vhgw")
        assert (o <= img).all() and (img <= c).all()
        assert np.array_equal(oracle.opening(o, w, w, method="direct"), o)
        assert np.array_equal(oracle.closing(c, w, w, method="direct"), c)


def _gradient_by_hand(img, wx, wy, ax, ay):
    """max - min over the window clipped to the image, pixel by pixel (pure Python;
    the definition of the gradient written out, not the oracle's code)."""
    H, W = img.shape
    out = np.zeros_like(img)
    for y in range(H):
        for x in range(W):
            vals = [int(img[yy, xx])
                    for yy in range(max(0, y - ay), min(H, y - ay + wy))
                    for xx in range(max(0, x - ax), min(W, x - ax + wx))]
            out[y, x] = max(vals) - min(vals)
    return out


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_gradient_pins(dtype):
    """The morphological gradient (dilation minus erosion, §2) against its
    definition by brute force on tiny images for every anchor, a step edge in closed
    form, and its invariants: zero on a constant image and for a 1x1 window,
    unchanged by taking the complement."""
    rng = np.random.default_rng(41)
    maxv = np.iinfo(dtype).max
    for H, W in ((1, 1), (3, 5), (6, 4)):
        img = rng.integers(0, maxv + 1, size=(H, W)).astype(dtype)
        for wx, wy in ((1, 1), (2, 3), (3, 2), (5, 4)):
            for ax, ay in itertools.product(range(wx), range(wy)):
                want = _gradient_by_hand(img, wx, wy, ax, ay)
                for m in ("direct", "vhgw"):
                    assert np.array_equal(oracle.gradient(img, wx, wy, ax, ay, method=m), want)
    # step edge: 0 left of column 10, v from it on; a w x 1 window straddles the edge
    # exactly at columns 10 - (w - 1 - a) .. 9 + a
    v = 200 if dtype == np.uint8 else 50000
    img = np.zeros((3, 24), dtype)
    img[:, 10:] = v
    for w, a in ((5, 2), (4, 0), (7, 6)):
        want = np.zeros_like(img)
        want[:, 10 - (w - 1 - a):10 + a] = v
        assert np.array_equal(oracle.gradient(img, w, 1, a, 0), want), (w, a)
    img = synth.uniform(20, 30, dtype, seed=7)
    assert not oracle.gradient(img, 1, 1).any()
    assert not oracle.gradient(np.full((9, 11), 77, dtype), 5, 3).any()
    g = oracle.gradient(img, 7, 3, method="vhgw")
    assert np.array_equal(oracle.gradient((maxv - img).astype(dtype), 7, 3), g)


def _extremum_by_hand(img, wx, wy, ax, ay, use_max):
    """Erosion (min) or dilation (max) over the clipped window, by pure Python loops."""
    H, W = img.shape
    out = np.zeros_like(img)
    f = max if use_max else min
    for y in range(H):
        for x in range(W):
            out[y, x] = f(int(img[yy, xx])
                          for yy in range(max(0, y - ay), min(H, y - ay + wy))
                          for xx in range(max(0, x - ax), min(W, x - ax + wx)))
    return out


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_tophat_blackhat_pins(dtype):
    """Top-hat (image minus opening) and black-hat (closing minus image), clamped at
    0, against openings and closings formed by hand on tiny images for every anchor
    (the differences are never negative for a centred anchor, and can be otherwise);
    a lone bright pixel, which an opening removes, is exactly the top-hat, and a lone
    dark pixel, which a closing fills, exactly the black-hat; each the other's mirror
    under the complement."""
    rng = np.random.default_rng(43)
    maxv = np.iinfo(dtype).max
    for H, W in ((1, 1), (4, 5), (6, 3)):
        img = rng.integers(0, maxv + 1, size=(H, W)).astype(dtype)
        for wx, wy in ((1, 1), (2, 3), (3, 2), (3, 3)):
            for ax, ay in itertools.product(range(wx), range(wy)):
                e = _extremum_by_hand(img, wx, wy, ax, ay, False)
                o = _extremum_by_hand(e, wx, wy, ax, ay, True)
                d = _extremum_by_hand(img, wx, wy, ax, ay, True)
                c = _extremum_by_hand(d, wx, wy, ax, ay, False)
                t = img.astype(np.int64) - o
                b = c.astype(np.int64) - img
                # the centred anchor keeps opening <= image <= closing
                if 2 * ax == wx - 1 and 2 * ay == wy - 1:
                    assert (t >= 0).all() and (b >= 0).all()
                assert np.array_equal(oracle.tophat(img, wx, wy, ax, ay),
                                      np.maximum(t, 0).astype(dtype))
                assert np.array_equal(oracle.blackhat(img, wx, wy, ax, ay),
                                      np.maximum(b, 0).astype(dtype))
    v = 180 if dtype == np.uint8 else 40000
    img = np.full((9, 9), 10, dtype)
    img[4, 4] = v
    want = np.zeros_like(img)
    want[4, 4] = v - 10
    assert np.array_equal(oracle.tophat(img, 3, 3), want)
    assert not oracle.blackhat(img, 3, 3).any()  # a closing keeps a lone peak as it is
    dark = np.full((9, 9), v, dtype)
    dark[4, 4] = 10
    want = np.zeros_like(dark)
    want[4, 4] = v - 10
    assert np.array_equal(oracle.blackhat(dark, 3, 3), want)
    img = synth.uniform(25, 31, dtype, seed=9)
    t = oracle.tophat(img, 5, 3)
    b = oracle.blackhat(img, 5, 3)
    assert np.array_equal(oracle.blackhat((maxv - img).astype(dtype), 5, 3), t)
    assert np.array_equal(oracle.tophat((maxv - img).astype(dtype), 5, 3), b)


def test_u8_u16_consistency_scaled_by_257():
    img = synth.uniform(19, 23, np.uint8, seed=14)
    img16 = img.astype(np.uint16) * 257
    for wx, wy in ((3, 3), (8, 5)):
        for op in (0, 1):
            a = oracle.morph(img, op, wx, wy, method="vhgw").astype(np.uint16) * 257
            b = oracle.morph(img16, op, wx, wy, method="vhgw")
            assert np.array_equal(a, b)


def test_hybrid_threads_and_thresholds():
    img = synth.uniform(64, 77, np.uint8, seed=15)
    ref = oracle.erode(img, 9, 21, method="direct")
    for t in ((1, 1), (9, 9), (100, 3), (3, 100)):
        for nt in (1, 4):
            assert np.array_equal(oracle.erode(img, 9, 21, method="hybrid", thresholds=t,
                                               nthreads=nt), ref)


def test_oracle_rejects_bad_arguments():
    img = np.zeros((4, 4), np.uint8)
    for bad in (dict(wx=0, wy=1), dict(wx=3, wy=3, ax=3), dict(wx=3, wy=2, ay=-2)):
        with pytest.raises(ValueError):
            oracle.erode(img, bad["wx"], bad["wy"], bad.get("ax", -1), bad.get("ay", -1))
    assert oracle.erode(np.zeros((0, 5), np.uint8), 3, 3).shape == (0, 5)


def test_synthetic_inputs_are_seeded():
    a = synth.document(64, 80, seed=3)
    b = synth.document(64, 80, seed=3)
    assert np.array_equal(a, b) and a.dtype == np.uint8
    assert (a > 128).mean() > 0.5  # white page
    s1 = synth.batch_specs(16, seed=5)
    s2 = synth.batch_specs(16, seed=5)
    assert s1 == s2
    assert all(64 <= s["H"] <= 2048 and 64 <= s["W"] <= 2048 for s in s1)
    assert all(s["w"] in synth.BATCH_WINDOWS for s in s1)
    reqs = synth.request_stream(100.0, 2.0, seed=6)
    assert all(r["w"] % 2 == 1 and 3 <= r["w"] <= 101 for r in reqs)
    assert all(r["y"] + r["H"] <= 4096 and r["x"] + r["W"] <= 4096 for r in reqs)
