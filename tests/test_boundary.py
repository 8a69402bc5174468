"""The C-ABI boundary without a GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before anything touches the device
(validation runs first, so fake pointers never reach HIP)."""
import ctypes
import json
import os
import re

import pytest

from paper_2002_09474_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "morph.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(morph_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_exports():
    assert _declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_symbol():
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name


FAKE_SRC = 0x10000
FAKE_DST = 0x20000000


def _erode(src=FAKE_SRC, dst=FAKE_DST, H=8, W=8, pitch=8, wx=3, wy=3, ax=-1, ay=-1, border=0):
    return _lib.lib().morph_erode(src, dst, H, W, pitch, wx, wy, ax, ay, border, None)


def test_validation_errors():
    E = _lib
    assert _erode(H=-1) == E.MORPH_EINVAL
    assert _erode(W=-3) == E.MORPH_EINVAL
    assert _erode(wx=0) == E.MORPH_EINVAL
    assert _erode(wy=0) == E.MORPH_EINVAL
    assert _erode(ax=3) == E.MORPH_EINVAL
    assert _erode(ay=-2) == E.MORPH_EINVAL
    assert _erode(pitch=7) == E.MORPH_EINVAL
    assert _erode(src=0) == E.MORPH_EINVAL
    assert _erode(border=1) == E.MORPH_EUNSUPPORTED
    assert _erode(dst=FAKE_SRC + 7 * 8) == E.MORPH_EALIAS      # last row overlaps
    assert _erode(H=0, src=0, dst=0) == E.MORPH_OK              # empty image: no-op
    assert _erode(W=0) == E.MORPH_OK
    L = _lib.lib()
    # uint16 rows must be 2-byte aligned, pitch a multiple of 2
    assert L.morph_erode_u16(FAKE_SRC + 1, FAKE_DST, 8, 8, 16, 3, 3, -1, -1, 0, None) == E.MORPH_EINVAL
    assert L.morph_dilate_u16(FAKE_SRC, FAKE_DST, 8, 8, 17, 3, 3, -1, -1, 0, None) == E.MORPH_EINVAL
    assert L.morph_dilate_u16(FAKE_SRC, FAKE_DST, 8, 8, 15, 3, 3, -1, -1, 0, None) == E.MORPH_EINVAL
    # bad op / dtype through the general entry
    assert L.morph_apply(7, 0, FAKE_SRC, FAKE_DST, 8, 8, 8, 3, 3, -1, -1, 0, None, None, 0,
                         None) == E.MORPH_EINVAL
    assert L.morph_apply(0, 5, FAKE_SRC, FAKE_DST, 8, 8, 8, 3, 3, -1, -1, 0, None, None, 0,
                         None) == E.MORPH_EUNSUPPORTED


def test_open_close_workspace_checks():
    L = _lib.lib()
    E = _lib
    assert L.morph_workspace_bytes(8, 8, 8, 1) == 64
    assert L.morph_workspace_bytes(0, 8, 8, 1) == 0
    ws = 0x40000000
    # (rows of unaligned pitch, 9 bytes for uint8 and 18 for uint16: the one-pass form
    # does not apply, the two launches need the workspace)
    assert L.morph_open(FAKE_SRC, FAKE_DST, 8, 8, 9, 3, 3, -1, -1, 0, None, 0, None) == E.MORPH_ENOMEM
    assert L.morph_close(FAKE_SRC, FAKE_DST, 8, 8, 9, 3, 3, -1, -1, 0, ws, 71, None) == E.MORPH_ENOMEM
    assert L.morph_open(FAKE_SRC, FAKE_DST, 8, 8, 9, 3, 3, -1, -1, 0, FAKE_SRC + 8, 72,
                        None) == E.MORPH_EALIAS
    assert L.morph_close_u16(FAKE_SRC, FAKE_DST, 8, 8, 18, 3, 3, -1, -1, 0, FAKE_DST - 16, 144,
                             None) == E.MORPH_EALIAS
    # (nor a vertical window over 15)
    assert L.morph_open(FAKE_SRC, FAKE_DST, 64, 8, 8, 3, 17, -1, -1, 0, None, 0,
                        None) == E.MORPH_ENOMEM
    # the gradient needs the workspace where its one-pass form does not apply: a
    # vertical window over 9 (the streaming kernel) or rows of unaligned pitch
    assert L.morph_gradient(FAKE_SRC, FAKE_DST, 8, 8, 8, 3, 15, -1, -1, 0, None, 0,
                            None) == E.MORPH_ENOMEM
    assert L.morph_gradient(FAKE_SRC, FAKE_DST, 8, 7, 7, 3, 3, -1, -1, 0, ws, 55,
                            None) == E.MORPH_ENOMEM
    assert L.morph_gradient_u16(FAKE_SRC, FAKE_DST, 8, 8, 16, 31, 31, -1, -1, 0, FAKE_SRC + 8,
                                128, None) == E.MORPH_EALIAS
    assert L.morph_apply(7, 0, FAKE_SRC, FAKE_DST, 8, 8, 8, 3, 3, -1, -1, 0, None, None, 0,
                         None) == E.MORPH_EINVAL
    # top-hat and black-hat need it where their opening or closing does
    assert L.morph_tophat(FAKE_SRC, FAKE_DST, 8, 8, 9, 3, 3, -1, -1, 0, None, 0,
                          None) == E.MORPH_ENOMEM
    assert L.morph_blackhat_u16(FAKE_SRC, FAKE_DST, 8, 8, 18, 3, 3, -1, -1, 0, FAKE_DST, 144,
                                None) == E.MORPH_EALIAS


def test_openclose_fused_argument_checks():
    """The single-pass opening/closing rejects bad arguments before any launch:
    windows above 16 per axis where the one-pass form does not apply (here rows of
    unaligned pitch), bad dtype, anchors, pitch, overlap, border."""
    L = _lib.lib()
    E = _lib

    def oc(dtype=0, opening=1, src=FAKE_SRC, dst=FAKE_DST, H=8, W=8, pitch=8, wx=3, wy=3,
           ax=-1, ay=-1, border=0):
        return L.morph_openclose_fused(dtype, opening, src, dst, H, W, pitch, wx, wy, ax, ay,
                                       border, None)

    assert oc(wx=17, pitch=9) == E.MORPH_EUNSUPPORTED
    assert oc(wy=17, opening=0, pitch=9) == E.MORPH_EUNSUPPORTED
    assert oc(H=64, wy=17, pitch=8) == E.MORPH_EUNSUPPORTED  # (wy over 15 and over 16)
    assert oc(dtype=5) == E.MORPH_EUNSUPPORTED
    assert oc(border=1) == E.MORPH_EUNSUPPORTED
    assert oc(ax=3) == E.MORPH_EINVAL
    assert oc(wx=0) == E.MORPH_EINVAL
    assert oc(pitch=7) == E.MORPH_EINVAL
    assert oc(dtype=1, pitch=15) == E.MORPH_EINVAL
    assert oc(dst=FAKE_SRC + 7 * 8) == E.MORPH_EALIAS
    assert oc(H=0, src=0, dst=0) == E.MORPH_OK


def test_forced_direct_plans_past_the_compiled_windows():
    import paper_2002_09474_amd as morph
    # the wave kernel's direct passes: horizontal up to 16, vertical up to 31 (its
    # tall form past 9); beyond them the tile kernel's tap loops
    p = morph.resolve_plan("u8", 64, 64, 16, 31, method_x="direct", method_y="direct")
    # (a 64-pixel row is one strip of its 16 quads: at most stream_quads(16) = 59)
    assert (p["kernel"], p["method_x"], p["method_y"], p["tile_w"]) == ("wave", "direct",
                                                                       "direct", 64)
    p = morph.resolve_plan("u8", 64, 64, 17, 1, method_x="direct")
    assert (p["kernel"], p["method_x"]) == ("tile", "direct")
    p = morph.resolve_plan("u16", 64, 64, 3, 32, method_y="direct")
    assert (p["kernel"], p["method_y"]) == ("tile", "direct")
    p = morph.resolve_plan("u8", 64, 64, 200, 200, method_x="direct", method_y="direct")
    assert (p["kernel"], p["method_x"], p["method_y"]) == ("tile", "direct", "direct")
    p = _lib.Plan(0, 0, 6, 0)  # tile width must be a multiple of 4
    rc = _lib.lib().morph_apply(0, 0, FAKE_SRC, FAKE_DST, 64, 64, 64, 3, 3, -1, -1, 0,
                                ctypes.byref(p), None, 0, None)
    assert rc == _lib.MORPH_EINVAL


# A fixed table for the plan checks below (the shipped one is the autotuner's
# measurement and may change): unit heights and thresholds of its own.
PLAN_TABLE = {"t_x": 9, "t_y": 9, "wave_rows": 24, "stream_rows": 48, "stream_rows_runs": 32,
              "wide_rows": 4, "batch_wave_rows": 32, "batch_stream_rows": 48,
              "batch_stream_rows_runs": 48, "batch_t_x": 9, "batch_t_y": 9, "coop_min_wy": 0,
              "tiles": [{"wmax": 9, "tq": 32, "tb": 64}, {"wmax": 16, "tq": 32, "tb": 64},
                        {"wmax": 64, "tq": 48, "tb": 64}, {"wmax": 1 << 30, "tq": 64, "tb": 64}]}


def test_plan_resolution_and_thresholds(tmp_path):
    import json
    import paper_2002_09474_amd as morph
    f0 = tmp_path / "plan_table.json"
    f0.write_text(json.dumps({"u8": PLAN_TABLE, "u16": PLAN_TABLE}))
    morph.load_tuning(str(f0))
    t0 = morph.get_thresholds("u8")
    try:
        morph.set_thresholds("u8", 9, 7)
        assert morph.get_thresholds("u8") == (9, 7)
        p = morph.resolve_plan("u8", 1080, 1920, 9, 9)
        assert p["method_x"] == "direct" and p["method_y"] == "vhgw"
        p = morph.resolve_plan("u8", 1080, 1920, 7, 7)
        assert p["method_x"] == "direct" and p["method_y"] == "direct"
        # both passes direct: one wave per strip of stream_quads(7) = 61 quads x 24
        # rows, on an image with enough units (17 strips x 171 units) to fill the GPU
        p = morph.resolve_plan("u8", 4096, 4096, 7, 7)
        assert (p["tile_w"], p["tile_h"], p["kernel"]) == (4 * 61, 24, "wave")
        # a smaller single image takes shorter units, until it has about 2048 of them
        # (in steps of 8 rows, no fewer than 8): 1080 x 1920 has 8 strips, so
        # ceil(1080 * 8 / 2048) = 5 rows -> 8
        assert morph.resolve_plan("u8", 1080, 1920, 7, 7)["tile_h"] == 8
        assert morph.resolve_plan("u8", 3000, 1920, 7, 7)["tile_h"] == 16
        # a window of 1 skips the pass
        assert morph.resolve_plan("u8", 100, 100, 1, 31)["method_x"] is None
        # larger windows: the streaming kernel (vertical vHGW, horizontal doubling)
        # up to 128 x 256, the tile kernel beyond
        p = morph.resolve_plan("u8", 1080, 1920, 31, 31)
        assert (p["method_x"], p["method_y"], p["kernel"]) == ("doubling", "vhgw", "stream")
        # streaming units of 32 rows for wy > 16 (run-total form), 48 below (LDS ring),
        # on images with units enough; 4096 x 4096 (19 strips) takes 40 for the ring.
        # Strips store at most stream_quads(31) = 55 quads, as even as possible: a
        # 1024-quad row in 19 strips of 54
        p = morph.resolve_plan("u8", 8192, 4096, 31, 31)
        assert (p["tile_w"], p["tile_h"]) == (4 * 54, 32)
        assert morph.resolve_plan("u8", 8192, 4096, 31, 15)["tile_h"] == 48
        assert morph.resolve_plan("u8", 4096, 4096, 31, 15)["tile_h"] == 40
        assert morph.resolve_plan("u8", 1080, 1920, 31, 15)["tile_h"] == 8
        p = morph.resolve_plan("u8", 1080, 1920, 7, 63)
        assert (p["method_x"], p["method_y"]) == ("direct", "vhgw")
        # doubling with a direct-size vertical window: the wave kernel, 24-row units
        # (8 on small images), strips of up to stream_quads(wx) quads (a 90-pixel row:
        # one strip of its 23 quads)
        p = morph.resolve_plan("u8", 100000, 90, 3, 3, method_x="doubling")
        assert (p["kernel"], p["tile_w"], p["tile_h"]) == ("wave", 4 * 23, 24)
        p = morph.resolve_plan("u8", 100000, 4000, 3, 3, method_x="doubling")
        assert (p["kernel"], p["tile_w"]) == ("wave", 4 * 59)  # 1000 quads: 17 strips
        assert morph.resolve_plan("u8", 20, 90, 3, 3, method_x="doubling")["tile_h"] == 8
        # automatic: wide and short windows stay on the wave kernel with doubling
        p = morph.resolve_plan("u8", 1080, 1920, 63, 1)  # 480 quads: 11 strips of <= 47
        assert (p["method_x"], p["kernel"], p["tile_w"]) == ("doubling", "wave", 4 * 44)
        p = morph.resolve_plan("u8", 1080, 1920, 101, 101)
        assert (p["method_x"], p["method_y"], p["kernel"]) == ("doubling", "vhgw", "stream")
        p = morph.resolve_plan("u8", 1080, 1920, 129, 129)
        assert (p["method_x"], p["method_y"], p["kernel"]) == ("vhgw", "vhgw", "tile")
        assert morph.resolve_plan("u8", 4096, 4096, 1, 255)["kernel"] == "stream"
        assert morph.resolve_plan("u8", 4096, 4096, 1, 257)["kernel"] == "tile"
        # uint8, vertical window 1, 128 < wx <= 1000: the wide-row kernel, whose strip
        # stores the 16-pixel lanes whose input fits in 1024: (1006 - wx) // 16 + 1
        p = morph.resolve_plan("u8", 4096, 4096, 255, 1)
        assert (p["method_x"], p["kernel"], p["tile_w"], p["tile_h"]) == \
            ("doubling", "rows", 16 * 47, 4)
        assert morph.resolve_plan("u8", 4096, 4096, 1000, 1)["tile_w"] == 16
        assert morph.resolve_plan("u8", 4096, 4096, 129, 1, method_x="doubling")["kernel"] == "rows"
        assert morph.resolve_plan("u16", 4096, 4096, 255, 1)["kernel"] == "rows"
        for kw in (dict(wx=1001), dict(wy=2), dict(method_x="vhgw"), dict(tile=(256, 16))):
            a = dict(dtype_name="u8", H=4096, W=4096, wx=255, wy=1)
            a.update(kw)
            assert morph.resolve_plan(**a)["kernel"] == "tile", kw
        with pytest.raises(morph.MorphError):
            morph.resolve_plan("u8", 4096, 4096, 300, 3, method_x="doubling")
        for bad_kw in (dict(method_y="doubling"), dict(method_x="doubling", tile=(64, 32))):
            with pytest.raises(morph.MorphError):
                morph.resolve_plan("u8", 100, 100, 15, 5, **bad_kw)
        # windows are clipped to the image: 255x1 on a 4-wide image is a 7-wide window
        p = morph.resolve_plan("u8", 4, 4, 255, 1, method_x="direct")
        assert p["method_x"] == "direct"
        # a tuning file replaces thresholds and tiles
        f = tmp_path / "t.json"
        f.write_text(json.dumps({"u8": {"t_x": 3, "t_y": 4, "tiles": [
            {"wmax": 8, "tq": 16, "tb": 32}, {"wmax": 1000000, "tq": 40, "tb": 16}]}}))
        morph.load_tuning(str(f))
        assert morph.get_thresholds("u8") == (3, 4)
        # forced vHGW without a tile runs across the lanes of the streaming kernel
        # (horizontal windows up to 128) ...
        p = morph.resolve_plan("u8", 1000, 1000, 5, 5, method_x="vhgw", method_y="vhgw")
        assert (p["kernel"], p["method_x"], p["method_y"]) == ("stream", "vhgw", "vhgw")
        p = morph.resolve_plan("u8", 1000, 1000, 33, 3, method_x="vhgw")
        assert (p["kernel"], p["method_x"]) == ("wave", "vhgw")  # vertical direct
        p = morph.resolve_plan("u8", 1000, 1000, 129, 3, method_x="vhgw")
        assert p["kernel"] == "tile"
        # ... and with a tile (here only its height given: the width from the rule), or
        # beyond, on the workgroup-tile kernel, whose input row fills tq quads:
        # tw + wx - 1 + 3 <= 4 tq
        v = dict(method_x="vhgw", method_y="vhgw")
        p = morph.resolve_plan("u8", 1000, 1000, 5, 5, tile=(0, 32), **v)
        assert (p["kernel"], p["tile_w"], p["tile_h"]) == ("tile", 64 - 8, 32)
        p = morph.resolve_plan("u8", 1000, 1000, 30, 30, tile=(0, 16), **v)
        assert (p["tile_w"], p["tile_h"]) == (160 - 32, 16)
        # automatic methods beyond the thresholds: the streaming kernel, whose strip
        # stores at most the quads whose input fits in 64, (250 - wx) // 4 + 1 of them,
        # the strips as even as that allows: 250 quads in 5 strips of 50
        p = morph.resolve_plan("u8", 100000, 1000, 5, 5)
        assert (p["method_x"], p["method_y"]) == ("doubling", "vhgw")
        assert (p["tile_w"], p["tile_h"]) == (4 * 50, 48)
        f.write_text(json.dumps({"u8": {"stream_rows": 100, "stream_rows_runs": 40,
                                        "wide_rows": 7}}))
        morph.load_tuning(str(f))
        assert morph.resolve_plan("u8", 100000, 1000, 5, 5)["tile_h"] == 100
        assert morph.resolve_plan("u8", 1000, 1000, 200, 1)["tile_h"] == 7
        assert morph.resolve_plan("u8", 100000, 1000, 5, 17)["tile_h"] == 40
        # batch unit heights and the fused batch dispatch are keys of their own
        f.write_text(json.dumps({"u8": {"batch_wave_rows": 16, "batch_stream_rows": 20,
                                        "batch_stream_rows_runs": 30, "fuse": 0,
                                        "fit_units": 0}}))
        morph.load_tuning(str(f))
        # fit_units 0: a small single image keeps the tuned height
        assert morph.resolve_plan("u8", 1080, 1920, 3, 3)["tile_h"] == 24
        f.write_text(json.dumps({"u8": {"oc_rows": 24, "oc_rows_tall": 64, "oc_t_x": 5,
                                        "oc_one_pass": 0}}))
        morph.load_tuning(str(f))  # the one-pass opening's keys
        for bad_t in ({"batch_wave_rows": 12}, {"fuse": 2}, {"batch_stream_rows": 0},
                      {"fit_units": 3}, {"oc_rows": 12}, {"oc_rows_tall": 0},
                      {"oc_one_pass": 2}, {"oc_t_x": 0}):
            f.write_text(json.dumps({"u8": bad_t}))
            with pytest.raises(morph.MorphError):
                morph.load_tuning(str(f))
        bad = tmp_path / "bad.json"
        bad.write_text('{"u8": {"t_x": 3, "tiles": [{"wmax": 8, "tq": 1, "tb": 32}]}}')
        with pytest.raises(morph.MorphError):
            morph.load_tuning(str(bad))
        with pytest.raises(morph.MorphError):
            morph.load_tuning(str(tmp_path / "missing.json"))
    finally:
        assert _lib.lib().morph_load_tuning(None) == 0  # built-in defaults back
        morph.load_tuning(None)  # and the package's table


def test_shipped_table_is_the_built_in_one():
    """The autotuner's table shipped beside the package (loaded at import) and the
    library's built-in table give the same plans: thresholds, unit heights of single
    and batched images, tile shapes."""
    import paper_2002_09474_amd as morph
    cases = [(H, W, wx, wy, b) for (H, W) in ((4096, 4096), (100000, 1000), (1080, 1920))
             for (wx, wy) in ((3, 3), (9, 9), (10, 10), (16, 3), (17, 31), (31, 32), (101, 101),
                              (1, 255), (255, 1), (300, 300))
             for b in (False, True)]
    tiles = [(w, t) for w in (5, 12, 30, 60, 101) for t in ((0, 32), (0, 64))]

    def plans():
        out = [morph.get_thresholds(d) for d in ("u8", "u16")]
        for d in ("u8", "u16"):
            out += [morph.resolve_plan(d, H, W, wx, wy, batch=b) for H, W, wx, wy, b in cases]
            out += [morph.resolve_plan(d, 4096, 4096, w, w, method_x="vhgw", method_y="vhgw",
                                       tile=t) for w, t in tiles]
        return out
    try:
        assert _lib.lib().morph_load_tuning(None) == 0
        built_in = plans()
        morph.load_tuning(None)  # the shipped table
        assert plans() == built_in
    finally:
        morph.load_tuning(None)


def test_tuning_h_vhgw_routes_large_horizontal_windows(tmp_path):
    """"h_vhgw": 1 sends single images' automatic large horizontal windows to the
    paper's vHGW across the lanes (wave kernel's short form, streaming kernel); the tall
    wave form and batches keep doubling; 0 (the default) is doubling everywhere."""
    import json
    import paper_2002_09474_amd as morph
    f = tmp_path / "t.json"
    try:
        for flag, want in ((1, "vhgw"), (0, "doubling")):
            f.write_text(json.dumps({"u8": {"h_vhgw": flag, "t_x": 9, "t_y": 31}}))
            morph.load_tuning(str(f))
            for wx, wy, kernel, mx in ((33, 3, "wave", want), (101, 1, "wave", want),
                                       (45, 20, "wave", "doubling"), (63, 63, "stream", want),
                                       (5, 5, "wave", "direct")):
                p = morph.resolve_plan("u8", 150, 777, wx, wy)
                assert (p["kernel"], p["method_x"]) == (kernel, mx), (flag, wx, wy, p)
            assert morph.resolve_plan("u8", 150, 777, 33, 3, batch=True)["method_x"] == "doubling"
        f.write_text(json.dumps({"u8": {"h_vhgw": 2}}))
        with pytest.raises(morph.MorphError):
            morph.load_tuning(str(f))
    finally:
        morph.load_tuning(None)


def test_tuning_routes_tall_vertical_windows_to_the_cooperative_form(tmp_path):
    """coop_min_wy / coop_rows: single images on aligned rows whose vertical pass is
    vHGW in run totals take the streaming kernel's cooperative form from coop_min_wy,
    with units of coop_rows rows (shorter on small images); batches, rows of odd pitch,
    windows under coop_min_wy and units whose LDS would pass 64 KB keep the streaming
    kernel; 0 turns it off."""
    import json
    import paper_2002_09474_amd as morph
    f = tmp_path / "t.json"
    try:
        f.write_text(json.dumps({"u8": {"coop_min_wy": 64, "coop_rows": 96, "t_y": 31},
                                 "u16": {"coop_min_wy": 17, "coop_rows": 512, "t_y": 16,
                                         "fit_units": 0}}))
        morph.load_tuning(str(f))
        p = morph.resolve_plan("u8", 4096, 4096, 1, 255)
        assert (p["kernel"], p["tile_h"]) == ("stream_coop", 96)
        assert morph.resolve_plan("u8", 4096, 4096, 101, 101)["kernel"] == "stream_coop"
        assert morph.resolve_plan("u8", 4096, 4096, 7, 63)["kernel"] == "stream"  # under 64
        assert morph.resolve_plan("u8", 4096, 4096, 1, 255, batch=True)["kernel"] == "stream"
        assert morph.resolve_plan("u8", 4096, 4095, 1, 255)["kernel"] == "stream"  # odd pitch
        assert morph.resolve_plan("u8", 4096, 4096, 5, 255, method_x="vhgw")["kernel"] == "stream"
        # uint16 units of 512 rows would need over 64 KB of LDS at wy 17
        assert morph.resolve_plan("u16", 4096, 4096, 1, 17)["kernel"] == "stream"
        assert morph.resolve_plan("u16", 4096, 4096, 1, 255)["kernel"] == "stream"
        f.write_text(json.dumps({"u16": {"coop_rows": 64}}))
        morph.load_tuning(str(f))
        assert morph.resolve_plan("u16", 4096, 4096, 1, 17)["kernel"] == "stream_coop"
        f.write_text(json.dumps({"u8": {"coop_min_wy": 0}}))
        morph.load_tuning(str(f))
        assert morph.resolve_plan("u8", 4096, 4096, 1, 255)["kernel"] == "stream"
        # batches by keys of their own
        f.write_text(json.dumps({"u8": {"batch_coop_min_wy": 33, "batch_coop_rows": 64,
                                        "batch_coop_waves": 4}}))
        morph.load_tuning(str(f))
        p = morph.resolve_plan("u8", 1000, 1000, 7, 63, batch=True)
        assert (p["kernel"], p["tile_h"]) == ("stream_coop", 64)
        assert morph.resolve_plan("u8", 4096, 4096, 1, 255)["kernel"] == "stream"
        for bad in ({"coop_rows": 12}, {"coop_rows": 2048}, {"coop_min_wy": -1}, {"coop_waves": 5},
                    {"batch_coop_waves": 2}, {"batch_coop_rows": 0}):
            f.write_text(json.dumps({"u8": bad}))
            with pytest.raises(morph.MorphError):
                morph.load_tuning(str(f))
    finally:
        morph.load_tuning(None)


def test_strerror():
    L = _lib.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert L.morph_strerror(s)
    assert L.morph_strerror(-99) == b"unknown status"


def test_multiply_high_division_is_exact():
    """The kernels divide work-unit indices u by d as mulhi(u, ceil(2^32 / d)); this
    is exact whenever u * d < 2^32 (the planner's guarantee)."""
    import math
    import random
    rnd = random.Random(5)
    for d in list(range(2, 600)) + [rnd.randrange(2, 1 << 16) for _ in range(300)]:
        m = math.ceil((1 << 32) / d)
        umax = ((1 << 32) - 1) // d
        for u in [0, 1, d - 1, d, d + 1, umax, umax - 1] + [rnd.randrange(0, umax + 1) for _ in range(40)]:
            assert (u * m) >> 32 == u // d, (u, d)
