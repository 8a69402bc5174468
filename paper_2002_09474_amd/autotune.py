"""Autotuner: measures, on the GPU it runs on, where the direct passes stop beating
the large-window passes (per pass and element type), how many rows the wave and
streaming kernels' units should hold, and which tile shapes the workgroup-tile
kernel should use, and writes the tuning table the library loads
(``morph_load_tuning``; the Python package loads ``tuning_gfx950.json`` next to
this file at start-up when it exists).

The paper chose its switch-over windows by timing both implementations of each
pass over a range of windows (§5.1.3, §5.2.3, §5.3); this does the same with the
GPU kernels the automatic plan picks between: for a pass of window w, the direct
pass (the register-only wave kernel when both passes are direct) against the
large-window pass (the streaming kernel: vHGW through an LDS ring vertically,
doubling across lanes horizontally), as single-pass sweeps along x (w x 1) and
along y (1 x w) on a 4096x4096 document page.  The threshold of a pass is the
largest window up to which direct is never slower by more than the timing noise.
On the same page, the large horizontal windows' two passes across the lanes, doubling
and the paper's vHGW, are timed against each other (h_vhgw).
The thresholds of batched images are then chosen on the whole benchmark batch
(direct passes that leave the fused dispatch can cost it more than they save).
Unit heights of batched images are then chosen on the whole 512-image batch of the
benchmark (one key at a time; then whether its run-total streaming units should take
the cooperative form), those of single images on 4096x4096 images: the wave
kernel's over 3x3 and 9x9, its tall form's over 15x15 and 1x31, the streaming
kernel's ring form at 15x15 with vHGW forced and its run-total form over 7x63,
101x101 and 1x255, its cooperative form's (with its waves a unit) over 7x63, 101x101,
1x155 and 1x255, the one-pass opening's over 3x3 and 9x9 and at 15x15 -- each the
height whose worst time over its windows, relative to the best height there, is
least.  Then the vertical window from which the cooperative form beats the streaming
kernel's own, whether the one-pass opening beats the two launches at all, the unit
height of the wide-row kernel (uint8, vertical window 1, wx > 128) on the same
images, and tile shapes of the tile kernel per window bucket.
As in the benchmark, timed launches take turns over copies of their images that
together hold more memory than the 256 MB Infinity Cache (four copies of the batch;
512 MB of 4096x4096 buffers), so that what is measured is the kernels reading HBM.  Run
``python -m paper_2002_09474_amd.autotune``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning_gfx950.json")
# largest windows of the library's direct passes (wave kernel) per axis
DIRECT_MAX = {"x": 16, "y": 31}
BUCKETS = ((9, 9), (16, 15), (32, 31), (64, 63), (1 << 30, 101))  # (wmax, representative w)
TQ = (16, 32, 48, 64, 96)
TB = (16, 32, 64, 128)
WAVE_ROWS = (8, 16, 24, 32, 48)
STREAM_ROWS = (32, 48, 64, 96)      # streaming units, LDS-ring form (wy <= 16)
STREAM_ROWS_RUNS = (24, 32, 48, 64)  # streaming units, run-total form (wy > 16)
# unit heights of single images, each timed on 4096x4096 images over its windows
# (wx, wy): the wave kernel's short form and its tall form (a kernel of its own); the
# streaming kernel's ring form (vertical windows up to 16, which the automatic plan
# takes direct: forced vHGW) and its run-total form
SINGLE_KEYS = (("wave_rows", WAVE_ROWS, ((3, 3), (9, 9)), {}),
               ("wave_rows_tall", WAVE_ROWS, ((15, 15), (1, 31)), {}),
               ("stream_rows", STREAM_ROWS, ((15, 15),), {"method_y": "vhgw"}),
               ("stream_rows_runs", STREAM_ROWS_RUNS, ((7, 63), (101, 101), (1, 255)), {}))
# the streaming kernel's cooperative form (single images, run-total windows): its unit
# heights over its windows, then the vertical window from which it beats the
# streaming kernel's own form (1 x wy at COOP_MIN)
COOP_ROWS = (48, 64, 96, 128, 192)
COOP_WAVES = (4, 8, 16)
COOP_WINDOWS = ((7, 63), (101, 101), (1, 155), (1, 255))
COOP_MIN = (33, 63, 101, 155, 255)
# unit heights of batched images, timed on the whole benchmark batch
BATCH_KEYS = (("batch_wave_rows", (16, 24, 32, 48)), ("batch_stream_rows", (32, 48, 64, 96)),
              ("batch_stream_rows_runs", (32, 48, 64)))
# unit heights of single images' one-pass openings, each timed on 4096x4096 images
# over its windows (the short kernel's, vertical windows up to 9, and the tall one's)
OC_KEYS = (("oc_rows", (8, 16, 24, 32, 48), (3, 9)), ("oc_rows_tall", (16, 32, 48, 64), (15,)))
BATCH_COPIES = 4  # copies of the batch that timed launches take turns over (1.3 GB of uint8)
WIDE_ROWS = (2, 4, 8, 16)            # wide-row units (uint8, wy = 1, wx > 128)
WIDE_WINDOWS = (200, 255, 511)


def _timer(torch, fn, iters, warmup=5):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(iters):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / iters * 1e3  # microseconds


def _bufs(torch, img, min_bytes=512 << 20):
    """Copies of `img` and as many outputs, at least four pairs and together at least
    `min_bytes` (launches take turns over them)."""
    n = max(4, -(-min_bytes // (2 * img.numel() * img.element_size())))
    srcs = [img.clone() for _ in range(n)]
    return srcs, [torch.empty_like(s) for s in srcs]


def _with_table(morph, table):
    """Load a tuning table given as a dict (through a temporary file)."""
    fd, path = tempfile.mkstemp(suffix=".json")
    try:
        with os.fdopen(fd, "w") as f:
            json.dump(table, f)
        morph.load_tuning(path)
    finally:
        os.unlink(path)


def pass_sweep(torch, morph, dname, srcs, dsts, iters=40, windows=None):
    """Time each single pass for w = 2 .. DIRECT_MAX[axis] (or the given windows per
    axis), direct (threshold >= w) against the large-window pass (threshold w - 1),
    with automatic methods."""
    rows = []
    t0 = morph.get_thresholds(dname)
    try:
        for axis in ("x", "y"):
            ws = windows[axis] if windows else range(2, DIRECT_MAX[axis] + 1)
            for w in ws:
                wx, wy = (w, 1) if axis == "x" else (1, w)
                t = {}
                for name, thr in (("direct", w), ("large", w - 1)):
                    morph.set_thresholds(dname, thr if axis == "x" else t0[0],
                                         thr if axis == "y" else t0[1])
                    k = [0]

                    def fn():
                        i = k[0] % len(srcs)
                        k[0] += 1
                        morph.apply("erode", srcs[i], wx, wy, out=dsts[i])
                    # the median of three timings
                    t[name] = sorted(_timer(torch, fn, iters) for _ in range(3))[1]
                rows.append({"axis": axis, "w": w, "direct_us": round(t["direct"], 3),
                             "large_us": round(t["large"], 3)})
    finally:
        morph.set_thresholds(dname, *t0)
    return rows


def threshold(rows, axis, tol=0.03):
    """The window before the first sustained loss of the direct pass: the largest
    swept w such that no two consecutive swept windows up to w + 1 both have
    direct > large * (1 + tol) (a single loss within the noise does not end the
    direct range; 1 if direct loses from the start)."""
    rs = sorted((r for r in rows if r["axis"] == axis), key=lambda r: r["w"])
    lose = [r["direct_us"] > r["large_us"] * (1 + tol) for r in rs]
    t = 1
    for i, r in enumerate(rs):
        if lose[i] and (i + 1 == len(rs) or lose[i + 1]):
            break
        if not lose[i]:
            t = r["w"]
    return t


H_WINDOWS = (13, 31, 63, 101)  # horizontal windows the doubling / vHGW choice is timed at


def h_vhgw_check(torch, morph, srcs, dsts, windows=H_WINDOWS, iters=20):
    """1 if the paper's vHGW across the lanes beats doubling over w x 1 passes at
    `windows` (the sum of medians of three timings), else 0; and the timings."""
    res = []
    for name in ("doubling", "vhgw"):
        us = []
        for w in windows:
            k = [0]

            def fn():
                i = k[0] % len(srcs)
                k[0] += 1
                morph.apply("erode", srcs[i], w, 1, out=dsts[i], method_x=name)
            us.append(round(sorted(_timer(torch, fn, iters) for _ in range(3))[1], 3))
        res.append({"method_x": name, "windows": list(windows), "us": us})
    return int(sum(res[1]["us"]) < sum(res[0]["us"])), res


def _time_batches(torch, morph, copies, iters):
    """Microseconds a launch of the batch, launches taking turns over its copies (so
    that, as in the benchmark, a launch does not find its images in the Infinity
    Cache): the median of three timings."""
    bs = []
    try:
        for items in copies:
            b = morph.Batch(len(items), 1 << 22)
            bs.append(b)
            b.set(items)
        k = [0]

        def fn():
            bs[k[0] % len(bs)].enqueue()
            k[0] += 1
        ts = sorted(_timer(torch, fn, iters, warmup=len(bs)) for _ in range(3))
        return ts[1]
    finally:
        for b in bs:
            b.close()


def batch_thresholds(torch, morph, dname, copies, base, tx, ty, iters=10):
    """(batch_t_x, batch_t_y): the thresholds under which the whole batch runs
    fastest, among the classic pair (9, 9), the single-image thresholds and mixes
    of them -- a pass taken off the fused dispatch can cost the batch more than it
    saves on its own images."""
    cands = sorted({(9, 9), (min(tx, 9), 9), (9, min(ty, 15)), (tx, min(ty, 15)), (tx, ty)})
    res = []
    for cx, cy in cands:
        _with_table(morph, {dname: dict(base, batch_t_x=cx, batch_t_y=cy)})
        us = _time_batches(torch, morph, copies, iters)
        res.append({"batch_t_x": cx, "batch_t_y": cy, "us": round(us, 2)})
    best = min(res, key=lambda r: r["us"])
    return best["batch_t_x"], best["batch_t_y"], res


def best_rows(torch, morph, dname, copies, key, choices, base, iters=10):
    """The `key` (a batch unit height) among `choices` that runs the batch (launches
    taking turns over its copies) fastest, the rest of the table being `base`."""
    res = []
    for c in choices:
        _with_table(morph, {dname: dict(base, **{key: c})})
        us = _time_batches(torch, morph, copies, iters)
        res.append({key: c, "us": round(us, 2)})
    best = min(res, key=lambda r: r["us"])[key]
    return best, res


def tile_sweep(torch, morph, srcs, dsts, dname, iters=20, buckets=BUCKETS, tqs=TQ, tbs=TB):
    """Tile shapes of the workgroup-tile kernel (forced vHGW passes) per window bucket."""
    rules, table = [], []
    H, W = srcs[0].shape
    v = dict(method_x="vhgw", method_y="vhgw")
    for wmax, w in buckets:
        best = None
        for tq in tqs:
            for tb in tbs:
                tw = max(4 * tq - ((w + 2 + 3) // 4 * 4), (2 * w + 3) // 4 * 4)
                try:
                    plan = morph.resolve_plan(dname, H, W, w, w, tile=(tw, tb), **v)
                except morph.MorphError:
                    continue
                k = [0]

                def fn():
                    i = k[0] % len(srcs)
                    k[0] += 1
                    morph.apply("erode", srcs[i], w, w, out=dsts[i], tile=(tw, tb), **v)
                try:
                    us = _timer(torch, fn, iters)
                except morph.MorphError:
                    continue
                table.append({"w": w, "tq": tq, "tb": tb, "tile": [plan["tile_w"], plan["tile_h"]],
                              "us": round(us, 3)})
                if best is None or us < best[0]:
                    best = (us, tq, plan["tile_h"])
        if best is not None:
            rules.append({"wmax": wmax, "tq": best[1], "tb": best[2]})
            _log("%s: tiles up to %d: tq %d, tb %d" % (dname, wmax, best[1], best[2]))
    return rules, table


def least_worst(res, key):
    """The choice (value of `key`) whose worst time relative to the best choice at each
    window is least: res rows hold `key` and "us" (a list over the same windows)."""
    n = len(res[0]["us"])
    best = [min(r["us"][i] for r in res) for i in range(n)]
    return min(res, key=lambda r: max(r["us"][i] / best[i] for i in range(n)))[key]


def best_single_rows(torch, morph, dname, srcs, dsts, key, choices, base, windows, iters=20,
                     kw=None):
    """The `key` (a single-image unit height) among `choices` whose worst erosion time
    of the images `srcs` over `windows` ((wx, wy) pairs, with the plan arguments `kw`;
    median of three timings), relative to the best choice there, is least; the rest of
    the table being `base`."""
    kw = kw or {}
    res = []
    for c in choices:
        _with_table(morph, {dname: dict(base, **{key: c})})
        us = []
        for wx, wy in windows:
            k = [0]

            def fn():
                i = k[0] % len(srcs)
                k[0] += 1
                morph.apply("erode", srcs[i], wx, wy, out=dsts[i], **kw)
            us.append(round(sorted(_timer(torch, fn, iters) for _ in range(3))[1], 3))
        res.append({key: c, "windows": ["%dx%d" % w for w in windows], "us": us})
    return least_worst(res, key), res


def coop_sweep(torch, morph, dname, srcs, dsts, base, iters=20, choices=COOP_ROWS,
               windows=COOP_WINDOWS, mins=COOP_MIN, tol=0.03):
    """The cooperative form's waves a unit and unit height (the pair least worst over
    `windows`, the form taken from wy 17), then coop_min_wy: the smallest swept wy
    (1 x wy) from which it is never slower than the streaming kernel's own form by more
    than `tol` (0 if it loses at the largest).  Returns (coop_waves, coop_rows,
    coop_min_wy, height table, threshold rows)."""
    table = []
    for nw in COOP_WAVES:
        _, t = best_single_rows(torch, morph, dname, srcs, dsts, "coop_rows", choices,
                                dict(base, coop_min_wy=17, coop_waves=nw), windows, iters)
        table += [dict(r, coop_waves=nw, coop=(nw, r["coop_rows"])) for r in t]
    waves_best, rows_best = least_worst(table, "coop")
    for r in table:
        del r["coop"]
    rows = []
    for wy in mins:
        t = {}
        for name, m in (("stream", 0), ("coop", 17)):
            _with_table(morph, {dname: dict(base, coop_min_wy=m, coop_rows=rows_best,
                                            coop_waves=waves_best)})
            k = [0]

            def fn():
                i = k[0] % len(srcs)
                k[0] += 1
                morph.apply("erode", srcs[i], 1, wy, out=dsts[i])
            t[name] = sorted(_timer(torch, fn, iters) for _ in range(3))[1]
        rows.append({"wy": wy, "stream_us": round(t["stream"], 3), "coop_us": round(t["coop"], 3)})
    thr = 0
    for r in reversed(rows):
        if r["coop_us"] > r["stream_us"] * (1 + tol):
            break
        thr = r["wy"]
    return waves_best, rows_best, thr, table, rows


def oc_rows_sweep(torch, morph, dname, srcs, dsts, key, choices, base, windows, iters=20):
    """The `key` (a unit height of the one-pass opening) among `choices` whose worst
    w x w opening time over `windows`, relative to the best choice there, is least; the
    rest of the table being `base`."""
    res = []
    for c in choices:
        _with_table(morph, {dname: dict(base, **{key: c})})
        us = []
        for w in windows:
            k = [0]

            def fn():
                i = k[0] % len(srcs)
                k[0] += 1
                morph.openclose_fused("open", srcs[i], w, w, out=dsts[i])
            us.append(round(sorted(_timer(torch, fn, iters) for _ in range(3))[1], 3))
        res.append({key: c, "windows": ["%dx%d" % (w, w) for w in windows], "us": us})
    return least_worst(res, key), res


def oc_one_pass_check(torch, morph, dname, srcs, dsts, base, windows=(3, 9, 15), iters=20):
    """1 if the one-pass openings beat the two launches through a workspace (the sum
    over `windows` of w x w openings), else 0; and the timings."""
    ws = [torch.empty_like(d) for d in dsts]
    res = []
    for one in (1, 0):
        _with_table(morph, {dname: dict(base, oc_one_pass=one)})
        us = 0.0
        for w in windows:
            k = [0]

            def fn():
                i = k[0] % len(srcs)
                k[0] += 1
                morph.apply("open", srcs[i], w, w, out=dsts[i], workspace=ws[i])
            us += _timer(torch, fn, iters)
        res.append({"oc_one_pass": one, "us": round(us, 3)})
    return int(res[0]["us"] <= res[1]["us"]), res


def wide_rows_sweep(torch, morph, srcs, dsts, base, iters=20, choices=WIDE_ROWS):
    """Rows of a wide-row unit: the sum over WIDE_WINDOWS (w x 1) on uint8 4096x4096
    images, per choice; the fastest."""
    res = []
    for c in choices:
        _with_table(morph, {"u8": dict(base, wide_rows=c)})
        us = 0.0
        for w in WIDE_WINDOWS:
            k = [0]

            def fn():
                i = k[0] % len(srcs)
                k[0] += 1
                morph.apply("erode", srcs[i], w, 1, out=dsts[i])
            us += _timer(torch, fn, iters)
        res.append({"wide_rows": c, "us": round(us, 2)})
    return min(res, key=lambda r: r["us"])["wide_rows"], res


def _batch_items(torch, morph, dev, dname, n=512, hi=2048, copies=BATCH_COPIES):
    """The benchmark's 512-image batch (uint8, or the same images scaled to uint16) in
    `copies` copies, each its own source and destination images; n and hi give a
    smaller batch of the same kind."""
    from . import synth
    specs = synth.batch_specs(n, seed=5, hi=hi)
    imgs = synth.batch_images(specs, seed=5)
    out = [[] for _ in range(copies)]
    for s, im in zip(specs, imgs):
        t = torch.from_numpy(im).to(dev)
        if dname == "u16":
            t = (t.to(torch.int32) * 257).to(torch.int16).view(torch.uint16)
        # rows padded to 64 bytes, as the benchmark lays the batch out
        es = t.element_size()
        p = (s["W"] * es + 63) // 64 * 64 // es
        for items in out:
            src = torch.zeros((s["H"], p), dtype=t.dtype, device=dev)[:, :s["W"]]
            src.copy_(t)
            dst = torch.empty((s["H"], p), dtype=t.dtype, device=dev)[:, :s["W"]]
            items.append(dict(src=src, dst=dst, wx=s["w"], wy=s["w"], op=s["op"]))
    return out


# the reduced grid: a few windows and choices per key on smaller images, for a
# check that the tuner runs end to end and writes a table the library loads
REDUCED = {"windows": {"x": (2, 3, 9, 12, 16), "y": (2, 3, 9, 15, 31)},
           "batch": (48, 300), "big": 1024,
           "batch_keys": tuple((k, c[:2]) for k, c in BATCH_KEYS),
           "single_keys": tuple((k, c[:2], w[:1], kw) for k, c, w, kw in SINGLE_KEYS),
           "oc_keys": tuple((k, c[:2], w) for k, c, w in OC_KEYS),
           "coop_rows": COOP_ROWS[:2], "coop_windows": ((1, 101),), "coop_min": (33, 101),
           "wide_rows": WIDE_ROWS[:2], "buckets": BUCKETS[:1], "tq": TQ[:2], "tb": TB[:2]}


def tune(out_path=DEFAULT_OUT, quick=False, reduced=False):
    import torch

    import paper_2002_09474_amd as morph
    from paper_2002_09474_amd import synth
    dev = torch.device("cuda")
    morph._lib.lib().morph_load_tuning(None)  # start from the built-in table
    # (on a stream of its own: the legacy default stream cannot be captured, so
    # batches launched there would not replay graphs as they do in use)
    side = torch.cuda.Stream()
    prev = torch.cuda.current_stream()
    torch.cuda.set_stream(side)
    try:
        return _tune(torch, morph, synth, dev, out_path, quick, reduced)
    finally:
        torch.cuda.synchronize()
        torch.cuda.set_stream(prev)


def _log(msg):
    print("[autotune] " + msg, file=sys.stderr, flush=True)


def _tune(torch, morph, synth, dev, out_path, quick, reduced):
    result = {"device": torch.cuda.get_device_name(0), "version": morph.version(),
              "grid": "reduced" if reduced else ("quick" if quick else "full")}
    R = REDUCED if reduced else None
    # the pass sweep's page: document-like content (as the 1920x1080 configuration)
    # at 4096 x 4096, where the kernels' time, not a launch's fixed cost, decides
    doc = torch.from_numpy(synth.document(540 if R else 4096, 960 if R else 4096, seed=2)).to(dev)
    for dname in ("u8", "u16"):
        img = doc if dname == "u8" else (doc.to(torch.int32) * 257).to(torch.int16).view(torch.uint16)
        srcs, dsts = _bufs(torch, img, (16 << 20) if R else (512 << 20))
        rows = pass_sweep(torch, morph, dname, srcs, dsts, iters=10 if R else (20 if quick else 40),
                          windows=R["windows"] if R else None)
        tx, ty = threshold(rows, "x"), threshold(rows, "y")
        _log("%s: pass sweep done, thresholds x %d, y %d" % (dname, tx, ty))
        hv, result[dname + "_h_vhgw_check"] = h_vhgw_check(
            torch, morph, srcs, dsts, (13, 31) if R else H_WINDOWS, 3 if R else 20)
        _log("%s: h_vhgw %d" % (dname, hv))
        del srcs, dsts
        base = {"t_x": tx, "t_y": ty, "h_vhgw": hv}
        copies = (_batch_items(torch, morph, dev, dname, *R["batch"], copies=2) if R
                  else _batch_items(torch, morph, dev, dname))
        it = 4 if R else (8 if quick else 16)
        btx, bty, bt_table = batch_thresholds(torch, morph, dname, copies, base, tx, ty, it)
        base.update(batch_t_x=btx, batch_t_y=bty)
        _log("%s: batch thresholds x %d, y %d" % (dname, btx, bty))
        result[dname + "_batch_threshold_sweep"] = bt_table
        for key, choices in (R["batch_keys"] if R else BATCH_KEYS):
            best, table = best_rows(torch, morph, dname, copies, key, choices, base, it)
            base[key] = best
            _log("%s: %s %d" % (dname, key, best))
            result[dname + "_" + key + "_sweep"] = table
        # the run-total streaming units in the cooperative form (a dispatch of their own)
        # against the fused dispatch: on or off
        bc = []
        for cmin in (0, 17):
            t = dict(base, batch_coop_min_wy=cmin, batch_coop_rows=64, batch_coop_waves=4)
            _with_table(morph, {dname: t})
            bc.append({"batch_coop_min_wy": cmin,
                       "us": round(_time_batches(torch, morph, copies, it), 2)})
        base["batch_coop_min_wy"] = min(bc, key=lambda r: r["us"])["batch_coop_min_wy"]
        if base["batch_coop_min_wy"]:
            base.update(batch_coop_rows=64, batch_coop_waves=4)
        result[dname + "_batch_coop_check"] = bc
        _log("%s: batch_coop_min_wy %d" % (dname, base["batch_coop_min_wy"]))
        del copies
        _with_table(morph, {dname: base})
        g = torch.Generator(device=dev).manual_seed(3)
        n = R["big"] if R else 4096
        big = torch.randint(0, 256 if dname == "u8" else 65536, (n, n), generator=g,
                            dtype=torch.int32, device=dev)
        big = big.to(torch.uint8) if dname == "u8" else big.to(torch.int16).view(torch.uint16)
        srcs, dsts = _bufs(torch, big, (16 << 20) if R else (512 << 20))
        for key, choices, ws, kw in (R["single_keys"] if R else SINGLE_KEYS):
            best, table = best_single_rows(torch, morph, dname, srcs, dsts, key, choices, base, ws,
                                           3 if R else (8 if quick else 20), kw)
            base[key] = best
            _log("%s: %s %d" % (dname, key, best))
            result[dname + "_" + key + "_sweep"] = table
        _with_table(morph, {dname: base})
        cw, cr, cmin, ctab, crows = coop_sweep(
            torch, morph, dname, srcs, dsts, base, 3 if R else (8 if quick else 20),
            choices=R["coop_rows"] if R else COOP_ROWS,
            windows=R["coop_windows"] if R else COOP_WINDOWS,
            mins=R["coop_min"] if R else COOP_MIN)
        base.update(coop_waves=cw, coop_rows=cr, coop_min_wy=cmin)
        result[dname + "_coop_rows_sweep"] = ctab
        result[dname + "_coop_threshold_sweep"] = crows
        _log("%s: coop_waves %d, coop_rows %d, coop_min_wy %d" % (dname, cw, cr, cmin))
        _with_table(morph, {dname: base})
        oc_it = 3 if R else (8 if quick else 20)
        for key, choices, ws in (R["oc_keys"] if R else OC_KEYS):
            best, table = oc_rows_sweep(torch, morph, dname, srcs, dsts, key, choices, base, ws,
                                        oc_it)
            base[key] = best
            _log("%s: %s %d" % (dname, key, best))
            result[dname + "_" + key + "_sweep"] = table
        base["oc_one_pass"], result[dname + "_oc_one_pass_check"] = oc_one_pass_check(
            torch, morph, dname, srcs, dsts, base, iters=oc_it)
        _log("%s: oc_one_pass %d" % (dname, base["oc_one_pass"]))
        _with_table(morph, {dname: base})
        if dname == "u8":
            wr2, wr2_table = wide_rows_sweep(torch, morph, srcs, dsts, base,
                                             3 if R else (8 if quick else 20),
                                             choices=R["wide_rows"] if R else WIDE_ROWS)
            base["wide_rows"] = wr2
            result["u8_wide_rows_sweep"] = wr2_table
            _with_table(morph, {dname: base})
        if R:
            rules, table = tile_sweep(torch, morph, srcs, dsts, dname, iters=3,
                                      buckets=R["buckets"], tqs=R["tq"], tbs=R["tb"])
        else:
            rules, table = tile_sweep(torch, morph, srcs, dsts, dname,
                                      iters=8 if quick else 20)
        del srcs, dsts, big
        result[dname] = dict(base, tiles=rules)
        result[dname + "_pass_sweep"] = rows
        result[dname + "_tile_sweep"] = table
        _log("%s: %s" % (dname, result[dname]))
    with open(out_path, "w") as f:
        json.dump(result, f, indent=1)
    morph.load_tuning(out_path)
    return result


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--reduced", action="store_true",
                    help="a few windows and choices per key on smaller images")
    a = ap.parse_args(argv)
    r = tune(a.out, a.quick, a.reduced)
    print(json.dumps({k: r[k] for k in ("device", "u8", "u16")}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
