"""Autotuner: measures, on the GPU it runs on, where the direct pass stops beating
van Herk/Gil-Werman (per pass and element type) and which tile shape is fastest
for each window bucket, and writes the tuning table the library loads
(``morph_load_tuning``; the Python package loads ``tuning_gfx950.json`` next to
this file at start-up when it exists).

The paper chose its switch-over windows by timing both implementations of each
pass over a range of windows (§5.1.3, §5.2.3, §5.3); this does the same with the
GPU kernels: single-pass sweeps along x (w x 1) and along y (1 x w) on the
1920x1080 document page, both methods forced.  The threshold of a pass is the
largest window up to which the direct pass is never slower than vHGW by more than
the timing noise.  Tile shapes (input quads per tile row ``tq`` and output rows
``tb``) are then timed per window bucket on 4096x4096 images with the chosen
thresholds.  Run ``python -m paper_2002_09474_amd.autotune``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning_gfx950.json")
DIRECT_MAX = 9
BUCKETS = ((9, 9), (16, 15), (32, 31), (64, 63), (1 << 30, 101))  # (wmax, representative w)
TQ = (16, 32, 48, 64, 96)
TB = (16, 32, 64, 128)


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


def _bufs(torch, img, n):
    srcs = [img.clone() for _ in range(n)]
    return srcs, [torch.empty_like(s) for s in srcs]


def pass_sweep(torch, morph, srcs, dsts, iters=40):
    """Time each single pass, direct vs vHGW, for w = 2 .. DIRECT_MAX."""
    rows = []
    for axis in ("x", "y"):
        for w in range(2, DIRECT_MAX + 1):
            wx, wy = (w, 1) if axis == "x" else (1, w)
            t = {}
            for m in ("direct", "vhgw"):
                k = [0]
                kw = {"method_x": m} if axis == "x" else {"method_y": m}

                def fn():
                    i = k[0] % len(srcs)
                    k[0] += 1
                    morph.apply("erode", srcs[i], wx, wy, out=dsts[i], **kw)
                t[m] = _timer(torch, fn, iters)
            rows.append({"axis": axis, "w": w, "direct_us": round(t["direct"], 3),
                         "vhgw_us": round(t["vhgw"], 3)})
    return rows


def threshold(rows, axis, tol=0.03):
    """Largest w such that direct <= vHGW * (1 + tol) for every w' <= w (1 if none)."""
    t = 1
    for r in sorted((r for r in rows if r["axis"] == axis), key=lambda r: r["w"]):
        if r["direct_us"] <= r["vhgw_us"] * (1 + tol):
            t = r["w"]
        else:
            break
    return t


def tile_sweep(torch, morph, srcs, dsts, dname, iters=20):
    rules, table = [], []
    H, W = srcs[0].shape
    for wmax, w in BUCKETS:
        best = None
        for tq in TQ:
            for tb in TB:
                tw = max(4 * tq - ((w + 2 + 3) // 4 * 4), (2 * w + 3) // 4 * 4)
                try:
                    plan = morph.resolve_plan(dname, H, W, w, w, tile=(tw, tb))
                except morph.MorphError:
                    continue
                k = [0]

                def fn():
                    i = k[0] % len(srcs)
                    k[0] += 1
                    morph.apply("erode", srcs[i], w, w, out=dsts[i], tile=(tw, tb))
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
    return rules, table


def tune(out_path=DEFAULT_OUT, quick=False):
    import torch

    import paper_2002_09474_amd as morph
    from paper_2002_09474_amd import synth
    dev = torch.device("cuda")
    morph._lib.lib().morph_load_tuning(None)  # start from the built-in table
    result = {"device": torch.cuda.get_device_name(0), "version": morph.version()}
    doc = torch.from_numpy(synth.document(1080, 1920, seed=2)).to(dev)
    for dname in ("u8", "u16"):
        img = doc if dname == "u8" else (doc.to(torch.int32) * 257).to(torch.int16).view(torch.uint16)
        srcs, dsts = _bufs(torch, img, 8)
        rows = pass_sweep(torch, morph, srcs, dsts, iters=20 if quick else 40)
        tx, ty = threshold(rows, "x"), threshold(rows, "y")
        morph.set_thresholds(dname, tx, ty)
        del srcs, dsts
        g = torch.Generator(device=dev).manual_seed(3)
        big = torch.randint(0, 256 if dname == "u8" else 65536, (4096, 4096), generator=g,
                            dtype=torch.int32, device=dev)
        big = big.to(torch.uint8) if dname == "u8" else big.to(torch.int16).view(torch.uint16)
        srcs, dsts = _bufs(torch, big, 6)
        rules, table = tile_sweep(torch, morph, srcs, dsts, dname, iters=8 if quick else 20)
        del srcs, dsts, big
        result[dname] = {"t_x": tx, "t_y": ty, "tiles": rules}
        result[dname + "_pass_sweep"] = rows
        result[dname + "_tile_sweep"] = table
        print("[autotune] %s: t_x=%d t_y=%d tiles=%s" % (dname, tx, ty, rules), file=sys.stderr,
              flush=True)
    with open(out_path, "w") as f:
        json.dump(result, f, indent=1)
    morph.load_tuning(out_path)
    return result


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true")
    a = ap.parse_args(argv)
    r = tune(a.out, a.quick)
    print(json.dumps({k: r[k] for k in ("device", "u8", "u16")}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
