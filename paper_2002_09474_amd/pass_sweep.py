"""Per-pass window sweep in the shape of the paper's own experiment (§5.1.3 and
§5.2.3, Figs. 3-4): one pass at a time, w x 1 (along x) and 1 x w (along y), w
swept, on an 800x600 uint8 page (the paper's image size).  Two comparisons:

- the paper's two methods on one kernel: the workgroup-tile kernel runs the direct
  pass (compiled per window up to 9, a loop over the taps beyond) and the vHGW
  pass for every w, so both curves cover the whole range and cross where the
  direct pass's O(w) work overtakes vHGW's constant work;
- along x, the paper's vHGW run across the wave kernel's lanes beside the
  doubling pass the library takes for large horizontal windows;
- the production choice: the library's direct pass (the register-only wave
  kernel: vertical windows up to 31, horizontal up to 16) against its
  large-window pass (vertically vHGW on the streaming kernel, horizontally
  doubling across lanes), each forced through the thresholds; this crossover is
  the threshold the tuning table ships.

Times are per launch, from 20 launches over 8 buffer pairs captured in one graph.
Run ``python -m paper_2002_09474_amd.pass_sweep [--out FILE.json]``.
"""
from __future__ import annotations

import argparse
import json
import sys

WINDOWS = (1, 2, 3, 4, 5, 7, 9, 11, 13, 15, 17, 19, 21, 25, 31, 45, 63, 101, 155, 255)
# largest windows of the library's direct pass per axis (wave kernel)
PROD_DIRECT_MAX = {"x": 16, "y": 31}


def _graph_us(torch, fns, reps=10):
    stream = torch.cuda.current_stream()
    for f in fns:  # warm up (and any lazy set-up) outside the capture
        f()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for f in fns:
            f()
    g.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        a.record(stream)
        g.replay()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e3 / len(fns))
    ts.sort()
    return ts[len(ts) // 2]


def sweep(H=600, W=800, windows=WINDOWS, dname="u8"):
    import torch

    import paper_2002_09474_amd as morph
    from paper_2002_09474_amd import synth
    dev = torch.device("cuda")
    img = torch.from_numpy(synth.document(H, W, seed=4)).to(dev)
    if dname == "u16":
        img = (img.to(torch.int32) * 257).to(torch.int16).view(torch.uint16)
    nbuf = 8
    srcs = [img.clone() for _ in range(nbuf)]
    dsts = [torch.empty_like(s) for s in srcs]
    t0 = morph.get_thresholds(dname)
    rows = []
    try:
        for axis in ("x", "y"):
            for w in windows:
                wx, wy = (w, 1) if axis == "x" else (1, w)
                r = {"axis": axis, "w": w,
                     "kernel": morph.resolve_plan(dname, H, W, wx, wy)["kernel"]}
                # the paper's two methods on the tile kernel (a tile plan keeps the
                # forced direct pass off the wave kernel): the tile the tuned rule for
                # w <= 9 gives
                tw = max(4 * 32 - ((w + 2 + 3) & ~3), (2 * w + 3) & ~3)
                variants = [("auto", {}),
                            ("tile_direct", {"method_x": "direct", "method_y": "direct",
                                             "tile": (tw, 64)}),
                            ("tile_vhgw", {"method_x": "vhgw", "method_y": "vhgw",
                                           "tile": (tw, 64)})]
                if axis == "x" and w <= 128:
                    # vHGW across the wave kernel's lanes, beside its doubling
                    variants.append(("lanes_vhgw", {"method_x": "vhgw"}))
                    variants.append(("lanes_doubling", {"method_x": "doubling"}))
                for name, kw in variants:
                    fns = [(lambda i=i: morph.apply("erode", srcs[i], wx, wy, out=dsts[i], **kw))
                           for i in range(nbuf) for _ in range(20 // nbuf + 1)][:20]
                    r[name + "_us"] = round(_graph_us(torch, fns), 2)
                # the library's own direct and large-window passes, through the
                # thresholds (w <= t: direct)
                if 2 <= w <= PROD_DIRECT_MAX[axis]:
                    for name, thr in (("direct", w), ("large", w - 1)):
                        morph.set_thresholds(dname, thr if axis == "x" else t0[0],
                                             thr if axis == "y" else t0[1])
                        r[name + "_kernel"] = morph.resolve_plan(dname, H, W, wx, wy)["kernel"]
                        fns = [(lambda i=i: morph.apply("erode", srcs[i], wx, wy, out=dsts[i]))
                               for i in range(nbuf) for _ in range(20 // nbuf + 1)][:20]
                        r[name + "_us"] = round(_graph_us(torch, fns), 2)
                    morph.set_thresholds(dname, *t0)
                rows.append(r)
                print(json.dumps(r), flush=True)
    finally:
        morph.set_thresholds(dname, *t0)
    return {"image": [H, W], "dtype": dname, "op": "erode", "thresholds": list(t0),
            "rows": rows}


def crossover(rows, axis, a, b):
    """Smallest swept w > 1 at which method b is faster than method a (None if never)."""
    for r in sorted((r for r in rows if r["axis"] == axis), key=lambda r: r["w"]):
        if r["w"] > 1 and a + "_us" in r and b + "_us" in r and r[b + "_us"] < r[a + "_us"]:
            return r["w"]
    return None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None)
    ap.add_argument("--dtype", default="u8", choices=("u8", "u16"))
    ap.add_argument("--size", default="800x600", help="WxH")
    a = ap.parse_args(argv)
    W, H = (int(v) for v in a.size.split("x"))
    res = sweep(H=H, W=W, dname=a.dtype)
    res["crossovers"] = {
        axis: {"tile_direct_to_vhgw": crossover(res["rows"], axis, "tile_direct", "tile_vhgw"),
               "direct_to_large": crossover(res["rows"], axis, "direct", "large"),
               "doubling_to_lanes_vhgw": crossover(res["rows"], axis, "lanes_doubling",
                                                    "lanes_vhgw")}
        for axis in ("x", "y")}
    print(json.dumps(res["crossovers"]), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
