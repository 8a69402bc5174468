"""Per-pass window sweep in the shape of the paper's own experiment (§5.1.3 and
§5.2.3, Figs. 3-4): one pass at a time on an 800x600 uint8 image, w x 1 (along x)
and 1 x w (along y), w swept, timing the paper's two methods as the workgroup-tile
kernel implements them (direct for w <= 9, vHGW for every w) beside the automatic
choice (wave, streaming or wide-row kernel).  Times are per launch, from 20 launches
over 8 buffer pairs captured in one graph.  Run
``python -m paper_2002_09474_amd.pass_sweep [--out FILE.json]``.
"""
from __future__ import annotations

import argparse
import json
import sys

WINDOWS = (1, 2, 3, 4, 5, 7, 9, 11, 15, 21, 31, 45, 63, 101, 155, 255)


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


def sweep(H=600, W=800, windows=WINDOWS):
    import torch

    import paper_2002_09474_amd as morph
    from paper_2002_09474_amd import synth
    dev = torch.device("cuda")
    img = torch.from_numpy(synth.document(H, W, seed=4)).to(dev)
    nbuf = 8
    srcs = [img.clone() for _ in range(nbuf)]
    dsts = [torch.empty_like(s) for s in srcs]
    rows = []
    for axis in ("x", "y"):
        for w in windows:
            wx, wy = (w, 1) if axis == "x" else (1, w)
            r = {"axis": axis, "w": w, "kernel": morph.resolve_plan("u8", H, W, wx, wy)["kernel"]}
            # the paper's direct pass on the tile kernel needs a tile (forced methods
            # without one plan the wave kernel): the tile the tuned rule for w <= 9 gives
            tw = max(4 * 32 - ((w + 2 + 3) & ~3), (2 * w + 3) & ~3)
            for name, kw in (("auto", {}),
                             ("direct", {"method_x": "direct", "method_y": "direct",
                                         "tile": (tw, 64)}),
                             ("vhgw", {"method_x": "vhgw", "method_y": "vhgw"})):
                if name == "direct" and w > 9:
                    continue
                fns = [(lambda i=i: morph.apply("erode", srcs[i], wx, wy, out=dsts[i], **kw))
                       for i in range(nbuf) for _ in range(20 // nbuf + 1)][:20]
                r[name + "_us"] = round(_graph_us(torch, fns), 2)
            rows.append(r)
            print(json.dumps(r), flush=True)
    return {"image": [H, W], "dtype": "u8", "op": "erode", "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = sweep()
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
