"""GPU parity of the batched persistent launch: every image of a mixed batch (sizes,
windows, anchors, ops, uint8 and uint16, aligned and unaligned rows) equals the
CPU oracle and the single-image call, on the first launch and on graph replays,
after re-setting the batch to a smaller one, and on a non-default stream."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2002_09474_amd as morph  # noqa: E402
from paper_2002_09474_amd import synth  # noqa: E402
from gpuutil import to_dev, to_host  # noqa: E402


def _items(n, seed, dtype_mix=True):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        H = int(rng.integers(1, 300))
        W = int(rng.integers(1, 300))
        dt = np.uint16 if (dtype_mix and i % 3 == 2) else np.uint8
        img = synth.uniform(H, W, dt, seed=seed * 1000 + i)
        w = int(rng.choice([1, 2, 3, 5, 9, 15, 31, 63, 200, 400]))
        # (wide windows along rows: the wide-row kernel for uint8)
        wy = 1 if w > 128 else int(rng.choice([w, 1, 3]))
        ax = int(rng.integers(-1, w))
        ay = int(rng.integers(-1, wy))
        op = "erode" if rng.integers(0, 2) else "dilate"
        pitch = W + int(rng.choice([0, 0, 1, 3, 61]))
        off = int(rng.choice([0, 0, 1]))
        src, _ = to_dev(img, pitch_elems=pitch, offset_elems=off)
        # the destination may have a row pitch of its own
        dpitch = W + int(rng.choice([0, 5, 64])) if i % 2 else pitch
        dst, _ = to_dev(np.zeros_like(img), pitch_elems=dpitch, offset_elems=off)
        out.append(dict(img=img, src=src, dst=dst, wx=w, wy=wy, ax=ax, ay=ay, op=op))
    return out


def _want(it):
    return oracle.morph(it["img"], 0 if it["op"] == "erode" else 1, it["wx"], it["wy"],
                        it["ax"], it["ay"], method="direct")


@pytest.mark.parametrize("fuse,fit,ty,coop", [(1, 1, 0, 0), (0, 1, 0, 0), (1, 0, 0, 0),
                                              (1, 1, 31, 0), (0, 1, 31, 0), (1, 1, 0, 17),
                                              (1, 0, 16, 17)])
def test_batch_matches_oracle_and_single_calls(fuse, fit, ty, coop, tmp_path):
    """With the wave and streaming groups fused into one dispatch per element type
    and row alignment (the default) and launched one group at a time; with units
    shortened to fill the GPU (the default for a batch this small) and at the tuned
    batch heights; with vertical windows up to 31 direct (the wave kernel's tall
    form, a dispatch of its own); with the run-total streaming units in the cooperative
    form (a dispatch of its own, 4 and 8 waves a unit)."""
    import json
    f = tmp_path / "t.json"
    t = {"fuse": fuse, "fit_units": fit}
    if ty:
        t["batch_t_y"] = ty
    if coop:
        t.update(batch_coop_min_wy=coop, batch_coop_rows=24 if fit else 64,
                 batch_coop_waves=4 if fit else 8)
    f.write_text(json.dumps({"u8": t, "u16": t}))
    morph.load_tuning(str(f))
    try:
        _batch_matches_oracle_and_single_calls()
    finally:
        morph.load_tuning(None)


def _batch_matches_oracle_and_single_calls():
    items = _items(40, seed=1)
    b = morph.Batch(64, 1 << 20)
    ntiles = b.set(items)
    assert ntiles > len(items) // 2
    for rep in range(3):  # first launch captures the graph, then two replays
        for it in items:
            it["dst"].zero_()
        torch.cuda.synchronize()
        b.enqueue()
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            got = to_host(it["dst"])
            assert np.array_equal(got, _want(it)), (rep, k, it["img"].shape, it["wx"], it["wy"])
    # the single-image call gives the same bytes
    for it in items[:10]:
        single = morph.apply(it["op"], it["src"], it["wx"], it["wy"], it["ax"], it["ay"])
        torch.cuda.synchronize()
        assert np.array_equal(to_host(single), to_host(it["dst"]))
    # a smaller batch on the same object, on another stream
    small = _items(5, seed=2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.set(small, stream=s)
        b.enqueue(stream=s)
        b.enqueue(stream=s)
    s.synchronize()
    for it in small:
        assert np.array_equal(to_host(it["dst"]), _want(it))
    b.close()


def test_batch_limits_and_errors():
    items = _items(3, seed=3, dtype_mix=False)
    b = morph.Batch(2, 1 << 20)
    with pytest.raises(morph.MorphError) as ei:
        b.set(items)
    assert ei.value.status == -5  # too many images
    b.close()
    b = morph.Batch(8, 1)
    with pytest.raises(morph.MorphError) as ei:
        b.set(items)
    assert ei.value.status == -5  # too many tiles
    b.close()
    b = morph.Batch(8, 1 << 20)
    bad = dict(items[0])
    bad["dst"] = bad["src"]
    with pytest.raises(morph.MorphError) as ei:
        b.set([bad])
    assert ei.value.status == -2  # src and dst overlap
    assert b.set([]) == 0
    b.enqueue()  # empty batch: nothing to do
    b.close()


def test_batch_of_document_images_like_the_benchmark():
    specs = synth.batch_specs(24, seed=5, hi=700)
    imgs = synth.batch_images(specs, seed=5)
    items = []
    for s, im in zip(specs, imgs):
        src, _ = to_dev(im, pitch_elems=(s["W"] + 63) // 64 * 64)
        dst, _ = to_dev(np.zeros_like(im), pitch_elems=(s["W"] + 63) // 64 * 64)
        items.append(dict(img=im, src=src, dst=dst, wx=s["w"], wy=s["w"], ax=-1, ay=-1,
                          op=s["op"]))
    b = morph.Batch(32, 1 << 20)
    b.set(items)
    b.enqueue()
    torch.cuda.synchronize()
    for it in items:
        assert np.array_equal(to_host(it["dst"]), _want(it))
    b.close()


def test_batch_with_many_wave_units(tmp_path):
    """A batch whose direct-window images give far more wave units than the chip
    holds waves at once (16 images of about 1000x1000 with 3x3 and 9x9 windows in
    8-row units: over 9000 units), mixed with 31x31 images on the streaming kernel:
    every unit is done."""
    import json
    f = tmp_path / "t.json"
    f.write_text(json.dumps({"u8": {"batch_wave_rows": 8}}))
    morph.load_tuning(str(f))
    try:
        items = []
        for i in range(24):
            img = synth.uniform(1000, 1000 - 3 * i, np.uint8, seed=4000 + i)
            src, _ = to_dev(img, pitch_elems=1024)
            dst, _ = to_dev(np.zeros_like(img), pitch_elems=1024)
            w = (3, 9, 31)[i % 3]
            items.append(dict(img=img, src=src, dst=dst, wx=w, wy=w, ax=-1, ay=-1,
                              op="erode" if i % 2 else "dilate"))
        b = morph.Batch(32, 1 << 20)
        assert b.set(items) > 9000  # wave units alone: more than 8192
        b.enqueue()
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            assert np.array_equal(to_host(it["dst"]), _want(it)), k
        b.close()
    finally:
        morph.load_tuning(None)


def _want_any(it):
    return oracle.apply(it["op"], it["img"], it["wx"], it["wy"], it["ax"], it["ay"],
                        method="vhgw" if max(it["wx"], it["wy"]) > 15 else "direct")


def test_batch_openings_and_closings_with_workspace():
    """Openings and closings as batch descriptors (§2: the dilation of the erosion and
    the erosion of the dilation, same rectangle and anchor), mixed with erosions and
    dilations, uint8 and uint16, odd pitches: the first operation into the enqueue
    workspace, the second from it, in one graph; each image equals the oracle and its
    single-image call, on the first launch, on a replay, and after the workspace is
    replaced by another buffer (the job table is rewritten, the graph kept)."""
    items = _items(36, seed=11)
    rng = np.random.default_rng(11)
    for it in items:
        it["op"] = str(rng.choice(["erode", "dilate", "open", "close", "open", "close"]))
    b = morph.Batch(64, 1 << 20)
    b.set(items)
    need = b.workspace_bytes
    n_oc = sum(it["op"] in ("open", "close") for it in items)
    assert n_oc > 10 and need > 0
    ws1 = torch.empty(need, dtype=torch.uint8, device="cuda")
    ws2 = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")[1000:1000 + need]
    for rep, ws in enumerate((ws1, ws1, ws2, ws1)):
        for it in items:
            it["dst"].zero_()
        torch.cuda.synchronize()
        b.enqueue(workspace=ws)
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            got = to_host(it["dst"])
            assert np.array_equal(got, _want_any(it)), (rep, k, it["op"], it["img"].shape,
                                                       it["wx"], it["wy"], it["ax"], it["ay"])
    for it in items[:12]:
        single = morph.apply(it["op"], it["src"], it["wx"], it["wy"], it["ax"], it["ay"])
        torch.cuda.synchronize()
        assert np.array_equal(to_host(single), to_host(it["dst"]))
    # a plain launch (no graph) with the binding's own workspace
    for it in items:
        it["dst"].zero_()
    b.launch()
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        assert np.array_equal(to_host(it["dst"]), _want_any(it)), ("launch", k)
    # workspace too small, missing, or overlapping an image of the batch
    for bad in (ws1[:need - 1], None):
        ptr = 0 if bad is None else bad.data_ptr()
        nb = 0 if bad is None else bad.numel()
        rc = morph._lib.lib().morph_batch_enqueue(b._h, ptr or None, nb, None)
        assert rc == -5, rc
    src0 = items[0]["src"]
    base = src0.data_ptr()
    rc = morph._lib.lib().morph_batch_enqueue(b._h, base, need, None)
    assert rc == -2, rc
    b.close()


def test_bench_batch_matches_oracle():
    """The benchmark's exact workload: the 512-image batch of document-like pages
    (H, W log-uniform 64..2048, windows 3..63, erosion or dilation; seed 5; 159.85
    Mpx in ~22.8k units) in one pool with 64-byte row pitches, captured then
    replayed; every output pixel of all 512 images equals the oracle's."""
    import os
    import bench
    specs, imgs, items, npx, pools = bench.build_batch(torch, morph, synth, torch.device("cuda"))
    assert len(items) == 512 and npx == 159_850_750
    b = morph.Batch(len(items), 1 << 22)
    assert b.set(items) > 20_000
    dst_pool = pools[1]
    nth = os.cpu_count() or 1
    for rep in range(2):  # capture, then replay into a cleared pool
        dst_pool.fill_(0x5a)
        b.enqueue()
        torch.cuda.synchronize()
        for k, (s, im, it) in enumerate(zip(specs, imgs, items)):
            want = oracle.apply(s["op"], im, s["w"], s["w"], method="hybrid", nthreads=nth)
            assert np.array_equal(to_host(it["dst"]), want), (rep, k, s)
    b.close()
