"""The autotuner on the GPU, on its reduced grid (a few windows and choices per key
on smaller images): it runs end to end, writes a table the library loads, and with
that table loaded the results of single images (windows on both sides of the
measured thresholds; openings and closings, one-pass windows among them) and of a
mixed batch still equal the CPU oracle bit for bit.
The package's default table is restored afterwards."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2002_09474_amd as morph  # noqa: E402
from paper_2002_09474_amd import autotune, synth  # noqa: E402
from gpuutil import to_dev, to_host  # noqa: E402


def test_reduced_tuning_table_loads_and_keeps_results(tmp_path):
    out = tmp_path / "tuning.json"
    try:
        res = autotune.tune(str(out), reduced=True)
        table = json.loads(out.read_text())
        for d in ("u8", "u16"):
            t = table[d]
            assert 1 <= t["t_x"] <= autotune.DIRECT_MAX["x"]
            assert 1 <= t["t_y"] <= autotune.DIRECT_MAX["y"]
            assert t["tiles"] and all(r["tq"] >= 2 for r in t["tiles"])
            assert morph.get_thresholds(d) == (t["t_x"], t["t_y"])  # loaded
            assert t["oc_rows"] % 8 == 0 and t["oc_rows_tall"] % 8 == 0
            assert t["oc_one_pass"] in (0, 1)
            assert len(res[d + "_pass_sweep"]) == 10
        for dt, seed in ((np.uint8, 41), (np.uint16, 42)):
            dn = "u8" if dt == np.uint8 else "u16"
            tx, ty = morph.get_thresholds(dn)
            img = synth.uniform(333, 517, dt, seed=seed)
            d, _ = to_dev(img)
            for wx, wy in ((tx, ty), (tx + 1, ty + 1), (max(1, tx - 1), ty), (3, 3), (31, 31),
                           (200, 1), (1, 101), (15, 15), (9, 12)):
                for op in ("erode", "dilate", "open", "close"):
                    got = to_host(morph.apply(op, d, wx, wy))
                    torch.cuda.synchronize()
                    want = oracle.apply(op, img, wx, wy, method="vhgw", nthreads=8)
                    assert np.array_equal(got, want), (dn, op, wx, wy)
        specs = synth.batch_specs(40, seed=43, hi=400)
        imgs = synth.batch_images(specs, seed=43)
        items = []
        for s, im in zip(specs, imgs):
            src, _ = to_dev(im, pitch_elems=(s["W"] + 63) // 64 * 64)
            dst, _ = to_dev(np.zeros_like(im), pitch_elems=(s["W"] + 63) // 64 * 64)
            items.append(dict(img=im, src=src, dst=dst, wx=s["w"], wy=s["w"], op=s["op"]))
        b = morph.Batch(64, 1 << 20)
        b.set(items)
        b.enqueue()
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            want = oracle.apply(it["op"], it["img"], it["wx"], it["wy"], method="vhgw", nthreads=8)
            assert np.array_equal(to_host(it["dst"]), want), k
        b.close()
    finally:
        morph.load_tuning(None)
