"""The serving loop on the GPU: a Poisson stream of mixed requests (crops of
device-resident images, erode/dilate/open/close, windows 3..101) where every
result equals the same request run alone (tolerance 0: integer min/max) and a
sample equals the CPU oracle; the byte budget holds."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2002_09474_amd as morph  # noqa: E402
from paper_2002_09474_amd import serve  # noqa: E402


def test_stream_results_equal_alone_and_oracle():
    pool = serve.make_pool(n=3, hw=1024, seed=9)
    budget = 64 << 20
    st, sch = serve.serve(rate=3000.0, duration=0.15, budget=budget, n_streams=3, max_batch=16,
                          seed=9, pool=pool, keep_outputs=lambda r: True)
    assert st["completed"] == st["requests"] > 100 and st["rejected"] == 0
    assert sch.max_inflight_bytes <= budget
    assert st["batches"] > 3
    host = [p.cpu().numpy() for p in pool]
    for k, r in enumerate(sorted(sch.done, key=lambda r: r.rid)):
        src = pool[r.img][r.y:r.y + r.H, r.x:r.x + r.W]
        alone = morph.apply(r.op, src, r.w, r.w)
        torch.cuda.synchronize()
        got = r.out.cpu().numpy()
        assert np.array_equal(got, alone.cpu().numpy()), (r.rid, r.op, r.w, r.H, r.W)
        if k % 15 == 0:
            crop = np.ascontiguousarray(host[r.img][r.y:r.y + r.H, r.x:r.x + r.W])
            want = oracle.apply(r.op, crop, r.w, r.w, method="vhgw", nthreads=8)
            assert np.array_equal(got, want), (r.rid, r.op, r.w)


def test_budget_smaller_than_requests_rejects_them():
    pool = serve.make_pool(n=1, hw=512, seed=3)
    st, sch = serve.serve(rate=2000.0, duration=0.05, budget=100_000, n_streams=2, max_batch=8,
                          seed=3, pool=pool)
    assert st["rejected"] > 0
    assert st["completed"] + st["rejected"] == st["requests"]
    assert sch.max_inflight_bytes <= 100_000


def test_serving_stream_shaped_like_the_request_config():
    """The request configuration's shape: a pool of 4096 x 4096 uint8 images, crops
    with H and W log-uniform 128..4096, odd windows 3..101, erosion, dilation,
    opening and closing, admission under the 8 GB budget.  Every one of the
    >= 200 results equals the same request run alone, and each equals the CPU
    oracle (tolerance 0)."""
    import os
    pool = serve.make_pool(n=4, hw=4096, seed=6)
    budget = 8 << 30
    st, sch = serve.serve(rate=2000.0, duration=0.12, budget=budget, n_streams=4, max_batch=64,
                          seed=6, pool=pool, keep_outputs=lambda r: True)
    assert st["completed"] == st["requests"] >= 200 and st["rejected"] == 0
    assert sch.max_inflight_bytes <= budget
    done = sorted(sch.done, key=lambda r: r.rid)
    assert {r.op for r in done} == {"erode", "dilate", "open", "close"}
    assert max(r.w for r in done) > 90 and max(max(r.H, r.W) for r in done) > 3000
    host = [p.cpu().numpy() for p in pool]
    nth = os.cpu_count() or 1
    for r in done:
        src = pool[r.img][r.y:r.y + r.H, r.x:r.x + r.W]
        alone = morph.apply(r.op, src, r.w, r.w)
        torch.cuda.synchronize()
        got = r.out.cpu().numpy()
        assert np.array_equal(got, alone.cpu().numpy()), (r.rid, r.op, r.w, r.H, r.W)
        crop = np.ascontiguousarray(host[r.img][r.y:r.y + r.H, r.x:r.x + r.W])
        want = oracle.apply(r.op, crop, r.w, r.w, method="hybrid", nthreads=nth)
        assert np.array_equal(got, want), (r.rid, r.op, r.w, r.H, r.W)


def test_saturating_stream_is_held_to_the_budget():
    """Ten times the configured rate under a 256 MB budget: admission binds (the
    micro-batches hold several requests, in-flight bytes stay within the budget)
    and every request completes with the result it has alone."""
    pool = serve.make_pool(n=2, hw=4096, seed=8)
    budget = 256 << 20
    st, sch = serve.serve(rate=20000.0, duration=0.03, budget=budget, n_streams=4,
                          max_batch=64, seed=8, pool=pool, keep_outputs=lambda r: True)
    assert st["completed"] + st["rejected"] == st["requests"] > 400
    assert sch.max_inflight_bytes <= budget
    assert st["mean_batch"] > 2.0, st
    for r in sorted(sch.done, key=lambda r: r.rid)[::7]:
        src = pool[r.img][r.y:r.y + r.H, r.x:r.x + r.W]
        alone = morph.apply(r.op, src, r.w, r.w)
        torch.cuda.synchronize()
        assert np.array_equal(r.out.cpu().numpy(), alone.cpu().numpy()), (r.rid, r.op, r.w)
