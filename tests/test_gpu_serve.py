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
