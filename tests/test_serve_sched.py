"""The serving scheduler on the CPU with a fake executor and a fake clock:
arrival-order admission, the byte budget is never exceeded, requests larger than
the budget are rejected without blocking others, completion releases bytes and
admits waiting requests, and latencies come from the clock."""
import math

from paper_2002_09474_amd.serve import Request, Scheduler


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Each micro-batch takes `cost` seconds per request after launch; `slots`
    batches may run at once."""

    def __init__(self, clock, slots=2, cost=1e-3):
        self.clock, self.slots, self.cost = clock, slots, cost
        self.running = []
        self.launched = []

    @staticmethod
    def need_bytes(r):
        return r.H * r.W * (2 if r.op in ("open", "close") else 1)

    def has_slot(self):
        return len(self.running) < self.slots

    def launch(self, reqs):
        h = {"end": self.clock() + self.cost * len(reqs), "reqs": [r.rid for r in reqs]}
        self.running.append(h)
        self.launched.append(h["reqs"])
        return h

    def finished(self, h):
        return self.clock() >= h["end"]

    def release(self, h):
        self.running.remove(h)


def _req(i, t, H=10, W=10, op="erode"):
    return Request(rid=i, t_arrive=t, img=0, y=0, x=0, H=H, W=W, w=3, op=op)


def test_fifo_budget_and_release():
    clk = FakeClock()
    ex = FakeExecutor(clk, slots=2, cost=1e-3)
    sch = Scheduler(ex, budget_bytes=350, max_batch=8, clock=clk)
    reqs = [_req(i, 0.0001 * i) for i in range(40)]  # 100 bytes each, 3 fit at once
    st = sch.run(reqs, sleep=clk.sleep)
    assert st["completed"] == 40 and st["rejected"] == 0
    assert sch.max_inflight_bytes <= 350
    order = [rid for batch in ex.launched for rid in batch]
    assert order == sorted(order)  # admitted in arrival order
    assert all(len(b) <= 3 for b in ex.launched)
    assert all(r.t_done >= r.t_admit >= r.t_arrive for r in sch.done)
    assert st["p50_ms"] is not None and st["p99_ms"] >= st["p50_ms"]


def test_oversized_request_is_rejected_without_blocking():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, budget_bytes=1000, clock=clk)
    reqs = [_req(0, 0.0), _req(1, 0.0, H=40, W=40), _req(2, 0.0), _req(3, 0.0, H=10, W=30, op="open")]
    st = sch.run(reqs, sleep=clk.sleep)
    assert [r.rid for r in sch.rejected] == [1]
    assert sorted(r.rid for r in sch.done) == [0, 2, 3]
    assert st["rejected"] == 1


def test_big_request_waits_for_memory_and_keeps_its_place():
    clk = FakeClock()
    ex = FakeExecutor(clk, slots=4, cost=1e-2)
    sch = Scheduler(ex, budget_bytes=500, max_batch=16, clock=clk)
    # r0 fills 400 B; r1 needs 400 B and must wait; r2 (100 B) arrives later and must
    # not overtake r1
    reqs = [_req(0, 0.0, H=20, W=20), _req(1, 0.001, H=20, W=20), _req(2, 0.002)]
    sch.run(reqs, sleep=clk.sleep)
    by = {r.rid: r for r in sch.done}
    assert by[1].t_admit >= by[0].t_done
    assert by[2].t_admit >= by[1].t_admit
    assert sch.max_inflight_bytes <= 500


def test_continuous_batching_overlaps_micro_batches():
    clk = FakeClock()
    ex = FakeExecutor(clk, slots=3, cost=5e-3)
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_batch=4, clock=clk)
    reqs = [_req(i, 0.001 * i) for i in range(30)]
    st = sch.run(reqs, sleep=clk.sleep)
    assert st["completed"] == 30
    assert st["batches"] >= 8
    # with 3 slots more than one micro-batch ran at the same time at some point
    assert max(len(b) for b in ex.launched) <= 4


def test_stats_percentiles():
    clk = FakeClock()
    sch = Scheduler(FakeExecutor(clk), budget_bytes=10 ** 6, clock=clk)
    for i, lat in enumerate([1.0, 2.0, 3.0, 4.0]):
        r = _req(i, 0.0)
        r.t_done = lat
        sch.done.append(r)
    st = sch.stats(10.0)
    assert math.isclose(st["p50_ms"], 2000.0) and math.isclose(st["p99_ms"], 4000.0)
