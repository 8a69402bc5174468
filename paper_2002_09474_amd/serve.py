"""Continuous-batching request loop for erosion / dilation / opening / closing.

Requests (a crop of a device-resident image, a square window, an op) arrive over
time.  The scheduler admits queued requests in arrival order while the device
memory they will hold (output, plus a workspace for opening/closing) fits in a
byte budget and an executor slot is free, groups everything admitted at that
moment into one micro-batch, and hands it to the executor, which runs it on one
of several streams as batched launches.  Work of different micro-batches
overlaps on the device; requests that arrive while others run are admitted as
soon as memory and a slot free up.  Completion releases the bytes and records
the latency (completion minus arrival).

The scheduler holds no GPU code and takes its clock as an argument, so its
admission and ordering logic can be exercised with a fake executor and a fake
clock.  ``GpuExecutor`` is the real executor (HIP batch launches through the C
ABI).  Run ``python -m paper_2002_09474_amd.serve`` for the Poisson stream.
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import time
from dataclasses import dataclass, field

OPS = ("erode", "dilate", "open", "close")


@dataclass
class Request:
    rid: int
    t_arrive: float
    img: int
    y: int
    x: int
    H: int
    W: int
    w: int
    op: str
    need: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    status: str = "new"
    out: object = field(default=None, repr=False)

    @property
    def pixels(self) -> int:
        return self.H * self.W


class Scheduler:
    """Byte-budget admission, FIFO order, continuous micro-batching."""

    def __init__(self, executor, budget_bytes: int, max_batch: int = 64, clock=time.perf_counter,
                 keep_outputs=None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.keep_outputs = keep_outputs or (lambda r: False)
        self.queue = collections.deque()
        self.inflight = []  # (handle, [requests])
        self.inflight_bytes = 0
        self.max_inflight_bytes = 0
        self.done = []
        self.rejected = []
        self.batches = 0

    def submit(self, req: Request) -> None:
        req.need = self.ex.need_bytes(req)
        if req.need > self.budget:
            req.status = "rejected"
            self.rejected.append(req)
            return
        req.status = "queued"
        self.queue.append(req)

    def poll(self) -> int:
        """Retire finished micro-batches; returns how many requests completed."""
        n = 0
        still = []
        for handle, reqs in self.inflight:
            if self.ex.finished(handle):
                now = self.clock()
                for r in reqs:
                    r.t_done = now
                    r.status = "done"
                    self.inflight_bytes -= r.need
                    if not self.keep_outputs(r):
                        r.out = None
                    self.done.append(r)
                    n += 1
                self.ex.release(handle)
            else:
                still.append((handle, reqs))
        self.inflight = still
        return n

    def admit(self) -> int:
        """Admit queued requests (in order, stopping at the first that does not fit)
        into one micro-batch if the executor has a free slot."""
        if not self.queue or not self.ex.has_slot():
            return 0
        take = []
        while self.queue and len(take) < self.max_batch:
            r = self.queue[0]
            if self.inflight_bytes + r.need > self.budget:
                break
            self.queue.popleft()
            self.inflight_bytes += r.need
            take.append(r)
        if not take:
            return 0
        now = self.clock()
        for r in take:
            r.t_admit = now
            r.status = "running"
        self.max_inflight_bytes = max(self.max_inflight_bytes, self.inflight_bytes)
        handle = self.ex.launch(take)
        self.inflight.append((handle, take))
        self.batches += 1
        return len(take)

    def step(self) -> bool:
        """One scheduling round; True if anything happened."""
        return bool(self.poll()) | bool(self.admit())

    def idle(self) -> bool:
        return not self.queue and not self.inflight

    def run(self, requests, sleep=time.sleep, poll_interval: float = 50e-6):
        """Feed `requests` (sorted by t_arrive, seconds from the start) in real time
        on this scheduler's clock and run until all are done or rejected."""
        t0 = self.clock()
        i = 0
        n = len(requests)
        while i < n or not self.idle():
            now = self.clock() - t0
            while i < n and requests[i].t_arrive <= now:
                r = requests[i]
                r.t_arrive += t0
                self.submit(r)
                i += 1
            if not self.step():
                nxt = requests[i].t_arrive - now if i < n else poll_interval
                sleep(max(0.0, min(nxt, poll_interval)))
        return self.stats(self.clock() - t0)

    def stats(self, wall: float) -> dict:
        lat = sorted(r.t_done - r.t_arrive for r in self.done)

        def pct(p):
            if not lat:
                return None
            return lat[min(len(lat) - 1, int(math.ceil(p * len(lat))) - 1)]
        px = sum(r.pixels for r in self.done)
        return {"completed": len(self.done), "rejected": len(self.rejected),
                "batches": self.batches, "wall_s": wall,
                "mean_batch": len(self.done) / self.batches if self.batches else None,
                "gpixel_s": px / wall / 1e9 if wall > 0 else None,
                "p50_ms": None if not lat else pct(0.50) * 1e3,
                "p99_ms": None if not lat else pct(0.99) * 1e3,
                "max_inflight_bytes": self.max_inflight_bytes, "budget_bytes": self.budget}


def _pitch(W: int) -> int:
    return (W + 63) // 64 * 64


class GpuExecutor:
    """Runs micro-batches as HIP batch launches on a ring of streams, one batch
    object per stream.  Openings and closings are batch descriptors of their own:
    both operations run in the same launch, the intermediates in a workspace
    allocated per micro-batch and held until it completes."""

    def __init__(self, pool, n_streams: int = 4, max_images: int = 256):
        import torch
        import paper_2002_09474_amd as morph
        self.torch = torch
        self.morph = morph
        self.pool = pool
        self.dev = pool[0].device
        self.slots = []
        for _ in range(n_streams):
            self.slots.append({"stream": torch.cuda.Stream(device=self.dev),
                               "batch": morph.Batch(max_images, 1 << 20),
                               "busy": None})

    @staticmethod
    def need_bytes(req: Request) -> int:
        """Device bytes a request holds while it runs: its output and, for an opening
        or closing, its intermediate in the batch workspace (rows padded to 64
        bytes, the image on a 256-byte boundary)."""
        out = req.H * _pitch(req.W)
        return out + ((out + 255) // 256 * 256 if req.op in ("open", "close") else 0)

    def has_slot(self) -> bool:
        return any(s["busy"] is None for s in self.slots)

    def _alloc(self, H, W):
        buf = self.torch.empty(H * _pitch(W), dtype=self.torch.uint8, device=self.dev)
        return buf.view(H, _pitch(W))[:, :W]

    def launch(self, reqs):
        torch = self.torch
        slot = next(s for s in self.slots if s["busy"] is None)
        st = slot["stream"]
        items = []
        with torch.cuda.stream(st):
            for r in reqs:
                src = self.pool[r.img][r.y:r.y + r.H, r.x:r.x + r.W]
                out = self._alloc(r.H, r.W)
                r.out = out
                items.append(dict(src=src, dst=out, wx=r.w, wy=r.w, op=r.op))
            b = slot["batch"]
            b.set(items, stream=st)
            nws = b.workspace_bytes
            ws = torch.empty(nws, dtype=torch.uint8, device=self.dev) if nws else None
            b.launch(stream=st, workspace=ws)
            ev = torch.cuda.Event()
            ev.record(st)
        slot["busy"] = (ev, ws)
        return slot

    def finished(self, slot) -> bool:
        return slot["busy"][0].query()

    def release(self, slot) -> None:
        slot["busy"] = None


def make_requests(rate: float, duration: float, seed: int = 6, pool_n: int = 32,
                  pool_hw: int = 4096):
    from . import synth
    raw = synth.request_stream(rate, duration, seed=seed, lo=min(128, pool_hw),
                               hi=min(4096, pool_hw), pool_h=pool_hw, pool_w=pool_hw,
                               pool_n=pool_n)
    return [Request(rid=i, t_arrive=d["t"], img=d["img"], y=d["y"], x=d["x"], H=d["H"],
                    W=d["W"], w=d["w"], op=d["op"]) for i, d in enumerate(raw)]


def make_pool(n: int = 32, hw: int = 4096, seed: int = 6):
    """Device-resident source images, uniform uint8 (erosion time does not depend on
    the pixel values)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    return [torch.randint(0, 256, (hw, hw), generator=g, dtype=torch.int32,
                          device="cuda").to(torch.uint8) for _ in range(n)]


def serve(rate=2000.0, duration=60.0, budget=8 << 30, n_streams=4, max_batch=64, seed=6,
          pool_n=32, pool_hw=4096, keep_outputs=None, pool=None):
    import torch
    pool = pool if pool is not None else make_pool(pool_n, pool_hw, seed)
    ex = GpuExecutor(pool, n_streams=n_streams)
    reqs = make_requests(rate, duration, seed=seed, pool_n=len(pool), pool_hw=pool[0].shape[0])
    torch.cuda.synchronize()
    sch = Scheduler(ex, budget, max_batch=max_batch, keep_outputs=keep_outputs)
    st = sch.run(reqs)
    torch.cuda.synchronize()
    st.update({"rate_req_s": rate, "duration_s": duration, "requests": len(reqs),
               "streams": n_streams, "max_batch": max_batch})
    return st, sch


def main(argv=None):
    ap = argparse.ArgumentParser(description="Poisson request stream through the GPU loop")
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--seed", type=int, default=6)
    a = ap.parse_args(argv)
    st, _ = serve(a.rate, a.duration, int(a.budget_gb * (1 << 30)), a.streams, a.max_batch, a.seed)
    print(json.dumps(st), flush=True)


if __name__ == "__main__":
    sys.exit(main())
