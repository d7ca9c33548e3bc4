"""Continuous-batching server for parameter-sweep discharges.

Requests (arrival time, configuration, number of steps) are admitted into the
slots of one library context as they arrive, while earlier requests are still
running: every admitted discharge advances in the same device steps as the
others, its particles stay in HBM between steps, and when it reaches its last
step its RF-averaged profiles are read back and its slot and memory are
returned to the pool for the next request.

Admission is first-come first-served and budgeted by HBM footprint: the head
of the queue is admitted when a slot is free and the pool's largest free block
holds the bytes its configuration needs (``slot_bytes``).  A request larger
than the whole pool is rejected.  The device is stepped in chunks that end
when the next running request is due to finish (at most ``chunk_max`` steps),
so finished requests leave, and waiting ones enter, at chunk boundaries.

Latency of a request = completion time - arrival time, on the host's
monotonic clock; completion is when its profiles are on the host.

The scheduling logic talks to a backend with the methods of ``GpuBackend``;
tests drive it with a host-side fake to check admission and accounting.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    cfg: dict
    steps: int
    admitted: float = -1.0
    done: float = -1.0
    slot: int = -1
    k: int = 0
    status: str = "waiting"  # waiting | running | done | rejected | failed
    result: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.done - self.arrival if self.done >= 0 else float("nan")


class GpuBackend:
    """The library context as the server's backend: ``n_slots`` empty slots
    over an arena whose pool holds ``pool_bytes``."""

    def __init__(self, n_slots, pool_bytes, precision=1):
        from . import _lib
        from .configs import base
        empty = base(n_cells=0, precision=precision)
        self._lib = _lib
        self.ctx = _lib.Context([empty] * n_slots, pool_bytes=pool_bytes)

    def slot_bytes(self, cfg):
        return self._lib.slot_bytes(cfg)

    def pool_free(self):
        return self.ctx.pool_free()

    def admit(self, slot, cfg):
        """Place cfg in slot; False when the pool cannot hold it."""
        return self.ctx.slot_reset(slot, cfg) == self._lib.PIC_OK

    def step(self, n):
        self.ctx.step(n)

    def collect(self, slot):
        """Profiles and counters of a finished discharge (synchronises)."""
        d = self.ctx.diagnostics(slot, allow_error=True)
        out = dict(self.ctx.profiles(slot))
        out["status"] = int(d["return_status"])
        out["particle_steps"] = int(d["particle_steps"])
        out["step"] = int(d["step"])
        return out

    def release(self, slot):
        self.ctx.slot_release(slot)

    def close(self):
        self.ctx.close()


class Server:
    def __init__(self, backend, n_slots, chunk_max=200, clock=time.monotonic, sleep=time.sleep):
        self.b = backend
        self.n_slots = n_slots
        self.chunk_max = chunk_max
        self.clock = clock
        self.sleep = sleep
        self.device_steps = 0
        self.chunks = 0

    def run(self, trace):
        """Serve ``trace`` (iterable of (arrival_s, cfg, steps)) in real time;
        returns the requests with their timings and results."""
        reqs = [Request(i, float(t), dict(cfg), int(n)) for i, (t, cfg, n) in enumerate(trace)]
        pending = deque(sorted(reqs, key=lambda r: (r.arrival, r.rid)))
        queue = deque()
        active = {}
        free = list(range(self.n_slots - 1, -1, -1))
        t0 = self.clock()

        def now():
            return self.clock() - t0

        while pending or queue or active:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            # Admission: FIFO, while a slot is free and the pool holds the head.
            while queue and free:
                r = queue[0]
                need = self.b.slot_bytes(r.cfg)
                if need > self.b.pool_free():
                    if not active:      # nothing will ever free more memory
                        queue.popleft()
                        r.status = "rejected"
                        r.done = now()
                        continue
                    break
                slot = free.pop()
                if not self.b.admit(slot, r.cfg):
                    free.append(slot)
                    if not active:
                        queue.popleft()
                        r.status = "rejected"
                        r.done = now()
                        continue
                    break
                queue.popleft()
                r.slot, r.k, r.status, r.admitted = slot, 0, "running", now()
                active[slot] = r
            if not active:
                if pending and not queue:
                    self.sleep(max(0.0, pending[0].arrival - now()))
                continue
            n = min(self.chunk_max, min(r.steps - r.k for r in active.values()))
            self.b.step(n)
            self.device_steps += n
            self.chunks += 1
            for slot in list(active):
                r = active[slot]
                r.k += n
                if r.k >= r.steps:
                    r.result = self.b.collect(slot)
                    r.done = now()
                    r.status = "done" if r.result.get("status", 0) == 0 else "failed"
                    self.b.release(slot)
                    free.append(slot)
                    del active[slot]
        return reqs


def summarise(reqs, wall_s):
    """p50 / p99 latency, throughput and counts of a served trace."""
    import numpy as np
    done = [r for r in reqs if r.status == "done"]
    lat = np.array([r.latency for r in done]) if done else np.array([float("nan")])
    ps = sum(r.result.get("particle_steps", 0) for r in done)
    return dict(requests=len(reqs), completed=len(done),
                rejected=sum(r.status == "rejected" for r in reqs),
                failed=sum(r.status == "failed" for r in reqs),
                failures=[dict(rid=r.rid, status=r.result.get("status"), step=r.result.get("step"),
                               steps=r.steps, cells=r.cfg.get("n_cells"),
                               n_per_species=r.cfg.get("n_per_species"), v_rf=r.cfg.get("v_rf"),
                               p_pa=r.cfg.get("p_pa"))
                          for r in reqs if r.status == "failed"],
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_queue_s=float(np.mean([r.admitted - r.arrival for r in done])) if done else None,
                particle_steps=int(ps), wall_s=wall_s,
                throughput=ps / wall_s if wall_s > 0 else None)
