"""Admission and accounting of the continuous-batching server, driven by a
host-side fake backend and a simulated clock (no GPU)."""
import math

import pytest

from paper_2308_13092_amd.serve import Server, summarise


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeBackend:
    """Pool of ``budget`` bytes; a step costs ``sec_per_step`` of simulated
    time whatever the number of running discharges (they share the device)."""

    def __init__(self, clock, budget, sec_per_step=1e-3):
        self.clock = clock
        self.budget = budget
        self.used = 0
        self.max_used = 0
        self.sec_per_step = sec_per_step
        self.slots = {}
        self.max_running = 0
        self.log = []

    def slot_bytes(self, cfg):
        return cfg["bytes"]

    def pool_free(self):
        return self.budget - self.used

    def admit(self, slot, cfg):
        assert slot not in self.slots
        if cfg["bytes"] > self.pool_free():
            return False
        self.used += cfg["bytes"]
        self.max_used = max(self.max_used, self.used)
        self.slots[slot] = dict(cfg=cfg, k=0)
        self.max_running = max(self.max_running, len(self.slots))
        self.log.append(("admit", cfg["name"], self.clock.t))
        return True

    def step(self, n):
        assert n > 0 and self.slots
        for s in self.slots.values():
            s["k"] = min(s["k"] + n, s["cfg"]["steps"])
        self.clock.t += n * self.sec_per_step

    def collect(self, slot):
        s = self.slots[slot]
        return dict(status=0, step=s["k"], particle_steps=s["k"] * s["cfg"]["np"],
                    name=s["cfg"]["name"])

    def release(self, slot):
        s = self.slots.pop(slot)
        self.used -= s["cfg"]["bytes"]
        self.log.append(("release", s["cfg"]["name"], self.clock.t))


def trace_of(specs):
    return [(t, dict(name=i, bytes=b, steps=n, np=100), n) for i, (t, b, n) in enumerate(specs)]


def serve(specs, budget, n_slots, chunk_max=50):
    clk = Clock()
    fb = FakeBackend(clk, budget)
    srv = Server(fb, n_slots, chunk_max=chunk_max, clock=clk, sleep=clk.sleep)
    reqs = srv.run(trace_of(specs))
    return reqs, fb, srv, clk


def test_every_request_runs_exactly_its_steps():
    specs = [(0.0, 10, 120), (0.01, 20, 30), (0.02, 10, 300), (0.5, 5, 7)]
    reqs, fb, srv, clk = serve(specs, budget=100, n_slots=4)
    for r in reqs:
        assert r.status == "done"
        assert r.result["step"] == r.steps
        assert r.arrival <= r.admitted <= r.done
    assert fb.used == 0 and not fb.slots


def test_budget_and_slots_are_respected():
    specs = [(0.001 * i, 30 + 7 * (i % 3), 50 + 10 * i) for i in range(20)]
    reqs, fb, srv, clk = serve(specs, budget=100, n_slots=3)
    assert fb.max_used <= 100
    assert fb.max_running <= 3
    assert all(r.status == "done" for r in reqs)


def test_admission_is_first_come_first_served():
    specs = [(0.0, 60, 100), (0.001, 60, 10), (0.002, 10, 10)]
    reqs, fb, srv, clk = serve(specs, budget=100, n_slots=4)
    admits = [name for ev, name, _ in fb.log if ev == "admit"]
    assert admits == [0, 1, 2]
    # request 2 fits beside 0 but waits behind 1 (no overtaking)
    assert reqs[2].admitted >= reqs[1].admitted


def test_requests_overlap_on_the_device():
    """A request arriving while another runs joins it before it finishes."""
    specs = [(0.0, 10, 1000), (0.05, 10, 100)]
    reqs, fb, srv, clk = serve(specs, budget=100, n_slots=2)
    assert reqs[1].admitted < reqs[0].done
    assert reqs[1].done < reqs[0].done
    # it waited at most one chunk for admission
    assert reqs[1].admitted - reqs[1].arrival <= 50 * 1e-3 + 1e-9


def test_oversized_request_is_rejected_and_others_served():
    specs = [(0.0, 10, 20), (0.0, 500, 20), (0.1, 10, 20)]
    reqs, fb, srv, clk = serve(specs, budget=100, n_slots=2)
    assert [r.status for r in reqs] == ["done", "rejected", "done"]


def test_idle_server_waits_for_arrivals():
    specs = [(1.0, 10, 10), (2.0, 10, 10)]
    reqs, fb, srv, clk = serve(specs, budget=100, n_slots=1)
    assert reqs[0].admitted >= 1.0 and reqs[1].admitted >= 2.0
    assert srv.device_steps == 20


def test_summary_percentiles():
    specs = [(0.0, 10, 10 * (i + 1)) for i in range(10)]
    reqs, fb, srv, clk = serve(specs, budget=1000, n_slots=10)
    s = summarise(reqs, clk.t)
    lat = sorted(r.latency for r in reqs)
    assert s["completed"] == 10
    assert s["p50_s"] == pytest.approx((lat[4] + lat[5]) / 2)
    assert s["p99_s"] <= lat[-1] + 1e-12
    assert s["particle_steps"] == sum(100 * r.steps for r in reqs)
    assert math.isclose(s["throughput"], s["particle_steps"] / clk.t)
