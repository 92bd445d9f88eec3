"""Scheduler logic of the continuous-batching service, on the CPU with fake
instances (no GPU): admission by footprint, slot limit, rejection of
requests larger than the budget, latency accounting and retirement."""

import threading
import time

import numpy as np

from paper_1511_08463_amd import serving


class FakeInstance:
    live = 0
    peak = 0
    lock = threading.Lock()

    def __init__(self, req, device):
        with FakeInstance.lock:
            FakeInstance.live += 1
            FakeInstance.peak = max(FakeInstance.peak, FakeInstance.live)
        self.req = req
        self.t = None

    def set_load(self, t):
        self.t = t

    def solve_step(self, raise_on_error=True):
        time.sleep(0.002 * self.req.params["cost"])
        code = -3 if self.req.params.get("fail_at") == self.t else 0
        return {"code": code, "sweeps": 1}

    def state(self):
        return (np.array([self.t]), None, None)

    def close(self):
        with FakeInstance.lock:
            FakeInstance.live -= 1


def _reqs():
    rng = np.random.default_rng(0)
    out = []
    t = 0.0
    for rid in range(12):
        t += rng.exponential(0.002)
        out.append(serving.Request(rid, {"mem": int(rng.integers(1, 4)), "cost": 1}, None,
                                   [0.1 * k for k in range(1, 5)], t))
    out.append(serving.Request(99, {"mem": 50, "cost": 1}, None, [0.1], t))    # too big
    out.append(serving.Request(98, {"mem": 1, "cost": 1, "fail_at": 0.2}, None,
                               [0.1, 0.2, 0.3], t))                           # fails at step 2
    return out


def test_admission_budget_slots_and_rejection():
    FakeInstance.live = FakeInstance.peak = 0
    svc = serving.Service(budget_bytes=5, max_slots=3, workers=3, factory=FakeInstance,
                          size_of=lambda p: p["mem"], keep_state=True)
    summary, results = svc.run(_reqs())
    assert summary["rejected"] == [99]
    assert summary["peak_used_bytes"] <= 5
    assert FakeInstance.peak <= 3 and FakeInstance.live == 0
    for rid in range(12):
        r = results[rid]
        assert len(r.latencies) == 4 and all(x > 0 for x in r.latencies)
        assert r.state[0][0] == 0.4                     # ran its whole load path in order
    assert results[98].codes == [0, -3]                 # retired on the failing step
    assert summary["failed_steps"] == 1
    assert summary["steps"] == 12 * 4 + 2
    assert summary["p99_ms"] >= summary["p50_ms"] > 0


def test_fifo_admission_waits_for_memory():
    """A big request at the head of the queue is admitted once memory frees,
    before later small ones (first come, first served)."""
    reqs = [serving.Request(0, {"mem": 4, "cost": 5}, None, [0.1, 0.2], 0.0),
            serving.Request(1, {"mem": 4, "cost": 1}, None, [0.1], 0.001),
            serving.Request(2, {"mem": 1, "cost": 1}, None, [0.1], 0.002)]
    svc = serving.Service(budget_bytes=5, max_slots=4, workers=2, factory=FakeInstance,
                          size_of=lambda p: p["mem"])
    _, results = svc.run(reqs)
    assert results[1].admitted_at >= results[0].finished_at - 1e-6
    assert results[2].admitted_at >= results[1].admitted_at
