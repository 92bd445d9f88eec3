"""Continuous-batching service for independent fracture simulations.

Requests (one quasi-static load path each, on its own mesh size) arrive over
time.  The scheduler:

* admits a waiting request when its device footprint
  (``fracture_workspace_bytes``) fits in the remaining memory budget and a
  slot is free (first come, first served; a request larger than the whole
  budget is rejected);
* keeps every admitted instance's state (u, alpha, alpha_prev) resident in
  its own device workspace and gives it its own HIP stream;
* runs load steps of whichever admitted instances are ready on a pool of
  host worker threads, so that steps of different instances execute on the
  device at the same time (the solver releases the Python interpreter lock
  inside each call);
* retires an instance after its last step and frees its workspace, which
  lets waiting requests in.

Each step's latency runs from the moment it becomes eligible (the request's
admission for its first step, the previous step's completion otherwise) to
its completion, so waiting for a worker counts; the wait for admission
(arrival to admission) is reported on its own.  Results do not depend on the
mix: every instance computes with its own buffers and fixed-order
reductions.
"""

import dataclasses
import heapq
import threading
import time

import numpy as np

from . import fracture


@dataclasses.dataclass
class Request:
    rid: int
    params: dict
    notch: np.ndarray
    loads: list
    arrival: float                    # seconds after the service starts


@dataclasses.dataclass
class Result:
    rid: int
    latencies: list
    stats: list
    state: tuple = None               # (u, alpha, alpha_prev) when kept
    admitted_at: float = 0.0
    queue_wait: float = 0.0           # arrival to admission, seconds
    finished_at: float = 0.0
    codes: list = dataclasses.field(default_factory=list)


def footprint(params):
    """Device bytes an instance holds while admitted."""
    return fracture.fracture_workspace_bytes(fracture.make_params(**params))


def gpu_instance(req, device):
    """A solver instance with its own HIP stream (default priority)."""
    import torch
    stream = torch.cuda.Stream(device=device)
    return fracture.Fracture(fracture.make_params(**req.params), req.notch, device=device,
                             stream=stream)


class Service:
    def __init__(self, budget_bytes, max_slots=16, workers=4, device="cuda:0", keep_state=False,
                 factory=None, size_of=footprint, progress=None):
        """keep_state: True keeps every request's final (u, alpha, alpha_prev)
        on the host, or a set of request ids keeps those only."""
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.workers = workers
        self.device = device
        self.keep_state = keep_state
        self.factory = factory or gpu_instance
        self.size_of = size_of
        self.progress = progress     # optional callable(finished, total, elapsed_s)

    def run(self, requests):
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        lock = threading.Condition()
        waiting = []                         # arrived, not admitted (FIFO by arrival)
        ready = []                           # heap of (eligible_time, rid)
        active = {}                          # rid -> dict(inst, next_step, eligible)
        results = {r.rid: Result(r.rid, [], []) for r in reqs}
        rejected = []
        used = [0]
        peak = [0]
        pending = list(reqs)
        finished = [0]
        n_total = len(reqs)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        stop = [False]
        error = []

        def admit_locked():
            # arrivals whose time has come join the waiting list
            while pending and pending[0].arrival <= now():
                waiting.append(pending.pop(0))
            while waiting and len(active) < self.max_slots:
                r = waiting[0]
                fp = self.size_of(r.params)
                if fp > self.budget:
                    waiting.pop(0)
                    rejected.append(r.rid)
                    finished[0] += 1
                    continue
                if used[0] + fp > self.budget:
                    break
                waiting.pop(0)
                inst = self.factory(r, self.device)
                used[0] += fp
                peak[0] = max(peak[0], used[0])
                t_adm = now()
                active[r.rid] = dict(req=r, inst=inst, k=0, fp=fp, eligible=t_adm)
                results[r.rid].admitted_at = t_adm
                results[r.rid].queue_wait = max(0.0, t_adm - r.arrival)
                heapq.heappush(ready, (t_adm, r.rid))
            lock.notify_all()

        def worker():
            while True:
                with lock:
                    while not ready and not stop[0]:
                        admit_locked()
                        if ready or stop[0]:
                            break
                        lock.wait(timeout=0.002)
                    if stop[0]:
                        return
                    elig, rid = heapq.heappop(ready)
                    slot = active[rid]
                inst, req, k = slot["inst"], slot["req"], slot["k"]
                try:
                    inst.set_load(req.loads[k])
                    st = inst.solve_step(raise_on_error=False)
                except Exception as e:  # pragma: no cover - surfaced to the caller
                    with lock:
                        error.append(e)
                        stop[0] = True
                        lock.notify_all()
                    return
                done_t = now()
                res = results[rid]
                res.latencies.append(done_t - elig)
                res.stats.append(st)
                res.codes.append(st["code"])
                with lock:
                    slot["k"] += 1
                    if slot["k"] >= len(req.loads) or st["code"] != fracture.FRACTURE_OK:
                        keep = self.keep_state
                        if keep is True or (keep and rid in keep):
                            res.state = inst.state()
                        inst.close()
                        del slot["inst"]
                        used[0] -= slot["fp"]
                        del active[rid]
                        res.finished_at = done_t
                        finished[0] += 1
                        if self.progress is not None:
                            self.progress(finished[0], n_total, done_t)
                        if finished[0] >= n_total:
                            stop[0] = True
                        admit_locked()
                    else:
                        heapq.heappush(ready, (done_t, rid))
                    lock.notify_all()

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.workers)]
        with lock:
            admit_locked()
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if error:
            raise error[0]
        wall = now()
        lat = np.array([x for r in results.values() for x in r.latencies])
        steps = int(lat.size)
        waits = np.array([r.queue_wait for r in results.values() if r.rid not in rejected])
        summary = {
            "peak_used_bytes": peak[0],
            "instances": n_total - len(rejected),
            "rejected": rejected,
            "steps": steps,
            "wall_s": wall,
            "steps_per_s": steps / wall if wall > 0 else 0.0,
            "instances_per_s": (n_total - len(rejected)) / wall if wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if steps else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if steps else None,
            "queue_wait_p50_s": float(np.percentile(waits, 50)) if waits.size else None,
            "queue_wait_p99_s": float(np.percentile(waits, 99)) if waits.size else None,
            "failed_steps": int(sum(c != 0 for r in results.values() for c in r.codes)),
        }
        return summary, results


def run_alone(req, device="cuda:0"):
    """The same request on a fresh instance with nothing else running."""
    inst = fracture.Fracture(fracture.make_params(**req.params), req.notch, device=device)
    stats = []
    for t in req.loads:
        inst.set_load(t)
        stats.append(inst.solve_step(raise_on_error=False))
    state = inst.state()
    inst.close()
    return state, stats
