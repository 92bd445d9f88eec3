"""The continuous-batching service on the GPU: instances of uneven sizes run
concurrently on their own streams under a memory budget, and each result is
bitwise equal to the same request run alone."""

import numpy as np
import pytest

from paper_1511_08463_amd import serving, workloads

pytestmark = pytest.mark.gpu


def _requests(n, steps=4, seed=3):
    out = []
    for r in workloads.config5(n_instances=n, seed=seed, sizes=(32, 64, 128), rate=400.0):
        out.append(serving.Request(r["rid"], r["params"], r["notch"], r["loads"][:steps], r["arrival"]))
    return out


def test_served_results_equal_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    reqs = _requests(8)
    fps = sorted(serving.footprint(r.params) for r in reqs)
    budget = sum(fps[-3:])                       # forces queueing behind the budget
    print(f"[serving] budget {budget / 1e6:.1f} MB for {len(reqs)} requests", flush=True)
    svc = serving.Service(budget, max_slots=4, workers=4, keep_state=True)
    summary, results = svc.run(reqs)
    print(f"  {summary}", flush=True)
    assert summary["failed_steps"] == 0 and not summary["rejected"]
    assert summary["peak_used_bytes"] <= budget
    for r in reqs[:4]:
        alone, _ = serving.run_alone(r)
        mixed = results[r.rid].state
        for a, b in zip(alone, mixed):
            assert np.array_equal(a, b), r.rid
