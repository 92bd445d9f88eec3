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


def test_served_subset_matches_oracle():
    """A seeded subset of the served stream (config-5 recipe: uneven mesh
    sides, ell in [0.01, 0.05], h = ell/4, seeded notches, loads to sqrt(L)),
    run through the service concurrently under a budget with the served
    solver's own settings (ORAM-N, inexact sweeps, stop ||Phi||_2 < 1e-9) in
    float64, against the oracle's ORAM-N (exact solves, the same switch and
    stop tests) on each instance: u and alpha to 1e-6 relative L2 after
    every load step."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import am, problems
    S = workloads.CONFIG2_SOLVER
    reqs = []
    for r in workloads.config5(n_instances=5, seed=11, sizes=(24, 32, 40), rate=400.0):
        p = dict(r["params"], precision=0)
        reqs.append(serving.Request(r["rid"], p, r["notch"], r["loads"][:6], r["arrival"]))
    fps = sorted(serving.footprint(r.params) for r in reqs)
    svc = serving.Service(sum(fps[-2:]), max_slots=3, workers=3, keep_state=True)
    summary, results = svc.run(reqs)
    print(f"[serving/oracle] {summary}", flush=True)
    assert summary["failed_steps"] == 0
    for r in reqs:
        p = r.params
        P = problems.tension_2d(p["nx"], p["ny"], p["lx"], p["ly"], **workloads.oracle_kwargs(p))
        st = am.initial_state(P, r.notch.astype(bool))
        for t in r.loads:
            am.solve_load_step(P, st, t, omega=1.0, newton_on=True, switch_tol=S["switch_tol"],
                               final_tol=S["final_tol"], max_am=20000)
        u, a, _ = results[r.rid].state
        eu = np.linalg.norm(u - st.u) / np.linalg.norm(st.u)
        ea = np.linalg.norm(a - st.alpha) / np.linalg.norm(st.alpha)
        print(f"  rid {r.rid} n={p['nx']} ell={p['ell']:.4f}: rel_u={eu:.2e} rel_a={ea:.2e}",
              flush=True)
        assert eu < 1e-6 and ea < 1e-6
