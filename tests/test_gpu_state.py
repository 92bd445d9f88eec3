"""The carried state of the quasi-static evolution (u_{i-1}, alpha_{i-1}) of
Algorithm 1: checkpoint and resume through get_state/set_state, and the
failure path for non-finite values.

* A handle resumed in a fresh instance from a checkpoint continues the load
  path bit for bit: a load step depends on (u, alpha, alpha_prev, load)
  alone.
* A non-finite damage value makes solve_step return FRACTURE_ENONFINITE and
  leaves the state exactly as it was at entry of the step; after a valid
  state is set the handle solves again.
"""

import numpy as np
import pytest

from paper_1511_08463_amd import fracture, workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bits(v):
    return np.ascontiguousarray(v, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_resume_is_bitwise(precision):
    _torch()
    n = 64
    p, notch, loads, _ = workloads.config2("AT1", 1.0, seed=0, n=n)
    params = fracture.make_params(**p, **workloads.CONFIG2_SOLVER, precision=precision)
    k_ck, k_end = 12, 17        # checkpoint after t = 1.2; the specimen breaks at t = 1.5
    a = fracture.Fracture(params, notch, device="cuda:0")
    for k in range(k_ck):
        a.set_load(loads[k])
        a.solve_step()
    ck = a.state()
    print(f"[resume] {precision}: checkpoint after t={loads[k_ck - 1]:.1f}", flush=True)
    b = fracture.Fracture(params, None, device="cuda:0")
    b.set_state(u=ck[0], alpha=ck[1], alpha_prev=ck[2])
    for k in range(k_ck, k_end):
        a.set_load(loads[k])
        sa = a.solve_step()
        b.set_load(loads[k])
        sb = b.solve_step()
        sta, stb = a.state(), b.state()
        print(f"  t={loads[k]:.1f} sweeps {sa['sweeps']}/{sb['sweeps']} pcg {sa['pcg_iters']}/"
              f"{sb['pcg_iters']} newton {sa['newton_iters']}/{sb['newton_iters']}", flush=True)
        for f in ("sweeps", "pcg_iters", "vi_iters", "vi_cg_iters", "newton_iters", "minres_iters"):
            assert sa[f] == sb[f], (k + 1, f, sa[f], sb[f])
        for va, vb in zip(sta, stb):
            assert np.array_equal(_bits(va), _bits(vb)), k + 1
        assert a.energy() == b.energy()
    # the path went through the propagation: the specimen is cut
    assert np.all((b.state()[1].reshape(n + 1, n + 1) > 0.5).any(axis=0))
    a.close()
    b.close()


def test_nonfinite_damage_rolls_back():
    _torch()
    n = 32
    p, notch, loads, _ = workloads.config2("AT1", 1.0, seed=0, n=n)
    s = fracture.Fracture(fracture.make_params(**p, **workloads.CONFIG2_SOLVER), notch,
                          device="cuda:0")
    for k in range(2):
        s.set_load(loads[k])
        s.solve_step()
    good = s.state()
    bad_alpha = good[1].copy()
    bad_alpha[(n + 1) * (n // 2) + n // 2] = np.nan
    s.set_state(alpha=bad_alpha)
    s.set_load(loads[2])
    entry = s.state()
    st = s.solve_step(raise_on_error=False)
    print(f"[nonfinite] code {st['code']}", flush=True)
    assert st["code"] == fracture.FRACTURE_ENONFINITE
    after = s.state()
    for va, vb in zip(entry, after):
        assert np.array_equal(_bits(va), _bits(vb))
    # a valid state again: the same handle solves the step
    s.set_state(u=good[0], alpha=good[1], alpha_prev=good[2])
    s.set_load(loads[2])
    st = s.solve_step()
    assert st["converged"]
    u, al, ap = s.state()
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(al)) and np.all(al >= ap)
    s.close()


def test_idle_sweep_tightens_and_converges():
    """Sub-solve tolerances looser than the stop test (PCG and damage solve to
    1e-3, stop at ||Phi||_2 < 1e-9): a sweep whose solves stop at once leaves
    the state unchanged, after which the step's sub-solves are tightened
    (instead of the idle sweep repeating to max_am) and every step reaches
    the oracle's converged state."""
    _torch()
    from oracle import am, problems
    n = 32
    p, notch, loads, _ = workloads.config2("AT1", 1.0, seed=0, n=n)
    params = fracture.make_params(**p, newton=0, am_stop=fracture.FRACTURE_STOP_PHI, final_tol=1e-9,
                                  pcg_rtol=1e-3, vi_tol=1e-3, max_am=3000)
    s = fracture.Fracture(params, notch, device="cuda:0")
    P = problems.tension_2d(n, n, p["lx"], p["ly"], **workloads.oracle_kwargs(p))
    st = am.initial_state(P, notch.astype(bool))
    for t in loads[:11]:
        s.set_load(t)
        r = s.solve_step()
        am.solve_load_step(P, st, t, am_tol=1e-10, max_am=3000)
        u, a, _ = s.state()
        eu = np.linalg.norm(u - st.u) / np.linalg.norm(st.u)
        ea = np.linalg.norm(a - st.alpha) / max(np.linalg.norm(st.alpha), 1e-300)
        print(f"  t={t:.1f} sweeps={r['sweeps']} pcg={r['pcg_iters']} phi={r['phi_l2']:.1e} "
              f"rel_u={eu:.1e} rel_a={ea:.1e}", flush=True)
        assert r["converged"] and r["phi_l2"] <= 1e-9 and r["sweeps"] < 3000
        assert eu < 1e-6 and ea < 1e-6
    s.close()


def test_failed_step_names_its_stage():
    """stats.stopped_in: the elastic PCG's iteration limit and the sweep limit
    are told apart (and the state is rolled back either way)."""
    _torch()
    n = 32
    p, notch, loads, _ = workloads.config2("AT1", 1.0, seed=0, n=n)
    s = fracture.Fracture(fracture.make_params(**p, max_pcg=1, pcg_rtol=1e-13), notch,
                          device="cuda:0")
    s.set_load(loads[0])
    r = s.solve_step(raise_on_error=False)
    assert r["code"] == fracture.FRACTURE_ENOTCONV and r["stopped_in"] == fracture.FRACTURE_STAGE_PCG
    s.close()
    s = fracture.Fracture(fracture.make_params(**p, max_am=1, am_tol=1e-12), notch, device="cuda:0")
    entry = s.state()
    s.set_load(loads[11])
    r = s.solve_step(raise_on_error=False)
    assert r["code"] == fracture.FRACTURE_ENOTCONV
    assert r["stopped_in"] == fracture.FRACTURE_STAGE_SWEEPS
    for va, vb in zip(entry[1:], s.state()[1:]):
        assert np.array_equal(_bits(va), _bits(vb))
    s.close()
