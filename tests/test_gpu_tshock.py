"""GPU parity of the 2D thermal shock (Sec. 4.3): the eigenstrain in the
residual, gradients, energy, damage Hessian and coupling blocks; the load
path through the x-homogeneous damage band, its bifurcation and the crack
array; and the purely elastic regime below the critical shock."""

import numpy as np
import pytest

from oracle import am, problems
from paper_1511_08463_amd import fracture, workloads

pytestmark = pytest.mark.gpu

OPS_TOL = 1e-12


def _solver(p, notch=None, **kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fracture.Fracture(fracture.make_params(**dict(p, **kw)), notch, device="cuda:0")


def _problem(p):
    return problems.thermal_shock_2d(p["nx"], p["ny"], **workloads.oracle_kwargs_tshock(p))


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _close(got, want, tol=OPS_TOL):
    return np.max(np.abs(got - want)) <= tol * max(np.max(np.abs(want)), 1e-300)


@pytest.mark.parametrize("model,ps", [("AT1", 0), ("AT2", 1)])
def test_tshock_operators_match_oracle(model, ps):
    """40 x 12 cells on 10 x 3 (h = ell/4), tau = 0.7, random u and alpha."""
    p = workloads.tshock(40, 12, lx=10.0, ly=3.0, ratio=3.0, model=model, plane_stress=ps)
    print(f"[tshock] operators {model} plane_stress={ps}", flush=True)
    P = _problem(p)
    M = P.model
    N = M.N
    s = _solver(p, newton=1)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(2 * N) * 0.3
    alpha = rng.uniform(0.0, 1.0, N)
    tau = 0.7
    s.set_load(tau)
    s.set_state(u=u, alpha=alpha, alpha_prev=np.zeros(N))
    e0 = P.eps0(tau)
    Eu, Ea = s.gradient()
    assert _close(Eu, M.grad_u(u, alpha, e0))
    assert _close(Ea, M.grad_alpha(u, alpha, e0), 1e-11)
    el, su = s.energy()
    oel, osu = M.energies(u, alpha, e0)
    assert abs(el - oel) <= 1e-12 * abs(oel) and abs(su - osu) <= 1e-12 * abs(osu)
    x = rng.standard_normal(N)
    assert _close(s.apply(fracture.FRACTURE_OP_DAMAGE_HESS, x), M.damage_hessian(u, e0) @ x)
    B = M.coupling(u, alpha, e0)
    w = rng.standard_normal(N)
    want = B @ w
    want[P.fixed] = 0.0
    assert _close(s.apply(fracture.FRACTURE_OP_COUPLING, w, out_len=2 * N), want)
    v = rng.standard_normal(2 * N) * P.free
    assert _close(s.apply(fracture.FRACTURE_OP_COUPLING_T, v, out_len=N), B.T @ v)
    # the plain operator carries no eigenstrain
    y = s.apply(fracture.FRACTURE_OP_ELASTICITY, u)
    assert _close(y, M.K(alpha) @ u)
    s.close()


@pytest.mark.parametrize("newton,omega,precision",
                         [(1, 1.0, 0), (0, 1.4, 0), (0, 0.8, 0), (1, 1.0, 1)])
def test_tshock_load_path_parity(newton, omega, precision):
    """64 x 16 cells on 16 x 4 (h = ell/4), DT = 2 DT_c, tau = 0.2 .. 2.0:
    the damage band, its bifurcation (tau ~ 1.6) and the cracks through the
    band (tau ~ 1.8); both sides to tight tolerances."""
    p = workloads.tshock(64, 16, lx=16.0, ly=4.0, ratio=2.0, omega=omega)
    print(f"[tshock] load path newton={newton} omega={omega} precision={precision}", flush=True)
    P = _problem(p)
    st = am.initial_state(P)
    kw = dict(newton=newton, precision=precision, max_am=4000, pcg_rtol=1e-12, vi_cg_rtol=1e-12)
    if newton:
        kw.update(final_tol=1e-10, minres_rtol=1e-8, max_newton=30)
    else:
        kw.update(am_tol=1e-9)
    s = _solver(p, **kw)
    taus = [round(0.2 * k, 10) for k in range(1, 11)]
    for tau in taus:
        s.set_load(tau)
        stats = s.solve_step()
        if newton:
            am.solve_load_step(P, st, tau, newton_on=True, final_tol=1e-10, max_am=4000,
                               max_newton=30)
        else:
            am.solve_load_step(P, st, tau, omega=omega, am_tol=1e-9, max_am=4000)
        u, a, _ = s.state()
        eu, ea = _rel(u, st.u), _rel(a, st.alpha)
        el, su = s.energy()
        oel, osu = P.model.energies(st.u, st.alpha, P.eps0(tau))
        print(f"  tau={tau} sweeps={stats['sweeps']} newton={stats['newton_iters']} "
              f"rel_u={eu:.2e} rel_a={ea:.2e} amax={a.max():.3f} Es={su:.6f}/{osu:.6f}",
              flush=True)
        assert stats["converged"]
        assert eu < 1e-6 and ea < 1e-6
        assert abs(su - osu) <= 1e-6 * max(abs(osu), 1e-12)
    assert a.max() == 1.0                    # cracks have formed
    s.close()


@pytest.mark.parametrize("ratio", [0.97, 1.1])
def test_tshock_elastic_regime(ratio):
    """Below DT_c the slab stays exactly undamaged at every tau; above it the
    cooled layer damages (the oracle's pin, on the GPU)."""
    p = workloads.tshock(64, 16, lx=16.0, ly=4.0, ratio=ratio)
    print(f"[tshock] elastic regime ratio={ratio}", flush=True)
    s = _solver(p, newton=1)
    for tau in (0.25, 1.0, 8.0):
        s.set_load(tau)
        assert s.solve_step()["converged"]
    u, a, _ = s.state()
    y = np.repeat(np.arange(17) * 0.25, 65)
    if ratio < 1:
        assert np.all(a == 0.0)
    else:
        assert a.max() > 1e-2
        assert np.all(y[a > 1e-3] < 2.0)
    s.close()
