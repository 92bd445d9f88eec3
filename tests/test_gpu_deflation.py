"""GPU parity of the crack-aware deflation of the elastic CG (Sec. 3.1's
per-fragment rigid modes): fragment labels bit-exact against the oracle's
breadth-first search, E = W^T K W to 1e-12, and load steps solved with the
deflated CG against the oracle's exact solves (1e-6), including a specimen
cut in two by its notch.  At 2049 x 2049 nodes the labels are checked on
strips whose fragments are known in closed form."""

import numpy as np
import pytest

from oracle import am, deflation, mesh, problems
from paper_1511_08463_amd import fracture, workloads

pytestmark = pytest.mark.gpu

OPS_TOL = 1e-12
STEP_TOL = 1e-6


def _solver(p, notch=None, **kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fracture.Fracture(fracture.make_params(**dict(p, **kw)), notch, device="cuda:0")


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _field(kind, nx, ny, seed):
    X, _ = mesh.structured_mesh_2d(nx, ny)
    x, y = X[:, 0], X[:, 1]
    rng = np.random.default_rng(seed)
    if kind == "random":
        return rng.uniform(0.0, 1.0, X.shape[0])
    if kind == "smooth":                       # a few random plane waves
        a = np.zeros(X.shape[0])
        for _ in range(6):
            k = rng.uniform(3.0, 12.0, 2)
            a += np.sin(k[0] * x + k[1] * y + rng.uniform(0, 6.3))
        return 0.5 + 0.25 * a / 6 ** 0.5 * 2.0
    if kind == "bands":                        # two full-width bands and a partial one
        a = np.zeros(X.shape[0])
        a[np.abs(y - 0.3) < 0.6 / ny] = 1.0
        a[np.abs(y - 0.7) < 0.6 / ny] = 0.9
        a[(np.abs(x - 0.5) < 0.6 / nx) & (y < 0.3)] = 0.8
        return a
    raise ValueError(kind)


CASES = [("random", 38, 22, 0.5, 1, 8), ("random", 64, 40, 0.45, 3, 8),
         ("random", 96, 32, 0.4, 1, 8), ("random", 64, 40, 0.65, 4, 5),
         ("smooth", 96, 80, 0.5, 1, 8), ("smooth", 128, 72, 0.45, 20, 3),
         ("bands", 68, 44, 0.5, 1, 8), ("bands", 68, 44, 0.95, 1, 8)]


@pytest.mark.parametrize("kind,nx,ny,theta,min_nodes,fmax", CASES)
def test_fragments_match_oracle(kind, nx, ny, theta, min_nodes, fmax):
    p = workloads.tension(nx, 0.1, "AT1", ny=ny)
    print(f"[deflation] fragments {kind} {nx}x{ny} theta={theta} min={min_nodes} max={fmax}",
          flush=True)
    alpha = _field(kind, nx, ny, seed=nx)
    X, T = mesh.structured_mesh_2d(nx, ny)
    N = X.shape[0]
    name = deflation.components(T, N, alpha < theta)
    _, sizes = np.unique(name[name >= 0], return_counts=True)
    assert (sizes >= min_nodes).sum() <= 256          # within the candidate list
    want, roots = deflation.fragments(T, N, alpha, theta, min_nodes, fmax)
    s = _solver(p, deflate=1, deflate_theta=theta, deflate_min_nodes=min_nodes,
                deflate_max_fragments=fmax)
    s.set_state(u=np.zeros(2 * N), alpha=alpha, alpha_prev=np.zeros(N))
    nf, fid = s.fragments()
    s.close()
    print(f"  oracle {len(roots)} of {len(sizes)} components, gpu {nf}", flush=True)
    assert nf == len(roots)
    assert np.array_equal(fid.astype(np.int64), want)


def test_fragments_full_size_strips():
    """2049 x 2049 nodes: three damaged columns cut strips of 300, 700, 448
    and 598 node columns; the fragments are those strips, largest first."""
    n = 2048
    p = workloads.tension(n, 4.0 / n, "AT1")
    print("[deflation] fragments 2048^2 strips", flush=True)
    i = np.tile(np.arange(n + 1), n + 1)
    alpha = np.zeros((n + 1) * (n + 1))
    for c in (300, 1001, 1450):
        alpha[i == c] = 1.0
    s = _solver(p, deflate=1)
    s.set_state(u=np.zeros(2 * alpha.size), alpha=alpha, alpha_prev=np.zeros(alpha.size))
    nf, fid = s.fragments()
    s.close()
    want = np.full(alpha.size, -1)
    for k, (lo, hi) in enumerate([(301, 1001), (1451, 2049), (1002, 1450), (0, 300)]):
        want[(i >= lo) & (i < hi)] = k
    assert nf == 4
    assert np.array_equal(fid.astype(np.int64), want)


@pytest.mark.parametrize("nx,ny,kind", [(48, 40, "bands"), (96, 80, "smooth")])
def test_deflation_matrix_matches_oracle(nx, ny, kind):
    p = workloads.tension(nx, 0.1, "AT1", ny=ny, lx=1.0, ly=0.8)
    print(f"[deflation] E {kind} {nx}x{ny}", flush=True)
    P = problems.tension_2d(nx, ny, 1.0, 0.8, **workloads.oracle_kwargs(p))
    M = P.model
    alpha = _field(kind, nx, ny, seed=3)
    fid, roots = deflation.fragments(M.T, M.N, alpha, 0.5, 64, 8)
    W = deflation.rigid_modes(M.X, P.fixed, fid, len(roots), 1.0, 0.8)
    want = deflation.coarse_matrix(M.K(alpha), W)
    s = _solver(p, deflate=1)
    s.set_state(u=np.zeros(2 * M.N), alpha=alpha, alpha_prev=np.zeros(M.N))
    E = s.deflation_matrix()
    s.close()
    assert len(roots) >= 2 and E.shape == want.shape
    assert np.max(np.abs(E - want)) <= OPS_TOL * np.max(np.abs(want))


def _run_both(p, notch, loads, **kw):
    s = _solver(p, notch, am_tol=1e-10, pcg_rtol=1e-13, vi_cg_rtol=1e-13, **kw)
    P = problems.tension_2d(p["nx"], p["ny"], 1.0, 1.0, **workloads.oracle_kwargs(p))
    st = am.initial_state(P, notch.astype(bool))
    out = []
    for t in loads:
        s.set_load(t)
        stats = s.solve_step()
        am.solve_load_step(P, st, t, am_tol=1e-10)
        u, a, _ = s.state()
        out.append((_rel(u, st.u), _rel(a, st.alpha), stats))
        print(f"  t={t} sweeps={stats['sweeps']} pcg={stats['pcg_iters']} "
              f"rel_u={out[-1][0]:.2e} rel_a={out[-1][1]:.2e}", flush=True)
    s.close()
    return out


@pytest.mark.parametrize("cut", [False, True])
def test_deflated_load_path_parity(cut):
    """48 x 48 notched square loaded until the crack grows, or (cut) with the
    notch across the whole width, so that the body starts in two pieces and
    the damage band about the cut widens; ORAM with the deflated elastic CG
    against the oracle's exact solves."""
    n = 48
    p, notch, (y0, a) = workloads.small_tension(n, "AT1", ell=0.08)
    loads = [0.3, 0.8, 1.1]
    if cut:
        notch = workloads.notch_mask_2d(n, n, y0, 1.0)
        loads = [0.1, 0.2, 0.4]
    print(f"[deflation] load path cut={cut}", flush=True)
    res = _run_both(p, notch, loads, deflate=1, deflate_min_nodes=16)
    for eu, ea, stats in res:
        assert stats["converged"]
        assert eu < STEP_TOL and ea < STEP_TOL


def test_deflated_and_plain_cg_agree_on_broken_specimen():
    """192 x 192, AT1 damage profile across the mid-line: one load step with
    and without deflation reaches the same state."""
    n = 192
    p = workloads.tension(n, 4.0 / n, "AT1")
    print("[deflation] broken specimen 192^2", flush=True)
    X, _ = mesh.structured_mesh_2d(n, n)
    d = np.abs(X[:, 1] - 0.5)
    alpha = np.clip(1.0 - d / (8.0 / n), 0.0, 1.0) ** 2
    res = {}
    for dfl in (0, 1):
        s = _solver(p, deflate=dfl, am_tol=1e-10, pcg_rtol=1e-12, vi_cg_rtol=1e-12)
        s.set_state(u=np.zeros(2 * alpha.size), alpha=alpha, alpha_prev=alpha)
        s.set_load(0.5)
        stats = s.solve_step()
        res[dfl] = (s.state(), stats)
        if dfl:
            nf, _ = s.fragments()
            assert nf == 2
        s.close()
        print(f"  deflate={dfl} sweeps={stats['sweeps']} pcg={stats['pcg_iters']}", flush=True)
    (u0, a0, _), st0 = res[0]
    (u1, a1, _), st1 = res[1]
    assert st0["converged"] and st1["converged"]
    assert _rel(u1, u0) < 1e-8 and _rel(a1, a0) < 1e-8


def test_degenerate_fragment_sets():
    """No undamaged node: no fragment, and the deflated solve is the plain one
    bit for bit.  No damage: one fragment, the whole body, E against the
    oracle."""
    n = 40
    p = workloads.tension(n, 0.1, "AT1")
    print("[deflation] degenerate fragment sets", flush=True)
    P = problems.tension_2d(n, n, **workloads.oracle_kwargs(p))
    M = P.model
    N = M.N
    ones = np.ones(N)
    states = []
    for dfl in (0, 1):
        s = _solver(p, deflate=dfl, am_tol=1e-9, pcg_rtol=1e-12)
        s.set_state(u=np.zeros(2 * N), alpha=ones, alpha_prev=ones)
        if dfl:
            nf, fid = s.fragments()
            assert nf == 0 and np.all(fid == -1)
            assert s.deflation_matrix().shape == (0, 0)
        s.set_load(0.3)
        s.solve_step()
        states.append(s.state()[0])
        s.close()
    assert np.array_equal(states[0], states[1])
    s = _solver(p, deflate=1)
    s.set_state(u=np.zeros(2 * N), alpha=np.zeros(N), alpha_prev=np.zeros(N))
    nf, fid = s.fragments()
    E = s.deflation_matrix()
    s.close()
    assert nf == 1 and np.all(fid == 0)
    W = deflation.rigid_modes(M.X, P.fixed, np.zeros(N, dtype=np.int64), 1, 1.0, 1.0)
    want = deflation.coarse_matrix(M.K(np.zeros(N)), W)
    assert np.max(np.abs(E - want)) <= OPS_TOL * np.max(np.abs(want))


def test_fragment_held_entirely_by_dirichlet_dofs():
    """Surfing slab (every boundary DOF fixed): damaging the row below the
    top edge leaves the top row as a fragment whose three modes vanish on
    every DOF; the factorisation drops them and the deflated load step
    reaches the plain one's state."""
    p, notch, _ = workloads.surfing(0.1)
    nx, ny = p["nx"], p["ny"]
    print(f"[deflation] Dirichlet-held fragment {nx}x{ny}", flush=True)
    N = (nx + 1) * (ny + 1)
    alpha = np.zeros(N)
    alpha[(ny - 1) * (nx + 1): ny * (nx + 1)] = 1.0
    states, stats = [], []
    for dfl in (0, 1):
        s = _solver(p, notch, deflate=dfl, deflate_min_nodes=8, newton=1, final_tol=1e-9,
                    pcg_rtol=1e-12, vi_cg_rtol=1e-12)
        s.set_state(u=np.zeros(2 * N), alpha=alpha, alpha_prev=alpha)
        if dfl:
            nf, fid = s.fragments()
            assert nf == 2 and int((fid == 1).sum()) == nx + 1
            E = s.deflation_matrix()
            assert np.all(E[3:, :] == 0.0) and np.all(E[:, 3:] == 0.0)
        s.set_load(0.1)
        st = s.solve_step()
        assert st["converged"]
        states.append(s.state())
        stats.append(st)
        s.close()
    print(f"  pcg plain/deflated {stats[0]['pcg_iters']}/{stats[1]['pcg_iters']}", flush=True)
    assert _rel(states[1][0], states[0][0]) < 1e-7 and _rel(states[1][1], states[0][1]) < 1e-7
