"""Parity at the benchmark's full size (2048 x 2048, config 2) in the launch
configuration bench.py times.  The oracle cannot assemble the whole problem
in a test, so it computes sampled outputs one by one: each node's row of an
operator involves only the elements around it, and the oracle assembles
exactly those (a patch of at most 2 x 2 cells) with the same spacing and the
same field values.  After converged load steps the first-order conditions
(eq. (kkt)) are checked at sampled nodes the same way, together with the
bounds at every node."""

import numpy as np
import pytest

from oracle import fem, mesh, vi
from paper_1511_08463_amd import fracture, workloads

pytestmark = pytest.mark.gpu

N_SIDE = 2048


def _patch(i, j, n, h, ny=None, hy=None):
    """Cells around node (i, j) of an n x ny grid (cells h x hy), clipped to
    the domain: (X, T, global ids, local id)."""
    ny = n if ny is None else ny
    hy = h if hy is None else hy
    i0, i1 = max(i - 1, 0), min(i + 1, n)
    j0, j1 = max(j - 1, 0), min(j + 1, ny)
    X, T = mesh.structured_mesh_2d(i1 - i0, j1 - j0, (i1 - i0) * h, (j1 - j0) * hy)
    X = X + np.array([i0 * h, j0 * hy])
    ii, jj = np.meshgrid(np.arange(i0, i1 + 1), np.arange(j0, j1 + 1), indexing="xy")
    gid = (ii + (n + 1) * jj).ravel()
    loc = (i - i0) + (i1 - i0 + 1) * (j - j0)
    return X, T, gid, loc


def _samples(n, rng, k=160):
    pts = {(0, 0), (n, 0), (0, n), (n, n), (0, n // 2), (n, n // 2), (n // 2, 0), (n // 2, n)}
    while len(pts) < k:
        pts.add((int(rng.integers(0, n + 1)), int(rng.integers(0, n + 1))))
    return sorted(pts)


def _model(p, X, T):
    return fem.Model(X, T, E=p["E"], nu=p["nu"], Gc=p["Gc"], ell=p["ell"], k_ell=p["k_ell"],
                     model=p["model"])


def test_full_size_operator_rows():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, notch, _, _ = workloads.config2()
    n, h = N_SIDE, 1.0 / N_SIDE
    params = fracture.make_params(**p, newton=1)
    s = fracture.Fracture(params, notch, device="cuda:0")
    N = s.N
    rng = np.random.default_rng(12)
    u = rng.standard_normal(2 * N) * 1e-3
    alpha = rng.uniform(0, 1, N)
    s.set_state(u=u, alpha=alpha, alpha_prev=np.zeros(N))
    y = s.apply(fracture.FRACTURE_OP_ELASTICITY, u)
    x = rng.standard_normal(N)
    hx = s.apply(fracture.FRACTURE_OP_DAMAGE_HESS, x)
    Eu, Ea = s.gradient()
    worst = 0.0
    for (i, j) in _samples(n, rng):
        X, T, gid, loc = _patch(i, j, n, h)
        M = _model(p, X, T)
        up = np.concatenate([u[gid], u[N + gid]])
        ap = alpha[gid]
        m = len(gid)
        row = M.K(ap) @ up
        g = i + (n + 1) * j
        want = np.array([row[loc], row[m + loc]])
        got = np.array([y[g], y[N + g]])
        scale = np.max(np.abs(M.K(ap).toarray()[[loc, m + loc]])) * np.max(np.abs(up))
        worst = max(worst, np.max(np.abs(got - want)) / scale)
        hrow = M.damage_hessian(up) @ x[gid]
        assert abs(hx[g] - hrow[loc]) <= 1e-12 * max(1e-300, np.max(np.abs(M.damage_hessian(up).toarray()[loc])) * np.max(np.abs(x[gid])))
        ga = M.grad_alpha(up, ap)
        assert abs(Ea[g] - ga[loc]) <= 1e-11 * max(abs(ga[loc]), np.max(np.abs(M.damage_linear(up))), 1e-300)
    assert worst < 1e-12, worst
    s.close()


def _patch3(i, j, k, nx, ny, nz, hx, hy, hz):
    """Hexahedra around node (i, j, k) of the structured Kuhn mesh, clipped
    to the domain: (X, T, global ids, local id)."""
    i0, i1 = max(i - 1, 0), min(i + 1, nx)
    j0, j1 = max(j - 1, 0), min(j + 1, ny)
    k0, k1 = max(k - 1, 0), min(k + 1, nz)
    X, T = mesh.structured_mesh_3d(i1 - i0, j1 - j0, k1 - k0, (i1 - i0) * hx, (j1 - j0) * hy,
                                   (k1 - k0) * hz)
    X = X + np.array([i0 * hx, j0 * hy, k0 * hz])
    kk, jj, ii = np.meshgrid(np.arange(k0, k1 + 1), np.arange(j0, j1 + 1), np.arange(i0, i1 + 1),
                             indexing="ij")
    gid = (ii + (nx + 1) * (jj + (ny + 1) * kk)).ravel()
    loc = (i - i0) + (i1 - i0 + 1) * ((j - j0) + (j1 - j0 + 1) * (k - k0))
    return X, T, gid, loc


def test_full_size_3d_operator_rows():
    """The 3D operator on the 128 x 128 x 32 slab (config 3) as the bench runs
    it: the element-centric kernels on the finest level (15 x 15 x 4-node
    tiles).  Rows of K(alpha) u at sampled nodes (corners, edges, tile seams
    in x, y and z, random nodes) against the oracle's assembly of each node's
    hexahedron patch (eq. (elasticity)), and the two kernel families'
    results against each other on the whole grid."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, _ = workloads.config3()
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    hx, hy, hz = p["lx"] / nx, p["ly"] / ny, p["lz"] / nz
    rng = np.random.default_rng(33)
    out = {}
    for kern, m in (("elem", 1 << 18), ("node", 1 << 30)):
        s = fracture.Fracture(fracture.make_params(**p, elem3d_min_nodes=m), None, device="cuda:0")
        N = s.N
        if kern == "elem":
            u = rng.standard_normal(3 * N) * 1e-3
            alpha = rng.uniform(0, 1, N)
        s.set_state(u=u, alpha=alpha, alpha_prev=np.zeros(N))
        out[kern] = s.apply(fracture.FRACTURE_OP_ELASTICITY, u)
        s.close()
    y = out["elem"]
    assert np.max(np.abs(y - out["node"])) <= 1e-12 * np.max(np.abs(y))
    pts = {(0, 0, 0), (nx, ny, nz), (0, ny, 0), (nx, 0, nz), (14, 15, 3), (15, 14, 4), (16, 30, 7),
           (29, 31, 8), (nx, 60, 16), (64, ny, 0)}
    while len(pts) < 60:
        pts.add((int(rng.integers(0, nx + 1)), int(rng.integers(0, ny + 1)), int(rng.integers(0, nz + 1))))
    worst = 0.0
    for (i, j, k) in sorted(pts):
        X, T, gid, loc = _patch3(i, j, k, nx, ny, nz, hx, hy, hz)
        M = fem.Model(X, T, E=p["E"], nu=p["nu"], Gc=p["Gc"], ell=p["ell"], k_ell=p["k_ell"],
                      model=p["model"])
        up = np.concatenate([u[gid], u[N + gid], u[2 * N + gid]])
        Kp = M.K(alpha[gid])
        row = Kp @ up
        mloc = len(gid)
        g = i + (nx + 1) * (j + (ny + 1) * k)
        want = np.array([row[loc], row[mloc + loc], row[2 * mloc + loc]])
        got = np.array([y[g], y[N + g], y[2 * N + g]])
        scale = np.max(np.abs(Kp.toarray()[[loc, mloc + loc, 2 * mloc + loc]])) * np.max(np.abs(up))
        worst = max(worst, np.max(np.abs(got - want)) / scale)
    assert worst < 1e-12, worst


def test_full_size_residual_rows():
    """The elastic PCG's residual kernel at 2048^2 (the column-tiled form the
    finest level runs): -K(alpha) x on free rows and zero on Dirichlet rows,
    at sampled nodes (corners, edges, the notch row and random nodes),
    against the oracle's assembly of each node's element patch (eq.
    (elasticity))."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, notch, _, (y0, _) = workloads.config2()
    n, h = N_SIDE, 1.0 / N_SIDE
    s = fracture.Fracture(fracture.make_params(**p, newton=1), notch, device="cuda:0")
    N = s.N
    rng = np.random.default_rng(21)
    u = rng.standard_normal(2 * N) * 1e-3
    alpha = rng.uniform(0, 1, N)
    alpha[notch.astype(bool)] = 1.0
    s.set_state(u=u, alpha=alpha, alpha_prev=np.zeros(N))
    r = s.apply(fracture.FRACTURE_OP_RESIDUAL, u)
    jn = int(round(y0 / h))
    pts = _samples(n, rng) + [(i, jn) for i in range(0, n + 1, 97)] + [(5, 0), (7, n), (0, 9)]
    worst = 0.0
    for (i, j) in pts:
        X, T, gid, loc = _patch(i, j, n, h)
        M = _model(p, X, T)
        up = np.concatenate([u[gid], u[N + gid]])
        Kp = M.K(alpha[gid])
        row = Kp @ up
        g = i + (n + 1) * j
        m = len(gid)
        # Dirichlet DOFs: u_y on the bottom and top rows, u_x at node (0, 0)
        fixed_x = i == 0 and j == 0
        fixed_y = j == 0 or j == n
        want = np.array([0.0 if fixed_x else -row[loc], 0.0 if fixed_y else -row[m + loc]])
        got = np.array([r[g], r[N + g]])
        if fixed_x:
            assert got[0] == 0.0
        if fixed_y:
            assert got[1] == 0.0
        scale = np.max(np.abs(Kp.toarray()[[loc, m + loc]])) * np.max(np.abs(up))
        worst = max(worst, np.max(np.abs(got - want)) / scale)
    assert worst < 1e-12, worst
    s.close()


def test_full_size_vcycle_symmetric_positive():
    """The V-cycle at 2048^2 (column-tiled finest-level smoothing, residual
    and prolongation-fused steps, per-node coarse levels, the LDS tail and
    the dense coarsest solve) is a symmetric positive definite operator, as
    the PCG needs: y.Mx = x.My and x.Mx > 0 for random x, y (zero on
    Dirichlet DOFs), with a cracked damage field."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, notch, _, _ = workloads.config2()
    n = N_SIDE
    s = fracture.Fracture(fracture.make_params(**p, newton=1), notch, device="cuda:0")
    N = s.N
    yy = np.repeat(np.arange(n + 1) / n, n + 1)
    xx = np.tile(np.arange(n + 1) / n, n + 1)
    # an AT1 damage band (half-width 2 ell) along y = 0.5 over x < 0.7
    alpha = np.where(xx < 0.7, np.clip(1.0 - np.abs(yy - 0.5) / (8.0 / n), 0.0, 1.0) ** 2, 0.0)
    s.set_state(u=np.zeros(2 * N), alpha=alpha, alpha_prev=alpha)
    fracture.fracture_update_coefficients(s.h)
    rng = np.random.default_rng(4)
    free = np.ones(2 * N, bool)
    free[0] = False                                     # u_x at (0, 0)
    free[N:N + n + 1] = False                           # u_y on the bottom row
    free[N + n * (n + 1):] = False                      # u_y on the top row
    x = np.where(free, rng.standard_normal(2 * N), 0.0)
    y = np.where(free, rng.standard_normal(2 * N), 0.0)
    Mx = s.apply(fracture.FRACTURE_OP_PRECOND, x)
    My = s.apply(fracture.FRACTURE_OP_PRECOND, y)
    assert np.all(Mx[~free] == 0.0) and np.all(My[~free] == 0.0)
    a, b = y @ Mx, x @ My
    scale = np.linalg.norm(x) * np.linalg.norm(Mx) + np.linalg.norm(y) * np.linalg.norm(My)
    print(f"[vcycle 2048] y.Mx={a:.12e} x.My={b:.12e} rel={abs(a - b) / scale:.2e}", flush=True)
    assert abs(a - b) <= 1e-10 * scale
    assert x @ Mx > 0 and y @ My > 0
    s.close()


def test_ragged_large_grid_operator_rows():
    """A grid large enough for the column-tiled operator kernels, with a
    one-node ragged tail in both directions (1537 columns: 24 whole 64-wide
    tiles and one node; 1409 rows: one row past any tile height the kernels
    use; both axes still halve down to a dense coarsest level) and unequal
    cell sides: operator rows at tile seams, the last rows and columns, and
    random nodes match the oracle's patch assembly, and so do the damage
    gradient's rows (E_alpha from the column-walking VI evaluation)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nx, ny = 1536, 1408
    p = workloads.tension(nx, 0.01, "AT2", nx=nx, ny=ny)
    hx, hy = 1.0 / nx, 1.0 / ny
    s = fracture.Fracture(fracture.make_params(**p), None, device="cuda:0")
    N = s.N
    rng = np.random.default_rng(21)
    u = rng.standard_normal(2 * N)
    alpha = rng.uniform(0, 1, N)
    s.set_state(u=u, alpha=alpha, alpha_prev=np.zeros(N))
    y = s.apply(fracture.FRACTURE_OP_ELASTICITY, u)
    # the damage VI evaluation (column-walking on this grid): E_alpha rows
    _, Ea = s.gradient()
    js = sorted({0, 1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32, 33, ny - 2, ny - 1, ny,
                 ny - ny % 16, ny - ny % 8, ny - ny % 4, ny - ny % 16 - 1, ny - ny % 8 - 1}
                | {int(v) for v in rng.integers(0, ny + 1, 12)})
    ii = sorted({0, 1, 62, 63, 64, 65, 127, 128, nx - 1, nx, nx - nx % 64, nx - nx % 64 - 1}
                | {int(v) for v in rng.integers(0, nx + 1, 6)})
    worst = 0.0
    for j in js:
        for i in ii:
            X, T, gid, loc = _patch(i, j, nx, hx, ny, hy)
            M = _model(p, X, T)
            up = np.concatenate([u[gid], u[N + gid]])
            K = M.K(alpha[gid])
            row = K @ up
            m = len(gid)
            g = i + (nx + 1) * j
            scale = np.max(np.abs(K.toarray()[[loc, m + loc]])) * np.max(np.abs(up))
            err = max(abs(y[g] - row[loc]), abs(y[N + g] - row[m + loc])) / scale
            worst = max(worst, err)
            assert err < 1e-12, (i, j, err)
            ga = M.grad_alpha(up, alpha[gid])
            assert abs(Ea[g] - ga[loc]) <= 1e-11 * max(abs(ga[loc]), np.max(np.abs(M.damage_linear(up))),
                                                       1e-300), (i, j)
    print(f"[ragged-large] {len(js)}x{len(ii)} nodes, worst {worst:.2e}", flush=True)
    s.close()


def _kkt_at_samples(p, s, notch, pts, bound, n, h):
    """Every component of Phi at the sampled nodes is within bound."""
    u, a, ap = s.state()
    N = s.N
    for (i, j) in pts:
        if not (0 <= i <= n and 0 <= j <= n):
            continue
        X, T, gid, loc = _patch(i, j, n, h)
        M = _model(p, X, T)
        up = np.concatenate([u[gid], u[N + gid]])
        m = len(gid)
        Eu = M.K(a[gid]) @ up
        g = i + (n + 1) * j
        if not (i == 0 and j == 0):
            assert abs(Eu[loc]) <= bound, (i, j, Eu[loc], bound)
        if 0 < j < n:
            assert abs(Eu[m + loc]) <= bound, (i, j, Eu[m + loc], bound)
        Fa = M.grad_alpha(up, a[gid])[loc]
        phi = vi.mcp_residual(np.array([a[g]]), np.array([Fa]), np.array([ap[g]]),
                              np.array([1.0]))[0]
        assert abs(phi) <= bound, (i, j, phi, a[g], Fa, bound)


def test_full_size_bench_path_kkt_through_propagation():
    """The benchmarked path itself (2048^2, the bench's solver settings):
    load steps 1..15 through crack initiation (t = 1.0) and the unstable
    propagation (t = 1.5).  After t = 1.0 and after t = 1.5 the bounds hold
    at every node, the crack has grown (and after t = 1.5 cut the specimen),
    and every component of Phi at sampled nodes, many along the crack, is
    within the reported ||Phi||_2 (eq. (kkt), Algorithm 3's stop test)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, notch, loads, (y0, _) = workloads.config2()
    n, h = N_SIDE, 1.0 / N_SIDE
    s = fracture.Fracture(fracture.make_params(**p, **workloads.CONFIG2_SOLVER), notch,
                          device="cuda:0")
    rng = np.random.default_rng(11)
    jn = int(round(y0 / h))
    for k, t in enumerate(loads[:15]):
        s.set_load(t)
        st = s.solve_step()
        assert st["converged"], (k + 1, st)
        if k + 1 not in (10, 15):
            continue
        print(f"[fullsize] t={t:.1f}: sweeps={st['sweeps']} phi={st['phi_l2']:.2e}", flush=True)
        u, a, ap = s.state()
        assert np.all(a >= ap) and np.all(a <= 1.0) and np.all(a[notch.astype(bool)] == 1.0)
        cols = (a.reshape(n + 1, n + 1) > 0.5).any(axis=0)
        if k + 1 == 15:
            assert np.all(cols)                       # the specimen is cut
        else:
            assert np.count_nonzero(a > 0.5) > np.count_nonzero(notch)
        # sample along the crack band and at random nodes
        rows = np.flatnonzero((a.reshape(n + 1, n + 1) > 0.1).any(axis=1))
        pts = _samples(n, rng, 80)
        for i in range(0, n + 1, 128):
            col = a.reshape(n + 1, n + 1)[:, i]
            jc = int(np.argmax(col)) if col.max() > 0.1 else jn
            pts += [(i, jc + dj) for dj in (-12, -6, -2, 0, 2, 6, 12)]
        assert rows.size > 0
        _kkt_at_samples(p, s, notch, pts, st["phi_l2"] * (1 + 1e-6) + 1e-13, n, h)
    s.close()


def test_full_size_load_step_kkt():
    """The first two bench load steps (ORAM-N): the bounds hold at every node
    and, at sampled nodes, every component of the residual Phi (the free rows
    of E_u and the box Fischer--Burmeister residual of the damage VI, as in
    Algorithm 3) is within the reported ||Phi||_2."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, notch, loads, _ = workloads.config2()
    n, h = N_SIDE, 1.0 / N_SIDE
    params = fracture.make_params(**p, newton=1, pcg_rtol=1e-8, max_am=5000)
    s = fracture.Fracture(params, notch, device="cuda:0")
    for t in loads[:2]:
        s.set_load(t)
        st = s.solve_step()
        print(f"[fullsize] t={t}: {st}", flush=True)
        assert st["converged"]
    u, a, ap = s.state()
    N = s.N
    assert np.all(a >= ap) and np.all(a <= 1.0) and np.all(a[notch.astype(bool)] == 1.0)
    assert np.count_nonzero(a > 0.5) > np.count_nonzero(notch)   # damage is active
    bound = st["phi_l2"] * (1 + 1e-6) + 1e-13
    rng = np.random.default_rng(5)
    rows, cols = notch.reshape(n + 1, n + 1).nonzero()
    tip_i, tip_j = int(cols.max()), int(rows[0])
    pts = _samples(n, rng, 120) + [(tip_i + di, tip_j + dj)
                                   for di in range(-3, 12, 2) for dj in range(-10, 11, 2)]
    for (i, j) in pts:
        if not (0 <= i <= n and 0 <= j <= n):
            continue
        X, T, gid, loc = _patch(i, j, n, h)
        M = _model(p, X, T)
        up = np.concatenate([u[gid], u[N + gid]])
        m = len(gid)
        Eu = M.K(a[gid]) @ up
        g = i + (n + 1) * j
        # free rows: u_x everywhere except the pinned corner (0, 0);
        # u_y except on the bottom and top edges
        if not (i == 0 and j == 0):
            assert abs(Eu[loc]) <= bound, (i, j, Eu[loc], bound)
        if 0 < j < n:
            assert abs(Eu[m + loc]) <= bound, (i, j, Eu[m + loc], bound)
        Fa = M.grad_alpha(up, a[gid])[loc]
        phi = vi.mcp_residual(np.array([a[g]]), np.array([Fa]), np.array([ap[g]]),
                              np.array([1.0]))[0]
        assert abs(phi) <= bound, (i, j, phi, a[g], Fa, bound)
    s.close()
