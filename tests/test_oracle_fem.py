"""Pins of the oracle's discretisation against mathematics it must satisfy.

None of these re-types an oracle formula: each checks a property that a
dropped term, a wrong sign, a transposed operand or a wrong index would break
(patch test, rigid-body kernel, independent quadrature, finite differences).
"""

import itertools
import math

import numpy as np
import pytest

from oracle import fem, mesh


def _rng(seed=0):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------- mesh

@pytest.mark.parametrize("nx,ny,lx,ly", [(4, 3, 1.0, 1.0), (8, 8, 2.0, 0.5)])
def test_mesh2d_tiles_domain(nx, ny, lx, ly):
    X, T = mesh.structured_mesh_2d(nx, ny, lx, ly)
    vol, _ = fem.geometry(X, T)
    assert X.shape == ((nx + 1) * (ny + 1), 2)
    assert np.allclose(vol, lx * ly / (2 * nx * ny))
    assert math.isclose(vol.sum(), lx * ly, rel_tol=1e-14)
    # positive orientation and the right-diagonal split: no triangle crosses the
    # anti-diagonal, every cell's two triangles share the diagonal (i,j)-(i+1,j+1)
    P = X[T]
    det = (P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0])
    assert np.all(det > 0)
    assert np.all(T[0::2, 0] == T[1::2, 0]) and np.all(T[0::2, 2] == T[1::2, 1])


def test_mesh3d_kuhn_tiles_cube():
    X, T = mesh.structured_mesh_3d(3, 2, 2, 1.5, 1.0, 0.5)
    vol, _ = fem.geometry(X, T)
    assert np.allclose(vol, (1.5 / 3) * (1.0 / 2) * (0.5 / 2) / 6)
    assert math.isclose(vol.sum(), 1.5 * 1.0 * 0.5, rel_tol=1e-13)
    # each node appears in at most 24 tetrahedra; interior nodes in exactly 24
    counts = np.bincount(T.ravel(), minlength=len(X))
    inner = mesh.node_id_3d(1, 1, 1, 3, 2)
    assert counts[inner] == 24 and counts.max() == 24
    # every hexahedron's 6 tets share the main diagonal (v0, v0 + (1,1,1))
    assert np.all(T[:, 0].reshape(-1, 6) == T[::6, 0][:, None])
    assert np.all(T[:, 3].reshape(-1, 6) == T[::6, 3][:, None])


def test_nested_2d_coarse_triangles_are_unions_of_fine():
    """Refining the coarse mesh by edge midpoints gives the fine mesh: each
    coarse triangle's area equals the sum of the 4 fine ones inside it."""
    Xc, Tc = mesh.structured_mesh_2d(4, 4)
    Xf, Tf = mesh.structured_mesh_2d(8, 8)
    cf = Xf[Tf].mean(axis=1)
    for e, tri in enumerate(Tc):
        A = Xc[tri]
        M = np.column_stack([A[1] - A[0], A[2] - A[0]])
        lam = np.linalg.solve(M, (cf - A[0]).T).T
        inside = (lam[:, 0] > -1e-12) & (lam[:, 1] > -1e-12) & (lam.sum(axis=1) < 1 + 1e-12)
        assert inside.sum() == 4


# --------------------------------------------------------------------------- geometry and strains

@pytest.mark.parametrize("dim", [2, 3])
def test_gradients_reproduce_affine_fields(dim):
    rng = _rng(1)
    if dim == 2:
        X, T = mesh.structured_mesh_2d(3, 4, 1.2, 0.7)
    else:
        X, T = mesh.structured_mesh_3d(2, 3, 2, 1.0, 0.8, 0.6)
    _, grad = fem.geometry(X, T)
    c = rng.standard_normal(dim)
    f = X @ c + 0.3
    g = np.einsum("ea,eak->ek", f[T], grad)
    assert np.allclose(g, c[None, :], atol=1e-12)
    # affine displacement u = G x + b has the constant strain sym(G)
    G = rng.standard_normal((dim, dim))
    u = (X @ G.T + rng.standard_normal(dim)).T.ravel()      # blocked
    eps = fem.element_strains(u, T, grad)
    S = G + G.T
    if dim == 2:
        want = np.array([G[0, 0], G[1, 1], S[0, 1]])
    else:
        want = np.array([G[0, 0], G[1, 1], G[2, 2], S[1, 2], S[0, 2], S[0, 1]])
    assert np.allclose(eps, want[None, :], atol=1e-12)


def test_voigt_D_gives_isotropic_stress():
    lam, mu = fem.lame(1.0, 0.3, 3)
    D = fem.voigt_D(3, lam, mu)
    rng = _rng(2)
    e = rng.standard_normal((3, 3))
    e = 0.5 * (e + e.T)
    sig = lam * np.trace(e) * np.eye(3) + 2 * mu * e
    ev = np.array([e[0, 0], e[1, 1], e[2, 2], 2 * e[1, 2], 2 * e[0, 2], 2 * e[0, 1]])
    sv = D @ ev
    assert np.allclose(sv, [sig[0, 0], sig[1, 1], sig[2, 2], sig[1, 2], sig[0, 2], sig[0, 1]])
    # Young's modulus and Poisson ratio recovered from uniaxial stress
    C = np.linalg.inv(D[:3, :3])
    assert math.isclose(1.0 / C[0, 0], 1.0, rel_tol=1e-12)
    assert math.isclose(-C[0, 1] / C[0, 0], 0.3, rel_tol=1e-12)


def test_c_w_values():
    """c_w = 4 int_0^1 sqrt(w): numerically integrated, not re-typed."""
    s = np.linspace(0, 1, 200001)
    for model, w in (("AT1", s), ("AT2", s * s)):
        val = 4 * np.trapezoid(np.sqrt(w), s)
        assert math.isclose(fem.c_w(model), val, rel_tol=1e-6)


# --------------------------------------------------------------------------- a(alpha) element average (P5)

def _quad_triangle_deg4():
    """Dunavant degree-4 rule (6 points) on the reference triangle, barycentric."""
    a1, w1 = 0.445948490915965, 0.223381589678011
    a2, w2 = 0.091576213509771, 0.109951743655322
    pts, wts = [], []
    for a, w in ((a1, w1), (a2, w2)):
        b = 1 - 2 * a
        for p in ((a, a, b), (a, b, a), (b, a, a)):
            pts.append(p)
            wts.append(w)
    return np.array(pts), np.array(wts)


def _quad_tet_collapsed(n=6):
    """Tensor Gauss rule mapped to the reference tet (exact for high degree)."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    pts, wts = [], []
    for i, j, k in itertools.product(range(n), repeat=3):
        u, v, t = x[i], x[j], x[k]
        a = u
        b = v * (1 - u)
        c = t * (1 - u) * (1 - v)
        jac = (1 - u) ** 2 * (1 - v)
        pts.append((1 - a - b - c, a, b, c))
        wts.append(w[i] * w[j] * w[k] * jac * 6.0)      # weights sum to 1
    return np.array(pts), np.array(wts)


@pytest.mark.parametrize("dim", [2, 3])
def test_abar_is_exact_average_of_degradation(dim):
    rng = _rng(3)
    if dim == 2:
        X, T = mesh.structured_mesh_2d(3, 3)
        P, W = _quad_triangle_deg4()
    else:
        X, T = mesh.structured_mesh_3d(2, 2, 2)
        P, W = _quad_tet_collapsed()
    alpha = rng.uniform(0, 1, len(X))
    k = 1e-6
    ab = fem.avg_degradation(alpha, T, k, dim)
    aq = alpha[T] @ P.T                        # [E, q]
    want = ((1 - aq) ** 2 + k) @ W / W.sum()
    assert np.allclose(ab, want, rtol=1e-13, atol=1e-15)
    assert np.all(ab >= k) and np.all(ab <= 1 + k)


# --------------------------------------------------------------------------- elasticity operator (P1-P3)

def _model2d(nx=6, ny=5, **kw):
    X, T = mesh.structured_mesh_2d(nx, ny, 1.0, 0.8)
    return fem.Model(X, T, **kw)


def _model3d(**kw):
    X, T = mesh.structured_mesh_3d(3, 3, 2, 1.0, 1.0, 0.5)
    return fem.Model(X, T, **kw)


def _rigid_modes(X):
    N, d = X.shape
    modes = []
    for c in range(d):
        r = np.zeros(d * N)
        r[c * N:(c + 1) * N] = 1
        modes.append(r)
    pairs = [(0, 1)] if d == 2 else [(0, 1), (1, 2), (0, 2)]
    for a, b in pairs:
        r = np.zeros(d * N)
        r[a * N:(a + 1) * N] = -X[:, b]
        r[b * N:(b + 1) * N] = X[:, a]
        modes.append(r)
    return modes


@pytest.mark.parametrize("mk", [_model2d, _model3d])
def test_rigid_body_kernel_for_any_damage(mk):
    M = mk()
    alpha = _rng(4).uniform(0, 1, M.N)
    K = M.K(alpha)
    scale = abs(K).max()
    for r in _rigid_modes(M.X):
        assert np.max(np.abs(K @ r)) < 1e-12 * scale * np.max(np.abs(r))


@pytest.mark.parametrize("mk", [_model2d, _model3d])
def test_patch_test_uniform_damage(mk):
    M = mk()
    alpha = np.full(M.N, 0.37)
    G = _rng(5).standard_normal((M.dim, M.dim))
    u = (M.X @ G.T).T.ravel()
    y = M.K(alpha) @ u
    interior = np.ones(M.N, bool)
    for k in range(M.dim):
        interior &= (M.X[:, k] > 1e-12) & (M.X[:, k] < M.X[:, k].max() - 1e-12)
    idx = np.concatenate([np.flatnonzero(interior) + c * M.N for c in range(M.dim)])
    assert np.max(np.abs(y[idx])) < 1e-12 * np.max(np.abs(y))
    assert np.max(np.abs(y)) > 1e-3          # boundary rows carry the traction


def test_operator_symmetric_positive_and_energy_consistent():
    M = _model2d()
    rng = _rng(6)
    alpha = rng.uniform(0, 1, M.N)
    K = M.K(alpha)
    assert abs(K - K.T).max() < 1e-15 * abs(K).max()
    u = rng.standard_normal(2 * M.N)
    # 1/2 u^T K u equals the elastic energy integrated with a separate rule:
    # the edge-midpoint rule is exact for the quadratic a(alpha) on triangles
    el, _ = M.energies(u, alpha)
    mids = 0.5 * (alpha[M.T][:, [0, 1, 2]] + alpha[M.T][:, [1, 2, 0]])
    amean = ((1 - mids) ** 2 + M.k_ell).mean(axis=1)
    eps = fem.element_strains(u, M.T, M.grad)
    el_q = 0.5 * np.sum(M.vol * amean * np.einsum("ei,ij,ej->e", eps, M.D, eps))
    assert math.isclose(0.5 * u @ (K @ u), el_q, rel_tol=1e-12)
    assert math.isclose(el, el_q, rel_tol=1e-12)
    # K restricted to DOFs that remove rigid motions is positive definite
    fixed = np.zeros(2 * M.N, bool)
    fixed[[0, M.N, M.N + mesh.node_id_2d(6, 0, 6)]] = True
    Kf = K[~fixed][:, ~fixed].toarray()
    assert np.linalg.eigvalsh(Kf).min() > 0


# --------------------------------------------------------------------------- scalar operators

def test_mass_laplacian_load_vector_closed_forms():
    X, T = mesh.structured_mesh_2d(7, 5, 1.0, 1.0)
    M = fem.assemble_mass(X, T)
    L = fem.assemble_laplacian(X, T)
    m = fem.load_vector(X, T)
    one = np.ones(len(X))
    assert np.allclose(M @ one, m, atol=1e-15)
    assert math.isclose(one @ (M @ one), 1.0, rel_tol=1e-13)
    x = X[:, 0]
    assert math.isclose(x @ (M @ x), 1.0 / 3.0, rel_tol=1e-13)   # int x^2 (x is P1-exact)
    assert np.max(np.abs(L @ one)) < 1e-13
    assert math.isclose(x @ (L @ x), 1.0, rel_tol=1e-13)          # int |grad x|^2
    xy = X[:, 0] + 2 * X[:, 1]
    assert math.isclose(xy @ (L @ xy), 5.0, rel_tol=1e-13)
    # right-diagonal P1 Laplacian is the 5-point stencil on a square grid
    X2, T2 = mesh.structured_mesh_2d(4, 4)
    L2 = fem.assemble_laplacian(X2, T2).toarray()
    c = mesh.node_id_2d(2, 2, 4)
    row = L2[c]
    assert math.isclose(row[c], 4.0)
    for n in (mesh.node_id_2d(1, 2, 4), mesh.node_id_2d(3, 2, 4), mesh.node_id_2d(2, 1, 4), mesh.node_id_2d(2, 3, 4)):
        assert math.isclose(row[n], -1.0)
    assert abs(row[mesh.node_id_2d(1, 1, 4)]) < 1e-15 and abs(row[mesh.node_id_2d(3, 3, 4)]) < 1e-15


# --------------------------------------------------------------------------- derivatives (P12, P14)

def _fd(fun, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (fun(x + e) - fun(x - e)) / (2 * h)
    return g


@pytest.mark.parametrize("model", ["AT1", "AT2"])
@pytest.mark.parametrize("thermal", [False, True])
def test_gradients_match_energy_finite_differences(model, thermal):
    X, T = mesh.structured_mesh_2d(3, 3)
    M = fem.Model(X, T, ell=0.3, k_ell=1e-3, model=model)
    rng = _rng(7)
    u = 0.2 * rng.standard_normal(2 * M.N)
    alpha = rng.uniform(0.1, 0.9, M.N)
    eps0 = fem.isotropic_eigenstrain(0.05 * rng.standard_normal(len(T)), 2) if thermal else None
    E = lambda uu, aa: sum(M.energies(uu, aa, eps0))
    gu = _fd(lambda v: E(v, alpha), u)
    ga = _fd(lambda v: E(u, v), alpha)
    assert np.allclose(M.grad_u(u, alpha, eps0), gu, rtol=1e-7, atol=1e-9)
    assert np.allclose(M.grad_alpha(u, alpha, eps0), ga, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("model", ["AT1", "AT2"])
def test_hessian_blocks_match_finite_differences(model):
    X, T = mesh.structured_mesh_2d(3, 2)
    M = fem.Model(X, T, ell=0.3, k_ell=1e-3, model=model)
    rng = _rng(8)
    u = 0.2 * rng.standard_normal(2 * M.N)
    alpha = rng.uniform(0.1, 0.9, M.N)
    K = M.K(alpha).toarray()
    B = M.coupling(u, alpha).toarray()
    C = M.damage_hessian(u).toarray()
    h = 1e-6
    for j in range(M.N):
        e = np.zeros(M.N)
        e[j] = h
        dGu = (M.grad_u(u, alpha + e) - M.grad_u(u, alpha - e)) / (2 * h)
        dGa = (M.grad_alpha(u, alpha + e) - M.grad_alpha(u, alpha - e)) / (2 * h)
        assert np.allclose(B[:, j], dGu, rtol=1e-6, atol=1e-8)
        assert np.allclose(C[:, j], dGa, rtol=1e-6, atol=1e-8)
    for j in range(2 * M.N):
        e = np.zeros(2 * M.N)
        e[j] = h
        dGu = (M.grad_u(u + e, alpha) - M.grad_u(u - e, alpha)) / (2 * h)
        dGa = (M.grad_alpha(u + e, alpha) - M.grad_alpha(u - e, alpha)) / (2 * h)
        assert np.allclose(K[:, j], dGu, rtol=1e-6, atol=1e-8)
        assert np.allclose(B[j, :], dGa, rtol=1e-6, atol=1e-8)


def test_uniform_eigenstrain_is_stress_free():
    """P13: a uniform isotropic eigenstrain with only rigid-mode pins gives
    u = s (x - x_pin) and zero elastic energy, for any damage."""
    X, T = mesh.structured_mesh_3d(3, 2, 2, 1.0, 1.0, 0.5)
    M = fem.Model(X, T, ell=0.2)
    s = -0.01
    eps0 = fem.isotropic_eigenstrain(np.full(len(T), s), 3)
    alpha = _rng(9).uniform(0, 0.9, M.N)
    K = M.K(alpha)
    f = M.f_eigen(alpha, eps0)
    N = M.N
    p0, p1, p2 = 0, mesh.node_id_3d(3, 0, 0, 3, 2), mesh.node_id_3d(0, 2, 0, 3, 2)
    fixed = np.zeros(3 * N, bool)
    fixed[[p0, N + p0, 2 * N + p0, N + p1, 2 * N + p1, 2 * N + p2]] = True
    u = np.zeros(3 * N)
    F = ~fixed
    import scipy.sparse.linalg as spla
    u[F] = spla.spsolve(K[F][:, F].tocsc(), f[F])
    want = (s * (X - X[p0])).T.ravel()
    assert np.allclose(u, want, atol=1e-11)
    el, _ = M.energies(u, alpha, eps0)
    assert abs(el) < 1e-20
