"""Pins of the oracle's complementarity machinery (Sec. 2.4, Algorithm 4).

The box QP solver is checked against SciPy's L-BFGS-B and a projected
gradient method written here (brute force on tiny problems); the residual
Phi against the case table of the mixed complementarity problem.
"""

import numpy as np
import pytest
import scipy.optimize as so

from oracle import fem, mesh, vi


def test_fischer_burmeister_zero_set():
    # phi(a,b) = 0 exactly on {a >= 0, b >= 0, ab = 0}
    for a, b in [(0, 0), (0, 3.0), (2.0, 0), (0, 1e-9)]:
        assert vi.fb(a, b) == 0.0
    for a, b in [(1, 1), (-1, 0), (0, -1), (-1, -1), (0.5, 2)]:
        assert vi.fb(a, b) != 0.0
    assert np.isclose(vi.fb(1.0, 1.0), np.sqrt(2) - 2)


def test_mcp_residual_cases():
    l = np.array([0.0, 0.0, 0.0, 0.2, 0.0, 0.0, -np.inf])
    u = np.array([1.0, 1.0, 1.0, 0.2, 1.0, 1.0, np.inf])
    x = np.array([0.5, 0.0, 1.0, 0.2, 0.5, 0.0, 3.0])
    F = np.array([0.0, 2.0, -3.0, 7.0, 0.1, -0.1, 0.0])
    phi = vi.mcp_residual(x, F, l, u)
    # interior with F=0; lower bound with F>0; upper bound with F<0; l=u any F; free with F=0
    assert np.all(phi[[0, 1, 2, 3, 6]] == 0)
    # interior with F != 0 and lower bound with F < 0 violate the MCP
    assert phi[4] != 0 and phi[5] != 0
    # free component: Phi = -F
    assert vi.mcp_residual(np.array([1.0]), np.array([0.25]), np.array([-np.inf]), np.array([np.inf]))[0] == -0.25


def test_merit_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    n = 7
    A = rng.standard_normal((n, n))
    H = A @ A.T + n * np.eye(n)
    g = rng.standard_normal(n)
    l = np.full(n, -0.2)
    u = np.full(n, 0.4)
    l[0], u[0] = -np.inf, np.inf
    u[1] = np.inf
    l[2] = -np.inf
    x = rng.uniform(-0.15, 0.35, n)
    psi = lambda y: 0.5 * np.sum(vi.mcp_residual(y, H @ y - g, l, u) ** 2)
    import scipy.sparse as sp
    gr = vi.mcp_merit_gradient(x, H @ x - g, sp.csr_matrix(H), l, u)
    h = 1e-7
    fd = np.array([(psi(x + h * e) - psi(x - h * e)) / (2 * h) for e in np.eye(n)])
    assert np.allclose(gr, fd, rtol=1e-5, atol=1e-8)


def _projected_gradient(H, g, l, u, x0, iters=200000):
    L = np.linalg.eigvalsh(H).max()
    x = np.clip(x0, l, u)
    for _ in range(iters):
        xn = np.clip(x - (H @ x - g) / L, l, u)
        if np.max(np.abs(xn - x)) < 1e-15:
            break
        x = xn
    return x


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_box_qp_matches_brute_force(seed):
    """P11: damage-type box QP on a tiny mesh (<= 50 nodes)."""
    rng = np.random.default_rng(seed)
    X, T = mesh.structured_mesh_2d(5, 5)
    M = fem.Model(X, T, ell=0.15, model="AT1")
    u = 0.8 * rng.standard_normal(2 * M.N)
    H = M.damage_hessian(u).toarray()
    g = M.damage_linear(u)
    lo = np.clip(rng.uniform(-0.3, 0.5, M.N), 0, None)
    hi = np.ones(M.N)
    x, info = vi.box_qp(H, g, lo, hi, lo.copy(), tol=1e-14)
    assert not info["failed"]
    f = lambda y: 0.5 * y @ H @ y - g @ y
    res = so.minimize(f, lo.copy(), jac=lambda y: H @ y - g, method="L-BFGS-B",
                      bounds=list(zip(lo, hi)), options={"ftol": 1e-15, "gtol": 1e-13, "maxiter": 10000})
    xp = _projected_gradient(H, g, lo, hi, lo.copy())
    assert np.allclose(x, xp, atol=1e-9)
    assert np.allclose(x, res.x, atol=1e-6)
    assert f(x) <= f(res.x) + 1e-14
    # KKT signs (P10)
    F = H @ x - g
    at_lo = x - lo <= 1e-12
    at_hi = hi - x <= 1e-12
    inner = ~(at_lo | at_hi)
    assert np.all(F[at_lo & ~at_hi] >= -1e-12)
    assert np.all(F[at_hi & ~at_lo] <= 1e-12)
    assert np.max(np.abs(F[inner]), initial=0) < 1e-12


def test_box_qp_reaches_exact_unconstrained_solution():
    rng = np.random.default_rng(5)
    n = 12
    A = rng.standard_normal((n, n))
    H = A @ A.T + np.eye(n)
    xs = rng.uniform(0.2, 0.8, n)
    g = H @ xs
    x, info = vi.box_qp(H, g, np.zeros(n), np.ones(n), np.zeros(n), tol=1e-13)
    assert np.allclose(x, xs, atol=1e-12)


def test_active_set_rule():
    x = np.array([0.0, 0.0, 1.0, 1.0, 0.5, 0.3])
    F = np.array([1.0, -1.0, -1.0, 1.0, 5.0, 2.0])
    l = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.3])
    u = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 0.3])
    A = vi.active_set(x, F, l, u, 1e-12)
    assert A.tolist() == [True, False, True, False, False, True]
