"""Pins of the oracle's crack-aware deflation (the per-fragment rigid modes
that Sec. 3.1 names as a possible improvement of the elastic solve).

The fragment search is checked against SciPy's graph components (a
different algorithm over a graph built here from the element list) and
against geometry whose answer is known by hand: a damaged band across the
whole width splits the square in two; one that stops short of an edge does
not; a one-node line of damage cuts the mesh along the diagonal of its
triangles but not across it (the element edges run (i, j)-(i+1, j+1) only).
The rigid modes are checked against the kernel of the undamaged stiffness
(rigid motions carry no strain), and deflated CG against a direct solve, the
invariant W^T r = 0 of its iterates, and the iteration count it saves on a
broken specimen whose upper piece is held in x only through the band.
"""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components
from scipy.sparse.linalg import spsolve

from oracle import deflation, fem, mesh, problems


def _graph_names(T, N, solid):
    rows = np.concatenate([T[:, 0], T[:, 1], T[:, 2]])
    cols = np.concatenate([T[:, 1], T[:, 2], T[:, 0]])
    keep = solid[rows] & solid[cols]
    A = sp.coo_matrix((np.ones(keep.sum()), (rows[keep], cols[keep])), shape=(N, N))
    _, lab = connected_components(A, directed=False)
    name = np.full(N, -1)
    for c in np.unique(lab[solid]):
        on = (lab == c) & solid
        name[on] = np.flatnonzero(on).min()
    return name


@pytest.mark.parametrize("seed,theta", [(0, 0.5), (1, 0.6), (2, 0.4), (3, 0.55)])
def test_components_match_graph_library(seed, theta):
    nx, ny = 17, 13
    X, T = mesh.structured_mesh_2d(nx, ny)
    N = X.shape[0]
    alpha = np.random.default_rng(seed).uniform(0.0, 1.0, N)
    solid = alpha < theta
    got = deflation.components(T, N, solid)
    assert np.array_equal(got, _graph_names(T, N, solid))
    assert len(np.unique(got[got >= 0])) > 3             # several components


def _idx(i, j, nx):
    return i + (nx + 1) * j


def test_band_geometry():
    nx = ny = 20
    X, T = mesh.structured_mesh_2d(nx, ny)
    N = X.shape[0]
    a = np.zeros(N)
    a[[_idx(i, 7, nx) for i in range(nx + 1)]] = 1.0      # full-width band, row 7
    fid, roots = deflation.fragments(T, N, a, min_nodes=1)
    assert len(roots) == 2
    sizes = sorted(int((fid == k).sum()) for k in range(2))
    assert sizes == [7 * 21, 13 * 21]
    assert roots == [_idx(0, 8, nx), 0]                   # larger (upper) piece first
    a[_idx(nx, 7, nx)] = 0.0                              # band stops one node short
    fid, roots = deflation.fragments(T, N, a, min_nodes=1)
    assert len(roots) == 1 and (fid == 0).sum() == N - nx


def test_diagonal_lines():
    n = 12
    X, T = mesh.structured_mesh_2d(n, n)
    N = X.shape[0]
    a = np.zeros(N)
    a[[_idx(k, k, n) for k in range(n + 1)]] = 1.0        # along the element diagonals
    _, roots = deflation.fragments(T, N, a, min_nodes=1)
    assert len(roots) == 2
    a = np.zeros(N)
    a[[_idx(k, n - k, n) for k in range(n + 1)]] = 1.0    # across them
    _, roots = deflation.fragments(T, N, a, min_nodes=1)
    assert len(roots) == 1


def test_selection_by_size_and_limits():
    nx, ny = 10, 20
    X, T = mesh.structured_mesh_2d(nx, ny)
    N = X.shape[0]
    a = np.zeros(N)
    for j in (2, 5, 11):                                   # strips of 2, 2, 5 and 9 rows
        a[[_idx(i, j, nx) for i in range(nx + 1)]] = 1.0
    fid, roots = deflation.fragments(T, N, a, min_nodes=1)
    assert [int((fid == k).sum()) for k in range(4)] == [99, 55, 22, 22]
    assert roots == [_idx(0, 12, nx), _idx(0, 6, nx), 0, _idx(0, 3, nx)]
    _, roots = deflation.fragments(T, N, a, min_nodes=30)
    assert len(roots) == 2
    fid, roots = deflation.fragments(T, N, a, min_nodes=1, max_fragments=3)
    assert len(roots) == 3 and np.all(fid[: 2 * (nx + 1)] == 2)


def test_rigid_modes_carry_no_strain():
    """Unmasked rigid modes of the whole undamaged body lie in the kernel of
    K(0); masked, they are zero on every fixed DOF."""
    P = problems.tension_2d(16, 12, lx=1.5, ly=1.0)
    M = P.model
    N = M.N
    fid = np.zeros(N, dtype=np.int64)
    W = deflation.rigid_modes(M.X, np.zeros(2 * N, bool), fid, 1, 1.5, 1.0)
    K = M.K(np.zeros(N))
    scale = abs(K).max() * np.abs(W).max()
    assert np.max(np.abs(K @ W)) <= 1e-12 * scale
    Wm = deflation.rigid_modes(M.X, P.fixed, fid, 1, 1.5, 1.0)
    assert np.all(Wm[P.fixed] == 0.0) and np.array_equal(Wm[P.free], W[P.free])
    # the rotation is (-(y - yc), x - xc) s
    assert np.allclose(W[:N, 2], -(M.X[:, 1] - 0.5) * (2 / 1.5))
    assert np.allclose(W[N:, 2], (M.X[:, 0] - 0.75) * (2 / 1.5))


def _broken_specimen(n):
    """Tension specimen cut by a horizontal AT1 damage profile about the
    mid-line (alpha = 1 on it, zero beyond 2 ell): the upper piece is held
    in x only through the degraded stiffness of the band."""
    ell = 4.0 / n
    P = problems.tension_2d(n, n, ell=ell)
    M = P.model
    d = np.abs(M.X[:, 1] - 0.5)
    alpha = np.clip(1.0 - d / (2 * ell), 0.0, 1.0) ** 2
    K = M.K(alpha)
    ud = np.zeros(2 * M.N)
    ud[P.fixed] = P.dirichlet_values(1.0)[P.fixed]
    f = P.free
    Kff = K[f][:, f].tocsr()
    b = -(K @ ud)[f]
    return P, alpha, Kff, b


def test_deflated_cg_solves_and_keeps_residual_orthogonal():
    P, alpha, Kff, b = _broken_specimen(24)
    M = P.model
    fid, roots = deflation.fragments(M.T, M.N, alpha, min_nodes=16)
    assert len(roots) == 2
    W = deflation.rigid_modes(M.X, P.fixed, fid, len(roots), 1.0, 1.0)[P.free]
    E = deflation.coarse_matrix(Kff, W)
    assert np.allclose(E, E.T, rtol=1e-12, atol=1e-14 * np.abs(E).max())
    assert np.all(np.linalg.eigvalsh(E) > 0)
    exact = spsolve(Kff.tocsc(), b)
    tol = 1e-10 * np.linalg.norm(b)
    dinv = 1.0 / Kff.diagonal()
    jac = lambda v: dinv * v                            # noqa: E731
    x, it_d, worst = deflation.deflated_cg(Kff, b, np.zeros_like(b), W, tol, Minv=jac)
    assert np.linalg.norm(x - exact) <= 1e-7 * np.linalg.norm(exact)
    assert worst <= 1e-9
    x0, it_0, _ = deflation.deflated_cg(Kff, b, np.zeros_like(b), W[:, :0], tol, Minv=jac)
    assert np.linalg.norm(x0 - exact) <= 1e-7 * np.linalg.norm(exact)
    # the upper piece's x-translation is near-null: deflating it saves iterations
    assert it_d < it_0
