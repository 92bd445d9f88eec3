"""Pins of the 3D thermal slab (the exponential-eigenstrain variant of
Sec. 4.3, eqs. (energytshock), (tempfielderfc)) in the oracle.

* The eigenstrain of each Kuhn tetrahedron is -DT exp(-x_c / depth) I at its
  centroid.  The centroid abscissae are derived here from the Kuhn
  construction itself: a tetrahedron whose axis ordering puts x first,
  second or third has vertex x-offsets (0, 1, 1, 1), (0, 0, 1, 1) or
  (0, 0, 0, 1), so each hexahedron holds two tetrahedra with centroid at
  (i + 3/4) h, two at (i + 1/2) h and two at (i + 1/4) h.
* The displacement conditions (u_x = 0 on x = lx and the three point pins
  that remove the y/z translations and the rotation about x) leave no
  rigid motion free and do not over-constrain: a uniform cooling s of the
  whole slab is a compatible strain, so the discrete solution is the
  stress-free contraction u = s (x - lx, y, z) with zero elastic energy, for
  any damage, and AT1 damage stays exactly zero however strong the cooling.
* The derivatives of the 3D energy with the eigenstrain (E_u, E_alpha, and
  the Jacobian blocks E_uu, E_ualpha, E_alphaalpha of eq. (newton)) match
  central finite differences on a small Kuhn mesh.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import am, fem, mesh, problems


def _rng(seed):
    return np.random.default_rng(seed)


def test_eigenstrain_at_kuhn_centroids():
    nx, ny, nz, lx, ly, lz, depth = 4, 3, 2, 1.0, 0.75, 0.5, 0.3
    P = problems.thermal_3d(nx, ny, nz, lx, ly, lz, depth=depth)
    h = lx / nx
    dT = 1.7
    e0 = P.eps0(dT)
    assert e0.shape == (6 * nx * ny * nz, 6)
    # expected centroid abscissa of tetrahedron p of hexahedron (i, j, k):
    # (i + offset) h with the offset set by where the ordering puts the x axis
    offsets = {0: 0.75, 1: 0.5, 2: 0.25}
    perms = mesh.kuhn_permutations()
    want = np.empty(6 * nx * ny * nz)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = i + nx * (j + ny * k)
                for p, perm in enumerate(perms):
                    xc = (i + offsets[perm.index(0)]) * h
                    want[6 * c + p] = -dT * math.exp(-xc / depth)
    for comp in range(3):
        assert np.allclose(e0[:, comp], want, rtol=1e-14, atol=0)
    assert np.all(e0[:, 3:] == 0.0)
    # linear in DT, zero at DT = 0
    assert np.allclose(P.eps0(-2 * dT)[:, 0], -2 * want, rtol=1e-14, atol=0)
    assert np.all(P.eps0(0.0) == 0.0)
    # the volume integral of the centroid values approaches the exact
    # integral of exp(-x/depth) over the slab (one-point rule, O(h^2))
    vol = P.model.vol
    exact = ly * lz * depth * (1.0 - math.exp(-lx / depth))
    approx = float(np.sum(vol * e0[:, 0])) / -dT
    assert abs(approx - exact) < 0.2 * (h / depth) ** 2 * exact


def test_pins_remove_every_rigid_mode_and_keep_K_spd():
    nx, ny, nz = 3, 3, 2
    P = problems.thermal_3d(nx, ny, nz, 1.0, 1.0, 0.25)
    M = P.model
    X, N = M.X, M.N
    # the six rigid motions: translations and infinitesimal rotations
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    zero, one = np.zeros(N), np.ones(N)
    R = np.stack([
        np.concatenate([one, zero, zero]), np.concatenate([zero, one, zero]),
        np.concatenate([zero, zero, one]),
        np.concatenate([-y, x, zero]), np.concatenate([zero, -z, y]), np.concatenate([z, zero, -x]),
    ], axis=1)
    assert np.allclose(M.K(np.zeros(N)) @ R, 0.0, atol=1e-12)
    # no rigid motion survives the Dirichlet set: R restricted to the fixed
    # DOFs has full column rank
    assert np.linalg.matrix_rank(R[P.fixed]) == 6
    # the set is minimal up to the clamped face: u_x = 0 on x = lx plus
    # exactly three point conditions
    right = np.isclose(x, 1.0)
    assert P.fixed[:N].sum() == right.sum() and np.all(P.fixed[:N] == right)
    assert P.fixed[N:].sum() == 3
    for alpha in (np.zeros(N), _rng(3).uniform(0.0, 1.0, N)):
        Kf = M.K(alpha)[P.free][:, P.free].toarray()
        ev = np.linalg.eigvalsh(Kf)
        assert ev.min() > 1e-8 * ev.max()


@pytest.mark.parametrize("damaged", [False, True])
def test_uniform_cooling_is_stress_free_contraction(damaged):
    nx, ny, nz, lx, ly, lz = 4, 3, 2, 1.0, 1.0, 0.25
    # depth -> infinity: exp(-x/depth) = 1 to rounding, a uniform cooling
    P = problems.thermal_3d(nx, ny, nz, lx, ly, lz, depth=1e18)
    M = P.model
    s = -0.02
    st = am.initial_state(P)
    if damaged:
        st.alpha = _rng(4).uniform(0.0, 0.95, M.N)
    am.set_load(P, st, -s)
    u = am.elastic_solve(P, st.u, st.alpha, -s)
    X = M.X
    want = np.concatenate([s * (X[:, 0] - lx), s * X[:, 1], s * X[:, 2]])
    assert np.max(np.abs(u - want)) < 1e-12
    el, _ = M.energies(u, st.alpha, P.eps0(-s))
    assert abs(el) < 1e-24


def test_uniform_cooling_never_damages_at1():
    """The contraction is stress free, so W2 = 0 everywhere and AT1 (an
    elastic phase below Gc / (c_w ell)) leaves alpha at zero exactly, even
    at a cooling fifty times the onset of a constrained layer."""
    P = problems.thermal_3d(4, 4, 2, 1.0, 1.0, 0.25, depth=1e18)
    st = am.initial_state(P)
    dTc = math.sqrt(3.0 * (1.0 - 0.3) / (16.0 * P.model.ell))
    o = am.solve_load_step(P, st, 50.0 * dTc, max_am=20)
    assert o["converged"]
    assert np.all(st.alpha == 0.0)
    assert np.max(P.model.W2(st.u, P.eps0(50.0 * dTc))) < 1e-20


def test_surface_layer_damages_and_interior_stays_intact():
    """With a thin heated layer (depth comparable to h), a strong shock
    damages nodes next to the face x = 0 only; a weak one none."""
    nx = 16
    P = problems.thermal_3d(nx, 8, 2, 1.0, 0.5, 0.125, ell=4.0 / nx, depth=0.05)
    dTc = math.sqrt(3.0 * (1.0 - 0.3) / (16.0 * P.model.ell))
    x = P.model.X[:, 0]
    st = am.initial_state(P)
    o = am.solve_load_step(P, st, 0.3 * dTc, max_am=50)
    assert o["converged"] and np.all(st.alpha == 0.0)
    o = am.solve_load_step(P, st, 16.0 * dTc, max_am=200)
    assert o["converged"]
    assert st.alpha.max() > 0.1
    assert np.all(x[st.alpha > 1e-3] < 0.5)


def _fd(fun, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (fun(x + e) - fun(x - e)) / (2 * h)
    return g


def _kuhn_model(model):
    X, T = mesh.structured_mesh_3d(2, 2, 1, 1.0, 1.0, 0.5)
    return fem.Model(X, T, ell=0.3, k_ell=1e-3, model=model)


@pytest.mark.parametrize("model", ["AT1", "AT2"])
def test_gradients_3d_match_energy_finite_differences(model):
    M = _kuhn_model(model)
    rng = _rng(11)
    u = 0.2 * rng.standard_normal(3 * M.N)
    alpha = rng.uniform(0.1, 0.9, M.N)
    eps0 = fem.isotropic_eigenstrain(0.05 * rng.standard_normal(len(M.T)), 3)
    E = lambda uu, aa: sum(M.energies(uu, aa, eps0))
    gu = _fd(lambda v: E(v, alpha), u)
    ga = _fd(lambda v: E(u, v), alpha)
    assert np.allclose(M.grad_u(u, alpha, eps0), gu, rtol=1e-7, atol=1e-9)
    assert np.allclose(M.grad_alpha(u, alpha, eps0), ga, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("model", ["AT1", "AT2"])
def test_hessian_blocks_3d_match_finite_differences(model):
    M = _kuhn_model(model)
    rng = _rng(12)
    u = 0.2 * rng.standard_normal(3 * M.N)
    alpha = rng.uniform(0.1, 0.9, M.N)
    eps0 = fem.isotropic_eigenstrain(0.05 * rng.standard_normal(len(M.T)), 3)
    K = M.K(alpha).toarray()
    B = M.coupling(u, alpha, eps0).toarray()
    C = M.damage_hessian(u, eps0).toarray()
    h = 1e-6
    for j in range(M.N):
        e = np.zeros(M.N)
        e[j] = h
        dGu = (M.grad_u(u, alpha + e, eps0) - M.grad_u(u, alpha - e, eps0)) / (2 * h)
        dGa = (M.grad_alpha(u, alpha + e, eps0) - M.grad_alpha(u, alpha - e, eps0)) / (2 * h)
        assert np.allclose(B[:, j], dGu, rtol=1e-6, atol=1e-8)
        assert np.allclose(C[:, j], dGa, rtol=1e-6, atol=1e-8)
    for j in range(3 * M.N):
        e = np.zeros(3 * M.N)
        e[j] = h
        dGu = (M.grad_u(u + e, alpha, eps0) - M.grad_u(u - e, alpha, eps0)) / (2 * h)
        dGa = (M.grad_alpha(u + e, alpha, eps0) - M.grad_alpha(u - e, alpha, eps0)) / (2 * h)
        assert np.allclose(K[:, j], dGu, rtol=1e-6, atol=1e-8)
        assert np.allclose(B[j, :], dGa, rtol=1e-6, atol=1e-8)


def test_thermal_step_solution_satisfies_kkt():
    """A converged 3D load step with the exponential eigenstrain: E_u = 0 on
    the free DOFs (solved directly here against the oracle's assembled
    operators) and the damage KKT signs of eq. (kkt)."""
    nx = 8
    P = problems.thermal_3d(nx, 4, 2, 1.0, 0.5, 0.25, ell=4.0 / nx, depth=0.1)
    M = P.model
    st = am.initial_state(P)
    dTc = math.sqrt(3.0 * (1.0 - 0.3) / (16.0 * M.ell))
    load = 10.0 * dTc
    o = am.solve_load_step(P, st, load, max_am=300, am_tol=1e-11)
    assert o["converged"]
    e0 = P.eps0(load)
    gu = M.grad_u(st.u, st.alpha, e0)[P.free]
    K = M.K(st.alpha)[P.free][:, P.free]
    scale = np.linalg.norm(M.f_eigen(st.alpha, e0))
    assert np.linalg.norm(gu) < 1e-8 * scale
    ga = M.grad_alpha(st.u, st.alpha, e0)
    lo = st.alpha <= st.alpha_prev + 1e-12
    hi = st.alpha >= 1.0 - 1e-12
    mid = ~lo & ~hi
    tol = 1e-8 * max(1.0, np.abs(ga).max())
    assert np.all(ga[lo] >= -tol) and np.all(ga[hi] <= tol)
    assert np.all(np.abs(ga[mid]) <= 1e3 * tol)
    # the elastic solve is exact: re-solving with the final alpha changes nothing
    u2 = st.u.copy()
    rhs = M.f_eigen(st.alpha, e0)[P.free] - M.K(st.alpha)[P.free][:, P.fixed] @ st.u[P.fixed]
    u2[P.free] = spla.spsolve(K.tocsc(), rhs)
    assert np.allclose(u2, st.u, atol=1e-9 * np.abs(st.u).max())
