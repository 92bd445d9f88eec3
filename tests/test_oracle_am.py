"""Pins of the oracle's alternate minimisation against closed forms.

* P6: homogeneous bar -- the discrete solution is exactly linear in u and
  uniform in alpha; AT1 stays undamaged up to the elastic limit
  sigma_c = sqrt(3 Gc E / (8 ell)) (Sec. 4, the relation ell = 3/8 Gc E/sigma_c^2,
  and the traction bar's t_c, Sec. 4.2) and beyond it alpha = 1 - 3Gc/(8 ell W2);
  AT2 gives alpha = W2 / (W2 + Gc/ell).
* P7: 1D localisation band -- a line of nodes at alpha = 1 develops the AT1
  profile (1 - |x|/(2 ell))^2 or the AT2 profile exp(-|x|/ell), and the
  surface energy per unit length tends to Gc.
* P8: with omega = 1 the energy never increases across a sub-step
  (Sec. 1.2: each AM sub-step minimises a convex problem).
* P9: bounds alpha_prev <= alpha <= 1 hold at every iterate.
* ORAM relaxation readings coincide for omega <= 1.
"""

import math
import os

import numpy as np
import pytest

from oracle import am, fem, mesh, problems

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def _bar(model, plane_stress, ell=0.1, nx=4, ny=4):
    return problems.tension_2d(nx, ny, ell=ell, k_ell=1e-6, model=model, plane_stress=plane_stress)


@pytest.mark.parametrize("plane_stress", [True, False])
def test_homogeneous_bar_elastic_limit_at1(plane_stress):
    g = _read_golden("traction_bar_elastic_limit.txt")
    ell = g["ell"]
    t_c = g["t_c"]                  # paper's closed form (1D / plane stress / 3D)
    P = _bar("AT1", plane_stress, ell=ell)
    nu = 0.3
    # in plane strain with free lateral edges the uniaxial-stress modulus is E/(1-nu^2)
    tc = t_c if plane_stress else t_c * math.sqrt(1 - nu * nu)
    for t, damaged in ((0.999 * tc, False), (1.02 * tc, True)):
        st = am.initial_state(P)
        stats = am.solve_load_step(P, st, t, am_tol=1e-13)
        if not damaged:
            assert np.all(st.alpha == 0.0)
        else:
            W2 = (1.0 if plane_stress else 1.0 / (1 - nu * nu)) * t * t
            want = 1 - 3.0 / (8 * ell * W2)
            assert want > 0
            assert np.allclose(st.alpha, want, rtol=1e-10, atol=1e-12)
            # uniform damage leaves u linear: one more sweep changes nothing
            assert stats["sweeps"] <= 3
        # u is exactly the uniaxial-stress linear field
        N = P.model.N
        X = P.model.X
        assert np.allclose(st.u[N:], t * X[:, 1], atol=1e-12)
        exx = st.u[:N] / np.where(X[:, 0] > 0, X[:, 0], 1.0)
        assert np.allclose(exx[X[:, 0] > 0], exx[X[:, 0] > 0][0], rtol=1e-9)


def test_homogeneous_bar_at2_closed_form():
    ell = 0.1
    P = _bar("AT2", True, ell=ell)
    st = am.initial_state(P)
    t = 0.7
    am.solve_load_step(P, st, t, am_tol=1e-14, max_am=200)
    # AM converges to the coupled fixed point: alpha = W2 / (W2 + Gc/ell), W2 = t^2
    W2 = t * t
    want = W2 / (W2 + 1.0 / ell)
    assert np.allclose(st.alpha, want, rtol=1e-9)
    el, surf = P.model.energies(st.u, st.alpha)
    area = 1.0
    a = (1 - want) ** 2 + 1e-6
    assert math.isclose(el, area * 0.5 * a * W2, rel_tol=1e-9)
    assert math.isclose(surf, area * (1.0 / 2.0) * want ** 2 / ell, rel_tol=1e-9)


def _band(model, ny, ell=0.05, nx=2):
    """A strip [0, 0.25] x [0, 1] with alpha = 1 on the node row y = 1/2."""
    P = problems.tension_2d(nx, ny, lx=0.25, ly=1.0, ell=ell, model=model)
    X = P.model.X
    notch = np.isclose(X[:, 1], 0.5)
    st = am.initial_state(P, notch)
    am.solve_load_step(P, st, 0.0, am_tol=1e-12, max_am=50)
    return P, st


@pytest.mark.parametrize("model", ["AT1", "AT2"])
def test_band_profile_and_surface_energy(model):
    ell = 0.05
    errs, energies = [], []
    for ny in (40, 80, 160):
        P, st = _band(model, ny, ell)
        X = P.model.X
        col = np.isclose(X[:, 0], 0.125)
        y = X[col, 1]
        a = st.alpha[col]
        r = np.abs(y - 0.5)
        if model == "AT1":
            exact = np.where(r < 2 * ell, (1 - r / (2 * ell)) ** 2, 0.0)
        else:
            exact = np.exp(-r / ell)
        errs.append(np.max(np.abs(a - exact)))
        _, surf = P.model.energies(st.u, st.alpha)
        energies.append(surf / 0.25)
        # AT1 (no mass term) keeps the profile one-dimensional on every
        # column; AT2's consistent mass couples the boundary columns to their
        # diagonal neighbours asymmetrically, a genuine 2D discretisation effect
        if model == "AT1":
            for i in (0, 2):
                c2 = np.isclose(X[:, 0], 0.125 * i)
                assert np.allclose(st.alpha[c2], a, atol=1e-10)
    # AT1: the band edge 2 ell falls on a node and the 1D P1 solution of a
    # constant-coefficient second-order problem is nodally exact; AT2's
    # exponential profile converges under refinement
    if model == "AT1":
        assert max(errs) < 1e-12
    else:
        assert errs[2] < errs[1] < errs[0]
        assert errs[2] < 0.02
    e = np.abs(np.array(energies) - 1.0)
    assert e[2] < e[1] < e[0]
    assert e[2] < 0.03


def test_energy_monotone_with_omega_one_and_bounds():
    """P8 and P9 on a notched square at a load that grows damage."""
    P = problems.tension_2d(16, 16, ell=0.1, model="AT1")
    X = P.model.X
    notch = np.isclose(X[:, 1], 0.5) & (X[:, 0] <= 0.3 + 1e-12)
    st = am.initial_state(P, notch)
    prev_alpha = st.alpha.copy()
    for t in (0.5, 1.0, 1.3):
        trace = []
        am.set_load(P, st, t)
        e0 = sum(P.model.energies(st.u, st.alpha))
        trace_e = [e0]
        lower = st.alpha_prev.copy()
        for _ in range(15):
            am.oram_sweep(P, st, 1.0, trace=trace)
            assert np.all(st.alpha >= lower) and np.all(st.alpha <= 1.0)
        trace_e += [sum(e) for _, e in trace]
        d = np.diff(trace_e)
        assert np.all(d <= 1e-12 * max(1.0, abs(trace_e[0])))
        st.alpha_prev = st.alpha.copy()
        assert np.all(st.alpha >= prev_alpha)
        prev_alpha = st.alpha.copy()
    assert st.alpha[~notch].max() > 0.5          # the crack did grow


def test_relaxation_modes():
    rng = np.random.default_rng(3)
    n = 200
    lower = rng.uniform(0, 0.5, n)
    alpha = np.clip(lower + rng.uniform(0, 0.5, n), lower, 1)
    target = np.clip(rng.uniform(-0.2, 1.2, n), lower, 1)
    d = target - alpha
    for w in (0.5, 0.8, 1.0):
        ref = alpha + w * d
        for mode in ("project", "ratio", "bisect"):
            assert np.allclose(am.relax_alpha(alpha, d, w, lower, mode), ref, atol=1e-15)
    w = 1.6
    # targets strictly inside the box: the exact ratio factor lies in (1, omega]
    target = lower + (1 - lower) * rng.uniform(0.05, 0.95, n)
    d = target - alpha
    r1 = am.relax_alpha(alpha, d, w, lower, "ratio")
    r2 = am.relax_alpha(alpha, d, w, lower, "bisect")
    r3 = am.relax_alpha(alpha, d, w, lower, "project")
    for r in (r1, r2, r3):
        assert np.all(r >= lower) and np.all(r <= 1)
    nz = np.abs(d) > 1e-3
    s1 = (r1 - alpha)[nz] / d[nz]
    wbar = s1[0]
    assert np.allclose(s1, wbar) and 1.0 < wbar <= w
    # largest common factor: one component sits on a bound, and any larger
    # factor leaves the box
    assert np.any(np.isclose(r1, 1.0, rtol=0, atol=1e-14) | np.isclose(r1, lower, rtol=0, atol=1e-14))
    bigger = alpha + (wbar * (1 + 1e-9)) * d
    assert np.any((bigger > 1) | (bigger < lower)) or wbar == w
    # bisection: a single factor in [1, omega], feasible, no larger than the ratio test
    s2 = (r2 - alpha)[nz] / d[nz]
    assert np.allclose(s2, s2[0]) and 1.0 <= s2[0] <= wbar + 1e-12
    # projection: pointwise, equals alpha + omega*d wherever that is feasible
    free = ((alpha + w * d) <= 1) & ((alpha + w * d) >= lower)
    assert np.allclose(r3[free], (alpha + w * d)[free])


def test_oram_n_reaches_am_fixed_point_and_recovers_from_failure():
    P = problems.tension_2d(12, 12, ell=0.1, model="AT1")
    X = P.model.X
    notch = np.isclose(X[:, 1], 0.5) & (X[:, 0] <= 0.3 + 1e-12)
    loads = [0.6, 1.2]
    ref = am.initial_state(P, notch)
    am.run(P, ref, loads, omega=1.0, am_stop="phi", final_tol=1e-11, max_am=5000)
    for kw in ({"max_newton": 10}, {"max_newton": 1}):
        st = am.initial_state(P, notch)
        out = am.run(P, st, loads, omega=1.2, newton_on=True, switch_tol=1e-3,
                     final_tol=1e-11, max_am=5000, **kw)
        assert all(o["converged"] for o in out)
        assert any(o["newton_its"] > 0 for o in out)
        assert np.allclose(st.alpha, ref.alpha, atol=1e-7)
        assert np.allclose(st.u, ref.u, atol=1e-7)
        nphi = np.linalg.norm(am.residual(P, st))
        assert nphi <= 1e-11


def test_block_preconditioner_identity():
    """The fieldsplit preconditioner with S ~ C (Sec. 3.3) read with the lower
    factor [[I, 0], [-B^T, I]]: its action y1 = A^-1 x1, y2 = C^-1 (x2 - B^T y1),
    z1 = A^-1 (x1 - B y2) equals the inverse of [[A, B], [B^T, C + B^T A^-1 B]]
    and the expanded block form printed in the paper."""
    rng = np.random.default_rng(0)
    n1, n2 = 7, 5
    X = rng.standard_normal((n1, n1)); A = X @ X.T + n1 * np.eye(n1)
    Y = rng.standard_normal((n2, n2)); C = Y @ Y.T + n2 * np.eye(n2)
    B = rng.standard_normal((n1, n2))
    Ai, Ci = np.linalg.inv(A), np.linalg.inv(C)
    x = rng.standard_normal(n1 + n2)
    y1 = Ai @ x[:n1]
    y2 = Ci @ (x[n1:] - B.T @ y1)
    z1 = Ai @ (x[:n1] - B @ y2)
    P = np.block([[A, B], [B.T, C + B.T @ Ai @ B]])
    assert np.allclose(np.concatenate([z1, y2]), np.linalg.solve(P, x))
    expanded = np.block([[Ai + Ai @ B @ Ci @ B.T @ Ai, -Ai @ B @ Ci], [-Ci @ B.T @ Ai, Ci]])
    assert np.allclose(expanded @ x, np.linalg.solve(P, x))
    # and it is symmetric positive definite
    assert np.allclose(expanded, expanded.T) and np.linalg.eigvalsh(expanded).min() > 0


def test_young_omega_matches_sor_theory():
    """The automatic factor is Young's optimum for SOR: for a consistently
    ordered matrix (the 1D Laplacian) with Gauss-Seidel convergence factor
    rho, the SOR iteration matrix at young_omega has the smallest spectral
    radius over omega, and that radius is omega - 1.  The window is the
    ||dalpha|| history a contraction by rho leaves."""
    n = 24
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    D = np.diag(np.diag(A))
    L = -np.tril(A, -1)
    U = -np.triu(A, 1)

    def sor_radius(w):
        T = np.linalg.solve(D - w * L, (1 - w) * D + w * U)
        return np.max(np.abs(np.linalg.eigvals(T)))

    rho = sor_radius(1.0)                       # Gauss-Seidel
    window = [rho ** k for k in range(am.OMEGA_PROBE + 1)]
    w = am.young_omega(window, 1.99)
    grid = np.linspace(1.0, 1.99, 397)
    best = grid[np.argmin([sor_radius(x) for x in grid])]
    assert abs(w - best) < 0.01
    assert abs(sor_radius(w) - (w - 1.0)) < 1e-3
    assert sor_radius(w) <= min(sor_radius(x) for x in grid) + 1e-3
    # closed form at rho = 0.81 and the cap
    assert abs(am.young_omega([0.81 ** k for k in range(5)], 1.9) - 2.0 / (1.0 + math.sqrt(0.19))) < 1e-12
    assert am.young_omega([0.99 ** k for k in range(5)], 1.5) == 1.5
    # no contraction, no estimate
    assert am.young_omega([1.0, 1.0, 1.0, 1.0, 2.0], 1.9) is None
    assert am.young_omega([0.0, 0.0, 0.0, 0.0, 0.0], 1.9) is None


def test_auto_omega_load_step():
    """Automatic over-relaxation on the surfing slab (ell = 0.1, the step
    from t = 0 to t = 0.1): omega stays 1 for the first probe window, then
    takes one value in (1, cap]; the step reaches the state of plain
    alternate minimisation in fewer sweeps.  A step that converges within
    the first window runs exactly as at omega = 1."""
    from paper_1511_08463_amd import workloads
    p, notch, _ = workloads.surfing(0.1, steps=4)
    P = problems.surfing_2d(p["nx"], p["ny"], **workloads.oracle_kwargs_surfing(p))
    ref = am.initial_state(P, notch.astype(bool))
    am.solve_load_step(P, ref, 0.0, am_tol=1e-8, max_am=3000)
    st = ref.copy()
    o1 = am.solve_load_step(P, ref, 0.1, am_tol=1e-9, max_am=3000)
    oa = am.solve_load_step(P, st, 0.1, omega=1.9, omega_auto=True, am_tol=1e-9, max_am=3000)
    assert o1["converged"] and oa["converged"]
    k = am.OMEGA_PROBE + 1
    assert oa["omega"][:k] == [1.0] * k
    later = set(oa["omega"][k:])
    assert len(later) == 1 and 1.0 < later.pop() <= 1.9
    assert oa["sweeps"] < 0.85 * o1["sweeps"]
    assert np.max(np.abs(st.alpha - ref.alpha)) < 1e-7
    assert np.linalg.norm(st.u - ref.u) < 1e-6 * np.linalg.norm(ref.u)
    # an undamaged bar below the elastic limit converges before any estimate
    B = problems.tension_2d(8, 8, ell=0.1, model="AT1")
    s1, s2 = am.initial_state(B), am.initial_state(B)
    q1 = am.solve_load_step(B, s1, 0.05, am_tol=1e-10)
    q2 = am.solve_load_step(B, s2, 0.05, omega=1.9, omega_auto=True, am_tol=1e-10)
    assert q1["sweeps"] <= am.OMEGA_PROBE and q2["omega"] == [1.0] * q2["sweeps"]
    assert np.array_equal(s1.alpha, s2.alpha) and np.array_equal(s1.u, s2.u)
