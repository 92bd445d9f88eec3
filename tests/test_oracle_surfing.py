"""Pins of the surfing problem (Sec. 4.1) in the oracle.

The boundary field u_bar of eq. (surfingloading) is checked against what
linear elastic fracture mechanics fixes independently of its printed form:
it solves the homogeneous Navier equations of plane stress, leaves the crack
faces traction free, and its opening stress ahead of the tip is
K_I / sqrt(2 pi r) (the definition of the stress intensity factor).  The
damage evolution is checked against Griffith's prediction quoted in Sec. 4.1:
at K_I = sqrt(Gc E) the crack runs at the imposed speed v and dissipates
Gc v per unit time (up to the O(h/ell) overestimate of the discrete
regularised surface energy).
"""

import numpy as np
import pytest

from oracle import am, fem, problems

E, NU, KI = 1.0, 0.3, 1.0


def _stress(X, Y, d=1e-5):
    """Plane-stress stress of u_bar by central differences of the field."""
    ux = lambda x, y: problems.mode_i_displacement(x, y, KI, E, NU)[0]
    uy = lambda x, y: problems.mode_i_displacement(x, y, KI, E, NU)[1]
    exx = (ux(X + d, Y) - ux(X - d, Y)) / (2 * d)
    eyy = (uy(X, Y + d) - uy(X, Y - d)) / (2 * d)
    gxy = (ux(X, Y + d) - ux(X, Y - d)) / (2 * d) + (uy(X + d, Y) - uy(X - d, Y)) / (2 * d)
    lam, mu = fem.lame(E, NU, 2, plane_stress=True)
    sxx = (lam + 2 * mu) * exx + lam * eyy
    syy = lam * exx + (lam + 2 * mu) * eyy
    sxy = mu * gxy
    return sxx, syy, sxy


def test_mode_i_field_is_plane_stress_equilibrium():
    rng = np.random.default_rng(0)
    r = rng.uniform(0.2, 1.0, 20)
    th = rng.uniform(-2.5, 2.5, 20)          # away from the crack faces
    X, Y = r * np.cos(th), r * np.sin(th)
    d = 1e-3
    sxx_p, _, sxy_p = _stress(X + d, Y)
    sxx_m, _, sxy_m = _stress(X - d, Y)
    _, syy_p, syx_p = _stress(X, Y + d)
    _, syy_m, syx_m = _stress(X, Y - d)
    div_x = (sxx_p - sxx_m) / (2 * d) + (syx_p - syx_m) / (2 * d)
    div_y = (sxy_p - sxy_m) / (2 * d) + (syy_p - syy_m) / (2 * d)
    scale = KI / np.sqrt(2 * np.pi * r) / r
    assert np.max(np.abs(div_x) / scale) < 1e-4
    assert np.max(np.abs(div_y) / scale) < 1e-4


def test_mode_i_field_faces_free_and_stress_intensity():
    r = np.array([0.1, 0.3, 0.7])
    # traction free faces: sigma_yy = sigma_xy = 0 just above and below the crack
    for sgn in (1.0, -1.0):
        X, Y = -r, sgn * 1e-9 * np.ones_like(r)
        _, syy, sxy = _stress(X, Y, d=1e-10)
        assert np.max(np.abs(syy) * np.sqrt(r)) < 1e-3
        assert np.max(np.abs(sxy) * np.sqrt(r)) < 1e-3
    # opening stress ahead of the tip
    _, syy, sxy = _stress(r, 0.0 * r)
    assert np.allclose(syy, KI / np.sqrt(2 * np.pi * r), rtol=1e-6)
    assert np.max(np.abs(sxy)) < 1e-6
    # square-root scaling and symmetry of the opening
    ux1, uy1 = problems.mode_i_displacement(0.3, 0.2, KI, E, NU)
    ux4, uy4 = problems.mode_i_displacement(1.2, 0.8, KI, E, NU)
    assert np.isclose(ux4, 2 * ux1) and np.isclose(uy4, 2 * uy1)
    uxm, uym = problems.mode_i_displacement(0.3, -0.2, KI, E, NU)
    assert np.isclose(uxm, ux1) and np.isclose(uym, -uy1)


def test_surfing_crack_runs_at_v_and_dissipates_gc_v():
    """ell = 0.1, h = ell/4, K_I = sqrt(Gc E), v = 1 (Sec. 4.1), AT1, ORAM-N:
    after the initial transient the tip moves by v dt per step and the
    surface energy grows at Gc v, within the +15% overestimate that the
    regularised energy has on a mesh with h = ell/4."""
    ell = 0.1
    nx, ny = 80, 40
    P = problems.surfing_2d(nx, ny, ell=ell, KI=np.sqrt(1.0 * E), v=1.0, Lc=0.05, E=E, nu=NU)
    st = am.initial_state(P, problems.surfing_notch(nx, ny))
    X = P.model.X
    mid = np.isclose(X[:, 1], 0.5)
    surf, tips, ts = [], [], np.round(np.arange(0.0, 0.81, 0.1), 10)
    for t in ts:
        o = am.solve_load_step(P, st, t, newton_on=True, max_am=3000)
        assert o["converged"]
        surf.append(P.model.energies(st.u, st.alpha)[1])
        tips.append(X[mid & (st.alpha > 0.5), 0].max())
        assert np.all(st.alpha >= st.alpha_prev - 1e-15) and np.all(st.alpha <= 1.0)
    surf, tips = np.array(surf), np.array(tips)
    late = ts >= 0.3 - 1e-12
    rate = np.polyfit(ts[late], surf[late], 1)[0]
    assert 1.0 <= rate <= 1.15, rate
    assert np.all(np.abs(np.diff(tips[late]) - 0.1) <= 2.0 / nx + 1e-12), tips
