"""Pins of the 2D thermal shock (Sec. 4.3) in the oracle.

The eigenstrain path of the elastic energy (eq. (energytshock)) is checked
against a closed form: a uniform cooling s = -DT of the slab held at zero
lateral displacement is uniaxial strain, u_x = 0 and
u_y = 2 (lam + mu) / (lam + 2 mu) s (y - ly), which P1 represents exactly.
The damage side is checked against the purely elastic regime of Sec. 4.3:
below the critical shock the slab stays undamaged at every time tau, above
it damage appears in the cooled layer, and AT2 (no elastic phase) damages at
any intensity.
"""

import numpy as np
import pytest
from scipy.special import erfc

from oracle import am, fem, problems

NU = 0.3


def test_uniform_cooling_is_uniaxial_strain():
    for ps in (False, True):
        lx, ly = 16.0, 4.0
        P = problems.thermal_shock_2d(32, 8, lx, ly, dT=1.7, nu=NU, plane_stress=ps)
        st = am.initial_state(P)
        tau = 1e15                                   # erfc(y / (ell tau)) = 1 to rounding
        am.set_load(P, st, tau)
        u = am.elastic_solve(P, st.u, st.alpha, tau)
        N = P.model.N
        lam, mu = fem.lame(1.0, NU, 2, plane_stress=ps)
        s = -1.7
        c = 2.0 * (lam + mu) / (lam + 2.0 * mu) * s
        y = P.model.X[:, 1]
        assert np.max(np.abs(u[:N])) < 1e-12
        assert np.max(np.abs(u[N:] - c * (y - ly))) < 1e-11 * abs(c) * ly
        # the element stress is uniaxial: sigma_xx = E' s' only
        el, _ = P.model.energies(u, st.alpha, P.eps0(tau))
        Ep = 1.0 if ps else 1.0 / (1.0 - NU * NU)
        assert np.isclose(el, 0.5 * (1.0 + 1e-6) * Ep * s * s * lx * ly, rtol=1e-9)


def test_eigenstrain_profile_is_erfc_at_centroids():
    P = problems.thermal_shock_2d(8, 4, 8.0, 2.0, dT=2.0, ell=0.5)
    e0 = P.eps0(1.5)
    yc = P.model.X[P.model.T].mean(axis=1)[:, 1]
    want = -2.0 * erfc(yc / (0.5 * 1.5))
    assert np.allclose(e0[:, 0], want, rtol=0, atol=1e-15)
    assert np.allclose(e0[:, 1], want, rtol=0, atol=1e-15)
    assert np.all(e0[:, 2] == 0.0)
    assert np.all(P.eps0(0.0) == 0.0)
    # cells of a row: T0 centroids at (j + 1/3) h, T1 at (j + 2/3) h
    assert np.allclose(yc[0::2][:8], 0.5 / 3) and np.allclose(yc[1::2][:8], 1.0 / 3)


@pytest.mark.parametrize("ratio,damaged", [(0.97, False), (1.1, True)])
def test_elastic_regime_below_critical_shock(ratio, damaged):
    """AT1, h = ell/4: no damage at any tau below DT_c; damage in the cooled
    layer above it once the profile has spread (tau = 8)."""
    dTc = problems.thermal_shock_dTc(nu=NU)
    P = problems.thermal_shock_2d(64, 16, 16.0, 4.0, dT=ratio * dTc, nu=NU)
    st = am.initial_state(P)
    for tau in (0.25, 1.0, 8.0):
        o = am.solve_load_step(P, st, tau, max_am=200)
        assert o["converged"]
    y = P.model.X[:, 1]
    if damaged:
        assert st.alpha.max() > 1e-2
        assert np.all(y[st.alpha > 1e-3] < 2.0)              # only the cooled layer
    else:
        assert np.all(st.alpha == 0.0)


def test_at2_has_no_elastic_phase():
    P = problems.thermal_shock_2d(32, 8, 16.0, 4.0, dT=0.3, model="AT2", nu=NU)
    st = am.initial_state(P)
    o = am.solve_load_step(P, st, 1.0, max_am=200)
    assert o["converged"]
    assert st.alpha.max() > 0.0
    assert problems.thermal_shock_dTc(model="AT2") is None
