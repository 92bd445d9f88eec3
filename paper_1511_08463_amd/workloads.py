"""Seeded synthetic inputs shared by the tests, the bench and the smoke run.

This module holds input recipes only (mesh sizes, material constants, notch
geometry, load sequences, seeds); none of the method's arithmetic.  Both the
HIP path and the CPU oracle receive the same values from here.

Recipes (the paper uses no dataset; these stand in for its test problems):

* ``tension(n)``: the unit square, n x n right-diagonal cells, plane strain,
  E = 1, nu = 0.3, Gc = 1 (Sec. 4 fixes Gc = E = 1, nu = 0.3), k_ell = 1e-6,
  bottom u_y = 0, top u_y = t, with an initial crack alpha = 1 on the nodes of
  a horizontal segment starting at x = 0.
* ``config1``: 64 x 64, AT1, ell = 0.05, notch y = 0.5, x in [0, 0.3],
  10 steps t = 0.002 k.
* ``config2(model, omega, seed)``: 2048 x 2048, ell = 4h, notch height y0 and
  length a drawn from U[0.1, 0.4] (seed 0) and snapped to nodes, 20 steps
  t = 0.1 k.
* ``small_tension``: the config-2 recipe at a small n (parity sizes).
* ``config3``: the 3D thermal-shock slab [0,1] x [0,1] x [0,0.25],
  128 x 128 x 32 hexahedra split into 6 Kuhn tetrahedra, AT1, ell = 4h,
  eigenstrain -DT exp(-x/0.05) I, u_x = 0 on x = 1 plus the pins that
  remove the remaining rigid motions, DT_k = (k/15) 16 DT_c for k = 1..15
  with DT_c = sqrt(3 Gc (1 - nu) / (16 E ell)) (the onset of a thick surface
  layer under biaxial in-plane constraint, beta = 1).  The heated layer's
  W2 decays over 0.025 < ell, so onset comes later than DT_c (near 3 DT_c);
  the ramp runs to 16 DT_c, the largest intensity ratio of the paper's
  thermal-shock study, to cover nucleation and growth.
* ``surfing(ell)``: the surfing test of Sec. 4.1: the slab [0, 2] x [0, 1]
  (the paper's [0, L] x [-H/2, H/2] shifted by H/2), uniform cells of side
  h = ell/4 (the paper refines a band to h = ell/5; a uniform mesh here),
  plane stress, E = Gc = 1, nu = 0.3, K_I = sqrt(Gc E), v = 1, L_c = 0.05,
  AT1, the preexisting crack as alpha = 1 on the mid-line nodes with
  x <= L_c, loads t = 0.1 k.
* ``config5``: a served stream of independent tension problems: side
  n ~ U{64, ..., 1024}, ell ~ U[0.01, 0.05], h = ell/4, domain side
  L = n h, the config-2 notch recipe scaled by L, 10-30 load steps with
  t_k = k t_max / steps, t_max = c sqrt(L) (the onset displacement of a
  notched square scales like sqrt(L)); c = 1 by default, which reaches crack
  onset at the last steps (c = 2 drives most instances through unstable
  propagation across the whole specimen), Poisson arrivals at rate 50/s
  (seed 1), AT1, omega = 1, mixed precision, no Newton.
"""

import numpy as np


def notch_mask_2d(nx, ny, y0, length, lx=1.0, ly=1.0):
    """Nodes on the row nearest y = y0 with x <= length (uint8, node order)."""
    j0 = int(round(y0 / (ly / ny)))
    x = np.arange(nx + 1) * (lx / nx)
    mask = np.zeros((ny + 1, nx + 1), dtype=np.uint8)
    mask[j0, x <= length + 1e-12] = 1
    return mask.ravel()


def tension(n, ell, model="AT1", omega=1.0, **extra):
    """Parameters (keywords of ``fracture.make_params`` and of the oracle)."""
    p = dict(dim=2, nx=n, ny=n, lx=1.0, ly=1.0, model=model, E=1.0, nu=0.3, Gc=1.0,
             ell=ell, k_ell=1e-6, omega=omega, plane_stress=0)
    p.update(extra)
    return p


def config1():
    p = tension(64, 0.05, "AT1", am_tol=1e-5)
    notch = notch_mask_2d(64, 64, 0.5, 0.3)
    loads = [0.002 * k for k in range(1, 11)]
    return p, notch, loads


def notch_config2(n, seed=0):
    rng = np.random.default_rng(seed)
    y0 = rng.uniform(0.1, 0.4)
    a = rng.uniform(0.1, 0.4)
    h = 1.0 / n
    y0 = round(y0 / h) * h
    a = round(a / h) * h
    return y0, a


def config2(model="AT1", omega=1.0, seed=0, n=2048):
    h = 1.0 / n
    p = tension(n, 4 * h, model, omega)
    y0, a = notch_config2(n, seed)
    notch = notch_mask_2d(n, n, y0, a)
    loads = [0.1 * k for k in range(1, 21)]
    return p, notch, loads, (y0, a)


# Solver settings of the config-2 benchmark (bench.py's defaults): ORAM-N at
# omega = 1, switching to Newton at ||Phi||_2 < 1e-3 and stopping at 1e-9.
# Inside ORAM sweeps the subproblems are solved inexactly, since the Newton
# phase's stop test fixes the accuracy of the converged state: the elastic
# PCG stops at 0.95 of its warm-start residual (or 1e-8 of the load), the
# damage active-set iteration at 0.3 of its starting max |Phi|, and each of
# its reduced CG solves at 0.1 relative.  MINRES forcing by Eisenstat-Walker,
# one V-cycle per action of A^-1, the block-diagonal Newton preconditioner.
# The stop tolerance is tighter than the 1e-7 the paper's experiments use:
# once the specimen is cut, the translation of the upper piece is held only by
# the k_ell stiffness of the crack band, so a residual of 1e-7 leaves that soft
# mode, and u, uncertain beyond 1e-6 relative.  The parity test of the
# benchmarked path runs with exactly these settings.
CONFIG2_SOLVER = dict(am_tol=1e-5, pcg_rtol=1e-8, vi_cg_rtol=0.1, max_am=30000, newton=1,
                      switch_tol=1e-3, final_tol=1e-9, minres_rtol=1e-6, newton_vcycles=1,
                      newton_forcing=0.1, newton_forcing_mode=1, pcg_reduction=0.95,
                      vi_reduction=0.3, cheb_degree=2, newton_precond=1)


def small_tension(n, model="AT1", omega=1.0, seed=0, ell=None):
    h = 1.0 / n
    p = tension(n, ell if ell is not None else 4 * h, model, omega)
    y0, a = notch_config2(n, seed)
    return p, notch_mask_2d(n, n, y0, a), (y0, a)


def random_fields(N, ndof, seed, notch=None):
    """Random displacement and damage fields for operator checks."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(ndof)
    alpha = rng.uniform(0.0, 1.0, N)
    if notch is not None:
        alpha[np.asarray(notch, bool)] = 1.0
    return u, alpha


def oracle_kwargs(p):
    """The subset of parameters the oracle's problem builders take."""
    return dict(E=p["E"], nu=p["nu"], Gc=p["Gc"], ell=p["ell"], k_ell=p["k_ell"],
                model=p["model"], plane_stress=bool(p.get("plane_stress", 0)))


def config5(n_instances=256, seed=1, sizes=(64, 128, 256, 512, 1024), rate=50.0,
            max_am=None, load_scale=1.0, solver="oramn"):
    """Requests of the served stream: (rid, params, notch, loads, arrival).
    solver "oramn": ORAM-N with the 2048^2 benchmark's inexact sweeps
    (CONFIG2_SOLVER; up to 2000 sweeps per step); "am": alternate
    minimisation to ||dalpha||_inf < 1e-5 (up to 400 sweeps per step)."""
    if solver == "oramn":
        extra = dict(CONFIG2_SOLVER, max_am=2000 if max_am is None else max_am)
    elif solver == "am":
        extra = dict(max_am=400 if max_am is None else max_am)
    else:
        raise ValueError(solver)
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n_instances):
        n = int(rng.choice(sizes))
        ell = float(rng.uniform(0.01, 0.05))
        h = ell / 4.0
        L = n * h
        steps = int(rng.integers(10, 31))
        y0 = round(rng.uniform(0.1, 0.4) * n) * h
        a = round(rng.uniform(0.1, 0.4) * n) * h
        t += float(rng.exponential(1.0 / rate))
        p = tension(n, ell, "AT1", 1.0, lx=L, ly=L, precision=1, **extra)
        notch = notch_mask_2d(n, n, y0, a, L, L)
        loads = [k * (load_scale * np.sqrt(L)) / steps for k in range(1, steps + 1)]
        out.append(dict(rid=rid, params=p, notch=notch, loads=loads, arrival=t))
    return out


def surfing(ell=0.05, h_factor=4, model="AT1", steps=9, dt=0.1, **extra):
    """Parameters, preexisting-crack mask and loads of the surfing slab."""
    ny = int(round(1.0 / (ell / h_factor)))
    ny += ny % 2                                  # a node row on the mid line
    nx = 2 * ny
    p = dict(dim=2, nx=nx, ny=ny, lx=2.0, ly=1.0, model=model, E=1.0, nu=0.3, Gc=1.0, ell=ell,
             k_ell=1e-6, plane_stress=1, load_kind=2, surf_ki=1.0, surf_v=1.0, surf_lc=0.05)
    p.update(extra)
    x = np.arange(nx + 1) * (2.0 / nx)
    mask = np.zeros((ny + 1, nx + 1), dtype=np.uint8)
    mask[ny // 2, x <= p["surf_lc"] + 1e-12] = 1
    loads = [round(dt * k, 12) for k in range(steps)]
    return p, mask.ravel(), loads


def oracle_kwargs_surfing(p):
    return dict(lx=p["lx"], ly=p["ly"], KI=p["surf_ki"], v=p["surf_v"], Lc=p["surf_lc"], E=p["E"],
                nu=p["nu"], Gc=p["Gc"], ell=p["ell"], k_ell=p["k_ell"], model=p["model"],
                plane_stress=bool(p["plane_stress"]))


def thermal(nx, ny, nz, lx=1.0, ly=1.0, lz=0.25, ell=None, model="AT1", depth=0.05, **extra):
    if ell is None:
        ell = 4.0 * lx / nx
    p = dict(dim=3, nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, model=model, E=1.0, nu=0.3,
             Gc=1.0, ell=ell, k_ell=1e-6, load_kind=1, thermal_depth=depth)
    p.update(extra)
    return p


def thermal_dtc(p):
    """Onset temperature drop of the biaxially constrained surface layer (AT1)."""
    return float(np.sqrt(3.0 * p["Gc"] * (1.0 - p["nu"]) / (16.0 * p["E"] * p["ell"])))


def config3(n=128, nz=32, steps=15, dt_max_factor=16.0):
    p = thermal(n, n, nz, 1.0, 1.0, 0.25)
    dtc = thermal_dtc(p)
    loads = [(k / steps) * dt_max_factor * dtc for k in range(1, steps + 1)]
    return p, loads


def oracle_kwargs3(p):
    return dict(E=p["E"], nu=p["nu"], Gc=p["Gc"], ell=p["ell"], k_ell=p["k_ell"],
                model=p["model"], depth=p["thermal_depth"])


def tshock_dtc(E=1.0, nu=0.3, Gc=1.0, ell=1.0, plane_stress=0):
    """Critical shock of the 2D slab (AT1, beta = 1): the cooled surface layer
    at zero lateral strain and zero normal stress stores E' (beta T)^2,
    E' = E/(1 - nu^2) in plane strain or E in plane stress, and damage
    starts where that reaches Gc/(c_w ell) with c_w = 8/3 (Sec. 4.3)."""
    Ep = E if plane_stress else E / (1.0 - nu * nu)
    return float(np.sqrt(3.0 * Gc / (8.0 * ell * Ep)))


def tshock(nx, ny, lx=40.0, ly=10.0, ratio=2.0, ell=1.0, model="AT1", **extra):
    """The 2D thermal shock of Sec. 4.3 on [0, lx] x [0, ly] (the paper's
    slab is 40 x 10 with ell = 1): shock intensity ratio * DT_c; the load
    of each step is the dimensionless time tau."""
    p = dict(dim=2, nx=nx, ny=ny, lx=lx, ly=ly, model=model, E=1.0, nu=0.3, Gc=1.0, ell=ell,
             k_ell=1e-6, plane_stress=0, load_kind=3)
    p.update(extra)
    p["thermal_dT"] = ratio * tshock_dtc(p["E"], p["nu"], p["Gc"], p["ell"], p["plane_stress"])
    return p


def oracle_kwargs_tshock(p):
    return dict(lx=p["lx"], ly=p["ly"], dT=p["thermal_dT"], E=p["E"], nu=p["nu"], Gc=p["Gc"],
                ell=p["ell"], k_ell=p["k_ell"], model=p["model"],
                plane_stress=bool(p["plane_stress"]))
