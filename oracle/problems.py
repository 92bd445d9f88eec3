"""Boundary-value problems the oracle solves.

Test infrastructure (see the package docstring).  A Problem bundles the
discrete model (``fem.Model``) with its Dirichlet data, the optional thermal
eigenstrain and the damage bounds:

* 2D tension (the traction-type load of Sec. 4.2 on a notched square):
  u_y = 0 on the bottom edge, u_y = t on the top edge, lateral edges free.
  The x-translation left free by these conditions is removed by u_x = 0 at
  the node (0, 0).
* Surfing (Sec. 4.1): the slab [0, lx] x [0, ly] (the paper's
  [0, L] x [-H/2, H/2] shifted by H/2) with u = u_bar(x - Lc - v t, y - ly/2)
  on the whole boundary, u_bar the asymptotic Mode-I crack-tip displacement
  of eq. (surfingloading) with kappa = (3 - nu)/(1 + nu) as printed.  On the
  crack line behind the tip (y = ly/2, x < Lc + v t) the two crack faces
  carry opposite u_y; a boundary node there takes their mean, u = 0.
* 2D thermal shock (Sec. 4.3, eqs. (energytshock), (tempfielderfc)): the
  slab [0, lx] x [0, ly] (the paper's [-L/2, L/2] x [0, H] shifted by L/2),
  cooled on its bottom face y = 0; eps0 = beta T I with T = -DT
  erfc(y / (ell tau)) evaluated at each triangle's centroid, the loading
  parameter being the dimensionless time tau (eps0 = 0 at tau = 0).  The
  displacement conditions of the paper's sketch are not in its text; the
  reading here: u_x = 0 on the lateral edges x = 0, lx and u_y = 0 on the
  top edge y = ly, the cooled face traction free.
* 3D thermal shock with an exponential temperature profile through x
  (a variant of Sec. 4.3, eqs. (energytshock), (tempfielderfc)): eps0 =
  -DT exp(-x / depth) I evaluated at each tetrahedron's centroid (beta = 1),
  u_x = 0 on the face x = lx; the y/z translations and the rotation about x
  that remain are removed by u_y = u_z = 0 at (lx, 0, 0) and u_z = 0 at
  (lx, ly, 0).

Damage bounds, Sec. 1.1 (the set D): alpha_prev <= alpha <= 1.  Nodes of an
initial notch carry alpha = alpha_prev = 1, so they are fixed.  No damage
Dirichlet condition is imposed anywhere else.
"""

import numpy as np

from . import fem, mesh


class Problem:
    def __init__(self, model, fixed, dirichlet, eps0=None):
        self.model = model
        self.fixed = fixed                  # bool over d*N displacement DOFs
        self.free = ~fixed
        self._dirichlet = dirichlet         # load -> values over d*N (used on fixed DOFs)
        self._eps0 = eps0                   # load -> [E, nvoigt] or None

    def dirichlet_values(self, load):
        return self._dirichlet(load)

    def eps0(self, load):
        return None if self._eps0 is None else self._eps0(load)


def tension_2d(nx, ny, lx=1.0, ly=1.0, E=1.0, nu=0.3, Gc=1.0, ell=0.05, k_ell=1e-6,
               model="AT1", plane_stress=False):
    X, T = mesh.structured_mesh_2d(nx, ny, lx, ly)
    M = fem.Model(X, T, E=E, nu=nu, Gc=Gc, ell=ell, k_ell=k_ell, model=model,
                  plane_stress=plane_stress)
    N = M.N
    fixed = np.zeros(2 * N, dtype=bool)
    bottom = np.flatnonzero(np.isclose(X[:, 1], 0.0))
    top = np.flatnonzero(np.isclose(X[:, 1], ly))
    fixed[N + bottom] = True
    fixed[N + top] = True
    fixed[0] = True                                         # u_x at node (0,0)

    def dirichlet(t):
        v = np.zeros(2 * N)
        v[N + top] = t
        return v

    return Problem(M, fixed, dirichlet)


def mode_i_displacement(X, Y, KI, E, nu):
    """u_bar of eq. (surfingloading): K_I / (2 mu) sqrt(r / 2pi)
    (kappa - cos theta) (cos(theta/2), sin(theta/2)), (r, theta) the polar
    coordinates of (X, Y) about the crack tip, theta in (-pi, pi]; zero on
    the crack line behind the tip (the mean of the two faces)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    mu = E / (2.0 * (1.0 + nu))
    kappa = (3.0 - nu) / (1.0 + nu)
    r = np.hypot(X, Y)
    theta = np.arctan2(Y, X)
    f = KI / (2.0 * mu) * np.sqrt(r / (2.0 * np.pi)) * (kappa - np.cos(theta))
    ux = f * np.cos(0.5 * theta)
    uy = f * np.sin(0.5 * theta)
    on_faces = (Y == 0.0) & (X < 0.0)
    ux = np.where(on_faces, 0.0, ux)
    uy = np.where(on_faces, 0.0, uy)
    return ux, uy


def surfing_2d(nx, ny, lx=2.0, ly=1.0, KI=1.0, v=1.0, Lc=0.05, E=1.0, nu=0.3, Gc=1.0,
               ell=0.05, k_ell=1e-6, model="AT1", plane_stress=True):
    X, T = mesh.structured_mesh_2d(nx, ny, lx, ly)
    M = fem.Model(X, T, E=E, nu=nu, Gc=Gc, ell=ell, k_ell=k_ell, model=model,
                  plane_stress=plane_stress)
    N = M.N
    x, y = X[:, 0], X[:, 1]
    edge = (np.isclose(x, 0.0) | np.isclose(x, lx) | np.isclose(y, 0.0) | np.isclose(y, ly))
    fixed = np.concatenate([edge, edge])
    # height above the mid line from the integer row index (exactly 0 on it)
    jrow = np.rint(y / (ly / ny))
    ymid = (2.0 * jrow - ny) * (0.5 * ly / ny)

    def dirichlet(t):
        ux, uy = mode_i_displacement(x - Lc - v * t, ymid, KI, E, nu)
        return np.concatenate([np.where(edge, ux, 0.0), np.where(edge, uy, 0.0)])

    return Problem(M, fixed, dirichlet)


def surfing_notch(nx, ny, lx=2.0, ly=1.0, Lc=0.05):
    """The preexisting crack: nodes of the mid line y = ly/2 with x <= Lc."""
    X, _ = mesh.structured_mesh_2d(nx, ny, lx, ly)
    return np.isclose(X[:, 1], 0.5 * ly) & (X[:, 0] <= Lc + 1e-12)


def thermal_shock_2d(nx, ny, lx=40.0, ly=10.0, dT=1.0, beta=1.0, E=1.0, nu=0.3, Gc=1.0,
                     ell=1.0, k_ell=1e-6, model="AT1", plane_stress=False):
    """The 2D thermal shock; the load passed to dirichlet/eps0 is tau."""
    from scipy.special import erfc
    X, T = mesh.structured_mesh_2d(nx, ny, lx, ly)
    M = fem.Model(X, T, E=E, nu=nu, Gc=Gc, ell=ell, k_ell=k_ell, model=model,
                  plane_stress=plane_stress)
    N = M.N
    fixed = np.zeros(2 * N, dtype=bool)
    fixed[np.flatnonzero(np.isclose(X[:, 0], 0.0) | np.isclose(X[:, 0], lx))] = True
    fixed[N + np.flatnonzero(np.isclose(X[:, 1], ly))] = True
    yc = X[T].mean(axis=1)[:, 1]

    def dirichlet(tau):
        return np.zeros(2 * N)

    def eps0(tau):
        if tau <= 0.0:
            return fem.isotropic_eigenstrain(np.zeros(len(T)), 2)
        return fem.isotropic_eigenstrain(-beta * dT * erfc(yc / (ell * tau)), 2)

    return Problem(M, fixed, dirichlet, eps0)


def thermal_shock_dTc(E=1.0, nu=0.3, Gc=1.0, ell=1.0, beta=1.0, model="AT1",
                      plane_stress=False):
    """Shock intensity below which the 2D slab stays undamaged (the purely
    elastic regime of Sec. 4.3), in the reading that the cooled surface layer
    is held at zero lateral strain and free of normal stress: there the
    effective strain energy density A0 eps_eff : eps_eff is E' (beta T)^2 with
    E' = E / (1 - nu^2) (plane strain) or E (plane stress), and AT1 damage
    starts where it reaches G_c / (c_w ell) (c_w = 8/3).  AT2 has no elastic
    phase (damage for any load), so None."""
    if model != "AT1":
        return None
    Ep = E if plane_stress else E / (1.0 - nu * nu)
    return np.sqrt(3.0 * Gc / (8.0 * ell * Ep)) / beta


def thermal_3d(nx, ny, nz, lx=1.0, ly=1.0, lz=0.25, E=1.0, nu=0.3, Gc=1.0, ell=None,
               k_ell=1e-6, model="AT1", depth=0.05):
    if ell is None:
        ell = 4.0 * lx / nx
    X, T = mesh.structured_mesh_3d(nx, ny, nz, lx, ly, lz)
    M = fem.Model(X, T, E=E, nu=nu, Gc=Gc, ell=ell, k_ell=k_ell, model=model)
    N = M.N
    fixed = np.zeros(3 * N, dtype=bool)
    right = np.flatnonzero(np.isclose(X[:, 0], lx))
    fixed[right] = True
    p0 = mesh.node_id_3d(nx, 0, 0, nx, ny)
    p1 = mesh.node_id_3d(nx, ny, 0, nx, ny)
    fixed[N + p0] = True
    fixed[2 * N + p0] = True
    fixed[2 * N + p1] = True
    xc = X[T].mean(axis=1)[:, 0]
    shape = np.exp(-xc / depth)

    def dirichlet(dT):
        return np.zeros(3 * N)

    def eps0(dT):
        return fem.isotropic_eigenstrain(-dT * shape, 3)

    return Problem(M, fixed, dirichlet, eps0)
