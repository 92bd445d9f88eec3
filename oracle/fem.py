"""Element integrals and assembled operators of the regularised energy.

Test infrastructure (see the package docstring).  Every function follows a
passage of the paper and integrates exactly:

* energy  E(u, a) = int 1/2 a(alpha) A0 eps(u):eps(u)
                   + Gc/c_w (w(alpha)/ell + ell grad alpha . grad alpha)
  -- eq. (regenergy), Sec. 1.1, with a(alpha) = (1-alpha)^2 + k_ell and
  w(alpha) = alpha (AT1, the model used in the rest of the paper) or alpha^2
  (AT2, the Ambrosio--Tortorelli choice), c_w = 4 int_0^1 sqrt(w).
* first derivatives E_u, E_alpha -- eq. (kkt), Sec. 1.2.
* second derivatives E_uu, E_ualpha, E_alphaalpha -- eqs. (elasticity),
  (offdiag), (helmholtz), Sec. 1.2.
* thermal eigenstrain eps_eff = eps(u) - eps0 -- eq. (energytshock), Sec. 4.3.

Readings of points the paper leaves open (quadrature of a(alpha) exact, i.e.
degree 2; consistent mass; eigenstrain constant per element at its centroid)
are stated where used.

Displacement DOF numbering is blocked: component c of node n is c*N + n.
Voigt order: 2D (xx, yy, 2xy); 3D (xx, yy, zz, 2yz, 2xz, 2xy).
"""

import math

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# material and model constants
# ----------------------------------------------------------------------------

def lame(E, nu, dim, plane_stress=False):
    """Lame constants of the isotropic A0 (sigma = lam tr(eps) I + 2 mu eps).

    In 2D plane stress the first constant becomes 2 lam mu / (lam + 2 mu).
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    if dim == 2 and plane_stress:
        lam = 2.0 * lam * mu / (lam + 2.0 * mu)
    return lam, mu


def voigt_D(dim, lam, mu):
    """A0 in Voigt form with engineering shear strains."""
    if dim == 2:
        return np.array([[lam + 2 * mu, lam, 0.0],
                         [lam, lam + 2 * mu, 0.0],
                         [0.0, 0.0, mu]])
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def c_w(model):
    """c_w = 4 int_0^1 sqrt(w(s)) ds (Sec. 1.1): AT1 w = s -> 8/3; AT2 w = s^2 -> 2."""
    if model == "AT1":
        return 8.0 / 3.0
    if model == "AT2":
        return 2.0
    raise ValueError(model)


# ----------------------------------------------------------------------------
# simplex geometry
# ----------------------------------------------------------------------------

def geometry(X, T):
    """Volumes |T_e| and gradients of the barycentric coordinates.

    Returns vol[E] and grad[E, d+1, d] with grad[e, a] = grad(phi_a) on T_e.
    """
    d = X.shape[1]
    P = X[T]                                   # [E, d+1, d]
    J = (P[:, 1:, :] - P[:, :1, :])            # rows: edge vectors v_a - v_0
    detJ = np.linalg.det(J)
    vol = np.abs(detJ) / math.factorial(d)
    # phi_a = lambda_a; for a >= 1, grad lambda = rows of inv(J)^T ... solve J g = e
    Jinv = np.linalg.inv(J)                    # [E, d, d]
    g = np.transpose(Jinv, (0, 2, 1))          # grad lambda_a (a=1..d) as rows
    grad = np.empty((len(T), d + 1, d))
    grad[:, 1:, :] = g
    grad[:, 0, :] = -g.sum(axis=1)
    return vol, grad


def strain_matrix(grad):
    """B[E, nvoigt, d*(d+1)] mapping local DOFs (component-major: c*(d+1)+a)
    to Voigt strains."""
    E, nv, d = grad.shape
    if d == 2:
        B = np.zeros((E, 3, 2 * nv))
        for a in range(nv):
            gx, gy = grad[:, a, 0], grad[:, a, 1]
            B[:, 0, 0 * nv + a] = gx
            B[:, 1, 1 * nv + a] = gy
            B[:, 2, 0 * nv + a] = gy
            B[:, 2, 1 * nv + a] = gx
        return B
    B = np.zeros((E, 6, 3 * nv))
    for a in range(nv):
        gx, gy, gz = grad[:, a, 0], grad[:, a, 1], grad[:, a, 2]
        B[:, 0, 0 * nv + a] = gx
        B[:, 1, 1 * nv + a] = gy
        B[:, 2, 2 * nv + a] = gz
        B[:, 3, 1 * nv + a] = gz
        B[:, 3, 2 * nv + a] = gy
        B[:, 4, 0 * nv + a] = gz
        B[:, 4, 2 * nv + a] = gx
        B[:, 5, 0 * nv + a] = gy
        B[:, 5, 1 * nv + a] = gx
    return B


def local_dofs(T, N, d):
    """Global DOF index of each local (component-major) DOF: [E, d*(d+1)]."""
    nv = T.shape[1]
    return np.concatenate([T + c * N for c in range(d)], axis=1)


def reference_mass(d):
    """Consistent P1 mass on a simplex divided by its volume:
    int phi_a phi_b = |T| (1 + delta_ab) / ((d+1)(d+2))."""
    nv = d + 1
    return (np.ones((nv, nv)) + np.eye(nv)) / ((d + 1) * (d + 2))


# ----------------------------------------------------------------------------
# coefficients a(alpha), strains and W2 = A0 eps:eps
# ----------------------------------------------------------------------------

def avg_degradation(alpha, T, k_ell, d):
    """Element average of a(alpha) = (1-alpha)^2 + k_ell with alpha P1,
    integrated exactly (degree 2): k + b^T M_ref b, b = 1 - alpha at the
    element's vertices."""
    b = 1.0 - alpha[T]
    Mr = reference_mass(d)
    return k_ell + np.einsum("ea,ab,eb->e", b, Mr, b)


def element_strains(u, T, grad):
    """Voigt strain of P1 displacement u (blocked) on each element."""
    E, nv, d = grad.shape
    N = u.size // d
    comps = [u[c * N:(c + 1) * N][T] for c in range(d)]       # [E, nv] each
    Gu = np.stack([np.einsum("ea,eak->ek", comps[c], grad) for c in range(d)], axis=1)  # [E, c, k] = du_c/dx_k
    if d == 2:
        return np.stack([Gu[:, 0, 0], Gu[:, 1, 1], Gu[:, 0, 1] + Gu[:, 1, 0]], axis=1)
    return np.stack([Gu[:, 0, 0], Gu[:, 1, 1], Gu[:, 2, 2],
                     Gu[:, 1, 2] + Gu[:, 2, 1],
                     Gu[:, 0, 2] + Gu[:, 2, 0],
                     Gu[:, 0, 1] + Gu[:, 1, 0]], axis=1)


def w2(eps_eff, D):
    """W2_e = A0 eps_eff : eps_eff (twice the undamaged energy density)."""
    return np.einsum("ei,ij,ej->e", eps_eff, D, eps_eff)


def isotropic_eigenstrain(s, dim):
    """Voigt form of eps0 = s I for per-element scalars s[E]."""
    out = np.zeros((len(s), 3 if dim == 2 else 6))
    out[:, :dim] = s[:, None]
    return out


# ----------------------------------------------------------------------------
# assembly
# ----------------------------------------------------------------------------

def _assemble(rows, cols, vals, n):
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()


def assemble_elasticity(X, T, coef, D):
    """K = sum_e coef_e |T_e| B_e^T D B_e, eq. (elasticity) with coef_e the
    element average of a(alpha)."""
    N, d = X.shape
    vol, grad = geometry(X, T)
    B = strain_matrix(grad)
    Ke = np.einsum("e,eik,ij,ejl->ekl", coef * vol, B, D, B)
    ld = local_dofs(T, N, d)
    rows = np.repeat(ld[:, :, None], ld.shape[1], axis=2)
    cols = np.repeat(ld[:, None, :], ld.shape[1], axis=1)
    return _assemble(rows, cols, Ke, d * N)


def eigenstrain_load(X, T, coef, D, eps0):
    """f = sum_e coef_e |T_e| B_e^T D eps0_e: the linear term of the elastic
    energy with eps_eff = eps(u) - eps0, eq. (energytshock)."""
    N, d = X.shape
    vol, grad = geometry(X, T)
    B = strain_matrix(grad)
    fe = np.einsum("e,eik,ij,ej->ek", coef * vol, B, D, eps0)
    ld = local_dofs(T, N, d)
    f = np.zeros(d * N)
    np.add.at(f, ld.ravel(), fe.ravel())
    return f


def assemble_weighted_mass(X, T, weight):
    """sum_e weight_e M_e with the consistent P1 mass M_e."""
    N, d = X.shape
    vol, _ = geometry(X, T)
    Mr = reference_mass(d)
    Me = (weight * vol)[:, None, None] * Mr[None]
    rows = np.repeat(T[:, :, None], d + 1, axis=2)
    cols = np.repeat(T[:, None, :], d + 1, axis=1)
    return _assemble(rows, cols, Me, N)


def assemble_mass(X, T):
    return assemble_weighted_mass(X, T, np.ones(len(T)))


def assemble_laplacian(X, T):
    """L_ab = int grad phi_a . grad phi_b (P1 stiffness of the Laplacian)."""
    N, d = X.shape
    vol, grad = geometry(X, T)
    Le = np.einsum("e,eak,ebk->eab", vol, grad, grad)
    rows = np.repeat(T[:, :, None], d + 1, axis=2)
    cols = np.repeat(T[:, None, :], d + 1, axis=1)
    return _assemble(rows, cols, Le, N)


def load_vector(X, T):
    """m_a = int phi_a = sum over elements containing a of |T|/(d+1)."""
    N, d = X.shape
    vol, _ = geometry(X, T)
    m = np.zeros(N)
    np.add.at(m, T.ravel(), np.repeat(vol / (d + 1), d + 1))
    return m


# ----------------------------------------------------------------------------
# the discrete model: energy, gradient, Hessian blocks
# ----------------------------------------------------------------------------

class Model:
    """Discrete regularised energy on a fixed mesh (eq. (regenergy)).

    Caches the alpha- and u-independent operators (L, M, m, B_e, |T_e|).
    """

    def __init__(self, X, T, E=1.0, nu=0.3, Gc=1.0, ell=0.05, k_ell=1e-6,
                 model="AT1", plane_stress=False):
        self.X = np.asarray(X, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.int64)
        self.N, self.dim = self.X.shape
        self.Gc, self.ell, self.k_ell, self.model = Gc, ell, k_ell, model
        self.cw = c_w(model)
        lam, mu = lame(E, nu, self.dim, plane_stress)
        self.D = voigt_D(self.dim, lam, mu)
        self.vol, self.grad = geometry(self.X, self.T)
        self.B = strain_matrix(self.grad)
        self.L = assemble_laplacian(self.X, self.T)
        self.M = assemble_mass(self.X, self.T)
        self.m = load_vector(self.X, self.T)
        self.ld = local_dofs(self.T, self.N, self.dim)

    # --- coefficients -------------------------------------------------------
    def abar(self, alpha):
        return avg_degradation(alpha, self.T, self.k_ell, self.dim)

    def eps_eff(self, u, eps0=None):
        eps = element_strains(u, self.T, self.grad)
        return eps if eps0 is None else eps - eps0

    def W2(self, u, eps0=None):
        return w2(self.eps_eff(u, eps0), self.D)

    # --- operators ----------------------------------------------------------
    def K(self, alpha):
        """E_uu, eq. (elasticity)."""
        return assemble_elasticity(self.X, self.T, self.abar(alpha), self.D)

    def f_eigen(self, alpha, eps0):
        if eps0 is None:
            return np.zeros(self.dim * self.N)
        return eigenstrain_load(self.X, self.T, self.abar(alpha), self.D, eps0)

    def damage_hessian(self, u, eps0=None):
        """E_alphaalpha, eq. (helmholtz) with a'' = 2: M_W + (2 Gc ell / c_w) L
        (+ (2 Gc / (c_w ell)) M for AT2, w'' = 2).  Independent of alpha."""
        Mw = assemble_weighted_mass(self.X, self.T, self.W2(u, eps0))
        H = Mw + (2.0 * self.Gc * self.ell / self.cw) * self.L
        if self.model == "AT2":
            H = H + (2.0 * self.Gc / (self.cw * self.ell)) * self.M
        return H.tocsr()

    def damage_linear(self, u, eps0=None):
        """g such that E_alpha(alpha) = H alpha - g (a quadratic in alpha):
        g = M_W 1 - [AT1] (Gc / (c_w ell)) m."""
        W = self.W2(u, eps0)
        Mw1 = np.zeros(self.N)
        np.add.at(Mw1, self.T.ravel(), np.repeat(W * self.vol / (self.dim + 1), self.dim + 1))
        g = Mw1
        if self.model == "AT1":
            g = g - (self.Gc / (self.cw * self.ell)) * self.m
        return g

    def grad_u(self, u, alpha, eps0=None):
        """E_u as a vector over all displacement DOFs: K(alpha) u - f."""
        return self.K(alpha) @ u - self.f_eigen(alpha, eps0)

    def grad_alpha(self, u, alpha, eps0=None):
        """E_alpha as a vector over nodes, eq. (kkt)."""
        return self.damage_hessian(u, eps0) @ alpha - self.damage_linear(u, eps0)

    def coupling(self, u, alpha, eps0=None):
        """E_ualpha, eq. (offdiag): B[v, j] = sum_e (-2 (M_e b)_j) (B_e^T D eps_eff_e)_v,
        b = 1 - alpha (a'(alpha) = -2(1-alpha), integrated exactly)."""
        d, N = self.dim, self.N
        sig = np.einsum("ij,ej->ei", self.D, self.eps_eff(u, eps0))
        fv = np.einsum("e,eik,ei->ek", self.vol, self.B, sig)          # [E, d*(d+1)]
        b = 1.0 - alpha[self.T]
        Mb = b @ reference_mass(d)                                     # [E, d+1] (per |T|)
        vals = -2.0 * fv[:, :, None] * Mb[:, None, :]
        rows = np.repeat(self.ld[:, :, None], d + 1, axis=2)
        cols = np.repeat(self.T[:, None, :], self.ld.shape[1], axis=1)
        return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(d * N, N)).tocsr()

    # --- energy -------------------------------------------------------------
    def energies(self, u, alpha, eps0=None):
        """(elastic, surface) parts of eq. (regenergy)."""
        el = 0.5 * np.sum(self.abar(alpha) * self.vol * self.W2(u, eps0))
        if self.model == "AT1":
            wint = self.m @ alpha
        else:
            wint = alpha @ (self.M @ alpha)
        surf = (self.Gc / self.cw) * (wint / self.ell + self.ell * alpha @ (self.L @ alpha))
        return el, surf
