"""Complementarity problems and the reduced-space active-set method.

Test infrastructure (see the package docstring).  Follows Sec. 2.4 of the
paper: the mixed complementarity problem MCP(F, l, u), the
Fischer--Burmeister NCP function, the residual Phi, and Algorithm 4 (the
reduced-space active set method) with the active set of eq. (reducedis) and
the reduced Newton step of eq. (reducednewton).

Readings where the paper is brief:

* The box (MCP) form of the residual, which the paper calls a straightforward
  extension of the NCP case: Phi_i = phi(x_i - l_i, phi(u_i - x_i, -F_i)).
  For an unbounded component (l = -inf, u = +inf) Phi_i = -F_i.
* Upper-bound activity mirrors the lower one: u_i - x_i <= zeta and F_i < 0.
  A component with l_i = u_i is always active.
* The reduced step solves J_NN d_N = -F_N (a descent step for the merit
  function; the printed system omits the sign).
* Line search: Armijo backtracking on psi = 1/2 ||Phi||^2 over the projected
  path pi[x + mu d], mu = 1, 1/2, ..., 2^-20, accepting when
  psi(trial) <= (1 - 2 sigma mu) psi(x), sigma = 1e-4.  If no step is
  accepted the steepest descent direction -grad psi is tried the same way.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

SIGMA = 1e-4
MAX_HALVINGS = 20


def fb(a, b):
    """Fischer--Burmeister NCP function phi(a, b) = sqrt(a^2 + b^2) - a - b
    (Sec. 2.4); zero iff a >= 0, b >= 0, ab = 0."""
    return np.hypot(a, b) - a - b


def _fb_partials(a, b):
    r = np.hypot(a, b)
    safe = r > 0
    da = np.where(safe, a / np.where(safe, r, 1.0), 1.0 / np.sqrt(2.0)) - 1.0
    db = np.where(safe, b / np.where(safe, r, 1.0), 1.0 / np.sqrt(2.0)) - 1.0
    return da, db


def mcp_residual(x, F, l, u):
    """Phi(x) for MCP(F, l, u) with the nested Fischer--Burmeister form."""
    x = np.asarray(x, dtype=np.float64)
    phi = np.empty_like(x)
    lo = np.isfinite(l)
    hi = np.isfinite(u)
    both = lo & hi
    onlylo = lo & ~hi
    onlyhi = ~lo & hi
    free = ~lo & ~hi
    phi[both] = fb(x[both] - l[both], fb(u[both] - x[both], -F[both]))
    phi[onlylo] = fb(x[onlylo] - l[onlylo], F[onlylo])
    phi[onlyhi] = -fb(u[onlyhi] - x[onlyhi], -F[onlyhi])
    phi[free] = -F[free]
    return phi


def mcp_merit_gradient(x, F, J, l, u):
    """grad of psi = 1/2 ||Phi||^2, i.e. V^T Phi with V an element of the
    generalised Jacobian of Phi (psi itself is continuously differentiable)."""
    n = x.size
    phi = mcp_residual(x, F, l, u)
    lo = np.isfinite(l)
    hi = np.isfinite(u)
    # d Phi_i / d x = ca_i e_i + cf_i (d F_i / d x)
    ca = np.zeros(n)
    cf = np.zeros(n)
    both = lo & hi
    if both.any():
        p = u[both] - x[both]
        q = -F[both]
        c = fb(p, q)
        a = x[both] - l[both]
        da_o, db_o = _fb_partials(a, c)
        da_i, db_i = _fb_partials(p, q)
        ca[both] = da_o - db_o * da_i
        cf[both] = -db_o * db_i
    m = lo & ~hi
    if m.any():
        da, db = _fb_partials(x[m] - l[m], F[m])
        ca[m] = da
        cf[m] = db
    m = ~lo & hi
    if m.any():
        da, db = _fb_partials(u[m] - x[m], -F[m])
        ca[m] = da
        cf[m] = db
    m = ~lo & ~hi
    cf[m] = -1.0
    return ca * phi + J.T @ (cf * phi)


def active_set(x, F, l, u, zeta):
    """Active components, eq. (reducedis), for box bounds."""
    lower = np.isfinite(l) & (x - l <= zeta) & (F > 0)
    upper = np.isfinite(u) & (u - x <= zeta) & (F < 0)
    fixed = np.isfinite(l) & np.isfinite(u) & (l == u)
    return lower | upper | fixed


def project(x, l, u):
    return np.minimum(np.maximum(x, l), u)


def reduced_space_active_set(Ffun, Jfun, x0, l, u, tol, zeta=1e-12, max_it=100,
                             solve=None, callback=None, norm="inf", descent_fallback=True):
    """Algorithm 4 for MCP(F, l, u).

    Ffun(x) -> F(x); Jfun(x) -> sparse Jacobian of F.  ``solve(Jnn, rhs)``
    solves the reduced system (default: sparse LU, i.e. exactly).
    Stops when ||Phi|| <= tol (``norm`` "inf" or "l2").  Returns (x, info)
    with info holding the iteration count, the final ||Phi||_2 and
    ||Phi||_inf, and a flag set when the line search failed (after the
    steepest-descent fallback, when enabled).
    """
    if solve is None:
        solve = lambda A, b: spla.splu(A.tocsc()).solve(b)
    x = project(np.array(x0, dtype=np.float64), l, u)
    info = {"iterations": 0, "failed": False, "linesearch_fallbacks": 0}
    for it in range(max_it + 1):
        F = Ffun(x)
        phi = mcp_residual(x, F, l, u)
        if callback is not None:
            callback(x, F, phi)
        if norm == "inf":
            nrm = np.max(np.abs(phi)) if phi.size else 0.0
        else:
            nrm = np.linalg.norm(phi)
        if nrm <= tol or it == max_it:
            break
        J = Jfun(x)
        A = active_set(x, F, l, u, zeta)
        N = ~A
        d = np.zeros_like(x)
        idx = np.flatnonzero(N)
        if idx.size:
            Jnn = J[idx][:, idx]
            d[idx] = solve(Jnn, -F[idx])
        psi0 = 0.5 * phi @ phi
        xn = _armijo(Ffun, x, d, l, u, psi0)
        if xn is None and not descent_fallback:
            info["failed"] = True
            break
        if xn is None:
            info["linesearch_fallbacks"] += 1
            g = mcp_merit_gradient(x, F, J, l, u)
            xn = _armijo(Ffun, x, -g, l, u, psi0, slope=-(g @ g))
            if xn is None:
                info["failed"] = True
                break
        x = xn
        info["iterations"] = it + 1
    F = Ffun(x)
    phi = mcp_residual(x, F, l, u)
    info["phi_l2"] = float(np.linalg.norm(phi))
    info["phi_inf"] = float(np.max(np.abs(phi))) if phi.size else 0.0
    return x, info


def _armijo(Ffun, x, d, l, u, psi0, slope=None):
    """Projected backtracking; slope defaults to -2 psi0 (a Newton direction)."""
    if slope is None:
        slope = -2.0 * psi0
    mu = 1.0
    for _ in range(MAX_HALVINGS + 1):
        xt = project(x + mu * d, l, u)
        phit = mcp_residual(xt, Ffun(xt), l, u)
        if 0.5 * phit @ phit <= psi0 + SIGMA * mu * slope:
            return xt
        mu *= 0.5
    return None


def box_qp(H, g, l, u, x0, tol, zeta=1e-12, max_it=100, solve=None):
    """min 1/2 x^T H x - g^T x  s.t. l <= x <= u, as MCP(Hx - g, l, u) by
    Algorithm 4 with exact reduced solves."""
    H = sp.csr_matrix(H)
    return reduced_space_active_set(lambda x: H @ x - g, lambda x: H, x0, l, u, tol,
                                    zeta=zeta, max_it=max_it, solve=solve)
