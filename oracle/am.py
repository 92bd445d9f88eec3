"""Alternate minimisation, its over-relaxed form and the Newton composition.

Test infrastructure (see the package docstring).

* One load step of the quasi-static evolution (Sec. 1.1, eq. (mainproblem)):
  minimise over u in C_ubar and alpha in D_{alpha_{i-1}}, then commit
  alpha_{i-1} <- alpha.
* Algorithm 1 (AM) and Algorithm 2 (ORAM): each sweep solves the elastic
  problem at fixed damage, relaxes u by omega, solves the damage variational
  inequality at fixed u, and relaxes alpha by a feasible factor.
* Algorithm 3 (ORAM-N): ORAM until the residual Phi of the optimality
  conditions is small, then the reduced-space active-set Newton method
  (Algorithm 4) on the coupled problem, reverting to ORAM when Newton fails.

Readings of points the paper leaves open:

* Dirichlet lifting: the new boundary value is written into u before the
  first sweep of a step, so the over-relaxed u never overshoots it.
* The damage step's largest feasible factor (Algorithm 2, Sec. 2.1) is read
  three ways, selected by ``relax``: "project" (pointwise projection of
  alpha + omega*dalpha onto the bounds, the default), "ratio" (the exact
  largest omega_bar <= omega keeping every component feasible) and "bisect"
  (the text's repeated midpoint of [1, omega_bar], at most 30 times, then 1).
  All three coincide for omega <= 1.
* The residual Phi stacks -E_u on the free displacement DOFs and the
  box Fischer--Burmeister residual of (alpha, E_alpha, alpha_prev, 1).
* ORAM-N switches to Newton when ||Phi||_2 drops below ``switch_tol``
  (absolute); after a Newton failure it runs ORAM until ||Phi||_2 has fallen
  by ``switch_rel`` relative to the value at the failure.  It stops when
  ||Phi||_2 <= ``final_tol``.
* The reduced Newton system is solved exactly (sparse LU): the inactive
  coupled Jacobian can be indefinite away from minimisers (Sec. 3.3).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import vi


class State:
    def __init__(self, u, alpha, alpha_prev, load=0.0):
        self.u = np.array(u, dtype=np.float64)
        self.alpha = np.array(alpha, dtype=np.float64)
        self.alpha_prev = np.array(alpha_prev, dtype=np.float64)
        self.load = load

    def copy(self):
        return State(self.u, self.alpha, self.alpha_prev, self.load)


def initial_state(problem, notch_mask=None):
    d, N = problem.model.dim, problem.model.N
    alpha = np.zeros(N)
    if notch_mask is not None:
        alpha[np.asarray(notch_mask, dtype=bool)] = 1.0
    return State(np.zeros(d * N), alpha, alpha.copy(), 0.0)


def set_load(problem, state, load):
    """Write the boundary values of the new load into u (lifting)."""
    state.load = load
    v = problem.dirichlet_values(load)
    state.u[problem.fixed] = v[problem.fixed]


# ----------------------------------------------------------------------------
# subproblems
# ----------------------------------------------------------------------------

def elastic_solve(problem, u, alpha, load):
    """u~ with E_u(u~, alpha; v) = 0 for all v in C_0 (Algorithm 1/2, first
    substep): K_FF u_F = f_F - K_FD u_D, solved exactly."""
    M = problem.model
    K = M.K(alpha)
    f = M.f_eigen(alpha, problem.eps0(load))
    F, D = problem.free, problem.fixed
    rhs = f[F] - K[F][:, D] @ u[D]
    out = u.copy()
    out[F] = spla.splu(K[F][:, F].tocsc()).solve(rhs)
    return out


def damage_solve(problem, u, alpha0, lower, load, tol=None, zeta=1e-12, max_it=200):
    """alpha~ in D_{alpha_prev} with E_alpha(u, alpha~; beta) >= 0 (second
    substep).  The damage energy is quadratic in alpha for AT1 and AT2, so the
    variational inequality is a box-constrained QP, solved by Algorithm 4."""
    M = problem.model
    eps0 = problem.eps0(load)
    H = M.damage_hessian(u, eps0)
    g = M.damage_linear(u, eps0)
    upper = np.ones_like(lower)
    if tol is None:
        tol = 1e-14 * max(1.0, np.max(np.abs(g)))
    return vi.box_qp(H, g, lower, upper, alpha0, tol, zeta=zeta, max_it=max_it)


def relax_alpha(alpha, dalpha, omega, lower, mode="project"):
    """alpha + omega_bar * dalpha kept inside [lower, 1] (Algorithm 2)."""
    upper = 1.0
    if mode == "project":
        return np.clip(alpha + omega * dalpha, lower, upper)
    if mode == "ratio":
        wb = omega
        pos = dalpha > 0
        neg = dalpha < 0
        if pos.any():
            wb = min(wb, np.min((upper - alpha[pos]) / dalpha[pos]))
        if neg.any():
            wb = min(wb, np.min((lower[neg] - alpha[neg]) / dalpha[neg]))
        # rounding guard: the exact factor is feasible by construction
        return np.clip(alpha + wb * dalpha, lower, upper)
    if mode == "bisect":
        wb = omega
        for _ in range(30):
            trial = alpha + wb * dalpha
            if np.all(trial >= lower) and np.all(trial <= upper):
                return trial
            wb = 0.5 * (1.0 + wb)
        return np.clip(alpha + dalpha, lower, upper)
    raise ValueError(mode)


def residual(problem, state):
    """Phi = [-E_u on free DOFs; box FB residual of (alpha, E_alpha)]."""
    M = problem.model
    eps0 = problem.eps0(state.load)
    Eu = M.grad_u(state.u, state.alpha, eps0)[problem.free]
    Ea = M.grad_alpha(state.u, state.alpha, eps0)
    phia = vi.mcp_residual(state.alpha, Ea, state.alpha_prev, np.ones_like(state.alpha))
    return np.concatenate([-Eu, phia])


# ----------------------------------------------------------------------------
# Algorithm 2 (ORAM); omega = 1 is Algorithm 1 (AM)
# ----------------------------------------------------------------------------

def oram_sweep(problem, state, omega=1.0, relax="project", qp_tol=None, trace=None):
    M = problem.model
    ut = elastic_solve(problem, state.u, state.alpha, state.load)
    u_new = state.u + omega * (ut - state.u)
    if trace is not None:
        trace.append(("u", M.energies(u_new, state.alpha, problem.eps0(state.load))))
    at, qinfo = damage_solve(problem, u_new, state.alpha, state.alpha_prev, state.load, tol=qp_tol)
    a_new = relax_alpha(state.alpha, at - state.alpha, omega, state.alpha_prev, relax)
    dinf = float(np.max(np.abs(a_new - state.alpha)))
    state.u = u_new
    state.alpha = a_new
    if trace is not None:
        trace.append(("alpha", M.energies(u_new, a_new, problem.eps0(state.load))))
    return dinf, qinfo


# ----------------------------------------------------------------------------
# coupled Newton (Algorithm 4 on the full optimality system)
# ----------------------------------------------------------------------------

def _pack(problem, state):
    return np.concatenate([state.u[problem.free], state.alpha])


def _unpack(problem, state, x):
    nf = int(problem.free.sum())
    state.u[problem.free] = x[:nf]
    state.alpha = x[nf:].copy()


def newton(problem, state, tol, max_it=10, zeta=1e-12):
    """Reduced-space active-set Newton with backtracking on the coupled
    MCP [E_u = 0 on free DOFs; E_alpha >= 0 complementarity on alpha]."""
    M = problem.model
    eps0 = problem.eps0(state.load)
    F_, D_ = problem.free, problem.fixed
    nf = int(F_.sum())
    u_fixed = state.u.copy()

    def split(x):
        u = u_fixed.copy()
        u[F_] = x[:nf]
        return u, x[nf:]

    def Ffun(x):
        u, a = split(x)
        return np.concatenate([M.grad_u(u, a, eps0)[F_], M.grad_alpha(u, a, eps0)])

    def Jfun(x):
        u, a = split(x)
        A = M.K(a)[F_][:, F_]
        B = M.coupling(u, a, eps0)[F_]
        C = M.damage_hessian(u, eps0)
        return sp.bmat([[A, B], [B.T, C]]).tocsr()

    l = np.concatenate([np.full(nf, -np.inf), state.alpha_prev])
    u = np.concatenate([np.full(nf, np.inf), np.ones(M.N)])
    x, info = vi.reduced_space_active_set(Ffun, Jfun, _pack(problem, state), l, u, tol,
                                          zeta=zeta, max_it=max_it, norm="l2",
                                          descent_fallback=False)
    _unpack(problem, state, x)
    return info


# ----------------------------------------------------------------------------
# one load step
# ----------------------------------------------------------------------------

# Automatic over-relaxation (an extension: the paper conjectures that the best
# omega minimises the spectral radius of the over-relaxed iteration, as in SOR
# theory (Sec. 2.2), and leaves its automatic choice to future work).  A load
# step starts at omega = 1; every OMEGA_PROBE + 1 sweeps at omega = 1 the
# convergence factor rho of plain alternate minimisation is estimated from the
# geometric mean of the OMEGA_PROBE successive ratios of ||dalpha||_inf, and
# once 0 < rho < 1 the step continues at Young's optimum for SOR,
# 2 / (1 + sqrt(1 - rho)), capped at the given omega.
OMEGA_PROBE = 4


def young_omega(dalpha_window, cap):
    """Young's optimal factor from OMEGA_PROBE + 1 successive ||dalpha||_inf
    values at omega = 1, capped at ``cap``; None when the window does not
    show a contraction (rho outside (0, 1))."""
    d0, dk = dalpha_window[0], dalpha_window[-1]
    if not d0 > 0:
        return None
    rho = (dk / d0) ** (1.0 / (len(dalpha_window) - 1))
    if not 0.0 < rho < 1.0:
        return None
    return min(cap, 2.0 / (1.0 + np.sqrt(1.0 - rho)))


def solve_load_step(problem, state, load, omega=1.0, relax="project", newton_on=False,
                    am_tol=1e-5, am_stop="dalpha", max_am=1000, switch_tol=1e-3,
                    switch_rel=1e-1, final_tol=1e-7, max_newton=10, qp_tol=None,
                    trace=None, omega_auto=False):
    """Minimise at load ``load`` starting from ``state`` (which holds
    u_{i-1}, alpha_{i-1}); commit alpha_prev <- alpha at the end.

    am_stop: "dalpha" stops ORAM on ||alpha^k - alpha^{k-1}||_inf < am_tol;
    "phi" stops on ||Phi||_2 <= final_tol.  With newton_on the stop is always
    ||Phi||_2 <= final_tol.  omega_auto: the factor of each sweep follows the
    automatic rule above, with ``omega`` as its cap.
    """
    set_load(problem, state, load)
    stats = {"sweeps": 0, "newton_its": 0, "newton_failures": 0, "converged": False,
             "dalpha_inf": [], "phi": [], "omega": []}
    threshold = switch_tol
    om = 1.0 if omega_auto else omega
    window = []
    while stats["sweeps"] < max_am:
        dinf, _ = oram_sweep(problem, state, om, relax, qp_tol=qp_tol, trace=trace)
        stats["sweeps"] += 1
        stats["dalpha_inf"].append(dinf)
        stats["omega"].append(om)
        if omega_auto and om == 1.0:
            window.append(dinf)
            if len(window) == OMEGA_PROBE + 1:
                w = young_omega(window, omega)
                if w is not None:
                    om = w
                window = []
        if not newton_on and am_stop == "dalpha":
            if dinf < am_tol:
                stats["converged"] = True
                break
            continue
        nphi = float(np.linalg.norm(residual(problem, state)))
        stats["phi"].append(nphi)
        if nphi <= final_tol:
            stats["converged"] = True
            break
        if newton_on and nphi < threshold:
            info = newton(problem, state, final_tol, max_it=max_newton)
            stats["newton_its"] += info["iterations"]
            nphi = info["phi_l2"]
            stats["phi"].append(nphi)
            if nphi <= final_tol:
                stats["converged"] = True
                break
            stats["newton_failures"] += 1
            threshold = switch_rel * nphi
    state.alpha_prev = state.alpha.copy()
    return stats


def run(problem, state, loads, **kw):
    out = []
    for t in loads:
        st = solve_load_step(problem, state, t, **kw)
        el, surf = problem.model.energies(state.u, state.alpha, problem.eps0(t))
        st["elastic"] = el
        st["surface"] = surf
        out.append(st)
    return out
