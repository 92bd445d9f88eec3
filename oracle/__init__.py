"""FP64 CPU oracle for the phase-field fracture hot path.

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(the HIP library and its Python binding) never imports, links or calls anything
here, and this package imports nothing from the product path.

It is a plain, slow, assembled-sparse implementation of what the method
computes, written from the paper (Farrell & Maurini, "Linear and nonlinear
solvers for variational phase-field models of brittle fracture"):

* ``mesh``  -- structured simplicial meshes (P1 discretisation, Sec. 1.2).
* ``fem``   -- element integrals and assembled operators for the regularised
               energy, eq. (regenergy), its first derivatives, eq. (kkt), and
               its second derivatives, eqs. (elasticity), (offdiag), (helmholtz).
* ``vi``    -- the Fischer--Burmeister NCP function and the reduced-space
               active-set method for complementarity problems (Sec. 2.4,
               Algorithm 4, eqs. (reducedis), (reducednewton)).
* ``am``    -- alternate minimisation (Algorithm 1), its over-relaxed form
               ORAM (Algorithm 2, Sec. 2.1) and the composition with Newton,
               ORAM-N (Algorithm 3, Sec. 2.3), plus the quasi-static load loop.

Every floating point quantity is float64.  Linear systems are solved exactly
(sparse LU) so that the oracle's iterates are the algorithm's iterates, not a
Krylov approximation of them.
"""
