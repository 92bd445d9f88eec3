/*
 * fracture.h -- C ABI of the MI355X (gfx950) phase-field fracture solver.
 *
 * The library computes quasi-static evolutions of the regularised brittle
 * fracture energy of Farrell & Maurini, "Linear and nonlinear solvers for
 * variational phase-field models of brittle fracture":
 *
 *   E(u, alpha) = int 1/2 a(alpha) A0 eps(u):eps(u)
 *                 + Gc/c_w (w(alpha)/ell + ell |grad alpha|^2)      eq. (regenergy)
 *
 * with a(alpha) = (1-alpha)^2 + k_ell, w = alpha (AT1) or alpha^2 (AT2),
 * minimised at each load step over u in C_ubar and alpha_prev <= alpha <= 1
 * (Sec. 1.1, eq. (mainproblem) and the set D).  One load step runs alternate
 * minimisation (Algorithm 1), over-relaxed by omega (ORAM, Algorithm 2), and
 * optionally composed with reduced-space active-set Newton (ORAM-N,
 * Algorithm 3 with Algorithm 4).  Discretisation: P1 on structured meshes
 * (right-diagonal triangles in 2D, Kuhn tetrahedra in 3D), Sec. 1.2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Node (i, j[, k]) has index n = i + (nx+1)*(j + (ny+1)*k); N nodes.
 * - Displacement vectors are "blocked": component c of node n is at c*N + n
 *   (length dim*N).  Damage vectors have length N.  All values are float64.
 * - Device memory: the caller allocates one workspace of
 *   fracture_workspace_bytes() bytes (any allocator; 256-byte alignment)
 *   and owns it; the library carves every array it needs out of it and
 *   never allocates device memory.  The caller also owns the HIP stream;
 *   every kernel of a handle is launched on that stream.
 * - Pointers documented as "device" must point to device memory; "host"
 *   pointers to host memory owned by the caller.
 * - Every int-returning function returns FRACTURE_OK (0) or a negative error
 *   code and never aborts.  fracture_strerror() names the code.
 * - A handle is not thread safe; use one handle per stream.
 */
#ifndef FRACTURE_H
#define FRACTURE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define FRACTURE_OK          0
#define FRACTURE_EINVAL     -1  /* invalid parameter or argument               */
#define FRACTURE_ENOMEM     -2  /* workspace smaller than required             */
#define FRACTURE_ENOTCONV   -3  /* iteration limit hit; state rolled back      */
#define FRACTURE_ENONFINITE -4  /* NaN/Inf met in a reduction; state rolled back */
#define FRACTURE_EDEVICE    -5  /* a HIP runtime call failed                   */
#define FRACTURE_ESCRATCH   -6  /* problem needs more than the static scratch of
                                   fracture_energy_noalloc                     */

/* ---- enumerations ------------------------------------------------------ */
#define FRACTURE_AT1 1          /* w(alpha) = alpha,   c_w = 8/3 (Sec. 1.1)     */
#define FRACTURE_AT2 2          /* w(alpha) = alpha^2, c_w = 2   (Sec. 1.1)     */

#define FRACTURE_LOAD_TENSION_2D 0  /* u_y = 0 at y = 0, u_y = t at y = ly,
                                       u_x = 0 at node (0,0); load = t       */
#define FRACTURE_LOAD_THERMAL_3D 1  /* eps0 = -load * exp(-x/depth) I at each
                                       element centroid (Sec. 4.3 variant);
                                       u_x = 0 on x = lx; u_y = u_z = 0 at
                                       (lx,0,0); u_z = 0 at (lx,ly,0)        */
#define FRACTURE_LOAD_SURFING_2D 2  /* surfing (Sec. 4.1): the whole boundary
                                       carries the asymptotic Mode-I crack
                                       displacement of eq. (surfingloading)
                                       about the tip (surf_lc + surf_v t,
                                       ly/2), kappa = (3-nu)/(1+nu) as
                                       printed; load = t.  On the crack line
                                       behind the tip the boundary node takes
                                       the mean of the two faces (zero).     */
#define FRACTURE_LOAD_THERMAL_SHOCK_2D 3
                                    /* thermal shock (Sec. 4.3, eqs.
                                       (energytshock), (tempfielderfc)): the
                                       slab is cooled on y = 0; eps0 =
                                       -thermal_dT * erfc(y_c / (ell t)) I at
                                       each triangle centroid y_c, load = t
                                       the dimensionless time tau (eps0 = 0
                                       for t <= 0); u_x = 0 on x = 0 and
                                       x = lx, u_y = 0 on y = ly, the cooled
                                       face traction free                    */

#define FRACTURE_RELAX_PROJECT 0  /* alpha <- clip(alpha + omega*dalpha)       */
#define FRACTURE_RELAX_RATIO   1  /* largest common feasible omega_bar <= omega */
#define FRACTURE_RELAX_BISECT  2  /* omega_bar <- (1 + omega_bar)/2 until feasible */

#define FRACTURE_STOP_DALPHA 0    /* ORAM stops on ||alpha^k - alpha^{k-1}||_inf */
#define FRACTURE_STOP_PHI    1    /* stops on ||Phi||_2 (residual of eq. (kkt))  */

#define FRACTURE_FP64  0          /* every kernel in float64                    */
#define FRACTURE_MIXED 1          /* float32 operator + multigrid inside a
                                     float64 flexible CG with float64 residuals */

/* ---- parameters -------------------------------------------------------- */
typedef struct {
  int dim;                  /* 2 or 3                                          */
  int nx, ny, nz;           /* cells per axis (nz ignored when dim == 2)       */
  double lx, ly, lz;        /* domain extents; origin at 0                     */
  int model;                /* FRACTURE_AT1 | FRACTURE_AT2                      */
  int plane_stress;         /* 2D only: 0 plane strain, 1 plane stress         */
  double E, nu, Gc, ell, k_ell;
  int load_kind;            /* FRACTURE_LOAD_*                                 */
  double thermal_depth;     /* decay length of the thermal eigenstrain         */
  double surf_ki;           /* surfing: stress intensity factor K_I            */
  double surf_v;            /* surfing: crack-tip speed v                      */
  double surf_lc;           /* surfing: initial tip abscissa L_c               */
  int precision;            /* FRACTURE_FP64 | FRACTURE_MIXED                  */
  double omega;             /* over-relaxation, in (0, 2) (Algorithm 2)        */
  int relax_mode;           /* FRACTURE_RELAX_*                                */
  int newton;               /* 0 ORAM only, 1 ORAM-N (Algorithm 3)             */
  int am_stop;              /* FRACTURE_STOP_* (ORAM only)                     */
  double am_tol;            /* tolerance of ||dalpha||_inf                     */
  double switch_tol;        /* ORAM-N: first switch when ||Phi||_2 < this      */
  double switch_rel;        /* ORAM-N: after a Newton failure, ORAM until
                               ||Phi||_2 falls by this factor                  */
  double final_tol;         /* ||Phi||_2 stop (ORAM-N, or am_stop == PHI)      */
  double pcg_rtol;          /* elastic PCG: ||r|| <= pcg_rtol * ||b_load||     */
  double vi_tol;            /* damage VI: ||Phi_alpha||_inf <= vi_tol          */
  double vi_cg_rtol;        /* reduced damage CG relative tolerance (default
                               1e-4: the active-set iteration around it still
                               drives the box residual to vi_tol)             */
  double minres_rtol;       /* Newton MINRES relative tolerance                */
  int max_am, max_pcg, max_vi, max_vi_cg, max_newton, max_minres;
                            /* iteration limits (defaults 2000 sweeps, 1000
                               PCG, 200 active-set and 2000 CG iterations per
                               damage solve, 10 Newton, 500 MINRES); reaching
                               one is FRACTURE_ENOTCONV                       */
  int cheb_degree;          /* Chebyshev smoothing steps per V-cycle side      */
  int coarse_max_dofs;      /* coarsen until the level has at most this many   */
  int newton_vcycles;       /* multigrid V-cycles per action of A^{-1} inside
                               the Newton block preconditioner, 1 or 2.  The
                               paper's setup (Sec. 3.3) uses two; the default
                               is one, which costs fewer V-cycles per Newton
                               solve on the structured meshes here.            */
  double newton_forcing;    /* > 0: adaptive forcing terms (the paper
                               recommends adaptive tolerances for practical
                               use, Sec. 5.3), never tighter than the
                               target newton_forcing * final_tol / ||Phi||
                               that lets the step reach final_tol and never
                               below minres_rtol; 0: always minres_rtol, as
                               in the paper's experiments                     */
  int use_graphs;           /* 1: record the fixed launch sequences (V-cycle,
                               block preconditioner) once per operand set and
                               replay them as HIP graphs; 0: launch eagerly.
                               Both run the same kernels in the same order,
                               so results are bitwise identical.               */
  int vcycle_tail;          /* 1: run the smallest 2D multigrid levels and the
                               coarsest solve of each V-cycle in one
                               workgroup with its data in LDS; 0: one kernel
                               per step.  Same per-node arithmetic.           */
  int newton_precond;       /* Newton MINRES preconditioner: 0 the paper's
                               symmetric multiplicative block form with
                               S ~ C (eq. (preconditioner): two actions of
                               A^{-1} and one of C^{-1}); 1 (default) the
                               block-diagonal form diag(A^{-1}, C^{-1}), one
                               of each, also SPD.  Both solve the same Newton
                               system to the same tolerance.                  */
  int newton_forcing_mode;  /* with newton_forcing > 0: 0 the target itself
                               (capped at 0.1); 1 (default) Eisenstat-Walker
                               choice 2, eta_k = 0.9 (||Phi_k||/||Phi_k-1||)^2
                               with eta_0 = 0.01 and their safeguard, capped
                               at 0.5                                         */
  double pcg_reduction;     /* ORAM-N only (newton = 1): the elastic solve of
                               an ORAM sweep may stop once its residual has
                               fallen by this factor from the warm start (or
                               at pcg_rtol, whichever is looser); the Newton
                               phase enforces the final accuracy.  0: always
                               pcg_rtol.  Default 0.01.                       */
  double newton_stall;      /* a Newton step that leaves more than this
                               fraction of ||Phi|| is an insufficient
                               reduction and ends the Newton phase (back to
                               ORAM, Sec. 2.3); 1 disables.  Default 0.9.     */
  int omega_auto;           /* 1: choose the over-relaxation factor per load
                               step: omega = 1 until the convergence factor
                               rho of plain alternate minimisation is
                               measured over 4 sweep ratios, then Young's SOR
                               optimum 2 / (1 + sqrt(1 - rho)), capped at
                               omega (the paper's hypothesis on the optimal
                               omega, Sec. 2.2; it leaves an automatic choice
                               to future work); 0: omega throughout           */
  double thermal_dT;        /* FRACTURE_LOAD_THERMAL_SHOCK_2D: shock intensity
                               beta * DT of the imposed temperature; finite,
                               any sign (negative heats)                      */
  int deflate;              /* 1: deflate the elastic CG of the sweeps by the
                               rigid modes of each undamaged fragment (the
                               per-piece near-null vectors Sec. 3.1 names as a
                               possible improvement; deflated CG of Saad,
                               Yeung, Erhel and Guyomarc'h, 2000), formed
                               anew from alpha at every elastic solve.  2D and
                               FRACTURE_FP64 only (else FRACTURE_EINVAL);
                               the Newton phase is unchanged.  Default 0.    */
  double deflate_theta;     /* a node is undamaged when alpha < this; in
                               (0, 1]; default 0.5                            */
  int deflate_min_nodes;    /* smallest fragment kept, in nodes (>= 1);
                               default 64                                     */
  int deflate_max_fragments;/* most fragments kept (1..8), the largest first;
                               default 8                                      */
  double vi_reduction;      /* ORAM-N only (newton = 1): the damage solve of
                               an ORAM sweep may stop once max |Phi| of its
                               box QP has fallen by this factor from the
                               sweep's starting alpha (or at vi_tol,
                               whichever is looser); the Newton phase
                               enforces the final accuracy.  In [0, 1);
                               0 (default): always vi_tol.                    */
  int elem3d_min_nodes;     /* 3D: multigrid levels with at least this many
                               nodes apply K with the element-centric kernels
                               (each tetrahedron formed once per block), the
                               smaller ones with one thread per node (more
                               workgroups).  >= 0; default 262144; 0: every
                               level.  Results agree to rounding.            */
} fracture_params;

/* Fill *p with the documented defaults for a 2D tension problem on an
   nx-by-ny unit square (AT1, FP64, omega = 1, ORAM only). */
void fracture_default_params(fracture_params* p, int nx, int ny);

typedef struct {
  int sweeps;               /* ORAM sweeps in the step                         */
  int pcg_iters;            /* elastic PCG iterations, summed                  */
  int vi_iters;             /* active-set iterations of the damage VI, summed  */
  int vi_cg_iters;          /* reduced damage CG iterations, summed            */
  int newton_iters;         /* coupled Newton iterations                       */
  int newton_failures;      /* Newton phases that reverted to ORAM             */
  int minres_iters;         /* MINRES iterations, summed                       */
  int converged;            /* 1 when the stop test was met                    */
  double dalpha_inf;        /* last ||alpha^k - alpha^{k-1}||_inf              */
  double phi_l2;            /* last ||Phi||_2 (when computed, else -1)         */
  double ms_total, ms_pcg, ms_vi, ms_newton;  /* device time, HIP events      */
  int stopped_in;           /* a failed step's stage (FRACTURE_STAGE_*), else
                               FRACTURE_STAGE_NONE                            */
} fracture_stats;

/* stats.stopped_in: where a step that did not return FRACTURE_OK stopped */
#define FRACTURE_STAGE_NONE        0
#define FRACTURE_STAGE_PCG         1  /* elastic PCG: max_pcg or non-finite      */
#define FRACTURE_STAGE_VI          2  /* damage VI: max_vi active-set iterations */
#define FRACTURE_STAGE_VI_SEARCH   3  /* damage VI: no acceptable line-search step */
#define FRACTURE_STAGE_NEWTON      4  /* Newton phase: non-finite MINRES or residual */
#define FRACTURE_STAGE_SWEEPS      5  /* max_am sweeps without the stop test     */
#define FRACTURE_STAGE_OTHER       6  /* device error, non-finite update         */

typedef struct fracture* fracture_t;   /* opaque; owned by the library          */

/* Bytes of device workspace the parameters need (0 on invalid parameters).
   Admission control uses this as the instance's device footprint. */
size_t fracture_workspace_bytes(const fracture_params* p);

/* Number of nodes N and of displacement DOFs dim*N. */
int fracture_sizes(const fracture_params* p, int64_t* nodes, int64_t* dofs);

/* Create a solver instance.
 *   notch_mask: host, N bytes (nonzero = node fixed at alpha = alpha_prev = 1,
 *               an initial crack), or NULL.
 *   d_workspace: device, >= fracture_workspace_bytes(p) bytes, 256-aligned;
 *               owned by the caller, used exclusively by this handle.
 *   hip_stream: a hipStream_t (NULL = the null stream).
 * Sets u = 0, alpha = alpha_prev = notch, load = 0.
 * Errors: EINVAL (parameters: dim, sizes not even-coarsenable to at least
 * one level, omega outside (0,2), ell <= 0, ...), ENOMEM, EDEVICE. */
int fracture_create(const fracture_params* p, const uint8_t* notch_mask,
                    void* d_workspace, size_t ws_bytes, void* hip_stream,
                    fracture_t* out);

/* Set the load of the next step (t for tension, DT for the thermal case) and
   write the new Dirichlet values into u (the lifting done before the first
   sweep, so that over-relaxation cannot overshoot them). */
int fracture_set_load(fracture_t h, double load);

/* Solve one load step (Algorithm 2, or 3 when params.newton) from the
   current state and commit alpha_prev <- alpha.  On ENOTCONV/ENONFINITE the
   state is rolled back to its value at entry (after the lifting).  `out`
   (host, may be NULL) receives the statistics. */
int fracture_solve_step(fracture_t h, fracture_stats* out);

/* One load step for each of n handles, run concurrently (one host thread per
   handle, each on its handle's stream, so the device overlaps their work).
   The handles must be distinct and should have distinct streams.  Results
   equal n separate fracture_solve_step calls; out (host) has n entries or
   is NULL; codes (host) has n entries or is NULL.  Returns the first
   non-zero code, else FRACTURE_OK. */
int fracture_solve_steps(fracture_t* hs, int n, fracture_stats* out, int* codes);

/* Progress monitor: when set, fn(user, sweep, dalpha_inf, phi_l2) is called
   on the host after every ORAM sweep and Newton iteration of solve_step
   (phi_l2 is -1 when not computed).  fn = NULL removes it.  fn must not
   call into the same handle: the solve keeps state between sweeps. */
typedef void (*fracture_monitor_fn)(void* user, int sweep, double dalpha_inf, double phi_l2);
int fracture_set_monitor(fracture_t h, fracture_monitor_fn fn, void* user);

/* Elastic and surface parts of eq. (regenergy) at the current state
   (host outputs). */
int fracture_energy(fracture_t h, double* elastic, double* surface);

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): the energies of
   fracture_energy for a state given by the caller, with no handle and no
   allocation of any kind.
   p:        problem parameters (validated as by fracture_create).
   load:     the load of the state (t, DT or tau; it sets the eigenstrain of
             the thermal loads and is ignored by the tension and surfing
             loads).
   d_u:      device, dim*N doubles, blocked layout; d_alpha: device, N doubles.
   hip_stream: the stream the kernels and the copy are queued on; it must
             belong to the current device.  Nothing is synchronised: the
             result is ready when the stream reaches this point.
   d_out:    device, 2 doubles: [elastic, surface] as fracture_energy returns.
   The partial sums, scalars and (3D) per-tetrahedron energies live in one
   32 MiB static device array per device, kept until the process ends.  2D
   meshes of any accepted size fit; 3D meshes fit up to about 690,000
   hexahedra (6 tetrahedra x 8 bytes each), larger ones return
   FRACTURE_ESCRATCH before anything is queued.  Every call on a device
   shares that device's array: calls that overlap on one device (on
   different streams, or from different threads) race and corrupt each
   other's result; serialise them.  The array needs no clearing between
   calls (every entry a call reads, it wrote first).
   Errors: EINVAL (bad parameters or NULL pointers), ESCRATCH, EDEVICE. */
int fracture_energy_noalloc(const fracture_params* p, double load, const double* d_u,
                            const double* d_alpha, void* hip_stream, double* d_out);

/* Copy the state out of / into the handle.  Pointers may be host or device
   (detected with hipPointerGetAttributes); lengths dim*N, N, N.  Any pointer
   may be NULL to skip that field. */
int fracture_get_state(fracture_t h, double* u, double* alpha, double* alpha_prev);
int fracture_set_state(fracture_t h, const double* u, const double* alpha,
                       const double* alpha_prev);

/* ---- operator actions (matrix-free; device in/out, float64) ------------
 * y = Op x at the current state.  `level` selects a multigrid level for
 * FRACTURE_OP_LEVEL (0 = finest).  Sizes: x and y as documented per op.
 *   ELASTICITY   K(alpha) x, eq. (elasticity): dim*N -> dim*N, no Dirichlet
 *                masking (the assembled operator).
 *   LEVEL        the level's Galerkin operator with Dirichlet rows and
 *                columns removed (rows zeroed): dim*N_l -> dim*N_l.
 *   DAMAGE_HESS  E_alphaalpha at the current u, eq. (helmholtz): N -> N.
 *   COUPLING     E_ualpha, eq. (offdiag): N -> dim*N (B x).
 *   COUPLING_T   its transpose: dim*N -> N (B^T x).
 *   PRECOND      one multigrid V-cycle (the PCG preconditioner) on the
 *                finest level, Dirichlet rows zero: dim*N -> dim*N.
 *   RESIDUAL     -K(alpha) x on the free rows, Dirichlet rows zero: the
 *                residual f - K x that the elastic PCG forms, for a zero
 *                load f (its kernel): dim*N -> dim*N.
 */
#define FRACTURE_OP_ELASTICITY  0
#define FRACTURE_OP_LEVEL       1
#define FRACTURE_OP_DAMAGE_HESS 2
#define FRACTURE_OP_COUPLING    3
#define FRACTURE_OP_COUPLING_T  4
#define FRACTURE_OP_PRECOND     5
#define FRACTURE_OP_RESIDUAL    6
int fracture_apply(fracture_t h, int op, int level, const double* d_x, double* d_y);

/* Refresh the multigrid coefficients (level averages of a(alpha) and the
   coarse inverse) from the current alpha.  solve_step does this itself; call
   it before FRACTURE_OP_LEVEL / FRACTURE_OP_PRECOND after set_state. */
int fracture_update_coefficients(fracture_t h);

/* Gradient of the energy at the current state (device outputs):
   Eu = K(alpha) u - f (dim*N, all rows), Ea = E_alpha (N), eq. (kkt). */
int fracture_gradient(fracture_t h, double* d_Eu, double* d_Ea);

/* Number of multigrid levels and the node counts per axis of one level. */
int fracture_levels(fracture_t h, int* nlevels);
int fracture_level_shape(fracture_t h, int level, int* nx, int* ny, int* nz);

/* ---- measurement hook ---------------------------------------------------
 * Launch one of the hot kernels `reps` times back to back on the handle's
 * stream on the handle's current buffers, bracketed by HIP events, and
 * return the mean duration per launch (host *avg_ms) and the kernel's
 * algorithmic (compulsory) bytes per launch (host *bytes): every distinct
 * input read once plus every output written once, from the level's sizes.
 *   APPLY    finest-level y = K(alpha) x: x 16 + alpha 8 + y 16 = 40 B
 *            per node.
 *   SMOOTH   finest-level Chebyshev step with iterate, rhs and update
 *            vectors: x 16 + alpha 8 + b 16 + d 16 in, x' 16 + d' 16 out
 *            = 88 B per node.
 *   VI_EVAL  damage residual, FB function and active set: alpha 8 +
 *            alpha_prev 8 + W2 16 in (2 per cell), F 8 + Phi 8 + mask 1 +
 *            inverse diagonal 8 out = 57 B per node.
 *   HELM     masked damage Hessian apply with the x.y reduction: x 8 +
 *            W2 16 + mask 1 in, y 8 out = 33 B per node.
 *   COPY     y = x for one displacement vector: 16 in + 16 out = 32 B per
 *            node.
 * The buffers are overwritten (call between load steps only). */
#define FRACTURE_KERNEL_APPLY   0
#define FRACTURE_KERNEL_SMOOTH  1
#define FRACTURE_KERNEL_VI_EVAL 2
#define FRACTURE_KERNEL_HELM    3
#define FRACTURE_KERNEL_COPY    4   /* plain copy of one displacement vector:
                                       the streaming reference (and the
                                       calibration kernel for HBM counters) */
int fracture_time_kernel(fracture_t h, int kernel, int reps, double* avg_ms, double* bytes);

/* Live timing of a kernel inside the solves (measurement hook).  After
   fracture_kernel_timing(h, FRACTURE_KERNEL_SMOOTH, capacity) every fifth
   float64 finest-level Chebyshev step of the multigrid V-cycles (a sample
   that cycles through the four steps of a V-cycle), whatever solve launches
   them, is bracketed by HIP events on the instance's stream, up to
   `capacity` steps, and each adds its algorithmic bytes (coefficients 8 B,
   b, x_in, a distinct d_in, x_out, d_out at 8 B per DOF, per node; the
   first post-smoothing step, which also applies the prolongation, adds the
   coarse correction at 8 B per coarse DOF); the
   durations include the dispatch around each kernel.  While it is active the V-cycles are launched
   eagerly (a recorded graph replay cannot hold the events).  The events are
   created here, up to 32768 steps; capacity 0 ends the timing.  Only
   FRACTURE_KERNEL_SMOOTH is accepted (else FRACTURE_EINVAL).
   fracture_kernel_timing_read waits for the recorded steps, returns their
   count, summed duration (ms) and summed algorithmic bytes, and clears the
   record (the capacity stays). */
int fracture_kernel_timing(fracture_t h, int kernel, int capacity);
int fracture_kernel_timing_read(fracture_t h, int* count, double* total_ms, double* total_bytes);

/* Crack-aware deflation (params.deflate = 1, else FRACTURE_EINVAL; 2D).
   Fragments are the connected components of the nodes with alpha <
   deflate_theta in the graph of the element edges; those of at least
   deflate_min_nodes nodes are kept, at most deflate_max_fragments of them,
   the largest first, ties by the smaller least node index (with more than
   256 components of at least deflate_min_nodes nodes, which of them are
   considered is unspecified).
   fracture_fragments labels the current alpha: d_fid (device, N ints)
   receives each node's fragment index, or -1 (damaged, or in a component
   not kept); *nfrag (host) the number kept.
   fracture_deflation_matrix forms E = W^T K(alpha) W (Sec. 3.1, eq.
   (elasticity)) for the current alpha; column 3f + t of W is, on fragment
   f, the x translation (t = 0), the y translation (t = 1) or the rotation
   (-(y - ly/2), x - lx/2) * 2 / max(lx, ly) (t = 2), zero elsewhere and on
   Dirichlet DOFs.  E (host, row-major m x m, room for 24 x 24 doubles)
   receives it and *m = 3 nfrag.  Both wait for the instance's stream. */
int fracture_fragments(fracture_t h, int* nfrag, int* d_fid);
int fracture_deflation_matrix(fracture_t h, int* m, double* E);

const char* fracture_strerror(int code);

/* Release the handle (host state only; the caller frees the workspace). */
void fracture_destroy(fracture_t h);

#ifdef __cplusplus
}
#endif
#endif /* FRACTURE_H */
