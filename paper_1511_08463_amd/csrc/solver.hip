// Host driver and C ABI (include/fracture.h).
//
// One load step (fracture_solve_step) runs Algorithm 2 of the paper (ORAM;
// omega = 1 is Algorithm 1) and, when enabled, its composition with Newton
// (Algorithm 3).  Every sweep:
//   1. coefficient update: multigrid level averages of a(alpha) and the
//      coarse inverse;
//   2. elastic subproblem E_u(u~, alpha; v) = 0 by multigrid-preconditioned CG
//      (matrix-free operator, Chebyshev/Jacobi smoothing, Galerkin coarse
//      levels, dense coarsest solve), warm-started from u;
//   3. u <- u + omega (u~ - u);
//   4. damage subproblem: the box QP of the quadratic damage energy, solved by
//      the reduced-space active-set method (Algorithm 4) with a Jacobi-CG on
//      the inactive Hessian block and a projected Armijo search on
//      1/2 ||Phi||^2;
//   5. alpha <- alpha + omega_bar (alpha~ - alpha), feasible.
// The host only reads convergence scalars (a few bytes) back from the device.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/fracture.h"
#include "common.h"
#include "launch.h"

using namespace frac;

namespace {

constexpr int MAXLEV = 16;
constexpr int DENSE_MAX = 1024;   // largest coarsest-level system inverted densely
// stalled ORAM sweeps (solve_step_impl): ||dalpha||_inf below STALL_DALPHA and
// no cut of ||Phi||_2 by the factor STALL_CUT within STALL_SWEEPS sweeps
constexpr double STALL_DALPHA = 1e-6;
constexpr double STALL_CUT = 0.9;
constexpr int STALL_SWEEPS = 50;
// The coarsest system is re-assembled and re-inverted once its coefficients
// drift by more than this relative amount from those of the current inverse.
constexpr double COARSE_DRIFT = 0.02;
constexpr int KT_MAX = 1 << 15;   // most finest-level steps timed at once
// every KT_STRIDE-th finest-level step is timed: a stride prime to the four
// steps of a V-cycle samples each kind alike, with a fifth of the events
constexpr int KT_STRIDE = 5;
constexpr double ARMIJO_SIGMA = 1e-4;
constexpr int MAX_HALVINGS = 20;
constexpr int MAX_GRAPHS = 16;
constexpr double NEWTON_ETA_MAX = 0.1;   // loosest forcing term of the target rule
constexpr double EW_ETA0 = 0.01;         // Eisenstat-Walker: first forcing term of a phase
constexpr double EW_ETA_MAX = 0.5;       // Eisenstat-Walker: loosest forcing term
constexpr int OMEGA_PROBE = 4;           // omega_auto: sweep ratios that estimate rho    // recorded launch sequences kept per instance

// Launch sequences recorded once and replayed as HIP graphs.
enum GraphOp { G_VCYCLE64 = 1, G_VCYCLE32 = 2, G_PRECOND = 3 };

struct Captured {
  int op;
  const void* a;
  const void* b;
  void* out;               // result buffer of the sequence
  hipGraphExec_t exec;
};

struct Level {
  Grid g;
  double* abar = nullptr;  // element coefficients (levels >= 1)
  double *b = nullptr, *xa = nullptr, *xb = nullptr, *d = nullptr, *r = nullptr;
  // float32 copies for the mixed-precision multigrid
  float* abar32 = nullptr;
  float *b32 = nullptr, *xa32 = nullptr, *xb32 = nullptr, *d32 = nullptr, *r32 = nullptr;
  // 3D smoothed levels: diag K(alpha) for the current coefficients
  double* dg = nullptr;
  float* dg32 = nullptr;
};

// Bump allocator over the caller's workspace (or a dry run that only counts).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* p) : base((char*)p) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace

struct fracture {
  fracture_params p;
  int dim = 2, nlev = 0;
  Level lv[MAXLEV];
  Mat mat;
  double lam_max = 0, lam_min = 0;
  double cheb_cd[16] = {}, cheb_cr[16] = {};
  double cw = 0, cL = 0, cM = 0, cm = 0, gc_cw = 0;
  hipStream_t st = nullptr;
  int64_t N = 0, n2 = 0;
  // state
  double *u = nullptr, *alpha = nullptr, *alpha_prev = nullptr, *u_entry = nullptr,
         *alpha_entry = nullptr;
  // elastic PCG
  double *x = nullptr, *r = nullptr, *pv = nullptr, *q = nullptr;
  // crack-aware deflation of the elastic CG (params.deflate)
  int *dfl_parent = nullptr, *dfl_label = nullptr, *dfl_fid = nullptr, *dfl_meta = nullptr;
  double *dfl_part = nullptr, *dfl_E = nullptr, *dfl_Einv = nullptr, *dfl_mu = nullptr;
  // damage VI
  double *w2 = nullptr, *F = nullptr, *phi = nullptr, *hdinv = nullptr, *atil = nullptr;
  double *vd = nullptr, *vr = nullptr, *vz = nullptr, *vp = nullptr, *vq = nullptr,
         *vt1 = nullptr, *vt2 = nullptr;
  uint8_t* mask = nullptr;
  // reductions
  double* S = nullptr;
  double* part = nullptr;
  int part_n = 0;
  // Newton (ORAM-N): 3N block vectors [u_x | u_y | alpha] and temporaries
  double *nv_prev = nullptr, *nv = nullptr, *naz = nullptr, *nz = nullptr, *nw_prev = nullptr,
         *nw = nullptr, *nx = nullptr;
  double *npu1 = nullptr, *npu2 = nullptr, *npa1 = nullptr, *npa2 = nullptr, *nca = nullptr,
         *ncb = nullptr, *ncd = nullptr, *nut = nullptr, *nat = nullptr, *nFu = nullptr;
  double chebC_cd[8] = {}, chebC_cr[8] = {};
  // mixed precision: float32 alpha and the inner flexible-CG vectors
  bool mixed = false;
  float *alpha32 = nullptr, *fe32 = nullptr, *fr32 = nullptr, *fp32 = nullptr, *fq32 = nullptr;
  // coarsest level
  double *dA = nullptr, *dAinv = nullptr;
  double* dref = nullptr;   // coarsest coefficients the dense inverse was formed from
  int dense_n = 0;
  // first level of the single-workgroup V-cycle tail per value type (-1: none)
  int tail64 = -1, tail32 = -1;
  // host side
  double* hS = nullptr;  // pinned copy of the scalar array (+ two lagged-read slots)
  hipEvent_t ev[10] = {};  // 0..7 timing, 8..9 lagged scalar reads
  // live timing of the finest-level Chebyshev steps (fracture_kernel_timing)
  hipEvent_t* kt_ev = nullptr;
  int kt_cap = 0, kt_used = 0, kt_seen = 0;
  double kt_bytes = 0.0;
  double load = 0.0;
  double bnorm = 0.0;
  Load2D load2d{};
  double omega_cur = 1.0;   // over-relaxation factor of the current sweep
  // sum of Phi^2 of the damage solve's final iterate (the box FB residual at
  // the sweep's u), valid until the next damage solve starts
  double vi_phi2 = 0.0;
  bool vi_phi2_valid = false;
  int vi_stop = FRACTURE_STAGE_VI;        // which VI limit ended a failed damage solve
  // absolute cap on the sub-solve tolerances of the current load step's
  // sweeps (INFINITY: none); set once a sweep leaves the state unchanged
  double sweep_cap = INFINITY;
  bool phi_reused = false;   // the last residual_launch took vi_phi2
  // r holds b - K(alpha) u (free rows; 0 on Dirichlet rows) at the current
  // u, alpha and load, and r_rr its squared norm: left by the last sweep's
  // residual for the next sweep's PCG, which then starts from it
  bool r_valid = false;
  double r_rr = 0.0;
  fracture_monitor_fn monitor = nullptr;
  void* monitor_user = nullptr;
  bool coef_valid = false;
  // recorded launch sequences: captured on a private stream, replayed on st
  std::vector<Captured> graphs;
  hipStream_t cap = nullptr;
  bool capturing = false;
  bool graph_error = false;
};

namespace {

int hip_ok(hipError_t e) { return e == hipSuccess ? FRACTURE_OK : FRACTURE_EDEVICE; }

#define HIPCHK(expr)                                       \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return FRACTURE_EDEVICE;         \
  } while (0)

// ---------------------------------------------------------------------------
// parameters, levels and workspace layout
// ---------------------------------------------------------------------------

int validate(const fracture_params* p) {
  if (!p) return FRACTURE_EINVAL;
  if (p->dim != 2 && p->dim != 3) return FRACTURE_EINVAL;
  if (p->nx < 2 || p->ny < 2) return FRACTURE_EINVAL;
  if (!(p->lx > 0) || !(p->ly > 0)) return FRACTURE_EINVAL;
  if (p->dim == 3 && (p->nz < 1 || !(p->lz > 0) || !(p->thermal_depth > 0))) return FRACTURE_EINVAL;
  if (p->model != FRACTURE_AT1 && p->model != FRACTURE_AT2) return FRACTURE_EINVAL;
  if (!(p->E > 0) || !(p->nu > -1.0 && p->nu < 0.5) || !(p->Gc > 0) || !(p->ell > 0) ||
      !(p->k_ell >= 0))
    return FRACTURE_EINVAL;
  if (!(p->omega > 0 && p->omega < 2)) return FRACTURE_EINVAL;
  if (p->relax_mode < 0 || p->relax_mode > 2) return FRACTURE_EINVAL;
  if (p->dim == 2 && p->load_kind != FRACTURE_LOAD_TENSION_2D &&
      p->load_kind != FRACTURE_LOAD_SURFING_2D && p->load_kind != FRACTURE_LOAD_THERMAL_SHOCK_2D)
    return FRACTURE_EINVAL;
  if (p->load_kind == FRACTURE_LOAD_THERMAL_SHOCK_2D && !std::isfinite(p->thermal_dT))
    return FRACTURE_EINVAL;
  if (p->load_kind == FRACTURE_LOAD_SURFING_2D &&
      (!std::isfinite(p->surf_ki) || !std::isfinite(p->surf_v) || !std::isfinite(p->surf_lc)))
    return FRACTURE_EINVAL;
  if (p->dim == 3 && p->load_kind != FRACTURE_LOAD_THERMAL_3D) return FRACTURE_EINVAL;
  if (p->precision != FRACTURE_FP64 && p->precision != FRACTURE_MIXED) return FRACTURE_EINVAL;
  if (p->newton && !(p->minres_rtol > 0 && p->max_minres >= 1 && p->max_newton >= 1)) return FRACTURE_EINVAL;
  if (p->max_am < 1 || p->max_pcg < 1 || p->max_vi < 1 || p->max_vi_cg < 1) return FRACTURE_EINVAL;
  if (p->cheb_degree < 1 || p->cheb_degree > 8) return FRACTURE_EINVAL;
  if (p->newton_vcycles < 1 || p->newton_vcycles > 2) return FRACTURE_EINVAL;
  if (p->use_graphs != 0 && p->use_graphs != 1) return FRACTURE_EINVAL;
  if (!(p->newton_forcing >= 0)) return FRACTURE_EINVAL;
  if (p->vcycle_tail != 0 && p->vcycle_tail != 1) return FRACTURE_EINVAL;
  if (p->newton_precond != 0 && p->newton_precond != 1) return FRACTURE_EINVAL;
  if (p->omega_auto != 0 && p->omega_auto != 1) return FRACTURE_EINVAL;
  if (p->newton_forcing_mode != 0 && p->newton_forcing_mode != 1) return FRACTURE_EINVAL;
  if (!(p->pcg_reduction >= 0 && p->pcg_reduction < 1)) return FRACTURE_EINVAL;
  if (!(p->vi_reduction >= 0 && p->vi_reduction < 1)) return FRACTURE_EINVAL;
  if (p->elem3d_min_nodes < 0) return FRACTURE_EINVAL;
  if (!(p->newton_stall > 0 && p->newton_stall <= 1)) return FRACTURE_EINVAL;
  if (p->deflate != 0 && p->deflate != 1) return FRACTURE_EINVAL;
  if (p->deflate &&
      (p->dim != 2 || p->precision != FRACTURE_FP64 || !(p->deflate_theta > 0 && p->deflate_theta <= 1) ||
       p->deflate_min_nodes < 1 || p->deflate_max_fragments < 1 ||
       p->deflate_max_fragments > DFL_FMAX))
    return FRACTURE_EINVAL;
  if ((int64_t)(p->nx + 1) * (p->ny + 1) * (p->dim == 3 ? p->nz + 1 : 1) > (int64_t)1 << 29)
    return FRACTURE_EINVAL;
  return FRACTURE_OK;
}

// Boundary-condition family of a 2D load kind.
int bc_kind2d(int load_kind) {
  if (load_kind == FRACTURE_LOAD_SURFING_2D) return BC_SURFING_2D;
  if (load_kind == FRACTURE_LOAD_THERMAL_SHOCK_2D) return BC_TSHOCK_2D;
  return BC_TENSION_2D;
}

// One structured level of the problem p with the given cells and spacings
// (no eigenstrain: with_load adds the load's).
Grid make_grid(const fracture_params* p, int nx, int ny, int nz, double hx, double hy, double hz) {
  Grid g{};
  g.nx = nx; g.ny = ny; g.nz = nz; g.hx = hx; g.hy = hy; g.hz = hz;
  g.N = (nx + 1) * (ny + 1) * (p->dim == 3 ? nz + 1 : 1);
  g.bc = p->dim == 3 ? BC_THERMAL_3D : bc_kind2d(p->load_kind);
  g.dim = p->dim;
  g.eig_dT = 0.0;
  g.eig_depth = p->thermal_depth;
  g.elem_min = p->elem3d_min_nodes;
  return g;
}

// Level shapes: halve both axes while they stay even and the level has more
// DOFs than coarse_max_dofs (at least once, so there is always a coarse level).
int level_shapes(const fracture_params* p, Grid* out) {
  const int dim = p->dim;
  int nx = p->nx, ny = p->ny, nz = dim == 3 ? p->nz : 0, L = 0;
  double hx = p->lx / nx, hy = p->ly / ny, hz = dim == 3 ? p->lz / nz : 0.0;
  for (;;) {
    out[L++] = make_grid(p, nx, ny, nz, hx, hy, hz);
    bool can = (nx % 2 == 0) && (ny % 2 == 0) && L < MAXLEV;
    if (dim == 2) can = can && nx >= 4 && ny >= 4;
    else can = can && (nz % 2 == 0) && nx >= 2 && ny >= 2 && nz >= 2;
    if (!can || (L >= 2 && dim * out[L - 1].N <= p->coarse_max_dofs)) break;
    nx /= 2; ny /= 2; hx *= 2; hy *= 2;
    if (dim == 3) { nz /= 2; hz *= 2; }
  }
  if (dim * out[L - 1].N > DENSE_MAX) return -1;
  if (L < 2) return -1;   // at least one coarse level
  return L;
}

// First level of the V-cycle tail that runs in one workgroup (2D only): the
// most levels, at most TAIL_MAX_LEVELS and never the finest, whose vectors,
// coefficients and coarsest system fit in LDS; -1 if none fits.
int tail_start(const Grid* gl, int L, int dim, int dn, size_t elem) {
  if (dim != 2) return -1;
  int best = -1;
  for (int lt = L - 2; lt >= 1 && L - 1 - lt <= TAIL_MAX_LEVELS; --lt)
    if (tail_lds_bytes(gl + lt, L - 1 - lt, dn, elem) <= (size_t)TAIL_LDS_BYTES) best = lt;
  return best;
}

size_t layout(const fracture_params* p, fracture* h, void* ws) {
  Grid gl[MAXLEV];
  const int L = level_shapes(p, gl);
  if (L < 1) return 0;
  Carver c(ws);
  const int dim = p->dim;
  const int64_t N = gl[0].N, n2 = dim * N;   // displacement DOFs
  const int64_t nelem = (int64_t)p->nx * p->ny * (dim == 3 ? 6 * (int64_t)p->nz : 2);
  fracture tmp;
  fracture* t = h ? h : &tmp;
  t->u = c.take<double>(n2);
  t->alpha = c.take<double>(N);
  t->alpha_prev = c.take<double>(N);
  t->u_entry = c.take<double>(n2);
  t->alpha_entry = c.take<double>(N);
  t->x = c.take<double>(n2);
  t->r = c.take<double>(n2);
  t->pv = c.take<double>(n2);
  t->q = c.take<double>(n2);
  t->w2 = c.take<double>(nelem);
  t->F = c.take<double>(N);
  t->phi = c.take<double>(N);
  t->hdinv = c.take<double>(N);
  t->atil = c.take<double>(N);
  t->vd = c.take<double>(N);
  t->vr = c.take<double>(N);
  t->vz = c.take<double>(N);
  t->vp = c.take<double>(N);
  t->vq = c.take<double>(N);
  t->vt1 = c.take<double>(N);
  t->vt2 = c.take<double>(N);
  t->mask = c.take<uint8_t>(N);
  for (int l = 0; l < L; ++l) {
    Level& v = t->lv[l];
    v.g = gl[l];
    const int64_t m2 = dim * (int64_t)gl[l].N;
    const int64_t ne = (int64_t)gl[l].nx * gl[l].ny * (dim == 3 ? 6 * (int64_t)gl[l].nz : 2);
    v.abar = l > 0 ? c.take<double>(ne) : nullptr;
    v.b = c.take<double>(m2);
    v.xa = c.take<double>(m2);
    v.xb = c.take<double>(m2);
    v.d = c.take<double>(m2);
    v.r = c.take<double>(m2);
    const bool smoothed3 = dim == 3 && l < L - 1;
    v.dg = smoothed3 ? c.take<double>(m2) : nullptr;
    if (p->precision == FRACTURE_MIXED) {
      v.dg32 = smoothed3 ? c.take<float>(m2) : nullptr;
      v.abar32 = l > 0 ? c.take<float>(ne) : nullptr;
      v.b32 = c.take<float>(m2);
      v.xa32 = c.take<float>(m2);
      v.xb32 = c.take<float>(m2);
      v.d32 = c.take<float>(m2);
      v.r32 = c.take<float>(m2);
    }
  }
  if (p->precision == FRACTURE_MIXED) {
    t->mixed = true;
    t->alpha32 = c.take<float>(N);
    t->fe32 = c.take<float>(n2);
    t->fr32 = c.take<float>(n2);
    t->fp32 = c.take<float>(n2);
    t->fq32 = c.take<float>(n2);
  }
  if (p->newton) {
    const int64_t n3 = n2 + N;   // [u block | alpha]
    t->nv_prev = c.take<double>(n3);
    t->nv = c.take<double>(n3);
    t->naz = c.take<double>(n3);
    t->nz = c.take<double>(n3);
    t->nw_prev = c.take<double>(n3);
    t->nw = c.take<double>(n3);
    t->nx = c.take<double>(n3);
    t->npu1 = c.take<double>(n2);
    t->npu2 = c.take<double>(n2);
    t->npa1 = c.take<double>(N);
    t->npa2 = c.take<double>(N);
    t->nca = c.take<double>(N);
    t->ncb = c.take<double>(N);
    t->ncd = c.take<double>(N);
    t->nut = c.take<double>(n2);
    t->nat = c.take<double>(N);
    t->nFu = c.take<double>(n2);
  }
  const int dn = dim * gl[L - 1].N;
  t->dA = c.take<double>((size_t)dn * dn);
  t->dAinv = c.take<double>((size_t)dn * dn);
  t->dref = c.take<double>((int64_t)gl[L - 1].nx * gl[L - 1].ny *
                           (dim == 3 ? 6 * (int64_t)gl[L - 1].nz : 2));
  int pn = node_blocks(gl[0]);
  if (vec_blocks(n2) > pn) pn = vec_blocks(n2);
  t->part_n = pn;
  t->part = c.take<double>(pn * C_SLOTS);
  if (p->deflate) {
    t->dfl_parent = c.take<int>(N);
    t->dfl_label = c.take<int>(N);
    t->dfl_fid = c.take<int>(N);
    t->dfl_meta = c.take<int>(DFL_META_INTS);
    t->dfl_part = c.take<double>((size_t)dfl_part_blocks(N) * DFL_M);
    t->dfl_E = c.take<double>(DFL_M * DFL_M);
    t->dfl_Einv = c.take<double>(DFL_M * DFL_M);
    t->dfl_mu = c.take<double>(DFL_M);
  }
  t->S = c.take<double>(S_COUNT);
  t->nlev = L;
  t->dense_n = dn;
  t->N = N;
  t->n2 = n2;
  t->tail64 = tail_start(gl, L, dim, dn, sizeof(double));
  t->tail32 = tail_start(gl, L, dim, dn, sizeof(float));
  return c.off + 256;
}

Mat make_mat(const fracture_params* p) {
  double lam = p->E * p->nu / ((1.0 + p->nu) * (1.0 - 2.0 * p->nu));
  const double mu = p->E / (2.0 * (1.0 + p->nu));
  if (p->dim == 2 && p->plane_stress) lam = 2.0 * lam * mu / (lam + 2.0 * mu);
  return Mat{lam + 2.0 * mu, lam, mu};
}

// Upper bound of lambda_max(D^{-1} K) for any damage: D^{-1}K's Gershgorin
// radius per row is a weighted mean of the element ratios
// sum_j |K_e,ij| / K_e,ii, so their maximum over the two triangle types
// bounds every level (all levels share the element shapes).
double chebyshev_bound2d(const Grid& g, const Mat& m) {
  const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy;
  double best = 0.0;
  for (int t = 0; t < 2; ++t) {
    double gx[3], gy[3];
    if (t == 0) { gx[0] = -ihx; gy[0] = 0; gx[1] = ihx; gy[1] = -ihy; gx[2] = 0; gy[2] = ihy; }
    else { gx[0] = 0; gy[0] = -ihy; gx[1] = ihx; gy[1] = 0; gx[2] = -ihx; gy[2] = ihy; }
    for (int v = 0; v < 3; ++v) {
      for (int comp = 0; comp < 2; ++comp) {
        double diag = 0, sum = 0;
        for (int b = 0; b < 3; ++b) {
          double kx, ky;
          if (comp == 0) {
            kx = m.l2m * gx[v] * gx[b] + m.mu * gy[v] * gy[b];
            ky = m.lam * gx[v] * gy[b] + m.mu * gy[v] * gx[b];
            if (b == v) diag = kx;
          } else {
            kx = m.lam * gy[v] * gx[b] + m.mu * gx[v] * gy[b];
            ky = m.l2m * gy[v] * gy[b] + m.mu * gx[v] * gx[b];
            if (b == v) diag = ky;
          }
          sum += std::fabs(kx) + std::fabs(ky);
        }
        if (sum / diag > best) best = sum / diag;
      }
    }
  }
  return best;
}

// The same bound for the six Kuhn tetrahedra (12 x 12 element matrices).
double chebyshev_bound3d(const Grid& g, const Mat& m) {
  static const int off[6][4][3] = {
    {{0,0,0},{1,0,0},{1,1,0},{1,1,1}}, {{0,0,0},{1,0,0},{1,0,1},{1,1,1}},
    {{0,0,0},{0,1,0},{1,1,0},{1,1,1}}, {{0,0,0},{0,1,0},{0,1,1},{1,1,1}},
    {{0,0,0},{0,0,1},{1,0,1},{1,1,1}}, {{0,0,0},{0,0,1},{0,1,1},{1,1,1}}};
  const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
  double best = 0.0;
  for (int p = 0; p < 6; ++p) {
    double gr[4][3] = {};
    for (int v = 0; v < 4; ++v) {
      for (int a = 0; a < 3; ++a) {
        if (v < 3 && off[p][v + 1][a] != off[p][v][a]) gr[v][a] -= ih[a];
        if (v > 0 && off[p][v][a] != off[p][v - 1][a]) gr[v][a] += ih[a];
      }
    }
    for (int v = 0; v < 4; ++v)
      for (int c = 0; c < 3; ++c) {
        double diag = 0, sum = 0;
        for (int w = 0; w < 4; ++w) {
          const double gg = gr[v][0] * gr[w][0] + gr[v][1] * gr[w][1] + gr[v][2] * gr[w][2];
          for (int d = 0; d < 3; ++d) {
            const double kv = m.lam * gr[v][c] * gr[w][d] + m.mu * gr[v][d] * gr[w][c] + (c == d ? m.mu * gg : 0.0);
            if (w == v && d == c) diag = kv;
            sum += std::fabs(kv);
          }
        }
        if (sum / diag > best) best = sum / diag;
      }
  }
  return best;
}

// The finest grid carrying the current load as thermal eigenstrain (3D: the
// load is DT; 2D thermal shock: the load is the time tau, the erfc length
// ell tau); the residual, W2, energy and coupling blocks of the actual
// problem use it, operator actions on error equations use the plain grid.
Grid with_load(Grid g, const fracture_params& p, double load) {
  if (g.dim == 3) {
    g.eig_dT = load;
  } else if (g.bc == BC_TSHOCK_2D && load > 0.0) {
    g.eig_dT = p.thermal_dT;
    g.eig_depth = p.ell * load;
  } else {
    g.eig_dT = 0.0;
  }
  return g;
}

Grid load_grid(const fracture* h) { return with_load(h->lv[0].g, h->p, h->load); }

Red red(fracture* h, int cslot, int sslot, int post = P_STORE) {
  return Red{h->part + (size_t)cslot * h->part_n, h->S, sslot, post};
}

// The device scalars into h->hS (pinned), then wait for the stream.  A small
// kernel writes them to host memory itself, which costs less than a runtime
// device-to-host copy on every convergence test.
int read_scalars(fracture* h) {
  if (h->graph_error) return FRACTURE_EDEVICE;
  launch_scalars_out(h->st, h->S, h->hS);
  HIPCHK(hipStreamSynchronize(h->st));
  return FRACTURE_OK;
}

// Lagged read of device scalars: the values of iteration k land in pinned
// slot k % 2 behind an event, and the host waits for iteration k - 1's (or
// k's) values while later work is already queued, so the device does not
// idle on the host's convergence test.
constexpr int LAG_W = 4;   // doubles per pinned slot

// Pinned host slot of iteration k's lagged scalars.  The kernel that
// produces them writes them there itself (Red::host, k_minres_b), so no copy
// is queued; lag_mark records the event the host waits on.
double* lag_slot(fracture* h, int k) { return h->hS + S_COUNT + LAG_W * (k & 1); }

void lag_mark(fracture* h, int k) { (void)hipEventRecord(h->ev[8 + (k & 1)], h->st); }

int lag_get(fracture* h, int k, int count, double* v) {
  if (h->graph_error) return FRACTURE_EDEVICE;
  HIPCHK(hipEventSynchronize(h->ev[8 + (k & 1)]));
  for (int q = 0; q < count; ++q) v[q] = h->hS[S_COUNT + LAG_W * (k & 1) + q];
  return FRACTURE_OK;
}

const double* level_coef(fracture* h, int l) { return l == 0 ? h->alpha : h->lv[l].abar; }

// ---------------------------------------------------------------------------
// multigrid
// ---------------------------------------------------------------------------

void update_coefficients(fracture* h) {
  for (int l = 1; l < h->nlev; ++l)
    launch_coarsen2d(h->st, h->lv[l - 1].g, l == 1, level_coef(h, l - 1), h->p.k_ell, h->lv[l].g,
                     h->lv[l].abar, h->mixed ? h->lv[l].abar32 : nullptr);
  if (h->mixed) launch_to_float(h->st, h->N, h->alpha, h->alpha32, 1.0);
  if (h->dim == 3)
    for (int l = 0; l < h->nlev - 1; ++l) {
      const Level& v = h->lv[l];
      launch_diag3d<double>(h->st, v.g, h->mat, l == 0, l == 0 ? h->alpha : v.abar, h->p.k_ell, v.dg);
      if (h->mixed)
        launch_diag3d<float>(h->st, v.g, h->mat, l == 0, l == 0 ? h->alpha32 : v.abar32, h->p.k_ell,
                             v.dg32);
    }
  const int Lc = h->nlev - 1;
  if (Lc >= 1)
    launch_dense_setup(h->st, h->lv[Lc].g, h->mat, h->lv[Lc].abar, h->dA, h->dAinv, h->dref, h->S,
                       COARSE_DRIFT);
  h->coef_valid = true;
}

// Coarsest level with nlev == 1 has no abar array; assemble from alpha then.
// (validate() guarantees nlev >= 2 for the sizes this driver accepts.)

// Buffers of a level in the value type of the cycle.
template <class T>
struct LevelBufs {
  T *b, *xa, *xb, *d, *r;
  const T* coef;
  const T* dg;   // 3D: the stored diagonal of K
};

template <class T>
LevelBufs<T> bufs(fracture* h, int l);

template <>
LevelBufs<double> bufs<double>(fracture* h, int l) {
  Level& v = h->lv[l];
  return {v.b, v.xa, v.xb, v.d, v.r, l == 0 ? h->alpha : v.abar, v.dg};
}

template <>
LevelBufs<float> bufs<float>(fracture* h, int l) {
  Level& v = h->lv[l];
  return {v.b32, v.xa32, v.xb32, v.d32, v.r32, l == 0 ? h->alpha32 : v.abar32, v.dg32};
}

// One Jacobi-Chebyshev step of the V-cycle; while fracture_kernel_timing is
// active every KT_STRIDE-th float64 step on the finest level is bracketed by
// events, with its algorithmic bytes (coefficients 8, b, x_in, a distinct
// d_in, x_out, d_out per node).
template <class T>
void smooth_step(fracture* h, const Grid& g, bool fine, const T* coef, const T* dg, double kell,
                 const T* x_in, T* x_out, const T* b, const T* din, T* dout, double cd, double cr,
                 const Grid* gc = nullptr, const T* xc = nullptr) {
  const bool timed = fine && sizeof(T) == sizeof(double) && h->kt_cap > 0 &&
                     (h->kt_seen++ % KT_STRIDE == 0) && h->kt_used < h->kt_cap;
  if (timed) (void)hipEventRecord(h->kt_ev[2 * h->kt_used], h->st);
  if (g.dim == 3)
    launch_smooth3d<T>(h->st, g, h->mat, fine, coef, dg, kell, x_in, x_out, b, din, dout, cd, cr);
  else if (xc)
    launch_prol_smooth2d<T>(h->st, g, *gc, h->mat, fine, coef, kell, x_in, xc, x_out, b, dout, cr);
  else
    launch_smooth2d<T>(h->st, g, h->mat, fine, coef, kell, x_in, x_out, b, din, dout, cd, cr);
  if (timed) {
    (void)hipEventRecord(h->kt_ev[2 * h->kt_used + 1], h->st);
    const double dv = 8.0 * g.dim;
    h->kt_bytes += (double)g.N * (8.0 + dv + (x_in ? dv : 0.0) + (din && din != x_in ? dv : 0.0) +
                                  dv + (dout ? dv : 0.0) + (g.dim == 3 ? dv : 0.0)) +
                   (xc ? dv * gc->N : 0.0);
    ++h->kt_used;
  }
}

// z = V-cycle(b) on level l; returns the buffer holding the result (final_out
// when given: the last post-smoothing step writes there).  The cycle is
// symmetric: pre- and post-smoothing apply the same Chebyshev polynomial, so
// it is a fixed SPD preconditioner in exact arithmetic.
template <class T>
T* vcycle_t(fracture* h, int l, const T* b, T* final_out = nullptr, bool first_done = false) {
  LevelBufs<T> v = bufs<T>(h, l);
  const Grid& g = h->lv[l].g;
  const int k = h->p.cheb_degree;
  const bool fine = l == 0;
  const double kell = h->p.k_ell;
  if (l == h->nlev - 1) {
    launch_dense_solve<T>(h->st, h->dense_n, h->dAinv, b, v.xa);
    return v.xa;
  }
  const int tail = sizeof(T) == sizeof(double) ? h->tail64 : h->tail32;
  if (h->p.vcycle_tail && l == tail) {
    TailArgs<T> ta{};
    ta.nl = h->nlev - 1 - l;
    for (int q = 0; q <= ta.nl; ++q) ta.g[q] = h->lv[l + q].g;
    for (int q = 0; q < ta.nl; ++q) ta.coef[q] = bufs<T>(h, l + q).coef;
    ta.m = h->mat;
    ta.kell = kell;
    ta.k = k;
    for (int s = 0; s < k; ++s) { ta.cd[s] = h->cheb_cd[s]; ta.cr[s] = h->cheb_cr[s]; }
    ta.Ainv = h->dAinv;
    ta.dense_n = h->dense_n;
    ta.b = b;
    ta.x = v.xa;
    launch_vtail2d<T>(h->st, ta);
    return v.xa;
  }
  // pre-smoothing from zero (first_done: the first step came with the
  // restriction, into xa and d)
  T* cur = nullptr;
  for (int s = 0; s < k; ++s) {
    T* out = (s % 2 == 0) ? v.xa : v.xb;
    if (s == 0 && first_done) {
      cur = out;
      continue;
    }
    const T* din = s == 0 ? nullptr : (s == 1 ? cur : v.d);
    T* dout = (s < k - 1) ? v.d : nullptr;
    smooth_step<T>(h, g, fine, v.coef, v.dg, kell, cur, out, b, din, dout, h->cheb_cd[s],
                   h->cheb_cr[s]);
    cur = out;
  }
  // residual, restriction, coarse correction
  Red none{};
  launch_resid2d<T>(h->st, g, h->mat, fine, v.coef, kell, cur, v.r, b, false, none);
  LevelBufs<T> c = bufs<T>(h, l + 1);
  // a next level smoothed by per-level kernels takes its first step from
  // zero together with the restriction
  const bool fuse = l + 1 < h->nlev - 1 && !(h->p.vcycle_tail && l + 1 == tail);
  if (fuse && g.dim == 3)
    launch_restrict_smooth3d<T>(h->st, g, h->lv[l + 1].g, v.r, c.b, c.dg, c.xa,
                                k > 1 ? c.d : nullptr, h->cheb_cr[0]);
  else if (fuse)
    launch_restrict_smooth2d<T>(h->st, g, h->lv[l + 1].g, h->mat, c.coef, kell, v.r, c.b, c.xa,
                                k > 1 ? c.d : nullptr, h->cheb_cr[0]);
  else
    launch_restrict2d<T>(h->st, g, h->lv[l + 1].g, v.r, c.b);
  T* xc = vcycle_t<T>(h, l + 1, c.b, nullptr, fuse);
  // in 2D the prolongation rides in the first post-smoothing step
  const bool prol_fused = g.dim == 2;
  if (!prol_fused) launch_prolong3d<T>(h->st, g, h->lv[l + 1].g, xc, cur);
  // post-smoothing (same polynomial: the V-cycle is symmetric)
  for (int s = 0; s < k; ++s) {
    T* out = (cur == v.xa) ? v.xb : v.xa;
    if (s == k - 1 && final_out) out = final_out;
    const T* din = s == 0 ? nullptr : v.d;
    T* dout = (s < k - 1) ? v.d : nullptr;
    const bool pr = s == 0 && prol_fused;
    smooth_step<T>(h, g, fine, v.coef, v.dg, kell, cur, out, b, din, dout, h->cheb_cd[s],
                   h->cheb_cr[s], pr ? &h->lv[l + 1].g : nullptr, pr ? xc : nullptr);
    cur = out;
  }
  return cur;
}

double* vcycle(fracture* h, int l, const double* b) { return vcycle_t<double>(h, l, b); }

// Runs body(), which launches on h->st and returns its result buffer.  With
// use_graphs the first call for an operand set (op, a, b) records the
// launches on the private stream h->cap as a HIP graph, later calls replay
// it on h->st.  A recorded sequence holds kernel launches only: no memset or
// copy node and no host synchronisation.  If recording fails the instance
// stops using graphs and launches eagerly (the same kernels in the same
// order).
template <class F>
void* graphed(fracture* h, int op, const void* a, const void* b, F&& body) {
  // eager while the finest-level steps are timed (no events inside a replay)
  if (!h->p.use_graphs || h->capturing || h->kt_cap > 0) return body();
  for (const Captured& c : h->graphs)
    if (c.op == op && c.a == a && c.b == b) {
      if (hipGraphLaunch(c.exec, h->st) != hipSuccess) h->graph_error = true;
      return c.out;
    }
  if ((int)h->graphs.size() >= MAX_GRAPHS) return body();
  if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) {
    h->cap = nullptr;
    h->p.use_graphs = 0;
    return body();
  }
  if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
    h->p.use_graphs = 0;
    return body();
  }
  hipStream_t user = h->st;
  h->st = h->cap;
  h->capturing = true;
  void* out = body();
  h->st = user;
  h->capturing = false;
  hipGraph_t gr = nullptr;
  hipGraphExec_t ex = nullptr;
  bool ok = hipStreamEndCapture(h->cap, &gr) == hipSuccess && gr;
  ok = ok && hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) == hipSuccess;
  if (gr) (void)hipGraphDestroy(gr);
  if (!ok) {
    (void)hipGetLastError();
    h->p.use_graphs = 0;
    return body();
  }
  h->graphs.push_back({op, a, b, out, ex});
  if (hipGraphLaunch(ex, h->st) != hipSuccess) h->graph_error = true;
  return out;
}

// V-cycle on the finest level (recorded per right-hand side buffer).
double* vcycle0(fracture* h, const double* b, double* final_out = nullptr) {
  return (double*)graphed(h, G_VCYCLE64, b, final_out,
                          [&] { return (void*)vcycle_t<double>(h, 0, b, final_out); });
}

float* vcycle0f(fracture* h, const float* b) {
  return (float*)graphed(h, G_VCYCLE32, b, nullptr, [&] { return (void*)vcycle_t<float>(h, 0, b); });
}

// ---------------------------------------------------------------------------
// elastic subproblem: x <- argmin at fixed alpha, warm start from u
// ---------------------------------------------------------------------------

// Stopping tolerance of one elastic solve inside ORAM: the absolute
// pcg_rtol * ||f||, or, under ORAM-N (whose Newton phase enforces the final
// accuracy of u and alpha), the looser of that and pcg_reduction times the
// residual at the warm start; never looser than the step's sweep cap.
double sweep_tol(const fracture* h, double tol, double r0) {
  if (h->p.newton && h->p.pcg_reduction > 0) tol = std::fmax(tol, h->p.pcg_reduction * r0);
  return std::fmin(tol, h->sweep_cap);
}

// Crack-aware deflation: label the fragments of the current alpha and form
// E = W^T K W (one operator action per mode, through pv and q) and its
// inverse on the device.  *m receives the number of modes (0: no fragment).
int dfl_setup(fracture* h, int* m) {
  const Grid& g = h->lv[0].g;
  hipStream_t st = h->st;
  launch_fragments2d(st, g, h->alpha, h->p.deflate_theta, h->p.deflate_min_nodes,
                     h->p.deflate_max_fragments, h->dfl_parent, h->dfl_label, h->dfl_fid,
                     h->dfl_meta);
  int nf = 0;
  HIPCHK(hipMemcpyAsync(&nf, h->dfl_meta + DFL_META_NFRAG, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *m = 3 * nf;
  Red none{};
  for (int k = 0; k < *m; ++k) {
    launch_dfl_mode(st, g, h->dfl_fid, k, h->pv);
    launch_apply2d<double>(st, g, h->mat, true, h->alpha, h->p.k_ell, h->pv, h->q, nullptr, 1, 0,
                           none);
    launch_dfl_wtv(st, g, h->dfl_fid, h->q, h->dfl_part, k, h->dfl_E, nullptr, nullptr);
  }
  if (*m) launch_dfl_invert(st, h->dfl_E, h->dfl_Einv, h->dfl_meta);
  return hip_ok(hipGetLastError());
}

// v -= W E^{-1} W^T K z (sign -1), the deflated CG direction correction, or
// x += W E^{-1} W^T r (sign +1, with Kz = nullptr: r itself).
void dfl_correct(fracture* h, const double* z, double* v, double sign) {
  const Grid& g = h->lv[0].g;
  const double* w = z;
  if (sign < 0) {
    Red none{};
    launch_apply2d<double>(h->st, g, h->mat, true, h->alpha, h->p.k_ell, z, h->q, nullptr, 1, 0,
                           none);
    w = h->q;
  }
  launch_dfl_wtv(h->st, g, h->dfl_fid, w, h->dfl_part, -1, nullptr, h->dfl_Einv, h->dfl_mu);
  launch_dfl_add(h->st, g, h->dfl_fid, h->dfl_mu, v, sign);
}

// Preconditioned CG on the elastic system, warm-started from u.  With
// params.deflate, deflated CG (Saad, Yeung, Erhel and Guyomarc'h, 2000):
// the start is corrected by W E^{-1} W^T r and every direction loses
// W E^{-1} W^T K z, which keeps W^T r = 0 at every iterate.
// The iterate: u itself at omega = 1 (the sweep keeps the elastic solution
// as is), else the separate x that the relaxation then blends into u.
double* pcg_iterate(fracture* h) { return h->omega_cur == 1.0 ? h->u : h->x; }

int pcg(fracture* h, double tol, int* iters) {
  const Grid& g = h->lv[0].g;
  const int64_t n2 = h->n2;
  hipStream_t st = h->st;
  double* x = pcg_iterate(h);
  if (x != h->u) HIPCHK(hipMemcpyAsync(x, h->u, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  const Grid gl = load_grid(h);
  int rc = FRACTURE_OK;
  double rr = h->r_rr;
  if (!h->r_valid) {
    launch_resid2d(st, gl, h->mat, true, h->alpha, h->p.k_ell, x, h->r, nullptr, true,
                   red(h, 0, S_RR));
    rc = read_scalars(h);
    if (rc) return rc;
    rr = h->hS[S_RR];
  }
  h->r_valid = false;
  if (!std::isfinite(rr)) return FRACTURE_ENONFINITE;
  *iters = 0;
  tol = sweep_tol(h, tol, std::sqrt(rr));
  if (std::sqrt(rr) <= tol) return FRACTURE_OK;
  int m = 0;
  if (h->p.deflate) {
    rc = dfl_setup(h, &m);
    if (rc) return rc;
  }
  if (m) {
    dfl_correct(h, h->r, x, 1.0);
    launch_resid2d(st, gl, h->mat, true, h->alpha, h->p.k_ell, x, h->r, nullptr, true,
                   red(h, 0, S_RR));
    rc = read_scalars(h);
    if (rc) return rc;
    rr = h->hS[S_RR];
    if (!std::isfinite(rr)) return FRACTURE_ENONFINITE;
    if (std::sqrt(rr) <= tol) return FRACTURE_OK;
  }
  double* z = vcycle0(h, h->r);
  launch_dot(st, n2, h->r, z, red(h, 1, S_RZ));
  // the first direction is z itself: it is copied into p only when a second
  // iteration needs the buffer that the next V-cycle overwrites (most
  // solves inside the sweeps stop after one)
  const double* p = z;
  if (m) {
    HIPCHK(hipMemcpyAsync(h->pv, z, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    dfl_correct(h, z, h->pv, -1.0);
    p = h->pv;
  }
  for (int it = 1; it <= h->p.max_pcg; ++it) {
    launch_apply2d(st, g, h->mat, true, h->alpha, h->p.k_ell, p, h->q, nullptr, 1, 1,
                   red(h, 2, S_PQ, P_CG_ALPHA));
    launch_cg_update(st, n2, x, h->r, p, h->q, h->S, red(h, 3, S_RR));
    rc = read_scalars(h);
    if (rc) return rc;
    rr = h->hS[S_RR];
    *iters = it;
    if (!std::isfinite(rr)) return FRACTURE_ENONFINITE;
    if (std::sqrt(rr) <= tol) return FRACTURE_OK;
    if (p != h->pv) {
      HIPCHK(hipMemcpyAsync(h->pv, p, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
      p = h->pv;
    }
    z = vcycle0(h, h->r);
    launch_dot(st, n2, h->r, z, red(h, 4, S_RZNEW, P_CG_BETA));
    launch_xpby(st, n2, z, h->pv, h->S);
    if (m) dfl_correct(h, z, h->pv, -1.0);
  }
  return FRACTURE_ENOTCONV;
}

// Mixed precision: iterative refinement in float64 around a float32
// flexible CG (FCG(1): p_k = z_k - (z_k.q_{k-1})/(p_{k-1}.q_{k-1}) p_{k-1},
// alpha_k = p_k.r_k / p_k.q_k) whose operator, V-cycle and vectors are all
// float32.  The float64 residual r = f - K x is recomputed before every
// inner solve, which sees it normalised to unit length.
constexpr double MIXED_INNER_RTOL = 1e-4;
constexpr double MIXED_LOOSE = 0.05;
constexpr int MIXED_MAX_OUTER = 30;

int pcg_mixed(fracture* h, double tol, int* iters) {
  const Grid& g = h->lv[0].g;
  const int64_t n2 = h->n2;
  hipStream_t st = h->st;
  *iters = 0;
  double* x = pcg_iterate(h);
  if (x != h->u) HIPCHK(hipMemcpyAsync(x, h->u, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  for (int outer = 0;; ++outer) {
    // the first residual may be the one the last sweep left in r
    int rc = FRACTURE_OK;
    double rr = h->r_rr;
    if (outer > 0 || !h->r_valid) {
      launch_resid2d<double>(st, load_grid(h), h->mat, true, h->alpha, h->p.k_ell, x, h->r, nullptr,
                             true, red(h, 0, S_RR));
      rc = read_scalars(h);
      if (rc) return rc;
      rr = h->hS[S_RR];
    }
    h->r_valid = false;
    if (!std::isfinite(rr)) return FRACTURE_ENONFINITE;
    const double rn = std::sqrt(rr);
    if (outer == 0) tol = sweep_tol(h, tol, rn);
    if (rn <= tol) return FRACTURE_OK;
    if (outer >= MIXED_MAX_OUTER || *iters >= h->p.max_pcg) return FRACTURE_ENOTCONV;
    // inner solve of K e = r / |r| in float32
    launch_to_float(st, n2, h->r, h->fr32, 1.0 / rn);
    HIPCHK(hipMemsetAsync(h->fe32, 0, n2 * sizeof(float), st));
    // the inner float32 recurrence tracks the true residual to about 1e-4
    // relative: a loose outer target (an ORAM sweep's reduction) is asked of
    // the inner solve almost as is, a tight one with a factor 2 to spare
    const double want = tol / rn;
    const double tin = std::fmax(MIXED_INNER_RTOL, (want >= MIXED_LOOSE ? 0.9 : 0.5) * want);
    // the first direction is z itself, copied into p only when a second
    // iteration needs the buffer that the next V-cycle overwrites
    float* z = vcycle0f(h, h->fr32);
    float* p = z;
    for (int it = 0;; ++it) {
      if (it > 0) {
        if (p != h->fp32) {
          HIPCHK(hipMemcpyAsync(h->fp32, p, n2 * sizeof(float), hipMemcpyDeviceToDevice, st));
          p = h->fp32;
        }
        z = vcycle0f(h, h->fr32);
        launch_dot_f(st, n2, z, h->fq32, red(h, 1, S_TMP0, P_FCG_BETA));
        launch_xpby_f(st, n2, z, h->fp32, h->S);
      }
      launch_apply2d<float>(st, g, h->mat, true, h->alpha32, h->p.k_ell, p, h->fq32, nullptr,
                            1, 1, red(h, 2, S_PQ));
      launch_dot_f(st, n2, p, h->fr32, red(h, 4, S_TMP1, P_FCG_ALPHA));
      launch_cg_update_f(st, n2, h->fe32, h->fr32, p, h->fq32, h->S, red(h, 3, S_RR));
      rc = read_scalars(h);
      if (rc) return rc;
      ++*iters;
      const double rin = h->hS[S_RR];
      if (!std::isfinite(rin)) return FRACTURE_ENONFINITE;
      if (std::sqrt(rin) <= tin || *iters >= h->p.max_pcg) break;
    }
    launch_add_scaled_f(st, n2, x, h->fe32, rn);
  }
}

// ||f - K u_D|| on free rows: the load the elastic problem carries (its RHS
// with a zero initial guess).  The PCG tolerance is relative to it.
int load_norm(fracture* h, double* out) {
  const Grid g = load_grid(h);
  HIPCHK(hipMemsetAsync(h->q, 0, h->n2 * sizeof(double), h->st));
  launch_lift2d(h->st, g, h->q, h->load, h->load2d);
  launch_resid2d(h->st, g, h->mat, true, h->alpha, h->p.k_ell, h->q, h->r, nullptr, true,
                 red(h, 0, S_RR));
  int rc = read_scalars(h);
  if (rc) return rc;
  *out = std::sqrt(h->hS[S_RR]);
  return FRACTURE_OK;
}

// ---------------------------------------------------------------------------
// damage subproblem: box QP by Algorithm 4 (atil <- argmin, start alpha)
// ---------------------------------------------------------------------------

// Projected Armijo search along vd on psi = 1/2 ||Phi||^2.  slope < 0.
// *phimax receives max |Phi| of the accepted point (its trial evaluation is
// that of the point the projected step then stores).
int line_search(fracture* h, double psi0, double slope, bool* accepted, double* phimax) {
  const Grid& g = h->lv[0].g;
  double mu = 1.0;
  *accepted = false;
  for (int k = 0; k <= MAX_HALVINGS; ++k) {
    launch_set_scalar(h->st, h->S, S_MU, mu);
    launch_vi_eval2d(h->st, g, h->cL, h->cM, h->cm, h->w2, h->atil, h->vd, h->alpha_prev, h->S,
                     S_MU, 1e-12, nullptr, nullptr, nullptr, nullptr, red(h, 5, S_TMP0),
                     red(h, 6, S_TMP1), red(h, 12, S_JLO), red(h, 13, S_JHI), true);
    int rc = read_scalars(h);
    if (rc) return rc;
    const double psi = 0.5 * h->hS[S_TMP0];
    if (!std::isfinite(psi)) return FRACTURE_ENONFINITE;
    if (psi <= psi0 + ARMIJO_SIGMA * mu * slope) {
      launch_proj_step(h->st, h->N, h->atil, h->vd, h->alpha_prev, h->S);
      *accepted = true;
      *phimax = h->hS[S_TMP1];
      return FRACTURE_OK;
    }
    mu *= 0.5;
  }
  return FRACTURE_OK;
}

// Under ORAM-N the damage solve of a sweep may stop at vi_reduction times
// its starting max |Phi| (the Newton phase enforces the final accuracy).
int damage_qp(fracture* h, int* vi_iters, int* cg_iters) {
  const Grid& g = h->lv[0].g;
  hipStream_t st = h->st;
  const int64_t N = h->N;
  HIPCHK(hipMemcpyAsync(h->atil, h->alpha, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  double stop = h->p.vi_tol;
  h->vi_phi2_valid = false;
  for (int it = 0;; ++it) {
    launch_vi_eval2d(st, g, h->cL, h->cM, h->cm, h->w2, h->atil, nullptr, h->alpha_prev, h->S,
                     S_MU, 1e-12, h->F, h->phi, h->mask, h->hdinv, red(h, 5, S_PHI2),
                     red(h, 6, S_PHIMAX), red(h, 12, S_JLO), red(h, 13, S_JHI), false);
    if (h->dim == 3) launch_irange3d(st, g, h->mask, red(h, 15, S_ILO), red(h, 16, S_IHI));
    int rc = read_scalars(h);
    if (rc) return rc;
    const double phimax = h->hS[S_PHIMAX], phi2 = h->hS[S_PHI2];
    if (!std::isfinite(phimax) || !std::isfinite(phi2)) return FRACTURE_ENONFINITE;
    if (it == 0 && h->p.newton && h->p.vi_reduction > 0)
      stop = std::fmax(h->p.vi_tol, h->p.vi_reduction * phimax);
    if (it == 0) stop = std::fmin(stop, h->sweep_cap);
    if (phimax <= stop) {
      h->vi_phi2 = phi2;
      h->vi_phi2_valid = true;
      return FRACTURE_OK;
    }
    if (it >= h->p.max_vi) {
      h->vi_stop = FRACTURE_STAGE_VI;
      return FRACTURE_ENOTCONV;
    }
    ++*vi_iters;
    // reduced Newton step: H_NN d_N = -F_N (Jacobi CG), d_A = 0.  The CG runs
    // on the row range that holds every inactive node (its vectors are zero
    // outside), which for crack bands is a thin strip of the grid.
    // In 3D the box is also cut to the columns that hold inactive nodes (a
    // damaged surface layer is thin in x but spans every row).
    const double jlo = -h->hS[S_JLO], jhi = h->hS[S_JHI];
    launch_neg_masked(st, N, h->F, h->mask, h->vr, h->vd);
    // no inactive node: d = 0, and the line search falls back to steepest descent
    const bool any_inactive = std::isfinite(jlo) && std::isfinite(jhi) && jhi >= jlo;
    const int j0 = any_inactive ? (int)jlo : 0, j1 = any_inactive ? (int)jhi : -1;
    int i0 = 0, i1 = g.nx;
    if (h->dim == 3 && any_inactive) {
      i0 = (int)(-h->hS[S_ILO]);
      i1 = (int)h->hS[S_IHI];
    }
    const int64_t W = g.nx + 1;
    const Box bx{(int64_t)j0 * W + i0, W, (int64_t)(i1 - i0 + 1),
                 any_inactive ? (int64_t)(j1 - j0 + 1) * (i1 - i0 + 1) : 0};
    // the direction update rides in the Hessian apply (p ping-pongs between
    // vp and vt1) and the preconditioner in the CG update, which in 2D also
    // finishes p.q itself, so an iteration is two kernels and one finishing
    // launch; the CG scalars live on the device and the host tests ||r|| one
    // iteration late (lag_mark / lag_get)
    // ||r_0||^2 reaches the host with the first lagged read (the second word
    // of iteration 1's slot), so no read stands between the start and the
    // first iterations; a zero r_0 makes those iterations leave d = 0
    if (any_inactive) {
      Red r0r = red(h, 7, S_TMP2);
      r0r.host = lag_slot(h, 1) + 1;
      launch_norm2_box(st, bx, h->vr, r0r);
      launch_jacobi_dot(st, bx, h->vr, h->hdinv, h->vz, red(h, 1, S_RZ));
    }
    double tol = 0.0;
    if (any_inactive) {
      double* pb[2] = {h->vp, h->vt1};
      for (int k = 1; k <= h->p.max_vi_cg; ++k) {
        double* pn = pb[k & 1];
        // in 2D the update forms alpha from the partials of p.q itself
        const Red rpq = red(h, 2, S_PQ, P_CG_ALPHA);
        const int npq = launch_helm_cg2d(st, g, h->cL, h->cM, h->w2, h->vz, pb[(k + 1) & 1], h->mask,
                                         pn, h->vq, j0, j1, i0, i1, h->S, k == 1, rpq, false);
        Red rr = red(h, 3, S_RR);
        rr.host = lag_slot(h, k);
        launch_cg_update_jac(st, bx, h->vd, h->vr, pn, h->vq, h->hdinv, h->vz, h->S, rr,
                             red(h, 4, S_RZNEW, P_CG_BETA), npq ? rpq.part : nullptr, npq);
        ++*cg_iters;
        lag_mark(h, k);
        if (k > 1) {
          double v[2] = {0.0, 0.0};
          rc = lag_get(h, k - 1, k == 2 ? 2 : 1, v);
          if (rc) return rc;
          if (k == 2) tol = h->p.vi_cg_rtol * std::sqrt(v[1]);
          if (!std::isfinite(v[0]) || !std::isfinite(tol)) return FRACTURE_ENONFINITE;
          if (std::sqrt(v[0]) <= tol) break;
        }
      }
      // an inexact step is still tried: the line search decides
    }
    bool ok = false;
    double phimax_new = INFINITY;
    const double psi0 = 0.5 * phi2;
    rc = line_search(h, psi0, -2.0 * psi0, &ok, &phimax_new);
    if (rc) return rc;
    if (!ok) {
      // steepest descent on psi: d = -(ca Phi + H (cf Phi))
      launch_merit_parts(st, N, h->atil, h->F, h->alpha_prev, h->vt1, h->vt2);
      Red none{};
      launch_helm_apply2d(st, g, h->cL, h->cM, h->w2, h->vt1, nullptr, h->vq, false, none);
      launch_neg_sum(st, N, h->vt2, h->vq, h->vd, red(h, 7, S_GG));
      rc = read_scalars(h);
      if (rc) return rc;
      rc = line_search(h, psi0, -h->hS[S_GG], &ok, &phimax_new);
      if (rc) return rc;
      if (!ok) {
        h->vi_stop = FRACTURE_STAGE_VI_SEARCH;
        return FRACTURE_ENOTCONV;
      }
    }
    // the accepted point already meets the stop test: no evaluation more
    if (phimax_new <= stop) {
      h->vi_phi2 = h->hS[S_TMP0];
      h->vi_phi2_valid = true;
      return FRACTURE_OK;
    }
  }
}

// ---------------------------------------------------------------------------
// residual of the optimality conditions, ||Phi||_2
// ---------------------------------------------------------------------------

// At omega = 1 the sweep's alpha is the damage solve's final iterate, whose
// FB residual (at the same u) that solve has just evaluated: only the
// elastic part is formed here.
// residual_launch queues the reductions, residual_value reads ||Phi||_2 from
// the scalars once the caller has read them (one read for the sweep).
void residual_launch(fracture* h) {
  const Grid g = load_grid(h);
  // -E_u on the free rows, kept in r for the next sweep's PCG
  launch_resid2d(h->st, g, h->mat, true, h->alpha, h->p.k_ell, h->u, h->r, nullptr, true,
                 red(h, 0, S_EU2));
  h->phi_reused = h->omega_cur == 1.0 && h->vi_phi2_valid;
  if (h->phi_reused) return;
  launch_w2_2d(h->st, g, h->mat, h->u, h->w2);
  launch_vi_eval2d(h->st, g, h->cL, h->cM, h->cm, h->w2, h->alpha, nullptr, h->alpha_prev, h->S,
                   S_MU, 1e-12, h->F, h->phi, h->mask, h->hdinv, red(h, 5, S_PHI2),
                   red(h, 6, S_PHIMAX), red(h, 12, S_JLO), red(h, 13, S_JHI), false);
}

double residual_value(const fracture* h) {
  return std::sqrt(h->hS[S_EU2] + (h->phi_reused ? h->vi_phi2 : h->hS[S_PHI2]));
}

// ---------------------------------------------------------------------------
// alpha relaxation (Algorithm 2); returns ||dalpha||_inf in S[S_DAMAX]
// ---------------------------------------------------------------------------

int relax_alpha(fracture* h) {
  hipStream_t st = h->st;
  const int64_t N = h->N;
  const double w = h->omega_cur;
  if (h->p.relax_mode == FRACTURE_RELAX_PROJECT || w <= 1.0) {
    launch_relax_alpha(st, N, h->alpha, h->atil, h->alpha_prev, w, h->S, -1, red(h, 8, S_DAMAX));
    return FRACTURE_OK;
  }
  if (h->p.relax_mode == FRACTURE_RELAX_RATIO) {
    launch_ratio(st, N, h->alpha, h->atil, h->alpha_prev, w, red(h, 9, S_RATIO, P_NEG));
    launch_relax_alpha(st, N, h->alpha, h->atil, h->alpha_prev, w, h->S, S_RATIO,
                       red(h, 8, S_DAMAX));
    return FRACTURE_OK;
  }
  // bisection toward 1 on [1, omega]
  double wb = w;
  bool feas = false;
  for (int k = 0; k < 30; ++k) {
    launch_violation(st, N, h->alpha, h->atil, h->alpha_prev, wb, red(h, 9, S_INFEAS));
    int rc = read_scalars(h);
    if (rc) return rc;
    if (h->hS[S_INFEAS] <= 0.0) { feas = true; break; }
    wb = 0.5 * (1.0 + wb);
  }
  if (!feas) wb = 1.0;
  launch_relax_alpha(st, N, h->alpha, h->atil, h->alpha_prev, wb, h->S, -1, red(h, 8, S_DAMAX));
  return FRACTURE_OK;
}

// ---------------------------------------------------------------------------
// Newton composition (Algorithm 3): reduced-space active-set Newton on the
// coupled optimality system, Jacobian solves by preconditioned MINRES
// ---------------------------------------------------------------------------

constexpr int CHEB_C = 4;            // Chebyshev steps approximating C^{-1}
constexpr double CHEB_C_LMAX = 2.0;  // lambda_max(D^{-1} C) <= 2 (element ratios of M and L)
constexpr double CHEB_C_LMIN = 0.04;

// Phi at (u, a): F_u = K(a) u (Dirichlet rows zero) into Fu; W2(u); F_a, Phi_a,
// the active set and the inverse diagonal via the VI evaluation.
// Returns ||Phi||^2 = sum over free rows of F_u^2 + sum Phi_a^2.
int coupled_residual(fracture* h, const double* u, const double* a, double* Fu, double* phi2) {
  const Grid g = load_grid(h);
  launch_apply2d(h->st, g, h->mat, true, a, h->p.k_ell, u, Fu, nullptr, 1, 2, red(h, 0, S_EU2));
  launch_w2_2d(h->st, g, h->mat, u, h->w2);
  launch_vi_eval2d(h->st, g, h->cL, h->cM, h->cm, h->w2, a, nullptr, h->alpha_prev, h->S, S_MU,
                   1e-12, h->F, h->phi, h->mask, h->hdinv, red(h, 5, S_PHI2), red(h, 6, S_PHIMAX),
                   red(h, 12, S_JLO), red(h, 13, S_JHI), false);
  int rc = read_scalars(h);
  if (rc) return rc;
  *phi2 = h->hS[S_EU2] + h->hS[S_PHI2];
  return std::isfinite(*phi2) ? FRACTURE_OK : FRACTURE_ENONFINITE;
}

// y = A^{-1} x approximated by newton_vcycles multigrid V-cycles from zero
// (the paper's preconditioner uses two): y = V x, then y += V (x - A y).
// Either way a fixed symmetric positive definite operator, as MINRES needs.
// In mixed precision the cycles run in float32 on the float32 copy of their
// right-hand side (MINRES vectors are normalised, so no scaling is needed);
// the residual between the cycles and y stay float64.
void apply_Ainv(fracture* h, const double* x, double* y) {
  const Grid& g = h->lv[0].g;
  const int64_t n2 = h->n2;
  Red none{};
  if (h->mixed) {
    launch_to_float(h->st, n2, x, h->fr32, 1.0);
    launch_from_float(h->st, n2, vcycle0f(h, h->fr32), y, 1.0);
    if (h->p.newton_vcycles == 1) return;
    launch_resid2d(h->st, g, h->mat, true, h->alpha, h->p.k_ell, y, h->npu2, x, false, none);
    launch_to_float(h->st, n2, h->npu2, h->fr32, 1.0);
    launch_add_scaled_f(h->st, n2, y, vcycle0f(h, h->fr32), 1.0);
    return;
  }
  vcycle0(h, x, y);
  if (h->p.newton_vcycles == 1) return;
  launch_resid2d(h->st, g, h->mat, true, h->alpha, h->p.k_ell, y, h->npu2, x, false, none);
  launch_axpby(h->st, n2, 1.0, vcycle0(h, h->npu2), 1.0, y);
}

// y = C^{-1} x approximated by CHEB_C Jacobi-Chebyshev steps on H_NN from 0.
void apply_Cinv(fracture* h, const double* x, double* y) {
  const Grid& g = h->lv[0].g;
  const double* cur = nullptr;
  double* bufs[2] = {h->nca, h->ncb};
  for (int s = 0; s < CHEB_C; ++s) {
    double* out = (s == CHEB_C - 1) ? y : bufs[s % 2];
    const double* din = s == 0 ? nullptr : (s == 1 ? cur : h->ncd);
    double* dout = (s < CHEB_C - 1) ? h->ncd : nullptr;
    launch_cheb_helm2d(h->st, g, h->cL, h->cM, h->w2, h->mask, cur, out, x, din, dout,
                       h->chebC_cd[s], h->chebC_cr[s]);
    cur = out;
  }
}

// Block preconditioner with S ~ C (eq. (preconditioner)), applied in the
// symmetric multiplicative order: y1 = A^{-1} x1; y2 = C^{-1}(x2 - B^T y1);
// z1 = A^{-1}(x1 - B y2); result [z1; y2].
void apply_P_body(fracture* h, const double* x, double* y) {
  const Grid g = load_grid(h);   // B and B^T carry the stress of u's effective strain
  const int64_t n2 = h->n2, N = h->N;
  Red none{};
  if (h->p.newton_precond == 1) {
    // block-diagonal variant: [A^{-1} x1; C^{-1} x2]
    apply_Ainv(h, x, y);
    apply_Cinv(h, x + n2, y + n2);
    return;
  }
  apply_Ainv(h, x, h->npu1);                                               // y1
  launch_jac2d(h->st, g, h->mat, h->p.k_ell, h->cL, h->cM, h->alpha, h->u, h->w2, h->mask,
               h->npu1, nullptr, nullptr, h->npa1, false, none, none, h->S + S_JLO);  // B^T y1
  launch_axpby(h->st, N, 1.0, x + n2, -1.0, h->npa1);                      // x2 - B^T y1
  apply_Cinv(h, h->npa1, y + n2);                                          // y2
  launch_jac2d(h->st, g, h->mat, h->p.k_ell, h->cL, h->cM, h->alpha, h->u, h->w2, h->mask,
               nullptr, y + n2, h->npu1, nullptr, false, none, none, h->S + S_JLO);   // B y2
  launch_axpby(h->st, n2, 1.0, x, -1.0, h->npu1);                          // x1 - B y2
  apply_Ainv(h, h->npu1, y);                                               // z1
}

void apply_P(fracture* h, const double* x, double* y) {
  graphed(h, G_PRECOND, x, y, [&] {
    apply_P_body(h, x, y);
    return (void*)y;
  });
}

// y = J x on the inactive coupled system; S[S_TMP0] + S[S_TMP1] = x.y.
// The displacement rows: A x_u by the column-tiled operator, then B x_a on
// the rows next to the inactive band (S_JLO, S_JHI as last read by the host,
// from the VI evaluation of this iterate), each adding its part of x_u.y_u.
void apply_J(fracture* h, const double* x, double* y) {
  const Grid g = load_grid(h);   // B and B^T carry the stress of u's effective strain
  const int64_t n2 = h->n2;
  launch_apply2d(h->st, h->lv[0].g, h->mat, true, h->alpha, h->p.k_ell, x, y, nullptr, 1,
                 1 /* dot */, red(h, 7, S_TMP0));
  const double jlo = -h->hS[S_JLO], jhi = h->hS[S_JHI];
  // B x_a reaches the rows within one cell of an inactive node: rows j +- 1
  // in 2D, row indices j + (ny + 1) k within +- (ny + 2) in 3D
  const int pad = h->dim == 3 ? g.ny + 2 : 1;
  if (std::isfinite(jlo) && std::isfinite(jhi) && jhi >= jlo)
    launch_couple_u2d(h->st, g, h->mat, h->alpha, h->u, x, x + n2, h->mask, y, (int)jlo - pad,
                      (int)jhi + pad, red(h, 14, S_TMP0, P_ADD));
  launch_jac2d(h->st, g, h->mat, h->p.k_ell, h->cL, h->cM, h->alpha, h->u, h->w2, h->mask, x,
               x + n2, nullptr, y + n2, true, red(h, 7, S_TMP0), red(h, 8, S_TMP1), h->S + S_JLO);
}

// MINRES (preconditioned; the three-term Lanczos recurrence with Givens
// rotations) for J d = rhs, rhs in nv.  Solution in nx.  The recurrence
// scalars live on the device (k_minres_a / k_minres_b), so the host only
// enqueues; it reads |eta| one step late through a pinned copy, and while it
// waits the device already applies J for the next iteration (discarded when
// the test passes).
int minres(fracture* h, double rtol, int* iters) {
  hipStream_t st = h->st;
  const int64_t n3 = h->n2 + h->N;   // [u block | alpha]
  HIPCHK(hipMemsetAsync(h->nx, 0, n3 * sizeof(double), st));
  HIPCHK(hipMemsetAsync(h->nv_prev, 0, n3 * sizeof(double), st));
  HIPCHK(hipMemsetAsync(h->nw_prev, 0, n3 * sizeof(double), st));
  HIPCHK(hipMemsetAsync(h->nw, 0, n3 * sizeof(double), st));
  double *v_prev = h->nv_prev, *v = h->nv, *az = h->naz, *z = h->nz, *w_prev = h->nw_prev,
         *w = h->nw;
  // The damage block of every Krylov vector vanishes off the inactive set
  // (the right-hand side, J and P all zero it there), so the vector updates
  // and dot products walk the displacement block and the rows of the
  // inactive band only (S_JLO, S_JHI from the VI evaluation of this
  // iterate's residual).
  const int64_t n2 = h->n2, W = h->lv[0].g.nx + 1;
  const double jlo = -h->hS[S_JLO], jhi = h->hS[S_JHI];
  Seg sg{n2, n2, n2};
  if (std::isfinite(jlo) && std::isfinite(jhi) && jhi >= jlo)
    sg = Seg{n2, n2 + (int64_t)jlo * W, n2 + ((int64_t)jhi - (int64_t)jlo + 1) * W};
  *iters = 0;
  apply_P(h, v, z);
  launch_dot_seg(st, sg, z, v, red(h, 9, S_TMP2));
  launch_minres_init(st, h->S);
  int rc = read_scalars(h);
  if (rc) return rc;
  if (h->hS[S_MN_BAD] != 0.0) return FRACTURE_ENONFINITE;
  const double g1 = h->hS[S_MN_G1];
  if (!(g1 > 0.0)) return FRACTURE_OK;
  apply_J(h, z, az);                                             // az = J z, S = z.J z
  for (int j = 1; j <= h->p.max_minres; ++j) {
    launch_minres_a(st, h->S);
    launch_lincomb3_s(st, sg, h->S, az, v, v_prev);              // az = v_{j+1}
    double* vn = az;
    apply_P(h, vn, v_prev);                                      // v_prev buffer <- z_{j+1}
    double* zn = v_prev;
    launch_dot_seg(st, sg, zn, vn, red(h, 9, S_TMP2));
    launch_minres_b(st, h->S, lag_slot(h, j));
    launch_minres_update_s(st, sg, h->S, z, w_prev, w, h->nx);   // w_prev <- w_{j+1}; x update
    lag_mark(h, j);
    // rotate buffers
    v_prev = v;                // v_{j}
    v = vn;                    // v_{j+1}
    az = z;                    // free buffer
    z = zn;                    // z_{j+1}
    std::swap(w_prev, w);      // w <- w_{j+1}, w_prev <- w_j
    *iters = j;
    if (j < h->p.max_minres) apply_J(h, z, az);                  // next iteration's J z
    double stat[3];
    rc = lag_get(h, j, 3, stat);
    if (rc) return rc;
    if (stat[2] != 0.0) return FRACTURE_ENONFINITE;
    if (stat[0] <= rtol * g1 || stat[1] == 0.0) return FRACTURE_OK;
  }
  return FRACTURE_OK;  // an inexact Newton direction is still tried by the line search
}

// One Newton phase (Algorithm 3, inner loop): iterate until ||Phi|| <=
// final_tol (converged), the line search fails or max_newton is reached
// (failed).  *nphi receives the final ||Phi||_2.
int newton_phase(fracture* h, fracture_stats* st, double* nphi, bool* converged) {
  hipStream_t s = h->st;
  const int64_t n2 = h->n2, N = h->N;
  *converged = false;
  double phi2 = 0;
  int rc = coupled_residual(h, h->u, h->alpha, h->nFu, &phi2);
  if (rc) return rc;
  double nphi_prev = 1.0, eta_prev = EW_ETA0;
  for (int it = 0; it < h->p.max_newton; ++it) {
    *nphi = std::sqrt(phi2);
    if (h->monitor) h->monitor(h->monitor_user, -(it + 1), -1.0, *nphi);
    if (*nphi <= h->p.final_tol) { *converged = true; return FRACTURE_OK; }
    update_coefficients(h);
    // rhs = -[F_u; F_a on the inactive set]
    launch_axpby(s, n2, -1.0, h->nFu, 0.0, h->nv);
    launch_neg_masked(s, N, h->F, h->mask, h->nv + n2, h->nca);
    // forcing term.  target: enough accuracy for this step to reach
    // final_tol.  Eisenstat-Walker (choice 2, gamma = 0.9, exponent 2, with
    // their safeguard): eta_k = 0.9 (||Phi_k|| / ||Phi_k-1||)^2, eta_0 =
    // EW_ETA0, never tighter than the target
    double eta = h->p.minres_rtol;
    if (h->p.newton_forcing > 0) {
      const double target = h->p.newton_forcing * h->p.final_tol / *nphi;
      if (h->p.newton_forcing_mode == 1) {
        double ew = EW_ETA0;
        if (it > 0) {
          ew = 0.9 * (*nphi / nphi_prev) * (*nphi / nphi_prev);
          const double sg = 0.9 * eta_prev * eta_prev;
          if (sg > 0.1) ew = std::fmax(ew, sg);
        }
        eta = std::fmax(h->p.minres_rtol, std::fmin(EW_ETA_MAX, std::fmax(ew, target)));
      } else {
        eta = std::fmax(h->p.minres_rtol, std::fmin(NEWTON_ETA_MAX, target));
      }
    }
    nphi_prev = *nphi;
    eta_prev = eta;
    int its = 0;
    rc = minres(h, eta, &its);
    st->minres_iters += its;
    if (rc) return rc;
    ++st->newton_iters;
    // projected Armijo search on psi = 1/2 ||Phi||^2 (Newton direction: slope -2 psi)
    const double psi0 = 0.5 * phi2;
    double mu = 1.0;
    bool ok = false;
    for (int k = 0; k <= MAX_HALVINGS; ++k) {
      launch_set_scalar(s, h->S, S_MU, mu);
      launch_trial_state(s, n2, N, h->u, h->alpha, h->nx, h->nx + n2, h->alpha_prev, h->S, h->nut,
                         h->nat);
      double p2t = 0;
      rc = coupled_residual(h, h->nut, h->nat, h->npu2, &p2t);
      if (rc == FRACTURE_ENONFINITE) { mu *= 0.5; continue; }
      if (rc) return rc;
      if (0.5 * p2t <= psi0 * (1.0 - 2.0 * ARMIJO_SIGMA * mu)) {
        HIPCHK(hipMemcpyAsync(h->u, h->nut, n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(h->alpha, h->nat, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(h->nFu, h->npu2, n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
        phi2 = p2t;
        ok = true;
        break;
      }
      mu *= 0.5;
    }
    if (!ok) {
      // restore the active set / residual of the accepted point for the caller
      rc = coupled_residual(h, h->u, h->alpha, h->nFu, &phi2);
      *nphi = std::sqrt(phi2);
      return rc;
    }
    // insufficient reduction: an accepted step that removes less than a
    // fraction 1 - newton_stall of ||Phi|| ends the phase (the iterate is
    // outside the region of fast Newton convergence); ORAM takes over
    if (h->p.newton_stall < 1.0 && std::sqrt(phi2) > h->p.newton_stall * *nphi &&
        std::sqrt(phi2) > h->p.final_tol) {
      *nphi = std::sqrt(phi2);
      return FRACTURE_OK;
    }
  }
  *nphi = std::sqrt(phi2);
  if (*nphi <= h->p.final_tol) *converged = true;
  return FRACTURE_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

int solve_step_impl(fracture* h, fracture_stats* s) {
  hipStream_t st = h->st;
  const int64_t N = h->N, n2 = h->n2;
  fracture_stats loc{};
  loc.phi_l2 = -1.0;
  HIPCHK(hipEventRecord(h->ev[0], st));
  // the coarsest inverse is formed anew from the state at the start of every
  // load step (NaN reference coefficients), so a step depends on (u, alpha,
  // alpha_prev, load) alone and a handle resumed from get_state/set_state
  // continues bit for bit
  {
    const Grid& gc = h->lv[h->nlev - 1].g;
    const size_t ne = (size_t)gc.nx * gc.ny * (gc.dim == 3 ? 6 * (size_t)gc.nz : 2);
    HIPCHK(hipMemsetAsync(h->dref, 0xFF, ne * sizeof(double), st));
  }
  HIPCHK(hipMemcpyAsync(h->u_entry, h->u, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->alpha_entry, h->alpha, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  int rc = FRACTURE_OK;
  double ms_pcg = 0, ms_vi = 0, ms_newton = 0;
  double threshold = h->p.switch_tol;
  double best_phi = INFINITY;   // smallest ||Phi||_2 of the step's sweeps so far
  int best_sweep = 0;           // the sweep that last cut it by STALL_CUT
  // omega: fixed, or (omega_auto) 1 until the convergence factor rho of the
  // plain alternate minimisation is measured, then Young's optimum
  // 2 / (1 + sqrt(1 - rho)) of SOR theory, capped at p.omega
  h->omega_cur = h->p.omega_auto ? 1.0 : h->p.omega;
  h->sweep_cap = INFINITY;
  h->r_valid = false;
  double da_hist[OMEGA_PROBE + 1] = {};
  for (int sweep = 1; sweep <= h->p.max_am; ++sweep) {
    update_coefficients(h);
    if (sweep == 1) {
      rc = load_norm(h, &h->bnorm);
      if (rc) break;
    }
    HIPCHK(hipEventRecord(h->ev[1], st));
    const int vi_before = loc.vi_iters;
    // elastic substep
    int it = 0;
    // tolerance: relative to the load vector; an absolute floor keeps zero loads finite
    const double tol = h->p.pcg_rtol * (h->bnorm > 0 ? h->bnorm : 1.0);
    rc = h->mixed ? pcg_mixed(h, tol, &it) : pcg(h, tol, &it);
    loc.pcg_iters += it;
    if (rc) { loc.stopped_in = FRACTURE_STAGE_PCG; break; }
    // at omega = 1 the PCG iterated on u itself
    if (h->omega_cur != 1.0) launch_relax_u(st, n2, h->u, h->x, h->omega_cur);
    HIPCHK(hipEventRecord(h->ev[2], st));
    // damage substep
    launch_w2_2d(st, load_grid(h), h->mat, h->u, h->w2);
    h->vi_stop = FRACTURE_STAGE_VI;
    rc = damage_qp(h, &loc.vi_iters, &loc.vi_cg_iters);
    if (rc) { loc.stopped_in = h->vi_stop; break; }
    rc = relax_alpha(h);
    if (rc) break;
    HIPCHK(hipEventRecord(h->ev[3], st));
    loc.sweeps = sweep;
    // the sweep's residual ||Phi||_2 (the stop and switch tests) is queued
    // before the one read of the sweep's scalars
    const bool want_phi = h->p.newton || h->p.am_stop != FRACTURE_STOP_DALPHA;
    if (want_phi) residual_launch(h);
    rc = read_scalars(h);
    if (rc) break;
    h->r_valid = want_phi;
    h->r_rr = h->hS[S_EU2];
    ms_pcg += elapsed(h->ev[1], h->ev[2]);
    ms_vi += elapsed(h->ev[2], h->ev[3]);
    loc.dalpha_inf = h->hS[S_DAMAX];
    if (!std::isfinite(loc.dalpha_inf)) { rc = FRACTURE_ENONFINITE; break; }
    if (h->p.omega_auto && h->omega_cur == 1.0) {
      // ||dalpha||_inf of the last OMEGA_PROBE + 1 sweeps at omega = 1
      const int q = (sweep - 1) % (OMEGA_PROBE + 1);
      da_hist[q] = loc.dalpha_inf;
      if (sweep % (OMEGA_PROBE + 1) == 0 && da_hist[0] > 0.0) {
        const double rho = std::pow(da_hist[OMEGA_PROBE] / da_hist[0], 1.0 / OMEGA_PROBE);
        if (rho > 0.0 && rho < 1.0)
          h->omega_cur = std::fmin(h->p.omega, 2.0 / (1.0 + std::sqrt(1.0 - rho)));
      }
    }
    if (h->monitor && (h->p.newton || h->p.am_stop != FRACTURE_STOP_PHI))
      h->monitor(h->monitor_user, sweep, loc.dalpha_inf, -1.0);
    if (!h->p.newton && h->p.am_stop == FRACTURE_STOP_DALPHA) {
      if (loc.dalpha_inf < h->p.am_tol) { loc.converged = 1; break; }
    } else {
      double nphi = residual_value(h);
      loc.phi_l2 = nphi;
      if (!std::isfinite(nphi)) { rc = FRACTURE_ENONFINITE; break; }
      if (h->monitor) h->monitor(h->monitor_user, sweep, loc.dalpha_inf, nphi);
      if (nphi <= h->p.final_tol) { loc.converged = 1; break; }
      // a sweep whose sub-solves all stopped at once (their tolerances are
      // looser than what is left of ||Phi||) changed nothing and every later
      // sweep would repeat it: the step's sweeps solve to a tenth of the
      // final tolerance from here on
      if (it == 0 && loc.vi_iters == vi_before && loc.dalpha_inf == 0.0)
        h->sweep_cap = 0.1 * h->p.final_tol;
      // the same when sweeps still move alpha, but only by a trace, and have
      // not cut ||Phi|| for STALL_SWEEPS sweeps: the sub-solves' errors (which
      // over-relaxation amplifies) hold ||Phi|| above the stop test
      if (nphi < STALL_CUT * best_phi) {
        best_phi = nphi;
        best_sweep = sweep;
      } else if (loc.dalpha_inf < STALL_DALPHA && sweep - best_sweep >= STALL_SWEEPS) {
        h->sweep_cap = 0.1 * h->p.final_tol;
      }
      if (h->p.newton && nphi < threshold) {
        h->r_valid = false;   // the Newton phase moves u and alpha
        HIPCHK(hipEventRecord(h->ev[1], st));
        bool conv = false;
        rc = newton_phase(h, &loc, &nphi, &conv);
        HIPCHK(hipEventRecord(h->ev[2], st));
        HIPCHK(hipEventSynchronize(h->ev[2]));
        ms_newton += elapsed(h->ev[1], h->ev[2]);
        if (rc) { loc.stopped_in = FRACTURE_STAGE_NEWTON; break; }
        loc.phi_l2 = nphi;
        if (conv) { loc.converged = 1; break; }
        ++loc.newton_failures;
        threshold = h->p.switch_rel * nphi;   // back to ORAM until Phi falls by switch_rel
      }
    }
  }
  if (rc == FRACTURE_OK && !loc.converged) {
    rc = FRACTURE_ENOTCONV;
    loc.stopped_in = FRACTURE_STAGE_SWEEPS;
  }
  if (rc != FRACTURE_OK && loc.stopped_in == FRACTURE_STAGE_NONE) loc.stopped_in = FRACTURE_STAGE_OTHER;
  if (rc == FRACTURE_OK) {
    HIPCHK(hipMemcpyAsync(h->alpha_prev, h->alpha, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else if (rc == FRACTURE_ENOTCONV || rc == FRACTURE_ENONFINITE) {
    (void)hipMemcpyAsync(h->u, h->u_entry, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(h->alpha, h->alpha_entry, N * sizeof(double), hipMemcpyDeviceToDevice, st);
    h->coef_valid = false;
  }
  (void)hipEventRecord(h->ev[4], st);
  (void)hipEventSynchronize(h->ev[4]);
  loc.ms_total = elapsed(h->ev[0], h->ev[4]);
  loc.ms_pcg = ms_pcg;
  loc.ms_vi = ms_vi;
  loc.ms_newton = ms_newton;
  if (s) *s = loc;
  return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of the no-allocation entry point (fracture_energy_noalloc)
// ---------------------------------------------------------------------------
//
// Callers that cannot allocate (graph capture, serving loops) get their
// reduction partials, scalars and (3D) element energies from this array
// instead of a handle's workspace.  Each device that loads the library holds
// its own copy until the process ends.  Host code never uses the symbol's
// name as an address: scratch_base() looks up the device address once per
// device with hipGetSymbolAddress and keeps it.

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;
constexpr size_t SCRATCH_S_BYTES = 1024;                          // S_COUNT doubles, padded
constexpr size_t SCRATCH_PART_BYTES = 2 * VGRID * sizeof(double);  // two partial-sum slots
static_assert(S_COUNT * sizeof(double) <= SCRATCH_S_BYTES, "scalar block");

size_t scratch_energy_bytes(const Grid& g) {
  size_t b = SCRATCH_S_BYTES + SCRATCH_PART_BYTES;
  if (g.dim == 3) b += (size_t)6 * g.nx * g.ny * g.nz * sizeof(double);   // W2 per tetrahedron
  return b;
}

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

// Device address of the current device's scratch (looked up once per device).
int scratch_base(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return FRACTURE_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FRACTURE_EDEVICE;
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return FRACTURE_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void fracture_default_params(fracture_params* p, int nx, int ny) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dim = 2;
  p->nx = nx;
  p->ny = ny;
  p->nz = 0;
  p->lx = 1.0;
  p->ly = 1.0;
  p->lz = 0.0;
  p->model = FRACTURE_AT1;
  p->plane_stress = 0;
  p->E = 1.0;
  p->nu = 0.3;
  p->Gc = 1.0;
  p->ell = 0.05;
  p->k_ell = 1e-6;
  p->load_kind = FRACTURE_LOAD_TENSION_2D;
  p->thermal_depth = 0.05;
  p->surf_ki = 1.0;
  p->surf_v = 1.0;
  p->surf_lc = 0.05;
  p->precision = FRACTURE_FP64;
  p->omega = 1.0;
  p->relax_mode = FRACTURE_RELAX_PROJECT;
  p->newton = 0;
  p->am_stop = FRACTURE_STOP_DALPHA;
  p->am_tol = 1e-5;
  p->switch_tol = 1e-3;
  p->switch_rel = 1e-1;
  p->final_tol = 1e-7;
  p->pcg_rtol = 1e-10;
  p->vi_tol = 1e-13;
  p->vi_cg_rtol = 1e-4;
  p->minres_rtol = 1e-6;
  p->max_am = 2000;
  p->max_pcg = 1000;
  p->max_vi = 200;
  p->max_vi_cg = 2000;
  p->max_newton = 10;
  p->max_minres = 500;
  p->cheb_degree = 2;
  p->coarse_max_dofs = 200;
  p->newton_vcycles = 1;
  p->newton_forcing = 0.1;
  p->use_graphs = 1;
  p->vcycle_tail = 1;
  p->newton_precond = 1;
  p->omega_auto = 0;
  p->newton_forcing_mode = 1;
  p->pcg_reduction = 0.01;
  p->newton_stall = 0.9;
  p->deflate = 0;
  p->deflate_theta = 0.5;
  p->deflate_min_nodes = 64;
  p->deflate_max_fragments = DFL_FMAX;
  p->vi_reduction = 0.0;
  p->elem3d_min_nodes = 1 << 18;
}

size_t fracture_workspace_bytes(const fracture_params* p) {
  if (validate(p) != FRACTURE_OK) return 0;
  return layout(p, nullptr, nullptr);
}

int fracture_sizes(const fracture_params* p, int64_t* nodes, int64_t* dofs) {
  if (!p || (p->dim != 2 && p->dim != 3) || p->nx < 1 || p->ny < 1) return FRACTURE_EINVAL;
  int64_t N = (int64_t)(p->nx + 1) * (p->ny + 1);
  if (p->dim == 3) N *= (p->nz + 1);
  if (nodes) *nodes = N;
  if (dofs) *dofs = N * p->dim;
  return FRACTURE_OK;
}

int fracture_create(const fracture_params* p, const uint8_t* notch_mask, void* d_workspace,
                    size_t ws_bytes, void* hip_stream, fracture_t* out) {
  if (!out) return FRACTURE_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  const size_t need = layout(p, nullptr, nullptr);
  if (need == 0) return FRACTURE_EINVAL;
  if (!d_workspace) return FRACTURE_EINVAL;
  if (((uintptr_t)d_workspace & 255) != 0) return FRACTURE_EINVAL;
  if (ws_bytes < need) return FRACTURE_ENOMEM;
  fracture* h = new (std::nothrow) fracture();
  if (!h) return FRACTURE_ENOMEM;
  h->p = *p;
  h->dim = p->dim;
  h->st = (hipStream_t)hip_stream;
  layout(p, h, d_workspace);
  h->mat = make_mat(p);
  h->load2d.kind = bc_kind2d(p->load_kind);
  h->load2d.ki2mu = p->surf_ki / (2.0 * h->mat.mu);
  h->load2d.kappa = (3.0 - p->nu) / (1.0 + p->nu);
  h->load2d.lc = p->surf_lc;
  h->load2d.v = p->surf_v;
  h->cw = p->model == FRACTURE_AT1 ? 8.0 / 3.0 : 2.0;
  h->gc_cw = p->Gc / h->cw;
  h->cL = 2.0 * p->Gc * p->ell / h->cw;
  h->cM = p->model == FRACTURE_AT2 ? 2.0 * p->Gc / (h->cw * p->ell) : 0.0;
  h->cm = p->model == FRACTURE_AT1 ? p->Gc / (h->cw * p->ell) : 0.0;
  // Chebyshev polynomial on [0.06 lmax, lmax]
  h->lam_max = p->dim == 3 ? chebyshev_bound3d(h->lv[0].g, h->mat) : chebyshev_bound2d(h->lv[0].g, h->mat);
  h->lam_min = 0.06 * h->lam_max;
  const double theta = 0.5 * (h->lam_max + h->lam_min), delta = 0.5 * (h->lam_max - h->lam_min);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  h->cheb_cd[0] = 0.0;
  h->cheb_cr[0] = 1.0 / theta;
  for (int s = 1; s < p->cheb_degree; ++s) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    h->cheb_cd[s] = rn * rho;
    h->cheb_cr[s] = 2.0 * rn / delta;
    rho = rn;
  }
  {
    const double th = 0.5 * (CHEB_C_LMAX + CHEB_C_LMIN), de = 0.5 * (CHEB_C_LMAX - CHEB_C_LMIN);
    const double sg = th / de;
    double rh = 1.0 / sg;
    h->chebC_cd[0] = 0.0;
    h->chebC_cr[0] = 1.0 / th;
    for (int k = 1; k < CHEB_C; ++k) {
      const double rn = 1.0 / (2.0 * sg - rh);
      h->chebC_cd[k] = rn * rh;
      h->chebC_cr[k] = 2.0 * rn / de;
      rh = rn;
    }
  }
  if (hipHostMalloc((void**)&h->hS, (S_COUNT + 2 * LAG_W) * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    delete h;
    return FRACTURE_EDEVICE;
  }
  for (int k = 0; k < 10; ++k) {
    const hipError_t e = k < 8 ? hipEventCreate(&h->ev[k])
                               : hipEventCreateWithFlags(&h->ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
      h->ev[k] = nullptr;
      fracture_destroy(h);
      return FRACTURE_EDEVICE;
    }
  }
  hipStream_t st = h->st;
  bool ok = true;
  ok &= hipMemsetAsync(h->S, 0, S_COUNT * sizeof(double), st) == hipSuccess;
  // NaN reference coefficients: the first coefficient update inverts
  {
    const Grid& gc = h->lv[h->nlev - 1].g;
    const size_t ne = (size_t)gc.nx * gc.ny * (gc.dim == 3 ? 6 * (size_t)gc.nz : 2);
    ok &= hipMemsetAsync(h->dref, 0xFF, ne * sizeof(double), st) == hipSuccess;
  }
  ok &= hipMemsetAsync(h->u, 0, h->n2 * sizeof(double), st) == hipSuccess;
  ok &= hipMemsetAsync(h->alpha, 0, h->N * sizeof(double), st) == hipSuccess;
  if (notch_mask) {
    // alpha = alpha_prev = 1 on notch nodes: staged through pinned memory
    double* tmp = nullptr;
    ok &= hipHostMalloc((void**)&tmp, h->N * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (ok) {
      for (int64_t k = 0; k < h->N; ++k) tmp[k] = notch_mask[k] ? 1.0 : 0.0;
      ok &= hipMemcpyAsync(h->alpha, tmp, h->N * sizeof(double), hipMemcpyHostToDevice, st) == hipSuccess;
      ok &= hipStreamSynchronize(st) == hipSuccess;
      (void)hipHostFree(tmp);
    }
  }
  ok &= hipMemcpyAsync(h->alpha_prev, h->alpha, h->N * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess;
  ok &= hipStreamSynchronize(st) == hipSuccess;
  if (!ok) {
    fracture_destroy(h);
    return FRACTURE_EDEVICE;
  }
  *out = h;
  return FRACTURE_OK;
}

int fracture_set_load(fracture_t h, double load) {
  if (!h || !std::isfinite(load)) return FRACTURE_EINVAL;
  h->load = load;
  launch_lift2d(h->st, h->lv[0].g, h->u, load, h->load2d);
  return hip_ok(hipGetLastError());
}

int fracture_solve_step(fracture_t h, fracture_stats* out) {
  if (!h) return FRACTURE_EINVAL;
  return solve_step_impl(h, out);
}

int fracture_solve_steps(fracture_t* hs, int n, fracture_stats* out, int* codes) {
  if (!hs || n < 0) return FRACTURE_EINVAL;
  // one host thread per handle: each drives its own stream, so the load
  // steps of different instances run on the device at the same time
  std::vector<int> rcs(n, FRACTURE_EINVAL);
  std::vector<std::thread> pool;
  pool.reserve(n);
  for (int k = 0; k < n; ++k) {
    if (!hs[k]) continue;
    pool.emplace_back([&, k]() { rcs[k] = solve_step_impl(hs[k], out ? out + k : nullptr); });
  }
  for (auto& t : pool) t.join();
  int worst = FRACTURE_OK;
  for (int k = 0; k < n; ++k) {
    if (codes) codes[k] = rcs[k];
    if (rcs[k] && !worst) worst = rcs[k];
  }
  return worst;
}

int fracture_set_monitor(fracture_t h, fracture_monitor_fn fn, void* user) {
  if (!h) return FRACTURE_EINVAL;
  h->monitor = fn;
  h->monitor_user = user;
  return FRACTURE_OK;
}

int fracture_energy(fracture_t h, double* elastic, double* surface) {
  if (!h) return FRACTURE_EINVAL;
  if (h->dim == 3) {
    launch_w2_3d(h->st, load_grid(h), h->mat, h->u, h->w2);
    launch_energy3d(h->st, h->lv[0].g, h->mat, h->p.k_ell, h->gc_cw, h->p.ell,
                    h->p.model == FRACTURE_AT2, h->w2, h->alpha, red(h, 10, S_EL), red(h, 11, S_SURF));
  } else {
    launch_energy2d(h->st, load_grid(h), h->mat, h->p.k_ell, h->gc_cw, h->p.ell,
                    h->p.model == FRACTURE_AT2, h->u, h->alpha, red(h, 10, S_EL), red(h, 11, S_SURF));
  }
  int rc = read_scalars(h);
  if (rc) return rc;
  if (elastic) *elastic = h->hS[S_EL];
  if (surface) *surface = h->hS[S_SURF];
  return FRACTURE_OK;
}

int fracture_energy_noalloc(const fracture_params* p, double load, const double* d_u,
                            const double* d_alpha, void* hip_stream, double* d_out) {
  if (!d_u || !d_alpha || !d_out || !std::isfinite(load)) return FRACTURE_EINVAL;
  int rc = validate(p);
  if (rc) return rc;
  // the fine grid and its element count decide the scratch it needs
  const int nz = p->dim == 3 ? p->nz : 0;
  const Grid g = with_load(make_grid(p, p->nx, p->ny, nz, p->lx / p->nx, p->ly / p->ny,
                                     p->dim == 3 ? p->lz / nz : 0.0),
                           *p, load);
  const size_t need = scratch_energy_bytes(g);
  if (need > SCRATCH_BYTES) return FRACTURE_ESCRATCH;
  char* base = nullptr;
  rc = scratch_base(&base);
  if (rc) return rc;
  double* S = (double*)base;
  double* part = (double*)(base + SCRATCH_S_BYTES);
  const Red rel{part, S, S_EL, P_STORE}, rsu{part + VGRID, S, S_SURF, P_STORE};
  const hipStream_t st = (hipStream_t)hip_stream;
  const Mat m = make_mat(p);
  const double gc_cw = p->Gc / (p->model == FRACTURE_AT1 ? 8.0 / 3.0 : 2.0);
  const int at2 = p->model == FRACTURE_AT2;
  if (p->dim == 3) {
    double* w2 = (double*)(base + SCRATCH_S_BYTES + SCRATCH_PART_BYTES);
    launch_w2_3d(st, g, m, d_u, w2);
    Grid gp = g;
    gp.eig_dT = 0.0;
    launch_energy3d(st, gp, m, p->k_ell, gc_cw, p->ell, at2, w2, d_alpha, rel, rsu);
  } else {
    launch_energy2d(st, g, m, p->k_ell, gc_cw, p->ell, at2, d_u, d_alpha, rel, rsu);
  }
  // S[S_EL], S[S_SURF] are adjacent: one device-to-device copy into the output
  HIPCHK(hipMemcpyAsync(d_out, S + S_EL, 2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  return hip_ok(hipGetLastError());
}

int fracture_get_state(fracture_t h, double* u, double* alpha, double* alpha_prev) {
  if (!h) return FRACTURE_EINVAL;
  if (u) HIPCHK(hipMemcpyAsync(u, h->u, h->n2 * sizeof(double), hipMemcpyDefault, h->st));
  if (alpha) HIPCHK(hipMemcpyAsync(alpha, h->alpha, h->N * sizeof(double), hipMemcpyDefault, h->st));
  if (alpha_prev)
    HIPCHK(hipMemcpyAsync(alpha_prev, h->alpha_prev, h->N * sizeof(double), hipMemcpyDefault, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return FRACTURE_OK;
}

int fracture_set_state(fracture_t h, const double* u, const double* alpha, const double* alpha_prev) {
  if (!h) return FRACTURE_EINVAL;
  if (u) HIPCHK(hipMemcpyAsync(h->u, u, h->n2 * sizeof(double), hipMemcpyDefault, h->st));
  if (alpha) HIPCHK(hipMemcpyAsync(h->alpha, alpha, h->N * sizeof(double), hipMemcpyDefault, h->st));
  if (alpha_prev)
    HIPCHK(hipMemcpyAsync(h->alpha_prev, alpha_prev, h->N * sizeof(double), hipMemcpyDefault, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  h->coef_valid = false;
  return FRACTURE_OK;
}

int fracture_update_coefficients(fracture_t h) {
  if (!h) return FRACTURE_EINVAL;
  update_coefficients(h);
  return hip_ok(hipStreamSynchronize(h->st));
}

int fracture_apply(fracture_t h, int op, int level, const double* d_x, double* d_y) {
  if (!h || !d_x || !d_y) return FRACTURE_EINVAL;
  const Grid& g = h->lv[0].g;
  Red none{};
  switch (op) {
    case FRACTURE_OP_ELASTICITY:
      launch_apply2d(h->st, g, h->mat, true, h->alpha, h->p.k_ell, d_x, d_y, nullptr, 0, 0, none);
      break;
    case FRACTURE_OP_LEVEL: {
      if (level < 0 || level >= h->nlev) return FRACTURE_EINVAL;
      if (!h->coef_valid) update_coefficients(h);
      launch_apply2d(h->st, h->lv[level].g, h->mat, level == 0, level_coef(h, level), h->p.k_ell,
                     d_x, d_y, nullptr, 1, 0, none);
    } break;
    case FRACTURE_OP_DAMAGE_HESS:
      launch_w2_2d(h->st, load_grid(h), h->mat, h->u, h->w2);
      launch_helm_apply2d(h->st, g, h->cL, h->cM, h->w2, d_x, nullptr, d_y, false, none);
      break;
    case FRACTURE_OP_COUPLING:
    case FRACTURE_OP_COUPLING_T: {
      // the full coupling block (no active set): mask cleared
      const Grid gl = load_grid(h);
      launch_w2_2d(h->st, gl, h->mat, h->u, h->w2);
      HIPCHK(hipMemsetAsync(h->mask, 0, h->N, h->st));
      if (op == FRACTURE_OP_COUPLING)
        launch_jac2d(h->st, gl, h->mat, h->p.k_ell, h->cL, h->cM, h->alpha, h->u, h->w2, h->mask,
                     nullptr, d_x, d_y, nullptr, false, none, none, nullptr);
      else
        launch_jac2d(h->st, gl, h->mat, h->p.k_ell, h->cL, h->cM, h->alpha, h->u, h->w2, h->mask,
                     d_x, nullptr, nullptr, d_y, false, none, none, nullptr);
    } break;
    case FRACTURE_OP_RESIDUAL:
      // the elastic PCG's residual kernel with a zero load: -K x on free rows
      launch_resid2d(h->st, g, h->mat, true, h->alpha, h->p.k_ell, d_x, d_y, nullptr, false, none);
      break;
    case FRACTURE_OP_PRECOND: {
      if (!h->coef_valid) update_coefficients(h);
      double* z = vcycle(h, 0, d_x);
      HIPCHK(hipMemcpyAsync(d_y, z, h->n2 * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    } break;
    default:
      return FRACTURE_EINVAL;
  }
  return hip_ok(hipStreamSynchronize(h->st));
}

int fracture_gradient(fracture_t h, double* d_Eu, double* d_Ea) {
  if (!h) return FRACTURE_EINVAL;
  const Grid g = load_grid(h);
  Red none{};
  if (d_Eu)
    launch_apply2d(h->st, g, h->mat, true, h->alpha, h->p.k_ell, h->u, d_Eu, nullptr, 0, 0, none);
  if (d_Ea) {
    launch_w2_2d(h->st, g, h->mat, h->u, h->w2);
    launch_vi_eval2d(h->st, g, h->cL, h->cM, h->cm, h->w2, h->alpha, nullptr, h->alpha_prev, h->S,
                     S_MU, 1e-12, h->F, h->phi, h->mask, h->hdinv, red(h, 5, S_PHI2),
                     red(h, 6, S_PHIMAX), red(h, 12, S_JLO), red(h, 13, S_JHI), false);
    HIPCHK(hipMemcpyAsync(d_Ea, h->F, h->N * sizeof(double), hipMemcpyDeviceToDevice, h->st));
  }
  return hip_ok(hipStreamSynchronize(h->st));
}

int fracture_fragments(fracture_t h, int* nfrag, int* d_fid) {
  if (!h || !nfrag || !d_fid || !h->p.deflate) return FRACTURE_EINVAL;
  const Grid& g = h->lv[0].g;
  launch_fragments2d(h->st, g, h->alpha, h->p.deflate_theta, h->p.deflate_min_nodes,
                     h->p.deflate_max_fragments, h->dfl_parent, h->dfl_label, d_fid, h->dfl_meta);
  HIPCHK(hipMemcpyAsync(nfrag, h->dfl_meta + DFL_META_NFRAG, sizeof(int), hipMemcpyDeviceToHost,
                        h->st));
  return hip_ok(hipStreamSynchronize(h->st));
}

int fracture_deflation_matrix(fracture_t h, int* m, double* E) {
  if (!h || !m || !E || !h->p.deflate) return FRACTURE_EINVAL;
  int rc = dfl_setup(h, m);
  if (rc) return rc;
  std::vector<double> full(DFL_M * DFL_M);
  HIPCHK(hipMemcpyAsync(full.data(), h->dfl_E, full.size() * sizeof(double), hipMemcpyDeviceToHost,
                        h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  for (int i = 0; i < *m; ++i)
    for (int j = 0; j < *m; ++j) E[i * *m + j] = full[i * DFL_M + j];
  return FRACTURE_OK;
}

int fracture_levels(fracture_t h, int* nlevels) {
  if (!h || !nlevels) return FRACTURE_EINVAL;
  *nlevels = h->nlev;
  return FRACTURE_OK;
}

int fracture_level_shape(fracture_t h, int level, int* nx, int* ny, int* nz) {
  if (!h || level < 0 || level >= h->nlev) return FRACTURE_EINVAL;
  if (nx) *nx = h->lv[level].g.nx;
  if (ny) *ny = h->lv[level].g.ny;
  if (nz) *nz = h->lv[level].g.nz;
  return FRACTURE_OK;
}

int fracture_time_kernel(fracture_t h, int kernel, int reps, double* avg_ms, double* bytes) {
  if (!h || reps < 1 || !avg_ms) return FRACTURE_EINVAL;
  const Level& L0 = h->lv[0];
  const Grid& g = L0.g;
  hipStream_t st = h->st;
  const double N = (double)h->N;
  const int64_t n2 = h->n2;
  // deterministic inputs: the current state
  HIPCHK(hipMemcpyAsync(L0.xa, h->u, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(L0.b, h->u, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemsetAsync(L0.d, 0, n2 * sizeof(double), st));
  launch_w2_2d(st, g, h->mat, h->u, h->w2);
  launch_vi_eval2d(st, g, h->cL, h->cM, h->cm, h->w2, h->alpha, nullptr, h->alpha_prev, h->S, S_MU,
                   1e-12, h->F, h->phi, h->mask, h->hdinv, red(h, 5, S_PHI2), red(h, 6, S_PHIMAX), red(h, 12, S_JLO),
                   red(h, 13, S_JHI), false);
  HIPCHK(hipMemsetAsync(h->vp, 0, h->N * sizeof(double), st));
  double b = 0;
  auto one = [&]() {
    switch (kernel) {
      case FRACTURE_KERNEL_APPLY:
        launch_apply2d(st, g, h->mat, true, h->alpha, h->p.k_ell, L0.xa, L0.xb, nullptr, 1, 0,
                       red(h, 2, S_PQ, P_STORE));
        break;
      case FRACTURE_KERNEL_COPY:
        launch_copy(st, n2, L0.xa, L0.xb);
        break;
      case FRACTURE_KERNEL_SMOOTH:
        if (g.dim == 3)
          launch_smooth3d<double>(st, g, h->mat, true, h->alpha, L0.dg, h->p.k_ell, L0.xa, L0.xb,
                                  L0.b, L0.d, L0.d, h->cheb_cd[1], h->cheb_cr[1]);
        else
          launch_smooth2d(st, g, h->mat, true, h->alpha, h->p.k_ell, L0.xa, L0.xb, L0.b, L0.d, L0.d,
                          h->cheb_cd[1], h->cheb_cr[1]);
        break;
      case FRACTURE_KERNEL_VI_EVAL:
        launch_vi_eval2d(st, g, h->cL, h->cM, h->cm, h->w2, h->alpha, nullptr, h->alpha_prev, h->S,
                         S_MU, 1e-12, h->F, h->phi, h->mask, h->hdinv, red(h, 5, S_PHI2),
                         red(h, 6, S_PHIMAX), red(h, 12, S_JLO), red(h, 13, S_JHI), false);
        break;
      case FRACTURE_KERNEL_HELM:
        launch_helm_apply2d(st, g, h->cL, h->cM, h->w2, h->vp, h->mask, h->vq, true,
                            red(h, 2, S_PQ, P_STORE));
        break;
      default:
        break;
    }
  };
  const double dv = 8.0 * h->dim;                 // one displacement vector, per node
  const double w2b = 8.0 * (h->dim == 3 ? 6 : 2);  // W2 per node (elements per node)
  switch (kernel) {
    case FRACTURE_KERNEL_APPLY: b = (2 * dv + 8.0) * N; break;
    case FRACTURE_KERNEL_SMOOTH: b = (5 * dv + 8.0 + (h->dim == 3 ? dv : 0.0)) * N; break;
    case FRACTURE_KERNEL_VI_EVAL: b = (8.0 + 8.0 + w2b + 8.0 + 8.0 + 1.0 + 8.0) * N; break;
    case FRACTURE_KERNEL_HELM: b = (8.0 + w2b + 1.0 + 8.0) * N; break;
    case FRACTURE_KERNEL_COPY: b = 2.0 * dv * N; break;
    default: return FRACTURE_EINVAL;
  }
  one();  // warm
  HIPCHK(hipEventRecord(h->ev[5], st));
  for (int k = 0; k < reps; ++k) one();
  HIPCHK(hipEventRecord(h->ev[6], st));
  HIPCHK(hipEventSynchronize(h->ev[6]));
  *avg_ms = elapsed(h->ev[5], h->ev[6]) / reps;
  if (bytes) *bytes = b;
  return FRACTURE_OK;
}

const char* fracture_strerror(int code) {
  switch (code) {
    case FRACTURE_OK: return "ok";
    case FRACTURE_EINVAL: return "invalid parameter or argument";
    case FRACTURE_ENOMEM: return "workspace too small";
    case FRACTURE_ENOTCONV: return "iteration limit reached (state rolled back)";
    case FRACTURE_ENONFINITE: return "non-finite value (state rolled back)";
    case FRACTURE_EDEVICE: return "HIP runtime error";
    case FRACTURE_ESCRATCH: return "problem larger than the static scratch of the no-allocation entry point";
    default: return "unknown error";
  }
}

static void kt_release(fracture* h) {
  if (h->kt_ev)
    for (int q = 0; q < 2 * h->kt_cap; ++q)
      if (h->kt_ev[q]) (void)hipEventDestroy(h->kt_ev[q]);
  delete[] h->kt_ev;
  h->kt_ev = nullptr;
  h->kt_cap = h->kt_used = h->kt_seen = 0;
  h->kt_bytes = 0.0;
}

int fracture_kernel_timing(fracture_t h, int kernel, int capacity) {
  if (!h || capacity < 0 || capacity > KT_MAX) return FRACTURE_EINVAL;
  if (capacity > 0 && kernel != FRACTURE_KERNEL_SMOOTH) return FRACTURE_EINVAL;
  if (h->st) HIPCHK(hipStreamSynchronize(h->st));
  kt_release(h);
  if (capacity == 0) return FRACTURE_OK;
  h->kt_ev = new (std::nothrow) hipEvent_t[2 * capacity]();
  if (!h->kt_ev) return FRACTURE_ENOMEM;
  h->kt_cap = capacity;
  for (int q = 0; q < 2 * capacity; ++q)
    if (hipEventCreate(&h->kt_ev[q]) != hipSuccess) {
      h->kt_ev[q] = nullptr;
      kt_release(h);
      return FRACTURE_EDEVICE;
    }
  return FRACTURE_OK;
}

int fracture_kernel_timing_read(fracture_t h, int* count, double* total_ms, double* total_bytes) {
  if (!h || !count || !total_ms || !total_bytes) return FRACTURE_EINVAL;
  double ms = 0.0;
  if (h->kt_used > 0) HIPCHK(hipEventSynchronize(h->kt_ev[2 * h->kt_used - 1]));
  for (int q = 0; q < h->kt_used; ++q) {
    float e = 0.0f;
    HIPCHK(hipEventElapsedTime(&e, h->kt_ev[2 * q], h->kt_ev[2 * q + 1]));
    ms += e;
  }
  *count = h->kt_used;
  *total_ms = ms;
  *total_bytes = h->kt_bytes;
  h->kt_used = 0;
  h->kt_bytes = 0.0;
  return FRACTURE_OK;
}

void fracture_destroy(fracture_t h) {
  if (!h) return;
  if (h->st) (void)hipStreamSynchronize(h->st);
  kt_release(h);
  for (Captured& c : h->graphs) (void)hipGraphExecDestroy(c.exec);
  h->graphs.clear();
  if (h->cap) (void)hipStreamDestroy(h->cap);
  for (int k = 0; k < 10; ++k)
    if (h->ev[k]) (void)hipEventDestroy(h->ev[k]);
  if (h->hS) (void)hipHostFree(h->hS);
  delete h;
}

}  // extern "C"
