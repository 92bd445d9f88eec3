// 2D kernels: P1 right-diagonal triangles on a structured grid.
//
// Cell (ci, cj) is split along its lower-left/upper-right diagonal into
//   T0 = [(ci,cj), (ci+1,cj), (ci+1,cj+1)]   and   T1 = [(ci,cj), (ci+1,cj+1), (ci,cj+1)].
// Element e = 2*(ci + nx*cj) + t.  Barycentric gradients (hx, hy the cell sides):
//   T0: (-1/hx, 0), (1/hx, -1/hy), (0, 1/hy);   T1: (0, -1/hy), (1/hx, 0), (-1/hx, 1/hy).
//
// The elasticity operator of eq. (elasticity) is applied matrix-free: one
// thread per node sums the forces of the six triangles around the node,
// f_v = abar_e |T| B_v^T D B_e u_e, reading neighbour data through the cache
// (no atomics, no assembled matrix).  abar_e, the exact element average of
// a(alpha) = (1-alpha)^2 + k_ell, is formed from nodal alpha on the finest
// level and read from a per-element array on coarser multigrid levels (the
// mean of the four children, which makes each coarse operator exactly the
// Galerkin product P^T K P of the finer one).
#include "common.h"
#include "launch.h"
#include "ops2d.h"

namespace frac {

// ---------------------------------------------------------------------------
// node kernels: apply / residual / Chebyshev step
// ---------------------------------------------------------------------------

// One thread per node (64 x NB_Y threads per tile, tiles in XCD-aware
// order): the short dependency chain suits the small, latency-bound
// multigrid levels.
template <int MODE, bool FA, bool HASX, int RED, class T, bool EIG = false>
__global__ __launch_bounds__(NB) void k_node2d(Grid g, Mat m, const T* __restrict__ coef, T kell,
                                               const T* __restrict__ x, T* __restrict__ y,
                                               const T* __restrict__ b, const T* __restrict__ din,
                                               T* __restrict__ dout, T cd, T cr, int mask, Red red) {
  const int nbx = gridDim.x, total = gridDim.x * gridDim.y;
  const int tt = xcd_tile(blockIdx.x + nbx * blockIdx.y, total);
  const int i = (tt % nbx) * NB_X + threadIdx.x;
  const int j = (tt / nbx) * NB_Y + threadIdx.y;
  double acc = 0.0;
  if (i <= g.nx && j <= g.ny) {
    const int N = g.N, n = i + (g.nx + 1) * j;
    T c[6];
    coef6<FA>(g, coef, kell, i, j, c);
    T fx, fy, dx, dy;
    node_force2d<HASX, MODE == M_SMOOTH, EIG>(g, m, c, x, x + N, i, j, fx, fy, dx, dy);
    const T xc = HASX ? x[n] : T(0), yc = HASX ? x[n + N] : T(0);
    node_out2d<MODE, RED>(g, i, j, fx, fy, dx, dy, xc, yc, y, b, din, dout, cd, cr, mask, acc);
  }
  if (RED != R_NONE) block_reduce<NB, false>(acc, red, total, tt, threadIdx.x + NB_X * threadIdx.y);
}

// Rows one thread of k_col2d walks: a column tile re-reads one grid row
// above and below it (x and alpha), so taller tiles read less, while
// shorter ones give more waves to hide latency with.  The Chebyshev step
// (seven streams) gains from 16 rows; apply and residual do best at 8.
constexpr int COL_NY = 8;
constexpr int COL_NY_SMOOTH = 16;
template <int MODE>
constexpr int col_rows() { return MODE == M_SMOOTH ? COL_NY_SMOOTH : COL_NY; }

// One wavefront per 64 x col_rows<MODE>() tile, thread i walking the tile's column
// (column2d): each element stress is formed once per thread and each row is
// loaded once, which pays on the large levels.  Tiles are taken in
// XCD-aware order (xcd_tile); there are no more of them than k_node2d's.
template <int MODE, bool FA, bool HASX, int RED, class T, bool EIG = false>
__global__ __launch_bounds__(NB_X) void k_col2d(Grid g, Mat m, const T* __restrict__ coef, T kell,
                                                const T* __restrict__ x, T* __restrict__ y,
                                                const T* __restrict__ b, const T* __restrict__ din,
                                                T* __restrict__ dout, T cd, T cr, int mask, Red red) {
  const int nbx = gridDim.x, total = gridDim.x * gridDim.y;
  const int t = xcd_tile(blockIdx.x + nbx * blockIdx.y, total);
  const int i = (t % nbx) * NB_X + threadIdx.x;
  const int j0 = (t / nbx) * col_rows<MODE>();
  double acc = 0.0;
  if (i <= g.nx) {
    column2d<col_rows<MODE>(), FA, HASX, MODE == M_SMOOTH, EIG>(
        g, m, coef, kell, x, i, j0, [&](int j, T fx, T fy, T dx, T dy, T xc, T yc) {
          node_out2d<MODE, RED>(g, i, j, fx, fy, dx, dy, xc, yc, y, b, din, dout, cd, cr, mask, acc);
        });
  }
  if (RED != R_NONE) block_reduce<NB_X, false>(acc, red, total, t, threadIdx.x);
}

// Levels with at least this many nodes use the column-blocked kernels.
constexpr int64_t COL_MIN_NODES = (int64_t)1 << 21;

static bool use_col2d(const Grid& g) { return (int64_t)(g.nx + 1) * (g.ny + 1) >= COL_MIN_NODES; }

static dim3 node_grid2(const Grid& g) {
  return dim3((g.nx + 1 + NB_X - 1) / NB_X, (g.ny + 1 + NB_Y - 1) / NB_Y);
}

// Grid of the operator kernels: column tiles of `rows` rows on large
// levels, else node tiles.
static dim3 op_grid2(const Grid& g, bool col, int rows) {
  if (!col) return node_grid2(g);
  static_assert(COL_NY % NB_Y == 0 && COL_NY_SMOOTH % NB_Y == 0,
                "column tiles cover whole node tiles");
  return dim3((g.nx + 1 + NB_X - 1) / NB_X, (g.ny + 1 + rows - 1) / rows);
}

int node_blocks2(const Grid& g) {
  dim3 gr = node_grid2(g);
  return (int)(gr.x * gr.y);
}

int node_blocks(const Grid& g) { return g.dim == 3 ? node_blocks3(g) : node_blocks2(g); }

// y = K x (mask: zero Dirichlet rows).  red (optional): R_DOT -> S[slot] = x.y,
// R_FREE2 -> S[slot] = sum over free rows of (K x - b)^2.
template <class T>
void launch_apply2d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* y, const ND<T>* b, int mask, int red, Red r) {
  if (g.dim == 3) return launch_apply3d<T>(st, g, m, fine, coef, kell, x, y, b, mask, red, r);
  const bool col = use_col2d(g);
  const dim3 gr = op_grid2(g, col, col_rows<M_APPLY>());
  const T k = T(kell);
  // the thermal-shock eigenstrain enters the operator of the actual problem
  // (finest level, load grid): y = K x - f
  const bool eig = fine && g.eig_dT != 0.0;
#define APPLY_CASE_E(FA, RD, EG)                                                                \
  do {                                                                                          \
  if (col)                                                                                      \
    hipLaunchKernelGGL((k_col2d<M_APPLY, FA, true, RD, T, EG>), gr, dim3(NB_X), 0, st, g, m, coef, \
                       k, x, y, b, (const T*)nullptr, (T*)nullptr, T(0), T(0), mask, r);       \
  else                                                                                          \
    hipLaunchKernelGGL((k_node2d<M_APPLY, FA, true, RD, T, EG>), gr, dim3(NB_X, NB_Y), 0, st, g, \
                       m, coef, k, x, y, b, (const T*)nullptr, (T*)nullptr, T(0), T(0), mask, r); \
  } while (0)
#define APPLY_CASE(FA, RD) APPLY_CASE_E(FA, RD, false)
  if (fine && eig) {
    if (red == R_NONE) APPLY_CASE_E(true, R_NONE, true);
    else if (red == R_DOT) APPLY_CASE_E(true, R_DOT, true);
    else APPLY_CASE_E(true, R_FREE2, true);
  } else if (fine) {
    if (red == R_NONE) APPLY_CASE(true, R_NONE);
    else if (red == R_DOT) APPLY_CASE(true, R_DOT);
    else APPLY_CASE(true, R_FREE2);
  } else {
    if (red == R_NONE) APPLY_CASE(false, R_NONE);
    else if (red == R_DOT) APPLY_CASE(false, R_DOT);
    else APPLY_CASE(false, R_FREE2);
  }
#undef APPLY_CASE
#undef APPLY_CASE_E
  if (red != R_NONE) launch_finish(st, r, (int)(gr.x * gr.y), false);
}

// r = b - K x on free rows, 0 on Dirichlet rows; optional ||r||^2 into S[slot].
template <class T>
void launch_resid2d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* r, const ND<T>* b, bool red, Red rr) {
  if (g.dim == 3) return launch_resid3d<T>(st, g, m, fine, coef, kell, x, r, b, red, rr);
  const bool col = use_col2d(g);
  const dim3 gr = op_grid2(g, col, col_rows<M_RESID>());
  const T k = T(kell);
  const bool eig = fine && g.eig_dT != 0.0;   // r = b - (K x - f) with the eigenstrain load
#define RES_CASE_E(FA, RD, EG)                                                                  \
  do {                                                                                          \
  if (col)                                                                                      \
    hipLaunchKernelGGL((k_col2d<M_RESID, FA, true, RD, T, EG>), gr, dim3(NB_X), 0, st, g, m, coef, \
                       k, x, r, b, (const T*)nullptr, (T*)nullptr, T(0), T(0), 1, rr);         \
  else                                                                                          \
    hipLaunchKernelGGL((k_node2d<M_RESID, FA, true, RD, T, EG>), gr, dim3(NB_X, NB_Y), 0, st, g, \
                       m, coef, k, x, r, b, (const T*)nullptr, (T*)nullptr, T(0), T(0), 1, rr); \
  } while (0)
#define RES_CASE(FA, RD) RES_CASE_E(FA, RD, false)
  if (fine && eig) {
    if (red) RES_CASE_E(true, R_DOT, true); else RES_CASE_E(true, R_NONE, true);
  } else if (fine) {
    if (red) RES_CASE(true, R_DOT); else RES_CASE(true, R_NONE);
  } else {
    if (red) RES_CASE(false, R_DOT); else RES_CASE(false, R_NONE);
  }
#undef RES_CASE
#undef RES_CASE_E
  if (red) launch_finish(st, rr, (int)(gr.x * gr.y), false);
}

// One Jacobi-preconditioned Chebyshev step:
//   d_new = cd * d_in + cr * D^{-1} (b - K x_in);  x_out = x_in + d_new
// x_in == nullptr means x_in = 0; d_in may be nullptr (0); d_out optional.
template <class T>
void launch_smooth2d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                     double kell, const ND<T>* x_in, T* x_out, const T* b, const ND<T>* d_in, ND<T>* d_out,
                     double cd, double cr) {
  // (3D levels: launch_smooth3d, with the level's stored diagonal)
  const bool col = use_col2d(g);
  const dim3 gr = op_grid2(g, col, col_rows<M_SMOOTH>());
  Red none{};
  const T k = T(kell);
#define SM_CASE(FA, HX)                                                                          \
  do {                                                                                          \
  if (col)                                                                                       \
    hipLaunchKernelGGL((k_col2d<M_SMOOTH, FA, HX, R_NONE, T>), gr, dim3(NB_X), 0, st, g, m, coef, \
                       k, x_in, x_out, b, d_in, d_out, T(cd), T(cr), 1, none);                  \
  else                                                                                           \
    hipLaunchKernelGGL((k_node2d<M_SMOOTH, FA, HX, R_NONE, T>), gr, dim3(NB_X, NB_Y), 0, st, g, m, \
                       coef, k, x_in, x_out, b, d_in, d_out, T(cd), T(cr), 1, none); \
  } while (0)
  if (fine) {
    if (x_in) SM_CASE(true, true); else SM_CASE(true, false);
  } else {
    if (x_in) SM_CASE(false, true); else SM_CASE(false, false);
  }
#undef SM_CASE
}

// ---------------------------------------------------------------------------
// multigrid transfers
// ---------------------------------------------------------------------------

// Coarse element coefficients: the mean of the four fine children.
//   coarse T0 of cell (I,J) = fine {(2I,2J) T0, (2I+1,2J) T0, (2I+1,2J) T1, (2I+1,2J+1) T0}
//   coarse T1 of cell (I,J) = fine {(2I,2J) T1, (2I,2J+1) T1, (2I,2J+1) T0, (2I+1,2J+1) T1}
// Always formed in float64 from the float64 fine data, then stored as T.
template <bool FA, class T>
__global__ __launch_bounds__(VB) void k_coarsen2d(Grid gf, const double* __restrict__ fine_a,
                                                  const T* __restrict__ fine_c, double kell,
                                                  Grid gc, double* __restrict__ coarse64,
                                                  T* __restrict__ coarse) {
  const int cell = blockIdx.x * VB + threadIdx.x;
  if (cell >= gc.nx * gc.ny) return;
  const int I = cell % gc.nx, J = cell / gc.nx;
  const int fi = 2 * I, fj = 2 * J;
  auto fc = [&](int ci, int cj, int t) -> double {
    if (FA) {
      const int W = gf.nx + 1, n = ci + W * cj;
      const double a00 = fine_a[n], a10 = fine_a[n + 1], a11 = fine_a[n + 1 + W], a01 = fine_a[n + W];
      return t == 0 ? abar3(a00, a10, a11, kell) : abar3(a00, a11, a01, kell);
    } else {
      return fine_a[2 * (ci + gf.nx * cj) + t];
    }
  };
  const double c0 = 0.25 * (fc(fi, fj, 0) + fc(fi + 1, fj, 0) + fc(fi + 1, fj, 1) + fc(fi + 1, fj + 1, 0));
  const double c1 = 0.25 * (fc(fi, fj, 1) + fc(fi, fj + 1, 1) + fc(fi, fj + 1, 0) + fc(fi + 1, fj + 1, 1));
  if (coarse64) { coarse64[2 * cell] = c0; coarse64[2 * cell + 1] = c1; }
  if (coarse) { coarse[2 * cell] = T(c0); coarse[2 * cell + 1] = T(c1); }
}

// Coarse coefficients from the finer level (alpha when fine_is_alpha); the
// float64 array coarse64 is always written, coarse32 (float copy) when given.
void launch_coarsen2d(hipStream_t st, const Grid& gf, bool fine_is_alpha, const double* fine,
                      double kell, const Grid& gc, double* coarse64, float* coarse32) {
  if (gc.dim == 3) return launch_coarsen3d(st, gf, fine_is_alpha, fine, kell, gc, coarse64, coarse32);
  const int n = gc.nx * gc.ny;
  dim3 gr((n + VB - 1) / VB), bl(VB);
  if (fine_is_alpha)
    hipLaunchKernelGGL((k_coarsen2d<true, float>), gr, bl, 0, st, gf, fine, (const float*)nullptr,
                       kell, gc, coarse64, coarse32);
  else
    hipLaunchKernelGGL((k_coarsen2d<false, float>), gr, bl, 0, st, gf, fine, (const float*)nullptr,
                       kell, gc, coarse64, coarse32);
}

// b_c = P^T r_f.  P interpolates linearly: fine node (2I,2J) takes coarse
// (I,J); a fine node at the midpoint of a coarse edge takes the mean of its
// two ends (edges along x, along y and along the cell diagonal).
template <class T>
__global__ __launch_bounds__(NB) void k_restrict2d(Grid gf, Grid gc, const T* __restrict__ rf,
                                                   T* __restrict__ bc) {
  const int I = blockIdx.x * NB_X + threadIdx.x;
  const int J = blockIdx.y * NB_Y + threadIdx.y;
  if (I > gc.nx || J > gc.ny) return;
  restrict_node2d(gf, gc, rf, bc, I, J);
}

template <class T>
void launch_restrict2d(hipStream_t st, const Grid& gf, const Grid& gc, const T* rf, T* bc) {
  if (gc.dim == 3) return launch_restrict3d<T>(st, gf, gc, rf, bc);
  dim3 gr(node_grid2(gc)), bl(NB_X, NB_Y);
  hipLaunchKernelGGL((k_restrict2d<T>), gr, bl, 0, st, gf, gc, rf, bc);
}

// b_c = P^T r_f and, from x = 0, the first Jacobi-Chebyshev step on the
// coarse level, x_c = cr D^{-1} b_c (d_c = x_c when dout): from zero the step
// reads no neighbour of x, so restriction and step are one pass over the
// coarse nodes.  Same arithmetic as k_restrict2d followed by k_node2d<SMOOTH>
// without x.
template <class T>
__global__ __launch_bounds__(NB) void k_restrict_smooth2d(Grid gf, Grid gc, Mat m,
                                                          const T* __restrict__ coef, T kell,
                                                          const T* __restrict__ rf,
                                                          T* __restrict__ bc, T* __restrict__ xout,
                                                          T* __restrict__ dout, T cr) {
  const int I = blockIdx.x * NB_X + threadIdx.x;
  const int J = blockIdx.y * NB_Y + threadIdx.y;
  if (I > gc.nx || J > gc.ny) return;
  restrict_node2d(gf, gc, rf, bc, I, J);
  T c[6];
  coef6<false>(gc, coef, kell, I, J, c);
  T fx, fy, dx, dy;
  node_force2d<false, true>(gc, m, c, (const T*)nullptr, (const T*)nullptr, I, J, fx, fy, dx, dy);
  double acc = 0.0;
  node_out2d<M_SMOOTH, R_NONE>(gc, I, J, fx, fy, dx, dy, T(0), T(0), xout, bc, (const T*)nullptr,
                               dout, T(0), cr, 1, acc);
}

template <class T>
void launch_restrict_smooth2d(hipStream_t st, const Grid& gf, const Grid& gc, const Mat& m,
                              const T* coef, double kell, const T* rf, T* bc, T* xout, T* dout,
                              double cr) {
  dim3 gr(node_grid2(gc)), bl(NB_X, NB_Y);
  hipLaunchKernelGGL((k_restrict_smooth2d<T>), gr, bl, 0, st, gf, gc, m, coef, T(kell), rf, bc,
                     xout, dout, T(cr));
}

// The prolongation x += P x_c folded into the first post-smoothing step,
// which starts from it: x_out = x + P x_c + cr D^{-1} (b - K (x + P x_c)),
// d_out = that step.  Same arithmetic as the prolongation (prolong_node2d)
// followed by the smoothing kernel of the level (k_node2d or k_col2d
// <SMOOTH>, with x and no d_in); x + P x_c itself is not stored.  FA:
// coefficients from alpha (finest level) or element averages.
template <bool FA, class T>
__global__ __launch_bounds__(NB) void k_prol_smooth2d(Grid g, Grid gc, Mat m,
                                                      const T* __restrict__ coef, T kell,
                                                      const T* __restrict__ x,
                                                      const T* __restrict__ xc,
                                                      T* __restrict__ y, const T* __restrict__ b,
                                                      T* __restrict__ dout, T cr) {
  constexpr int PH = NB_Y / 2 + 2;
  static_assert(NB_Y % 2 == 0 && NB_X % 2 == 0, "tiles start on even rows and columns");
  __shared__ T sx[PH * PROL_PW], sy[PH * PROL_PW];
  const int nbx = gridDim.x, total = gridDim.x * gridDim.y;
  const int tt = xcd_tile(blockIdx.x + nbx * blockIdx.y, total);
  const int i0 = (tt % nbx) * NB_X, j0 = (tt / nbx) * NB_Y;
  const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
  // the coarse nodes of fine columns i0 - 1 .. i0 + NB_X, rows j0 - 1 .. j0 + NB_Y
  const int cc0 = (i0 >> 1) - 1, cr0 = (j0 >> 1) - 1, Wc = gc.nx + 1;
  for (int q = threadIdx.x + NB_X * threadIdx.y; q < PH * PROL_PW; q += NB) {
    const int cy = cr0 + q / PROL_PW, cx = cc0 + q % PROL_PW;
    const bool ok = cy >= 0 && cy <= gc.ny && cx >= 0 && cx <= gc.nx;
    sx[q] = ok ? xc[cx + Wc * cy] : T(0);
    sy[q] = ok ? xc[gc.N + cx + Wc * cy] : T(0);
  }
  __syncthreads();
  if (i > g.nx || j > g.ny) return;
  const int N = g.N, n = i + (g.nx + 1) * j;
  const AddProl<T> pr{sx, sy, cc0, cr0};
  T c[6];
  coef6<FA>(g, coef, kell, i, j, c);
  T fx, fy, dx, dy;
  node_force2d<true, true, false, true>(g, m, c, x, x + N, i, j, fx, fy, dx, dy, &pr);
  T xn = x[n], yn = x[n + N];
  add_prol(g, pr, i, j, xn, yn);
  double acc = 0.0;
  node_out2d<M_SMOOTH, R_NONE>(g, i, j, fx, fy, dx, dy, xn, yn, y, b, (const T*)nullptr, dout,
                               T(0), cr, 1, acc);
}

// Column-tiled form: the coarse nodes the tile's rows j0 - 1 .. j0 + ROWS
// and columns i0 - 1 .. i0 + NB_X touch are staged in LDS first (coarse
// columns (i0 - 1) >> 1 .. (i0 + NB_X) >> 1, rows (j0 - 1) >> 1 ..
// (j0 + ROWS) >> 1 + 1, zero outside the coarse grid).
template <bool FA, class T>
__global__ __launch_bounds__(NB_X) void k_col_prol_smooth2d(Grid g, Grid gc, Mat m,
                                                            const T* __restrict__ coef, T kell,
                                                            const T* __restrict__ x,
                                                            const T* __restrict__ xc,
                                                            T* __restrict__ y,
                                                            const T* __restrict__ b,
                                                            T* __restrict__ dout, T cr) {
  constexpr int ROWS = col_rows<M_SMOOTH>();
  constexpr int PH = ROWS / 2 + 2;
  static_assert(ROWS % 2 == 0 && NB_X % 2 == 0, "tiles start on even rows and columns");
  __shared__ T sx[PH * PROL_PW], sy[PH * PROL_PW];
  const int nbx = gridDim.x, total = gridDim.x * gridDim.y;
  const int t = xcd_tile(blockIdx.x + nbx * blockIdx.y, total);
  const int i0 = (t % nbx) * NB_X, i = i0 + threadIdx.x;
  const int j0 = (t / nbx) * ROWS;
  const int cc0 = (i0 >> 1) - 1, cr0 = (j0 >> 1) - 1, Wc = gc.nx + 1;
  for (int q = threadIdx.x; q < PH * PROL_PW; q += NB_X) {
    const int cy = cr0 + q / PROL_PW, cx = cc0 + q % PROL_PW;
    const bool ok = cy >= 0 && cy <= gc.ny && cx >= 0 && cx <= gc.nx;
    sx[q] = ok ? xc[cx + Wc * cy] : T(0);
    sy[q] = ok ? xc[gc.N + cx + Wc * cy] : T(0);
  }
  __syncthreads();
  if (i > g.nx) return;
  double acc = 0.0;
  column2d<ROWS, FA, true, true, false>(
      g, m, coef, kell, x, i, j0,
      [&](int j, T fx, T fy, T dx, T dy, T xn, T yn) {
        node_out2d<M_SMOOTH, R_NONE>(g, i, j, fx, fy, dx, dy, xn, yn, y, b, (const T*)nullptr,
                                     dout, T(0), cr, 1, acc);
      },
      AddProl<T>{sx, sy, cc0, cr0});
}

template <class T>
void launch_prol_smooth2d(hipStream_t st, const Grid& g, const Grid& gc, const Mat& m, bool fine,
                          const T* coef, double kell, const T* x, const T* xc, T* y, const T* b,
                          T* dout, double cr) {
  const T k = T(kell), c = T(cr);
  if (use_col2d(g)) {
    const dim3 gr = op_grid2(g, true, col_rows<M_SMOOTH>());
    if (fine)
      hipLaunchKernelGGL((k_col_prol_smooth2d<true, T>), gr, dim3(NB_X), 0, st, g, gc, m, coef, k,
                         x, xc, y, b, dout, c);
    else
      hipLaunchKernelGGL((k_col_prol_smooth2d<false, T>), gr, dim3(NB_X), 0, st, g, gc, m, coef, k,
                         x, xc, y, b, dout, c);
  } else if (fine) {
    hipLaunchKernelGGL((k_prol_smooth2d<true, T>), node_grid2(g), dim3(NB_X, NB_Y), 0, st, g, gc, m,
                       coef, k, x, xc, y, b, dout, c);
  } else {
    hipLaunchKernelGGL((k_prol_smooth2d<false, T>), node_grid2(g), dim3(NB_X, NB_Y), 0, st, g, gc,
                       m, coef, k, x, xc, y, b, dout, c);
  }
}

#define INST(T)                                                                                  \
  template void launch_apply2d<T>(hipStream_t, const Grid&, const Mat&, bool, const T*, double,   \
                                  const T*, T*, const ND<T>*, int, int, Red);                         \
  template void launch_resid2d<T>(hipStream_t, const Grid&, const Mat&, bool, const T*, double,   \
                                  const T*, T*, const ND<T>*, bool, Red);                             \
  template void launch_smooth2d<T>(hipStream_t, const Grid&, const Mat&, bool, const T*, double,  \
                                   const ND<T>*, T*, const T*, const ND<T>*, ND<T>*, double, double);        \
  template void launch_restrict2d<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);        \
  template void launch_restrict_smooth2d<T>(hipStream_t, const Grid&, const Grid&, const Mat&,     \
                                            const T*, double, const T*, T*, T*, T*, double);       \
  template void launch_prol_smooth2d<T>(hipStream_t, const Grid&, const Grid&, const Mat&, bool,   \
                                        const T*, double, const T*, const T*, T*, const T*, T*,   \
                                        double);
INST(float)
INST(double)
#undef INST

// ---------------------------------------------------------------------------
// Dirichlet lifting (tension): u_y = 0 at j = 0, u_y = t at j = ny, u_x(0,0) = 0
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(VB) void k_lift2d(Grid g, double* __restrict__ u, double t) {
  const int i = blockIdx.x * VB + threadIdx.x;
  if (i > g.nx) return;
  const int W = g.nx + 1;
  u[g.N + i] = 0.0;
  u[g.N + i + W * g.ny] = t;
  if (i == 0) u[0] = 0.0;
}

// Surfing (Sec. 4.1, eq. (surfingloading)): every boundary node takes the
// asymptotic Mode-I displacement about the tip (lc + v t, ly/2); on the crack
// line behind the tip the two faces' values average to zero.  The height
// above the mid line is formed from the integer row index, exactly zero on it.
__global__ __launch_bounds__(VB) void k_lift_surf2d(Grid g, Load2D ld, double* __restrict__ u,
                                                    double t) {
  const int n = blockIdx.x * VB + threadIdx.x;
  if (n >= g.N) return;
  const int W = g.nx + 1, i = n % W, j = n / W;
  if (!(i == 0 || i == g.nx || j == 0 || j == g.ny)) return;
  const double X = i * g.hx - ld.lc - ld.v * t;
  const double Y = (2.0 * j - g.ny) * (0.5 * g.hy);
  double ux = 0.0, uy = 0.0;
  if (!(Y == 0.0 && X < 0.0)) {
    const double r = hypot(X, Y), th = atan2(Y, X);
    const double f = ld.ki2mu * sqrt(r / (2.0 * M_PI)) * (ld.kappa - cos(th));
    ux = f * cos(0.5 * th);
    uy = f * sin(0.5 * th);
  }
  u[n] = ux;
  u[g.N + n] = uy;
}

// Thermal shock: the lateral u_x and the top u_y are held at zero.
__global__ __launch_bounds__(VB) void k_lift_tshock2d(Grid g, double* __restrict__ u) {
  const int n = blockIdx.x * VB + threadIdx.x;
  if (n >= g.N) return;
  const int W = g.nx + 1, i = n % W, j = n / W;
  if (fixed_x2(g, i, j)) u[n] = 0.0;
  if (fixed_y2(g, i, j)) u[g.N + n] = 0.0;
}

void launch_lift2d(hipStream_t st, const Grid& g, double* u, double t, const Load2D& ld) {
  if (g.dim == 3) return launch_lift3d(st, g, u);
  if (ld.kind == BC_TSHOCK_2D) {
    hipLaunchKernelGGL(k_lift_tshock2d, dim3((g.N + VB - 1) / VB), dim3(VB), 0, st, g, u);
    return;
  }
  if (ld.kind == BC_SURFING_2D) {
    hipLaunchKernelGGL(k_lift_surf2d, dim3((g.N + VB - 1) / VB), dim3(VB), 0, st, g, ld, u, t);
    return;
  }
  hipLaunchKernelGGL(k_lift2d, dim3((g.nx + 1 + VB - 1) / VB), dim3(VB), 0, st, g, u, t);
}

// ---------------------------------------------------------------------------
// damage subproblem: W2 per element, Helmholtz operator, VI residual
// ---------------------------------------------------------------------------

// W2_e = A0 eps_e : eps_e for both triangles of every cell, eps_e the
// effective strain eps(u) - eps0 when the grid carries the thermal-shock
// eigenstrain.
__global__ __launch_bounds__(VB) void k_w2_2d(Grid g, Mat m, const double* __restrict__ u,
                                              double* __restrict__ w2) {
  const int cell = blockIdx.x * VB + threadIdx.x;
  if (cell >= g.nx * g.ny) return;
  const int ci = cell % g.nx, cj = cell / g.nx, W = g.nx + 1;
  const int n00 = ci + W * cj, n10 = n00 + 1, n11 = n00 + 1 + W, n01 = n00 + W;
  const double* ux = u;
  const double* uy = u + g.N;
  const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy;
  double s0 = 0.0, s1 = 0.0;
  if (g.eig_dT != 0.0) eig_row2d(g, cj, s0, s1);
  {
    const double exx = (ux[n10] - ux[n00]) * ihx - s0, eyy = (uy[n11] - uy[n10]) * ihy - s0;
    const double gam = (uy[n10] - uy[n00]) * ihx + (ux[n11] - ux[n10]) * ihy;
    w2[2 * cell] = m.l2m * (exx * exx + eyy * eyy) + 2.0 * m.lam * exx * eyy + m.mu * gam * gam;
  }
  {
    const double exx = (ux[n11] - ux[n01]) * ihx - s1, eyy = (uy[n01] - uy[n00]) * ihy - s1;
    const double gam = (uy[n11] - uy[n01]) * ihx + (ux[n01] - ux[n00]) * ihy;
    w2[2 * cell + 1] = m.l2m * (exx * exx + eyy * eyy) + 2.0 * m.lam * exx * eyy + m.mu * gam * gam;
  }
}

void launch_w2_2d(hipStream_t st, const Grid& g, const Mat& m, const double* u, double* w2) {
  if (g.dim == 3) return launch_w2_3d(st, g, m, u, w2);
  const int n = g.nx * g.ny;
  hipLaunchKernelGGL(k_w2_2d, dim3((n + VB - 1) / VB), dim3(VB), 0, st, g, m, u, w2);
}

// Helmholtz data: H = M_W + cL L + cM M, g = M_W 1 - cm m (eq. (helmholtz),
// quadratic damage energy).  M_W = sum_e W2_e M_e with the consistent mass.
struct Helm {
  double cL, cM, cm;      // cL = 2 Gc ell / c_w; cM = 2 Gc/(c_w ell) (AT2) or 0; cm = Gc/(c_w ell) (AT1) or 0
};

// Gradients of the three vertices of an element type, scaled by (1/hx, 1/hy).
__device__ __forceinline__ void tri_grads(int t, double ihx, double ihy, double gx[3], double gy[3]) {
  if (t == 0) {
    gx[0] = -ihx; gy[0] = 0.0; gx[1] = ihx; gy[1] = -ihy; gx[2] = 0.0; gy[2] = ihy;
  } else {
    gx[0] = 0.0; gy[0] = -ihy; gx[1] = ihx; gy[1] = 0.0; gx[2] = -ihx; gy[2] = ihy;
  }
}

// The six triangles around node (i,j): cell offsets, type and the node's local vertex.
__device__ __constant__ int c_tri_di[6] = {0, 0, -1, -1, -1, 0};
__device__ __constant__ int c_tri_dj[6] = {0, 0, 0, -1, -1, -1};
__device__ __constant__ int c_tri_t[6] = {0, 1, 0, 0, 1, 1};
__device__ __constant__ int c_tri_v[6] = {0, 0, 1, 2, 1, 2};

// Node offsets (di, dj) of the local vertices of a triangle type, from the cell corner.
__device__ __forceinline__ void tri_nodes(int t, int di[3], int dj[3]) {
  di[0] = 0; dj[0] = 0;
  if (t == 0) { di[1] = 1; dj[1] = 0; di[2] = 1; dj[2] = 1; }
  else { di[1] = 1; dj[1] = 1; di[2] = 0; dj[2] = 1; }
}

// Triangle K (0..5) around a node, in the order of c_tri_*: cell offset
// (di, dj), type t, the node's local vertex v, and the node offset of local
// vertex Q from the node — all compile-time constants.
template <int K>
struct Tri2 {
  static constexpr int di = (K == 2 || K == 3 || K == 4) ? -1 : 0;
  static constexpr int dj = K >= 3 ? -1 : 0;
  static constexpr int t = (K == 1 || K == 4 || K == 5) ? 1 : 0;
  static constexpr int v = K <= 1 ? 0 : ((K == 2 || K == 4) ? 1 : 2);
  template <int Q>
  static constexpr int slot() {   // (dx + 1) + 3 (dy + 1) in the node's 3x3 neighbourhood
    return (di + (Q == 0 ? 0 : (t == 0 ? 1 : (Q == 1 ? 1 : 0))) + 1) +
           3 * (dj + (Q == 0 ? 0 : (t == 0 ? (Q == 1 ? 0 : 1) : 1)) + 1);
  }
};

// Triangle K's part of (H a)_v, g_v and H_vv; av holds the field on the
// node's 3x3 neighbourhood.
template <int K>
__device__ __forceinline__ void tri_helm2(const Grid& g, const Helm& hp,
                                          const double* __restrict__ w2, const double (&av)[9],
                                          int i, int j, double ihx, double ihy, double area,
                                          double& Ha, double& gv, double& Hd) {
  using TK = Tri2<K>;
  const int ci = i + TK::di, cj = j + TK::dj;
  if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) return;
  double gx[3], gy[3];
  tri_grads(TK::t, ihx, ihy, gx, gy);
  const double a0 = av[TK::template slot<0>()], a1 = av[TK::template slot<1>()];
  const double a2 = av[TK::template slot<2>()];
  const double we = w2[2 * (ci + g.nx * cj) + TK::t];
  const double sum = a0 + a1 + a2;
  const double aV = TK::v == 0 ? a0 : (TK::v == 1 ? a1 : a2);
  const double mass = area / 12.0 * (aV + sum);                 // (M_e a)_v
  const double grx = a0 * gx[0] + a1 * gx[1] + a2 * gx[2];
  const double gry = a0 * gy[0] + a1 * gy[1] + a2 * gy[2];
  const double lap = area * (gx[TK::v] * grx + gy[TK::v] * gry);  // (L_e a)_v
  Ha += (we + hp.cM) * mass + hp.cL * lap;
  // (constant factors grouped: the divisions are loop-invariant, one per thread)
  gv += (we - hp.cm) * (area / 3.0);
  Hd += (we + hp.cM) * (area / 6.0) + hp.cL * area * (gx[TK::v] * gx[TK::v] + gy[TK::v] * gy[TK::v]);
}

// (H a)_v, g_v and H_vv at node (i,j) for the damage field a; when TRIAL the
// field is clip(a + mu*d, lo, 1) evaluated on the fly; MASKIN reads it as
// zero on active nodes, and with XPBY as a + mu*d (a CG direction update)
// there.  The field is read once on the node's seven-point neighbourhood.
template <bool TRIAL, bool MASKIN = false, bool XPBY = false>
__device__ __forceinline__ void helm_node2d(const Grid& g, const Helm& hp,
                                            const double* __restrict__ w2,
                                            const double* __restrict__ a,
                                            const double* __restrict__ d,
                                            const double* __restrict__ lo, double mu, int i, int j,
                                            double& Ha, double& gv, double& Hd,
                                            const uint8_t* __restrict__ mask = nullptr) {
  const int W = g.nx + 1, n = i + W * j;
  const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy, area = 0.5 * g.hx * g.hy;
  Ha = 0.0; gv = 0.0; Hd = 0.0;
  auto val = [&](int q) -> double {
    if (TRIAL) return fmin(fmax(a[q] + mu * d[q], lo[q]), 1.0);
    if (MASKIN && XPBY) return mask[q] ? 0.0 : a[q] + mu * d[q];
    if (MASKIN) return mask[q] ? 0.0 : a[q];
    return a[q];
  };
  double av[9];
#define LDH2(DX, DY)                                                                          \
  av[(DX + 1) + 3 * (DY + 1)] =                                                               \
      (i + DX >= 0 && i + DX <= g.nx && j + DY >= 0 && j + DY <= g.ny) ? val(n + DX + W * DY) \
                                                                        : 0.0;
  LDH2(0, 0) LDH2(1, 0) LDH2(1, 1) LDH2(0, 1) LDH2(-1, 0) LDH2(-1, -1) LDH2(0, -1)
#undef LDH2
  tri_helm2<0>(g, hp, w2, av, i, j, ihx, ihy, area, Ha, gv, Hd);
  tri_helm2<1>(g, hp, w2, av, i, j, ihx, ihy, area, Ha, gv, Hd);
  tri_helm2<2>(g, hp, w2, av, i, j, ihx, ihy, area, Ha, gv, Hd);
  tri_helm2<3>(g, hp, w2, av, i, j, ihx, ihy, area, Ha, gv, Hd);
  tri_helm2<4>(g, hp, w2, av, i, j, ihx, ihy, area, Ha, gv, Hd);
  tri_helm2<5>(g, hp, w2, av, i, j, ihx, ihy, area, Ha, gv, Hd);
}

// F = H a - g, Phi (box FB with bounds [lo, 1]), active mask (eq. (reducedis)
// with the upper-bound mirror), inverse diagonal of H on inactive nodes.
// Reductions: S[slot2] = sum Phi^2, S[slotm] = max |Phi| (NaN -> inf).
template <bool TRIAL>
__global__ __launch_bounds__(NB) void k_vi_eval2d(Grid g, Helm hp, const double* __restrict__ w2,
                                                  const double* __restrict__ a,
                                                  const double* __restrict__ d,
                                                  const double* __restrict__ lo,
                                                  const double* __restrict__ S, int mu_slot,
                                                  double zeta, double* __restrict__ F,
                                                  double* __restrict__ phi,
                                                  uint8_t* __restrict__ mask,
                                                  double* __restrict__ hdinv, Red r2, Red rm,
                                                  Red rlo, Red rhi) {
  const int i = blockIdx.x * NB_X + threadIdx.x;
  const int j = blockIdx.y * NB_Y + threadIdx.y;
  double p2 = 0.0, pm = 0.0, jlo = -INFINITY, jhi = -INFINITY;
  if (i <= g.nx && j <= g.ny) {
    const int n = i + (g.nx + 1) * j;
    const double mu = TRIAL ? S[mu_slot] : 0.0;
    double Ha, gv, Hd;
    helm_node2d<TRIAL>(g, hp, w2, a, d, lo, mu, i, j, Ha, gv, Hd);
    const double x = TRIAL ? fmin(fmax(a[n] + mu * d[n], lo[n]), 1.0) : a[n];
    const double l = lo[n];
    const double Fv = Ha - gv;
    const double ph = mcp_fb(x, Fv, l, 1.0);
    p2 = ph * ph;
    pm = nan_to_inf(fabs(ph));
    if (!TRIAL) {
      F[n] = Fv;
      phi[n] = ph;
      const bool act = (x - l <= zeta && Fv > 0.0) || (1.0 - x <= zeta && Fv < 0.0) || (l >= 1.0);
      mask[n] = act ? 1 : 0;
      hdinv[n] = act ? 0.0 : 1.0 / Hd;
      if (!act) { jlo = -(double)j; jhi = (double)j; }
    }
  }
  const int nb = gridDim.x * gridDim.y, bid = blockIdx.x + gridDim.x * blockIdx.y;
  const int tid = threadIdx.x + NB_X * threadIdx.y;
  block_reduce<NB, false>(p2, r2, nb, bid, tid);
  block_reduce<NB, true>(pm, rm, nb, bid, tid);
  if (!TRIAL) {
    block_reduce<NB, true>(jlo, rlo, nb, bid, tid);
    block_reduce<NB, true>(jhi, rhi, nb, bid, tid);
  }
}

// Triangle K's part of (H a)_v, g_v and H_vv with the element's W2 given
// (tri_helm2 with w2 read by the caller): the same arithmetic.
template <int K>
__device__ __forceinline__ void tri_helm2v(const Grid& g, const Helm& hp, double we,
                                           const double (&av)[9], int i, int j, double ihx,
                                           double ihy, double area, double& Ha, double& gv,
                                           double& Hd) {
  using TK = Tri2<K>;
  const int ci = i + TK::di, cj = j + TK::dj;
  if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) return;
  double gx[3], gy[3];
  tri_grads(TK::t, ihx, ihy, gx, gy);
  const double a0 = av[TK::template slot<0>()], a1 = av[TK::template slot<1>()];
  const double a2 = av[TK::template slot<2>()];
  const double sum = a0 + a1 + a2;
  const double aV = TK::v == 0 ? a0 : (TK::v == 1 ? a1 : a2);
  const double mass = area / 12.0 * (aV + sum);
  const double grx = a0 * gx[0] + a1 * gx[1] + a2 * gx[2];
  const double gry = a0 * gy[0] + a1 * gy[1] + a2 * gy[2];
  const double lap = area * (gx[TK::v] * grx + gy[TK::v] * gry);
  Ha += (we + hp.cM) * mass + hp.cL * lap;
  // (constant factors grouped: the divisions are loop-invariant, one per thread)
  gv += (we - hp.cm) * (area / 3.0);
  Hd += (we + hp.cM) * (area / 6.0) + hp.cL * area * (gx[TK::v] * gx[TK::v] + gy[TK::v] * gy[TK::v]);
}

// LDS-staged form for large grids: a block of 256 threads takes a 64 x 16
// node tile, first loads the tile's field (with a one-node halo) and the W2
// of its cells (cell columns i-1 and i of every node) into LDS with all loads
// in flight together, then each thread evaluates four nodes of one column
// from LDS.  Each field row and cell row is read from HBM once per tile (18
// of 16 rows, 17 of 16 cell rows).  Per node the same arithmetic as
// k_vi_eval2d (helm_node2d's six triangles in the same order).
constexpr int VL_ROWS = 16;
constexpr int VL_W = NB_X + 2;             // field tile width (halo on both sides)
constexpr int VL_CW = NB_X + 1;            // cell columns (i0 - 1 .. i0 + 63)

template <bool TRIAL>
__global__ __launch_bounds__(NB) void k_vi_eval_lds2d(Grid g, Helm hp, const double* __restrict__ w2,
                                                      const double* __restrict__ a,
                                                      const double* __restrict__ d,
                                                      const double* __restrict__ lo,
                                                      const double* __restrict__ S, int mu_slot,
                                                      double zeta, double* __restrict__ F,
                                                      double* __restrict__ phi,
                                                      uint8_t* __restrict__ mask,
                                                      double* __restrict__ hdinv, Red r2, Red rm,
                                                      Red rlo, Red rhi) {
  __shared__ double sa[VL_ROWS + 2][VL_W];         // field rows j0-1 .. j0+16
  __shared__ double sw[VL_ROWS + 1][VL_CW][2];     // W2 of cell rows j0-1 .. j0+15
  const int nbx = gridDim.x, total = gridDim.x * gridDim.y;
  const int t = xcd_tile(blockIdx.x + nbx * blockIdx.y, total);
  const int i0 = (t % nbx) * NB_X, j0 = (t / nbx) * VL_ROWS;
  const int tid = threadIdx.x + NB_X * threadIdx.y;
  const int W = g.nx + 1, nx = g.nx;
  const double mu = TRIAL ? S[mu_slot] : 0.0;
  for (int e = tid; e < (VL_ROWS + 2) * VL_W; e += NB) {
    const int rr = e / VL_W, cc = e % VL_W;
    const int ii = i0 - 1 + cc, r = j0 - 1 + rr;
    double v = 0.0;
    if (ii >= 0 && ii <= g.nx && r >= 0 && r <= g.ny) {
      const int q = ii + W * r;
      v = TRIAL ? fmin(fmax(a[q] + mu * d[q], lo[q]), 1.0) : a[q];
    }
    sa[rr][cc] = v;
  }
  for (int e = tid; e < (VL_ROWS + 1) * VL_CW * 2; e += NB) {
    const int rr = e / (2 * VL_CW), rem = e % (2 * VL_CW);
    const int cc = rem / 2, tt = rem % 2;
    const int ci = i0 - 1 + cc, cj = j0 - 1 + rr;
    sw[rr][cc][tt] = (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) ? 0.0 : w2[2 * (ci + nx * cj) + tt];
  }
  __syncthreads();
  const int tx = threadIdx.x, i = i0 + tx;
  const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy, area = 0.5 * g.hx * g.hy;
  double p2 = 0.0, pm = 0.0, jlo = -INFINITY, jhi = -INFINITY;
  if (i <= g.nx) {
    for (int s = 0; s < VL_ROWS / NB_Y; ++s) {
      const int rl = threadIdx.y * (VL_ROWS / NB_Y) + s;   // tile row of the node
      const int j = j0 + rl;
      if (j > g.ny) break;
      // the 3x3 neighbourhood in helm_node2d's slot order: (dx + 1) + 3 (dy + 1)
      const double av[9] = {sa[rl][tx], sa[rl][tx + 1], sa[rl][tx + 2],
                            sa[rl + 1][tx], sa[rl + 1][tx + 1], sa[rl + 1][tx + 2],
                            sa[rl + 2][tx], sa[rl + 2][tx + 1], sa[rl + 2][tx + 2]};
      // cells (i-1, j-1), (i, j-1) in cell row rl, (i-1, j), (i, j) in rl + 1
      double Ha = 0.0, gvv = 0.0, Hd = 0.0;
      tri_helm2v<0>(g, hp, sw[rl + 1][tx + 1][0], av, i, j, ihx, ihy, area, Ha, gvv, Hd);
      tri_helm2v<1>(g, hp, sw[rl + 1][tx + 1][1], av, i, j, ihx, ihy, area, Ha, gvv, Hd);
      tri_helm2v<2>(g, hp, sw[rl + 1][tx][0], av, i, j, ihx, ihy, area, Ha, gvv, Hd);
      tri_helm2v<3>(g, hp, sw[rl][tx][0], av, i, j, ihx, ihy, area, Ha, gvv, Hd);
      tri_helm2v<4>(g, hp, sw[rl][tx][1], av, i, j, ihx, ihy, area, Ha, gvv, Hd);
      tri_helm2v<5>(g, hp, sw[rl][tx + 1][1], av, i, j, ihx, ihy, area, Ha, gvv, Hd);
      const int n = i + W * j;
      const double x = av[4];
      const double l = lo[n];
      const double Fv = Ha - gvv;
      const double ph = mcp_fb(x, Fv, l, 1.0);
      p2 += ph * ph;
      pm = fmax(pm, nan_to_inf(fabs(ph)));
      if (!TRIAL) {
        F[n] = Fv;
        phi[n] = ph;
        const bool act = (x - l <= zeta && Fv > 0.0) || (1.0 - x <= zeta && Fv < 0.0) || (l >= 1.0);
        mask[n] = act ? 1 : 0;
        hdinv[n] = act ? 0.0 : 1.0 / Hd;
        if (!act) { jlo = fmax(jlo, -(double)j); jhi = fmax(jhi, (double)j); }
      }
    }
  }
  block_reduce<NB, false>(p2, r2, total, t, tid);
  block_reduce<NB, true>(pm, rm, total, t, tid);
  if (!TRIAL) {
    block_reduce<NB, true>(jlo, rlo, total, t, tid);
    block_reduce<NB, true>(jhi, rhi, total, t, tid);
  }
}

void launch_vi_eval2d(hipStream_t st, const Grid& g, double cL, double cM, double cm,
                      const double* w2, const double* a, const double* d, const double* lo,
                      const double* S, int mu_slot, double zeta, double* F, double* phi,
                      uint8_t* mask, double* hdinv, Red r2, Red rm, Red rlo, Red rhi, bool trial) {
  if (g.dim == 3)
    return launch_vi_eval3d(st, g, cL, cM, cm, w2, a, d, lo, S, mu_slot, zeta, F, phi, mask, hdinv,
                            r2, rm, rlo, rhi, trial);
  Helm hp{cL, cM, cm};
  if (use_col2d(g)) {
    static_assert(VL_ROWS % NB_Y == 0, "whole rows per thread");
    const dim3 gr((g.nx + 1 + NB_X - 1) / NB_X, (g.ny + 1 + VL_ROWS - 1) / VL_ROWS);
    if (trial)
      hipLaunchKernelGGL((k_vi_eval_lds2d<true>), gr, dim3(NB_X, NB_Y), 0, st, g, hp, w2, a, d, lo,
                         S, mu_slot, zeta, F, phi, mask, hdinv, r2, rm, rlo, rhi);
    else
      hipLaunchKernelGGL((k_vi_eval_lds2d<false>), gr, dim3(NB_X, NB_Y), 0, st, g, hp, w2, a, d, lo,
                         S, mu_slot, zeta, F, phi, mask, hdinv, r2, rm, rlo, rhi);
    const FinishSet fs{{r2, rm, rlo, rhi}, 0b1110, trial ? 2 : 4};
    launch_finish_multi(st, fs, (int)(gr.x * gr.y));
    return;
  }
  dim3 gr = node_grid2(g), bl(NB_X, NB_Y);
  if (trial)
    hipLaunchKernelGGL((k_vi_eval2d<true>), gr, bl, 0, st, g, hp, w2, a, d, lo, S, mu_slot, zeta,
                       F, phi, mask, hdinv, r2, rm, rlo, rhi);
  else
    hipLaunchKernelGGL((k_vi_eval2d<false>), gr, bl, 0, st, g, hp, w2, a, d, lo, S, mu_slot, zeta,
                       F, phi, mask, hdinv, r2, rm, rlo, rhi);
  // the four (trial: two) reductions are finished by one launch
  const FinishSet fs{{r2, rm, rlo, rhi}, 0b1110, trial ? 2 : 4};
  launch_finish_multi(st, fs, (int)(gr.x * gr.y));
}

// y = H x (MASKED: rows and columns of active nodes removed, i.e. x is taken
// as zero on active nodes and y is zero there).  Optional x.y into r.
template <bool MASKED, bool DOT>
__global__ __launch_bounds__(NB) void k_helm_apply2d(Grid g, Helm hp, const double* __restrict__ w2,
                                                     const double* __restrict__ x,
                                                     const uint8_t* __restrict__ mask,
                                                     double* __restrict__ y, int j0, int j1,
                                                     Red r) {
  const int i = blockIdx.x * NB_X + threadIdx.x;
  const int j = j0 + blockIdx.y * NB_Y + threadIdx.y;
  double acc = 0.0;
  if (i <= g.nx && j <= j1) {
    const int n = i + (g.nx + 1) * j;
    double Hx, gv, Hd;
    // MASKED: x is read as zero on active nodes, so values outside the
    // processed row range (all active) never enter
    helm_node2d<false, MASKED>(g, hp, w2, x, nullptr, nullptr, 0.0, i, j, Hx, gv, Hd, mask);
    if (MASKED && mask[n]) Hx = 0.0;
    y[n] = Hx;
    if (DOT) acc = (MASKED && mask[n]) ? 0.0 : x[n] * Hx;
  }
  if (DOT)
    block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y, blockIdx.x + gridDim.x * blockIdx.y,
                             threadIdx.x + NB_X * threadIdx.y);
}

void launch_helm_apply2d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                         const double* x, const uint8_t* mask, double* y, bool dot, Red r,
                         int j0, int j1) {
  if (g.dim == 3) return launch_helm_apply3d(st, g, cL, cM, w2, x, mask, y, dot, r, j0, j1);
  Helm hp{cL, cM, 0.0};
  if (j0 < 0) j0 = 0;
  if (j1 < 0 || j1 > g.ny) j1 = g.ny;
  if (j1 < j0) return;
  dim3 gr((g.nx + 1 + NB_X - 1) / NB_X, (j1 - j0 + 1 + NB_Y - 1) / NB_Y), bl(NB_X, NB_Y);
#define HELM_CASE(M, D) \
  hipLaunchKernelGGL((k_helm_apply2d<M, D>), gr, bl, 0, st, g, hp, w2, x, mask, y, j0, j1, r)
  if (mask) {
    if (dot) HELM_CASE(true, true); else HELM_CASE(true, false);
  } else {
    if (dot) HELM_CASE(false, true); else HELM_CASE(false, false);
  }
#undef HELM_CASE
  if (dot) launch_finish(st, r, (int)(gr.x * gr.y), false);
}

// One direction step of the Jacobi-preconditioned CG on H_NN over rows
// j0..j1: p_new = z + beta p_old (beta = S[S_BETA]; FIRST: p_new = z), formed
// on the fly wherever the stencil reads it, q = H_NN p_new, and the partial
// sums of p_new.q.  p_old and p_new are distinct buffers.
template <bool FIRST>
__global__ __launch_bounds__(NB) void k_helm_cg2d(Grid g, Helm hp, const double* __restrict__ w2,
                                                  const double* __restrict__ z,
                                                  const double* __restrict__ p_old,
                                                  const uint8_t* __restrict__ mask,
                                                  double* __restrict__ p_new,
                                                  double* __restrict__ q, int j0, int j1,
                                                  int i0, int i1, const double* __restrict__ S,
                                                  Red r) {
  const int i = i0 + blockIdx.x * NB_X + threadIdx.x;
  const int j = j0 + blockIdx.y * NB_Y + threadIdx.y;
  const double beta = FIRST ? 0.0 : S[S_BETA];
  double acc = 0.0;
  if (i <= i1 && j <= j1) {
    const int n = i + (g.nx + 1) * j;
    double Hx, gv, Hd;
    // active nodes read as zero, so rows outside j0..j1 (all active) never enter
    if (FIRST)
      helm_node2d<false, true>(g, hp, w2, z, nullptr, nullptr, 0.0, i, j, Hx, gv, Hd, mask);
    else
      helm_node2d<false, true, true>(g, hp, w2, z, p_old, nullptr, beta, i, j, Hx, gv, Hd, mask);
    const bool act = mask[n] != 0;
    const double pn = act ? 0.0 : (FIRST ? z[n] : z[n] + beta * p_old[n]);
    if (act) Hx = 0.0;
    p_new[n] = pn;
    q[n] = Hx;
    acc = pn * Hx;
  }
  block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y, blockIdx.x + gridDim.x * blockIdx.y,
                          threadIdx.x + NB_X * threadIdx.y);
}

// Rows j0..j1 (3D: row indices j + (ny + 1) k) and columns i0..i1.
int launch_helm_cg2d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                     const double* z, const double* p_old, const uint8_t* mask, double* p_new,
                     double* q, int j0, int j1, int i0, int i1, const double* S, bool first,
                     Red r, bool finish) {
  if (g.dim == 3)
    return launch_helm_cg3d(st, g, cL, cM, w2, z, p_old, mask, p_new, q, j0, j1, i0, i1, S, first, r,
                            finish);
  Helm hp{cL, cM, 0.0};
  if (j0 < 0) j0 = 0;
  if (j1 < 0 || j1 > g.ny) j1 = g.ny;
  if (i0 < 0) i0 = 0;
  if (i1 < 0 || i1 > g.nx) i1 = g.nx;
  if (j1 < j0 || i1 < i0) return 0;
  dim3 gr((i1 - i0 + 1 + NB_X - 1) / NB_X, (j1 - j0 + 1 + NB_Y - 1) / NB_Y), bl(NB_X, NB_Y);
  if (first)
    hipLaunchKernelGGL((k_helm_cg2d<true>), gr, bl, 0, st, g, hp, w2, z, p_old, mask, p_new, q, j0,
                       j1, i0, i1, S, r);
  else
    hipLaunchKernelGGL((k_helm_cg2d<false>), gr, bl, 0, st, g, hp, w2, z, p_old, mask, p_new, q, j0,
                       j1, i0, i1, S, r);
  if (!finish) return (int)(gr.x * gr.y);
  launch_finish(st, r, (int)(gr.x * gr.y), false);
  return 0;
}

// ---------------------------------------------------------------------------
// energy (eq. (regenergy)), per cell, deterministic sums
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(VB) void k_energy2d(Grid g, Mat m, double kell, double gc_cw,
                                                 double ell, int at2, const double* __restrict__ u,
                                                 const double* __restrict__ a, Red rel, Red rsu) {
  const int ncell = g.nx * g.ny;
  const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy, area = 0.5 * g.hx * g.hy;
  double el = 0.0, su = 0.0;
  for (int cell = blockIdx.x * VB + threadIdx.x; cell < ncell; cell += gridDim.x * VB) {
    const int ci = cell % g.nx, cj = cell / g.nx, W = g.nx + 1;
    const int n00 = ci + W * cj, n10 = n00 + 1, n11 = n00 + 1 + W, n01 = n00 + W;
    const double* ux = u;
    const double* uy = u + g.N;
    double es[2] = {0.0, 0.0};   // thermal-shock eigenstrain of the cell's T0, T1
    if (g.eig_dT != 0.0) eig_row2d(g, cj, es[0], es[1]);
    for (int t = 0; t < 2; ++t) {
      const int nA = n00, nB = t == 0 ? n10 : n11, nC = t == 0 ? n11 : n01;
      double exx, eyy, gam;
      if (t == 0) {
        exx = (ux[n10] - ux[n00]) * ihx; eyy = (uy[n11] - uy[n10]) * ihy;
        gam = (uy[n10] - uy[n00]) * ihx + (ux[n11] - ux[n10]) * ihy;
      } else {
        exx = (ux[n11] - ux[n01]) * ihx; eyy = (uy[n01] - uy[n00]) * ihy;
        gam = (uy[n11] - uy[n01]) * ihx + (ux[n01] - ux[n00]) * ihy;
      }
      exx -= es[t];
      eyy -= es[t];
      const double w2 = m.l2m * (exx * exx + eyy * eyy) + 2.0 * m.lam * exx * eyy + m.mu * gam * gam;
      const double a0 = a[nA], a1 = a[nB], a2 = a[nC];
      el += 0.5 * abar3(a0, a1, a2, kell) * area * w2;
      double gx[3], gy[3];
      tri_grads(t, ihx, ihy, gx, gy);
      const double grx = a0 * gx[0] + a1 * gx[1] + a2 * gx[2];
      const double gry = a0 * gy[0] + a1 * gy[1] + a2 * gy[2];
      const double s = a0 + a1 + a2;
      const double wint = at2 ? area / 12.0 * (a0 * a0 + a1 * a1 + a2 * a2 + s * s) : area / 3.0 * s;
      su += gc_cw * (wint / ell + ell * area * (grx * grx + gry * gry));
    }
  }
  block_reduce<VB, false>(el, rel, gridDim.x, blockIdx.x, threadIdx.x);
  block_reduce<VB, false>(su, rsu, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_energy2d(hipStream_t st, const Grid& g, const Mat& m, double kell, double gc_cw,
                     double ell, int at2, const double* u, const double* a, Red rel, Red rsu) {
  const int ncell = g.nx * g.ny;
  int nb = (ncell + VB - 1) / VB;
  if (nb > VGRID) nb = VGRID;
  hipLaunchKernelGGL(k_energy2d, dim3(nb), dim3(VB), 0, st, g, m, kell, gc_cw, ell, at2, u, a, rel, rsu);
  const FinishSet fs{{rel, rsu, Red{}, Red{}}, 0, 2};
  launch_finish_multi(st, fs, nb);
}

}  // namespace frac

namespace frac {

// ---------------------------------------------------------------------------
// coupled Jacobian (Newton step of Algorithm 3 / 4 on the full problem)
// ---------------------------------------------------------------------------
//
// E_ualpha of eq. (offdiag) with a'(alpha) = -2 (1 - alpha), integrated
// exactly with P1 alpha:  B[v, j] = sum_e -2 |T| (B_e^T D eps_e(u))_v (M_ref b_e)_j,
// b = 1 - alpha, M_ref = (1 + delta_ab)/12.
//
// k_jac_u2d:  y_u = A x_u + B x_a   (A = K(alpha), Dirichlet rows zero)
// k_jac_a2d:  y_a = B^T x_u + C x_a (C = H, rows and columns of active nodes removed)
// Either operand may be absent (nullptr) to apply one block only.

// (M_ref b)-weighted pairing w_e^T M_ref b_e of a triangle's three nodes.
__device__ __forceinline__ double mref_pair(double w0, double w1, double w2, double b0, double b1,
                                            double b2) {
  return (w0 * b0 + w1 * b1 + w2 * b2 + (w0 + w1 + w2) * (b0 + b1 + b2)) * (1.0 / 12.0);
}

// (B x_a) at node (i, j): the coupling coefficients c_e = -2 w_e^T M_ref b_e
// of the six triangles around the node, w = x_a masked to the inactive set,
// applied to the stress of u (its effective strain when EIG).
template <bool EIG>
__device__ __forceinline__ void coupling_force2d(const Grid& g, const Mat& m,
                                                 const double* __restrict__ alpha,
                                                 const double* __restrict__ u,
                                                 const double* __restrict__ xa,
                                                 const uint8_t* __restrict__ mask, int i, int j,
                                                 double& gx, double& gy) {
  const int W = g.nx + 1, N = g.N, n = i + W * j;
  const bool L = i > 0, R = i < g.nx, D = j > 0, U = j < g.ny;
  auto w_at = [&](bool ok, int k) -> double { return (ok && !mask[k]) ? xa[k] : 0.0; };
  auto b_at = [&](bool ok, int k) -> double { return ok ? 1.0 - alpha[k] : 0.0; };
  const double wC = w_at(true, n), wE = w_at(R, n + 1), wNE = w_at(R && U, n + 1 + W),
               wN = w_at(U, n + W), wW = w_at(L, n - 1), wSW = w_at(L && D, n - 1 - W),
               wS = w_at(D, n - W);
  const double bC = b_at(true, n), bE = b_at(R, n + 1), bNE = b_at(R && U, n + 1 + W),
               bN = b_at(U, n + W), bW = b_at(L, n - 1), bSW = b_at(L && D, n - 1 - W),
               bS = b_at(D, n - W);
  double c[6];
  c[0] = -2.0 * mref_pair(wC, wE, wNE, bC, bE, bNE);
  c[1] = -2.0 * mref_pair(wC, wNE, wN, bC, bNE, bN);
  c[2] = -2.0 * mref_pair(wW, wC, wN, bW, bC, bN);
  c[3] = -2.0 * mref_pair(wSW, wS, wC, bSW, bS, bC);
  c[4] = -2.0 * mref_pair(wSW, wC, wW, bSW, bC, bW);
  c[5] = -2.0 * mref_pair(wS, wE, wC, bS, bE, bC);
  double dx, dy;
  node_force2d<true, false, EIG>(g, m, c, u, u + N, i, j, gx, gy, dx, dy);
}

template <bool HAS_XU, bool HAS_XA, bool DOT, bool EIG>
__global__ __launch_bounds__(NB) void k_jac_u2d(Grid g, Mat m, double kell,
                                                const double* __restrict__ alpha,
                                                const double* __restrict__ u,
                                                const double* __restrict__ xu,
                                                const double* __restrict__ xa,
                                                const uint8_t* __restrict__ mask,
                                                double* __restrict__ yu, Red r,
                                                const double* __restrict__ band) {
  const int i = blockIdx.x * NB_X + threadIdx.x;
  const int j = blockIdx.y * NB_Y + threadIdx.y;
  double acc = 0.0;
  // B x_a vanishes at nodes with no inactive node within one row: with band
  // = (-j_lo, j_hi) of the inactive rows, only rows j_lo - 1 .. j_hi + 1 carry
  // it (band == nullptr: every row)
  bool couple = HAS_XA;
  if (HAS_XA && band) {
    const double jlo = -band[0], jhi = band[1];
    couple = jlo <= jhi && (double)j >= jlo - 1.0 && (double)j <= jhi + 1.0;
  }
  if (i <= g.nx && j <= g.ny) {
    const int N = g.N, n = i + (g.nx + 1) * j;
    double fx = 0, fy = 0, dx, dy;
    if (HAS_XU) {
      double c[6];
      coef6<true>(g, alpha, kell, i, j, c);
      node_force2d<true, false>(g, m, c, xu, xu + N, i, j, fx, fy, dx, dy);
    }
    if (couple) {
      double gx, gy;
      coupling_force2d<EIG>(g, m, alpha, u, xa, mask, i, j, gx, gy);
      fx += gx;
      fy += gy;
    }
    if (fixed_x2(g, i, j)) fx = 0.0;
    if (fixed_y2(g, i, j)) fy = 0.0;
    yu[n] = fx;
    yu[n + N] = fy;
    if (DOT) acc = xu[n] * fx + xu[n + N] * fy;
  }
  if (DOT)
    block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y, blockIdx.x + gridDim.x * blockIdx.y,
                            threadIdx.x + NB_X * threadIdx.y);
}

// Strain (exx, eyy, gamma) of a P1 field on triangle type t with local nodes 0..2.
__device__ __forceinline__ void tri_strain(int t, double ihx, double ihy, const double vx[3],
                                           const double vy[3], double& exx, double& eyy,
                                           double& gam) {
  double gx[3], gy[3];
  tri_grads(t, ihx, ihy, gx, gy);
  exx = gx[0] * vx[0] + gx[1] * vx[1] + gx[2] * vx[2];
  eyy = gy[0] * vy[0] + gy[1] * vy[1] + gy[2] * vy[2];
  gam = gy[0] * vx[0] + gy[1] * vx[1] + gy[2] * vx[2] + gx[0] * vy[0] + gx[1] * vy[1] + gx[2] * vy[2];
}

template <bool HAS_XU, bool HAS_XA, bool DOT, bool EIG>
__global__ __launch_bounds__(NB) void k_jac_a2d(Grid g, Mat m, Helm hp,
                                                const double* __restrict__ alpha,
                                                const double* __restrict__ u,
                                                const double* __restrict__ w2,
                                                const double* __restrict__ xu,
                                                const double* __restrict__ xa,
                                                const uint8_t* __restrict__ mask,
                                                double* __restrict__ ya, Red r) {
  const int i = blockIdx.x * NB_X + threadIdx.x;
  const int j = blockIdx.y * NB_Y + threadIdx.y;
  double acc = 0.0;
  if (i <= g.nx && j <= g.ny) {
    const int N = g.N, W = g.nx + 1, n = i + W * j;
    double y = 0.0;
    if (!mask[n]) {
      if (HAS_XA) {
        double Hx, gv, Hd;
        helm_node2d<false, true>(g, hp, w2, xa, nullptr, nullptr, 0.0, i, j, Hx, gv, Hd, mask);
        y += Hx;
      }
      if (HAS_XU) {
        const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy, area = 0.5 * g.hx * g.hy;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const int ci = i + c_tri_di[k], cj = j + c_tri_dj[k];
          if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
          const int t = c_tri_t[k], v = c_tri_v[k];
          int di[3], dj[3];
          tri_nodes(t, di, dj);
          double ux[3], uy[3], vx[3], vy[3], bb[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const int nn = ci + di[q] + W * (cj + dj[q]);
            ux[q] = u[nn]; uy[q] = u[nn + N];
            vx[q] = xu[nn]; vy[q] = xu[nn + N];
            bb[q] = 1.0 - alpha[nn];
          }
          double e0, e1, e2, f0, f1, f2;
          tri_strain(t, ihx, ihy, ux, uy, e0, e1, e2);
          tri_strain(t, ihx, ihy, vx, vy, f0, f1, f2);
          if (EIG) {   // effective strain of u
            double s0, s1;
            eig_row2d(g, cj, s0, s1);
            const double se = t == 0 ? s0 : s1;
            e0 -= se;
            e1 -= se;
          }
          // sigma(u) : eps(v) with sigma = D eps (engineering shear)
          const double s = (m.l2m * e0 + m.lam * e1) * f0 + (m.lam * e0 + m.l2m * e1) * f1 + m.mu * e2 * f2;
          const double mb = (bb[v] + bb[0] + bb[1] + bb[2]) * (1.0 / 12.0);
          y += -2.0 * area * s * mb;
        }
      }
    }
    ya[n] = y;
    if (DOT) acc = (HAS_XA && !mask[n]) ? xa[n] * y : 0.0;
  }
  if (DOT)
    block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y, blockIdx.x + gridDim.x * blockIdx.y,
                            threadIdx.x + NB_X * threadIdx.y);
}

// y_u = A x_u + B x_a (either part optional); y_a = B^T x_u + C x_a.
// dot: S[slot_u] = x_u . y_u and S[slot_a] = x_a . y_a (inactive part).
void launch_jac2d(hipStream_t st, const Grid& g, const Mat& m, double kell, double cL, double cM,
                  const double* alpha, const double* u, const double* w2, const uint8_t* mask,
                  const double* xu, const double* xa, double* yu, double* ya, bool dot, Red ru,
                  Red ra, const double* band) {
  if (g.dim == 3)
    return launch_jac3d(st, g, m, kell, cL, cM, alpha, u, w2, mask, xu, xa, yu, ya, dot, ru, ra,
                        band);
  dim3 gr = node_grid2(g), bl(NB_X, NB_Y);
  Helm hp{cL, cM, 0.0};
  // the coupling blocks carry the stress of u's effective strain: the
  // thermal-shock eigenstrain when the (load) grid has one
  const bool eig = g.eig_dT != 0.0;
  if (yu) {
#define JU(A, B, D)                                                                                \
  do {                                                                                             \
    if (eig && B)                                                                                  \
      hipLaunchKernelGGL((k_jac_u2d<A, B, D, true>), gr, bl, 0, st, g, m, kell, alpha, u, xu, xa,  \
                         mask, yu, ru, band);                                                      \
    else                                                                                           \
      hipLaunchKernelGGL((k_jac_u2d<A, B, D, false>), gr, bl, 0, st, g, m, kell, alpha, u, xu, xa, \
                         mask, yu, ru, band);                                                      \
  } while (0)
    if (xu && xa) { if (dot) JU(true, true, true); else JU(true, true, false); }
    else if (xu) { if (dot) JU(true, false, true); else JU(true, false, false); }
    else JU(false, true, false);
#undef JU
    if (dot && xu) launch_finish(st, ru, (int)(gr.x * gr.y), false);
  }
  if (ya) {
#define JA(A, B, D)                                                                                \
  do {                                                                                             \
    if (eig && A)                                                                                  \
      hipLaunchKernelGGL((k_jac_a2d<A, B, D, true>), gr, bl, 0, st, g, m, hp, alpha, u, w2, xu, xa, \
                         mask, ya, ra);                                                            \
    else                                                                                           \
      hipLaunchKernelGGL((k_jac_a2d<A, B, D, false>), gr, bl, 0, st, g, m, hp, alpha, u, w2, xu,   \
                         xa, mask, ya, ra);                                                        \
  } while (0)
    if (xu && xa) { if (dot) JA(true, true, true); else JA(true, true, false); }
    else if (xa) { if (dot) JA(false, true, true); else JA(false, true, false); }
    else JA(true, false, false);
#undef JA
    if (dot && xa) launch_finish(st, ra, (int)(gr.x * gr.y), false);
  }
}

// y_u += B x_a on rows r0..r1 (the rows next to the inactive set, the only
// ones B x_a reaches), Dirichlet rows left alone; partial sums of x_u . B x_a.
template <bool EIG>
__global__ __launch_bounds__(NB) void k_couple_u2d(Grid g, Mat m, const double* __restrict__ alpha,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ xu,
                                                   const double* __restrict__ xa,
                                                   const uint8_t* __restrict__ mask,
                                                   double* __restrict__ yu, int r0, int r1, Red r) {
  const int i = blockIdx.x * NB_X + threadIdx.x;
  const int j = r0 + blockIdx.y * NB_Y + threadIdx.y;
  double acc = 0.0;
  if (i <= g.nx && j <= r1) {
    const int N = g.N, n = i + (g.nx + 1) * j;
    double gx, gy;
    coupling_force2d<EIG>(g, m, alpha, u, xa, mask, i, j, gx, gy);
    if (fixed_x2(g, i, j)) gx = 0.0;
    if (fixed_y2(g, i, j)) gy = 0.0;
    yu[n] += gx;
    yu[n + N] += gy;
    acc = xu[n] * gx + xu[n + N] * gy;
  }
  block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y, blockIdx.x + gridDim.x * blockIdx.y,
                          threadIdx.x + NB_X * threadIdx.y);
}

void launch_couple_u2d(hipStream_t st, const Grid& g, const Mat& m, const double* alpha,
                       const double* u, const double* xu, const double* xa, const uint8_t* mask,
                       double* yu, int r0, int r1, Red r) {
  if (g.dim == 3) return launch_couple_u3d(st, g, m, alpha, u, xu, xa, mask, yu, r0, r1, r);
  if (r0 < 0) r0 = 0;
  if (r1 > g.ny) r1 = g.ny;
  if (r1 < r0) return;
  dim3 gr((g.nx + 1 + NB_X - 1) / NB_X, (r1 - r0 + 1 + NB_Y - 1) / NB_Y), bl(NB_X, NB_Y);
  if (g.eig_dT != 0.0)
    hipLaunchKernelGGL((k_couple_u2d<true>), gr, bl, 0, st, g, m, alpha, u, xu, xa, mask, yu, r0,
                       r1, r);
  else
    hipLaunchKernelGGL((k_couple_u2d<false>), gr, bl, 0, st, g, m, alpha, u, xu, xa, mask, yu, r0,
                       r1, r);
  launch_finish(st, r, (int)(gr.x * gr.y), false);
}

// Jacobi-preconditioned Chebyshev step on C = H_NN (the damage block of the
// Newton Jacobian): d_new = cd d_in + cr D^{-1} (b - C x_in); x_out = x_in + d_new.
__global__ __launch_bounds__(NB) void k_cheb_helm2d(Grid g, Helm hp, const double* __restrict__ w2,
                                                    const uint8_t* __restrict__ mask,
                                                    const double* __restrict__ x_in,
                                                    double* __restrict__ x_out,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ d_in,
                                                    double* __restrict__ d_out, double cd,
                                                    double cr) {
  const int i = blockIdx.x * NB_X + threadIdx.x;
  const int j = blockIdx.y * NB_Y + threadIdx.y;
  if (i > g.nx || j > g.ny) return;
  const int n = i + (g.nx + 1) * j;
  if (mask[n]) {
    x_out[n] = 0.0;
    if (d_out) d_out[n] = 0.0;
    return;
  }
  double Hx = 0.0, gv, Hd;
  if (x_in) helm_node2d<false, true>(g, hp, w2, x_in, nullptr, nullptr, 0.0, i, j, Hx, gv, Hd, mask);
  else helm_node2d<false, true>(g, hp, w2, b, nullptr, nullptr, 0.0, i, j, Hx, gv, Hd, mask);
  if (!x_in) Hx = 0.0;
  double dn = cr * (b[n] - Hx) / Hd;
  if (d_in) dn += cd * d_in[n];
  x_out[n] = (x_in ? x_in[n] : 0.0) + dn;
  if (d_out) d_out[n] = dn;
}

void launch_cheb_helm2d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                        const uint8_t* mask, const double* x_in, double* x_out, const double* b,
                        const double* d_in, double* d_out, double cd, double cr) {
  if (g.dim == 3)
    return launch_cheb_helm3d(st, g, cL, cM, w2, mask, x_in, x_out, b, d_in, d_out, cd, cr);
  Helm hp{cL, cM, 0.0};
  dim3 gr = node_grid2(g), bl(NB_X, NB_Y);
  hipLaunchKernelGGL(k_cheb_helm2d, gr, bl, 0, st, g, hp, w2, mask, x_in, x_out, b, d_in, d_out, cd, cr);
}

// Trial state of the coupled line search: u_t = u + mu d_u on free DOFs,
// alpha_t = clip(alpha + mu d_a, lo, 1); mu = S[S_MU].
__global__ __launch_bounds__(VB) void k_trial_state(int64_t n2, int64_t N, const double* __restrict__ u,
                                                    const double* __restrict__ a,
                                                    const double* __restrict__ du,
                                                    const double* __restrict__ da,
                                                    const double* __restrict__ lo,
                                                    const double* __restrict__ S,
                                                    double* __restrict__ ut,
                                                    double* __restrict__ at) {
  const double mu = S[S_MU];
  for (int64_t k = (int64_t)blockIdx.x * VB + threadIdx.x; k < n2 + N; k += (int64_t)gridDim.x * VB) {
    if (k < n2) ut[k] = u[k] + mu * du[k];
    else {
      const int64_t q = k - n2;
      at[q] = fmin(fmax(a[q] + mu * da[q], lo[q]), 1.0);
    }
  }
}

void launch_trial_state(hipStream_t st, int64_t n2, int64_t N, const double* u, const double* a,
                        const double* du, const double* da, const double* lo, const double* S,
                        double* ut, double* at) {
  int64_t nb = (n2 + N + VB - 1) / VB;
  if (nb > VGRID) nb = VGRID;
  hipLaunchKernelGGL(k_trial_state, dim3((int)nb), dim3(VB), 0, st, n2, N, u, a, du, da, lo, S, ut, at);
}

}  // namespace frac
