// Device code of the 2D operator (right-diagonal P1 triangles) shared by the
// stencil kernels: per-node forms (coupled Jacobian rows) and the
// column-blocked form (elasticity apply, residual, Chebyshev smoothing).
#pragma once

#include "common.h"

namespace frac {

// ---------------------------------------------------------------------------
// boundary conditions
// ---------------------------------------------------------------------------

// tension: u_x at node (0,0), u_y on the bottom and top edges;
// surfing: both components on the whole boundary;
// thermal shock: u_x on the lateral edges, u_y on the top edge
__device__ __forceinline__ bool on_edge2(const Grid& g, int i, int j) {
  return i == 0 || i == g.nx || j == 0 || j == g.ny;
}
__device__ __forceinline__ bool fixed_x2(const Grid& g, int i, int j) {
  if (g.bc == BC_SURFING_2D) return on_edge2(g, i, j);
  if (g.bc == BC_TSHOCK_2D) return i == 0 || i == g.nx;
  return (g.bc == BC_TENSION_2D) && i == 0 && j == 0;
}
__device__ __forceinline__ bool fixed_y2(const Grid& g, int i, int j) {
  if (g.bc == BC_SURFING_2D) return on_edge2(g, i, j);
  if (g.bc == BC_TSHOCK_2D) return j == g.ny;
  return (g.bc == BC_TENSION_2D) && (j == 0 || j == g.ny);
}

// Thermal-shock eigenstrain eps0 = s I of the triangles of cell row cj
// (eq. (tempfielderfc) at the centroid): T0 (s0) has its centroid at
// (cj + 1/3) hy, T1 (s1) at (cj + 2/3) hy.  Zero outside the grid rows.
__device__ __forceinline__ void eig_row2d(const Grid& g, int cj, double& s0, double& s1) {
  if (cj < 0 || cj >= g.ny) { s0 = s1 = 0.0; return; }
  const double r = g.hy / g.eig_depth;
  s0 = -g.eig_dT * erfc((cj + 1.0 / 3.0) * r);
  s1 = -g.eig_dT * erfc((cj + 2.0 / 3.0) * r);
}

// ---------------------------------------------------------------------------
// the node operator
// ---------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T abar3(T a0, T a1, T a2, T k) {
  const T b0 = T(1) - a0, b1 = T(1) - a1, b2 = T(1) - a2, s = b0 + b1 + b2;
  return k + (b0 * b0 + b1 * b1 + b2 * b2 + s * s) * (T(1) / T(12));
}

// Coefficients of the six triangles around node (i, j), in the order
// (a) cell(i,j) T0, (b) cell(i,j) T1, (c) cell(i-1,j) T0,
// (d) cell(i-1,j-1) T0, (e) cell(i-1,j-1) T1, (f) cell(i,j-1) T1.
// FA: from nodal alpha (finest level); otherwise from the element array.
template <bool FA, class T>
__device__ __forceinline__ void coef6(const Grid& g, const T* __restrict__ coef, T kell, int i,
                                      int j, T c[6]) {
  const int W = g.nx + 1, n = i + W * j;
  const bool L = i > 0, R = i < g.nx, D = j > 0, U = j < g.ny;
  if (FA) {
    const T aC = coef[n];
    const T aE = R ? coef[n + 1] : T(0);
    const T aNE = (R && U) ? coef[n + 1 + W] : T(0);
    const T aN = U ? coef[n + W] : T(0);
    const T aW = L ? coef[n - 1] : T(0);
    const T aSW = (L && D) ? coef[n - 1 - W] : T(0);
    const T aS = D ? coef[n - W] : T(0);
    c[0] = abar3(aC, aE, aNE, kell);
    c[1] = abar3(aC, aNE, aN, kell);
    c[2] = abar3(aW, aC, aN, kell);
    c[3] = abar3(aSW, aS, aC, kell);
    c[4] = abar3(aSW, aC, aW, kell);
    c[5] = abar3(aS, aE, aC, kell);
  } else {
    const int nx = g.nx;
    c[0] = (R && U) ? coef[2 * (i + nx * j)] : T(0);
    c[1] = (R && U) ? coef[2 * (i + nx * j) + 1] : T(0);
    c[2] = (L && U) ? coef[2 * (i - 1 + nx * j)] : T(0);
    c[3] = (L && D) ? coef[2 * (i - 1 + nx * (j - 1))] : T(0);
    c[4] = (L && D) ? coef[2 * (i - 1 + nx * (j - 1)) + 1] : T(0);
    c[5] = (R && D) ? coef[2 * (i + nx * (j - 1)) + 1] : T(0);
  }
}

// What the operator loads add to x: nothing (NoProl), or the coarse
// correction P x_c interpolated on the fly (AddProl), as after the V-cycle's
// prolongation: at fine node (i, j), half the sum of coarse nodes
// (i >> 1, j >> 1) and ((i + 1) >> 1, (j + 1) >> 1) (the nested P1
// interpolation of the right-diagonal triangles, prolong_node2d), zero on
// Dirichlet DOFs.  AddProl reads x_c from a block of coarse nodes staged in
// LDS: sx, sy hold the two components of coarse columns cc0 .. cc0 +
// PROL_PW - 1 of rows cr0, cr0 + 1, ... (row pitch PROL_PW), the coarse
// nodes that a tile NB_X fine columns wide touches.
constexpr int PROL_PW = NB_X / 2 + 2;
struct NoProl {};
template <class T>
struct AddProl {
  const T* sx;
  const T* sy;
  int cc0, cr0;
};
template <class T>
__device__ __forceinline__ void add_prol(const Grid&, const NoProl&, int, int, T&, T&) {}
template <class T>
__device__ __forceinline__ void add_prol(const Grid& g, const AddProl<T>& pr, int i, int j, T& vx,
                                         T& vy) {
  const int a = ((j >> 1) - pr.cr0) * PROL_PW + ((i >> 1) - pr.cc0);
  const int b = (((j + 1) >> 1) - pr.cr0) * PROL_PW + (((i + 1) >> 1) - pr.cc0);
  vx += fixed_x2(g, i, j) ? T(0) : T(0.5) * (pr.sx[a] + pr.sx[b]);
  vy += fixed_y2(g, i, j) ? T(0) : T(0.5) * (pr.sy[a] + pr.sy[b]);
}

// Force (fx, fy) = (K x) at node (i, j) and, when DIAG, the diagonal entries
// (dx, dy) of K for the node's two DOFs.
//
// EIG (thermal shock, finest level): the forces of the effective strain
// eps(x) - eps0, i.e. K x - f with f the eigenstrain load of eq.
// (energytshock).
// PROL: x is taken as x + P x_c (*pr), as after the V-cycle's prolongation.
template <bool HASX, bool DIAG, bool EIG = false, bool PROL = false, class T>
__device__ __forceinline__ void node_force2d(const Grid& g, const Mat& m, const T c[6],
                                             const T* __restrict__ ux, const T* __restrict__ uy,
                                             int i, int j, T& fx, T& fy, T& dx, T& dy,
                                             const AddProl<T>* pr = nullptr) {
  const int W = g.nx + 1, n = i + W * j;
  const bool L = i > 0, R = i < g.nx, D = j > 0, U = j < g.ny;
  const T ihx = T(1.0 / g.hx), ihy = T(1.0 / g.hy), area = T(0.5 * g.hx * g.hy);
  const T l2m = T(m.l2m), lam = T(m.lam), mu = T(m.mu);
  T cx = 0, cy = 0, ex = 0, ey = 0, nex = 0, ney = 0, nnx = 0, nny = 0;
  T wx = 0, wy = 0, swx = 0, swy = 0, sx = 0, sy = 0;
  if (HASX) {
    cx = ux[n];
    cy = uy[n];
    if (R) { ex = ux[n + 1]; ey = uy[n + 1]; }
    if (R && U) { nex = ux[n + 1 + W]; ney = uy[n + 1 + W]; }
    if (U) { nnx = ux[n + W]; nny = uy[n + W]; }
    if (L) { wx = ux[n - 1]; wy = uy[n - 1]; }
    if (L && D) { swx = ux[n - 1 - W]; swy = uy[n - 1 - W]; }
    if (D) { sx = ux[n - W]; sy = uy[n - W]; }
  }
  if (PROL) {
    add_prol(g, *pr, i, j, cx, cy);
    if (R) add_prol(g, *pr, i + 1, j, ex, ey);
    if (R && U) add_prol(g, *pr, i + 1, j + 1, nex, ney);
    if (U) add_prol(g, *pr, i, j + 1, nnx, nny);
    if (L) add_prol(g, *pr, i - 1, j, wx, wy);
    if (L && D) add_prol(g, *pr, i - 1, j - 1, swx, swy);
    if (D) add_prol(g, *pr, i, j - 1, sx, sy);
  }
  fx = fy = dx = dy = T(0);
  const T hxx = ihx * ihx, hyy = ihy * ihy;
  // eigenstrain of the cell rows above (j) and below (j - 1) the node
  T su0 = 0, su1 = 0, sd0 = 0, sd1 = 0;
  if (EIG) {
    double a0, a1, b0, b1;
    eig_row2d(g, j, a0, a1);
    eig_row2d(g, j - 1, b0, b1);
    su0 = T(a0); su1 = T(a1); sd0 = T(b0); sd1 = T(b1);
  }
  // (a) cell(i,j) T0: node is vertex 0, gradient (-1/hx, 0)
  if (R && U) {
    const T w = c[0] * area;
    if (HASX) {
      const T exx = (ex - cx) * ihx - su0, eyy = (ney - ey) * ihy - su0;
      const T gam = (ey - cy) * ihx + (nex - ex) * ihy;
      const T sxx = l2m * exx + lam * eyy, sxy = mu * gam;
      fx += w * (-sxx * ihx);
      fy += w * (-sxy * ihx);
    }
    if (DIAG) { dx += w * l2m * hxx; dy += w * mu * hxx; }
  }
  // (b) cell(i,j) T1: vertex 0, gradient (0, -1/hy)
  if (R && U) {
    const T w = c[1] * area;
    if (HASX) {
      const T exx = (nex - nnx) * ihx - su1, eyy = (nny - cy) * ihy - su1;
      const T gam = (ney - nny) * ihx + (nnx - cx) * ihy;
      const T syy = lam * exx + l2m * eyy, sxy = mu * gam;
      fx += w * (-sxy * ihy);
      fy += w * (-syy * ihy);
    }
    if (DIAG) { dx += w * mu * hyy; dy += w * l2m * hyy; }
  }
  // (c) cell(i-1,j) T0: vertex 1, gradient (1/hx, -1/hy)
  if (L && U) {
    const T w = c[2] * area;
    if (HASX) {
      const T exx = (cx - wx) * ihx - su0, eyy = (nny - cy) * ihy - su0;
      const T gam = (cy - wy) * ihx + (nnx - cx) * ihy;
      const T sxx = l2m * exx + lam * eyy, syy = lam * exx + l2m * eyy, sxy = mu * gam;
      fx += w * (sxx * ihx - sxy * ihy);
      fy += w * (sxy * ihx - syy * ihy);
    }
    if (DIAG) { dx += w * (l2m * hxx + mu * hyy); dy += w * (l2m * hyy + mu * hxx); }
  }
  // (d) cell(i-1,j-1) T0: vertex 2, gradient (0, 1/hy)
  if (L && D) {
    const T w = c[3] * area;
    if (HASX) {
      const T exx = (sx - swx) * ihx - sd0, eyy = (cy - sy) * ihy - sd0;
      const T gam = (sy - swy) * ihx + (cx - sx) * ihy;
      const T syy = lam * exx + l2m * eyy, sxy = mu * gam;
      fx += w * (sxy * ihy);
      fy += w * (syy * ihy);
    }
    if (DIAG) { dx += w * mu * hyy; dy += w * l2m * hyy; }
  }
  // (e) cell(i-1,j-1) T1: vertex 1, gradient (1/hx, 0)
  if (L && D) {
    const T w = c[4] * area;
    if (HASX) {
      const T exx = (cx - wx) * ihx - sd1, eyy = (wy - swy) * ihy - sd1;
      const T gam = (cy - wy) * ihx + (wx - swx) * ihy;
      const T sxx = l2m * exx + lam * eyy, sxy = mu * gam;
      fx += w * (sxx * ihx);
      fy += w * (sxy * ihx);
    }
    if (DIAG) { dx += w * l2m * hxx; dy += w * mu * hxx; }
  }
  // (f) cell(i,j-1) T1: vertex 2, gradient (-1/hx, 1/hy)
  if (R && D) {
    const T w = c[5] * area;
    if (HASX) {
      const T exx = (ex - cx) * ihx - sd1, eyy = (cy - sy) * ihy - sd1;
      const T gam = (ey - cy) * ihx + (cx - sx) * ihy;
      const T sxx = l2m * exx + lam * eyy, syy = lam * exx + l2m * eyy, sxy = mu * gam;
      fx += w * (-sxx * ihx + sxy * ihy);
      fy += w * (-sxy * ihx + syy * ihy);
    }
    if (DIAG) { dx += w * (l2m * hxx + mu * hyy); dy += w * (l2m * hyy + mu * hxx); }
  }
}

// ---------------------------------------------------------------------------
// node outputs of the apply / residual / Chebyshev-step kernels
// ---------------------------------------------------------------------------

enum { M_APPLY = 0, M_RESID = 1, M_SMOOTH = 2 };
enum { R_NONE = 0, R_DOT = 1, R_FREE2 = 2 };

// Output of a node kernel at node (i, j) from the node's force (fx, fy) = K x,
// diagonal (dx, dy) and iterate (xc, yc); acc collects the optional reduction.
template <int MODE, int RED, class T>
__device__ __forceinline__ void node_out2d(const Grid& g, int i, int j, T fx, T fy, T dx, T dy,
                                           T xc, T yc, T* __restrict__ y,
                                           const T* __restrict__ b, const T* __restrict__ din,
                                           T* __restrict__ dout, T cd, T cr, int mask,
                                           double& acc) {
  const int N = g.N, n = i + (g.nx + 1) * j;
  const bool fxd = fixed_x2(g, i, j), fyd = fixed_y2(g, i, j);
  if (MODE == M_APPLY) {
    const T yx = (mask && fxd) ? T(0) : fx;
    const T yy = (mask && fyd) ? T(0) : fy;
    y[n] = yx;
    y[n + N] = yy;
    if (RED == R_DOT) acc += (double)xc * yx + (double)yc * yy;
    if (RED == R_FREE2) {
      const double rx = (double)fx - (b ? (double)b[n] : 0.0);
      const double ry = (double)fy - (b ? (double)b[n + N] : 0.0);
      acc += (fxd ? 0.0 : rx * rx) + (fyd ? 0.0 : ry * ry);
    }
  } else if (MODE == M_RESID) {
    const T rx = fxd ? T(0) : (b ? b[n] : T(0)) - fx;
    const T ry = fyd ? T(0) : (b ? b[n + N] : T(0)) - fy;
    y[n] = rx;
    y[n + N] = ry;
    if (RED == R_DOT) acc += (double)rx * rx + (double)ry * ry;
  } else {
    const T rx = (b ? b[n] : T(0)) - fx, ry = (b ? b[n + N] : T(0)) - fy;
    T ddx = cr * rx / dx, ddy = cr * ry / dy;
    if (din) { ddx += cd * din[n]; ddy += cd * din[n + N]; }
    T xo = xc + ddx, yo = yc + ddy;
    if (fxd) { xo = T(0); ddx = T(0); }
    if (fyd) { yo = T(0); ddy = T(0); }
    y[n] = xo;
    y[n + N] = yo;
    if (dout) { dout[n] = ddx; dout[n + N] = ddy; }
  }
}

// ---------------------------------------------------------------------------
// column-blocked operator: one thread walks NB_Y consecutive nodes of a grid
// column, so that every element stress is formed once per thread and each
// grid row is loaded once (a sliding window of two rows in registers).
// ---------------------------------------------------------------------------

// Nodal values of grid row r at columns i-1, i, i+1 (zero outside the grid):
// displacement components and, on the finest level, alpha.
template <class T>
struct Row3 {
  T ux[3], uy[3], a[3];
};

template <bool FA, bool HASX, class T, class PR = NoProl>
__device__ __forceinline__ void load_row3(const Grid& g, const T* __restrict__ x,
                                          const T* __restrict__ coef, int i, int r, Row3<T>& R,
                                          const PR& pr = PR()) {
  const int W = g.nx + 1, N = g.N;
  const bool ok = r >= 0 && r <= g.ny;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ii = i - 1 + k;
    const bool in = ok && ii >= 0 && ii <= g.nx;
    const int n = ii + W * r;
    R.ux[k] = (HASX && in) ? x[n] : T(0);
    R.uy[k] = (HASX && in) ? x[n + N] : T(0);
    if (in) add_prol(g, pr, ii, r, R.ux[k], R.uy[k]);
    R.a[k] = (FA && in) ? coef[n] : T(0);
  }
}

// Forces (K x, or K x - f with the thermal-shock eigenstrain load when EIG)
// and, when DIAG, diagonal entries of K at nodes (i, j) for
// j = j0 .. min(j0 + ROWS - 1, ny); fin(j, fx, fy, dx, dy, x_x, x_y) receives
// each node's values (x_x, x_y: x at the node, zero without HASX).
// The cells of row cj left and right of the column, L = (i-1, cj) and
// C = (i, cj), hold the four triangles the column's nodes share:
//   L.T0 = [(i-1,cj), (i,cj), (i,cj+1)]      -> node (i,cj) as vertex 1, (i,cj+1) as vertex 2
//   L.T1 = [(i-1,cj), (i,cj+1), (i-1,cj+1)]  -> node (i,cj+1) as vertex 1
//   C.T0 = [(i,cj), (i+1,cj), (i+1,cj+1)]    -> node (i,cj) as vertex 0
//   C.T1 = [(i,cj), (i+1,cj+1), (i,cj+1)]    -> node (i,cj) as vertex 0, (i,cj+1) as vertex 2
// (the six triangles around a node are the three above it in cell row j and
// the three below it in cell row j-1).  pr: what the row loads add to x
// (NoProl, or AddProl: x + P x_c).  Precondition: 0 <= i <= nx,
// 0 <= j0 <= ny.
template <int ROWS, bool FA, bool HASX, bool DIAG, bool EIG, class T, class Fin,
          class PR = NoProl>
__device__ __forceinline__ void column2d(const Grid& g, const Mat& m, const T* __restrict__ coef,
                                         T kell, const T* __restrict__ x, int i, int j0,
                                         Fin&& fin, const PR& pr = PR()) {
  const T ihx = T(1.0 / g.hx), ihy = T(1.0 / g.hy), area = T(0.5 * g.hx * g.hy);
  const T l2m = T(m.l2m), lam = T(m.lam), mu = T(m.mu);
  const T hxx = ihx * ihx, hyy = ihy * ihy;
  const bool hasL = i >= 1, hasC = i < g.nx;
  const int nx = g.nx;
  Row3<T> lo, hi;
  load_row3<FA, HASX>(g, x, coef, i, j0 - 1, lo, pr);
  T fcx = 0, fcy = 0, dcx = 0, dcy = 0;   // node (i, cj)
  T fnx = 0, fny = 0, dnx = 0, dny = 0;   // node (i, cj + 1)
#pragma unroll
  for (int s = 0; s <= ROWS; ++s) {
    const int cj = j0 - 1 + s;
    if (cj > g.ny) break;
    load_row3<FA, HASX>(g, x, coef, i, cj + 1, hi, pr);
    T s0 = 0, s1 = 0;   // eigenstrain of the row's T0 / T1 triangles (EIG)
    if (EIG) {
      double e0, e1;
      eig_row2d(g, cj, e0, e1);
      s0 = T(e0); s1 = T(e1);
    }
    if (cj >= 0 && cj < g.ny) {
      if (hasL) {
        const T wl0 = area * (FA ? abar3(lo.a[0], lo.a[1], hi.a[1], kell) : coef[2 * (i - 1 + nx * cj)]);
        const T wl1 = area * (FA ? abar3(lo.a[0], hi.a[1], hi.a[0], kell) : coef[2 * (i - 1 + nx * cj) + 1]);
        T sxx = 0, syy = 0, sxy = 0, txx = 0, txy = 0;
        if (HASX) {
          // L.T0 strain: grads (-1/hx, 0), (1/hx, -1/hy), (0, 1/hy)
          const T exx = (lo.ux[1] - lo.ux[0]) * ihx - s0, eyy = (hi.uy[1] - lo.uy[1]) * ihy - s0;
          const T gam = (hi.ux[1] - lo.ux[1]) * ihy + (lo.uy[1] - lo.uy[0]) * ihx;
          sxx = l2m * exx + lam * eyy; syy = lam * exx + l2m * eyy; sxy = mu * gam;
          // L.T1 strain: grads (0, -1/hy), (1/hx, 0), (-1/hx, 1/hy)
          const T fxx = (hi.ux[1] - hi.ux[0]) * ihx - s1, fyy = (hi.uy[0] - lo.uy[0]) * ihy - s1;
          const T fam = (hi.ux[0] - lo.ux[0]) * ihy + (hi.uy[1] - hi.uy[0]) * ihx;
          txx = l2m * fxx + lam * fyy; txy = mu * fam;
        }
        // L.T0 -> (i,cj) vertex 1 (1/hx, -1/hy); (i,cj+1) vertex 2 (0, 1/hy)
        fcx += wl0 * (sxx * ihx - sxy * ihy);
        fcy += wl0 * (sxy * ihx - syy * ihy);
        fnx += wl0 * (sxy * ihy);
        fny += wl0 * (syy * ihy);
        // L.T1 -> (i,cj+1) vertex 1 (1/hx, 0)
        fnx += wl1 * (txx * ihx);
        fny += wl1 * (txy * ihx);
        if (DIAG) {
          dcx += wl0 * (l2m * hxx + mu * hyy);
          dcy += wl0 * (l2m * hyy + mu * hxx);
          dnx += wl0 * mu * hyy + wl1 * l2m * hxx;
          dny += wl0 * l2m * hyy + wl1 * mu * hxx;
        }
      }
      if (hasC) {
        const T wc0 = area * (FA ? abar3(lo.a[1], lo.a[2], hi.a[2], kell) : coef[2 * (i + nx * cj)]);
        const T wc1 = area * (FA ? abar3(lo.a[1], hi.a[2], hi.a[1], kell) : coef[2 * (i + nx * cj) + 1]);
        T sxx = 0, sxy = 0, txx = 0, tyy = 0, txy = 0;
        if (HASX) {
          // C.T0 strain
          const T exx = (lo.ux[2] - lo.ux[1]) * ihx - s0, eyy = (hi.uy[2] - lo.uy[2]) * ihy - s0;
          const T gam = (hi.ux[2] - lo.ux[2]) * ihy + (lo.uy[2] - lo.uy[1]) * ihx;
          sxx = l2m * exx + lam * eyy; sxy = mu * gam;
          // C.T1 strain
          const T fxx = (hi.ux[2] - hi.ux[1]) * ihx - s1, fyy = (hi.uy[1] - lo.uy[1]) * ihy - s1;
          const T fam = (hi.ux[1] - lo.ux[1]) * ihy + (hi.uy[2] - hi.uy[1]) * ihx;
          txx = l2m * fxx + lam * fyy; tyy = lam * fxx + l2m * fyy; txy = mu * fam;
        }
        // C.T0 -> (i,cj) vertex 0 (-1/hx, 0)
        fcx -= wc0 * (sxx * ihx);
        fcy -= wc0 * (sxy * ihx);
        // C.T1 -> (i,cj) vertex 0 (0, -1/hy); (i,cj+1) vertex 2 (-1/hx, 1/hy)
        fcx -= wc1 * (txy * ihy);
        fcy -= wc1 * (tyy * ihy);
        fnx += wc1 * (txy * ihy - txx * ihx);
        fny += wc1 * (tyy * ihy - txy * ihx);
        if (DIAG) {
          dcx += wc0 * l2m * hxx + wc1 * mu * hyy;
          dcy += wc0 * mu * hxx + wc1 * l2m * hyy;
          dnx += wc1 * (l2m * hxx + mu * hyy);
          dny += wc1 * (l2m * hyy + mu * hxx);
        }
      }
    }
    if (s >= 1) fin(cj, fcx, fcy, dcx, dcy, lo.ux[1], lo.uy[1]);
    fcx = fnx; fcy = fny; dcx = dnx; dcy = dny;
    fnx = fny = dnx = dny = T(0);
    lo = hi;
  }
}

// b_c(I,J) = (P^T r_f)(I,J): the coincident fine node plus half of the six
// fine nodes at the midpoints of the coarse edges through (I,J).
template <class T>
__device__ __forceinline__ void restrict_node2d(const Grid& gf, const Grid& gc,
                                                const T* __restrict__ rf, T* __restrict__ bc,
                                                int I, int J) {
  const int Wf = gf.nx + 1, Nf = gf.N, fi = 2 * I, fj = 2 * J, f = fi + Wf * fj;
  const int nc = I + (gc.nx + 1) * J;
  for (int comp = 0; comp < 2; ++comp) {
    const T* r = rf + comp * Nf;
    T s = r[f];
    T h = 0;
    if (fi > 0) h += r[f - 1];
    if (fi < gf.nx) h += r[f + 1];
    if (fj > 0) h += r[f - Wf];
    if (fj < gf.ny) h += r[f + Wf];
    if (fi < gf.nx && fj < gf.ny) h += r[f + 1 + Wf];
    if (fi > 0 && fj > 0) h += r[f - 1 - Wf];
    s += T(0.5) * h;
    const bool fixed = comp == 0 ? fixed_x2(gc, I, J) : fixed_y2(gc, I, J);
    bc[comp * gc.N + nc] = fixed ? T(0) : s;
  }
}

// x_f(i,j) += (P x_c)(i,j): the coarse value at a coincident node, else the
// mean of the two ends of the coarse edge (x, y or diagonal) holding it.
template <class T>
__device__ __forceinline__ void prolong_node2d(const Grid& gf, const Grid& gc,
                                               const T* __restrict__ xc, T* __restrict__ xf,
                                               int i, int j) {
  const int Wc = gc.nx + 1, n = i + (gf.nx + 1) * j;
  const int I0 = i >> 1, J0 = j >> 1, I1 = (i + 1) >> 1, J1 = (j + 1) >> 1;
  for (int comp = 0; comp < 2; ++comp) {
    const T* c = xc + comp * gc.N;
    const T v = T(0.5) * (c[I0 + Wc * J0] + c[I1 + Wc * J1]);
    const bool fixed = comp == 0 ? fixed_x2(gf, i, j) : fixed_y2(gf, i, j);
    if (!fixed) xf[comp * gf.N + n] += v;
  }
}

}  // namespace frac
