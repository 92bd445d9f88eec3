// Per-node device code of the 2D operator (right-diagonal P1 triangles),
// shared by the stencil kernels and the fused coarse-level kernel.
#pragma once

#include "common.h"

namespace frac {

// ---------------------------------------------------------------------------
// boundary conditions
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool fixed_x2(const Grid& g, int i, int j) {
  return (g.bc == BC_TENSION_2D) && i == 0 && j == 0;
}
__device__ __forceinline__ bool fixed_y2(const Grid& g, int i, int j) {
  return (g.bc == BC_TENSION_2D) && (j == 0 || j == g.ny);
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

// Force (fx, fy) = (K x) at node (i, j) and, when DIAG, the diagonal entries
// (dx, dy) of K for the node's two DOFs.
template <bool HASX, bool DIAG, class T>
__device__ __forceinline__ void node_force2d(const Grid& g, const Mat& m, const T c[6],
                                             const T* __restrict__ ux, const T* __restrict__ uy,
                                             int i, int j, T& fx, T& fy, T& dx, T& dy) {
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
  fx = fy = dx = dy = T(0);
  const T hxx = ihx * ihx, hyy = ihy * ihy;
  // (a) cell(i,j) T0: node is vertex 0, gradient (-1/hx, 0)
  if (R && U) {
    const T w = c[0] * area;
    if (HASX) {
      const T exx = (ex - cx) * ihx, eyy = (ney - ey) * ihy;
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
      const T exx = (nex - nnx) * ihx, eyy = (nny - cy) * ihy;
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
      const T exx = (cx - wx) * ihx, eyy = (nny - cy) * ihy;
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
      const T exx = (sx - swx) * ihx, eyy = (cy - sy) * ihy;
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
      const T exx = (cx - wx) * ihx, eyy = (wy - swy) * ihy;
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
      const T exx = (ex - cx) * ihx, eyy = (cy - sy) * ihy;
      const T gam = (ey - cy) * ihx + (cx - sx) * ihy;
      const T sxx = l2m * exx + lam * eyy, syy = lam * exx + l2m * eyy, sxy = mu * gam;
      fx += w * (-sxx * ihx + sxy * ihy);
      fy += w * (-sxy * ihx + syy * ihy);
    }
    if (DIAG) { dx += w * (l2m * hxx + mu * hyy); dy += w * (l2m * hyy + mu * hxx); }
  }
}

// ---------------------------------------------------------------------------
// per-node multigrid updates (one node (i, j) of level g)
// ---------------------------------------------------------------------------

// One Jacobi-Chebyshev step at a node: d = cd d_in + cr D^{-1}(b - K x_in),
// x_out = x_in + d (x_in == nullptr: zero iterate).  FA: coefficients from
// nodal alpha.
template <bool FA, class T>
__device__ __forceinline__ void smooth_node2d(const Grid& g, const Mat& m, const T* __restrict__ coef,
                                              T kell, const T* __restrict__ x_in,
                                              T* __restrict__ x_out, const T* __restrict__ b,
                                              const T* __restrict__ d_in, T* __restrict__ d_out,
                                              T cd, T cr, int i, int j) {
  const int N = g.N, n = i + (g.nx + 1) * j;
  T c[6];
  coef6<FA>(g, coef, kell, i, j, c);
  T fx = 0, fy = 0, dx, dy;
  if (x_in) node_force2d<true, true>(g, m, c, x_in, x_in + N, i, j, fx, fy, dx, dy);
  else node_force2d<false, true>(g, m, c, x_in, x_in, i, j, fx, fy, dx, dy);
  T ddx = cr * (b[n] - fx) / dx, ddy = cr * (b[n + N] - fy) / dy;
  if (d_in) { ddx += cd * d_in[n]; ddy += cd * d_in[n + N]; }
  T xo = (x_in ? x_in[n] : T(0)) + ddx, yo = (x_in ? x_in[n + N] : T(0)) + ddy;
  if (fixed_x2(g, i, j)) { xo = T(0); ddx = T(0); }
  if (fixed_y2(g, i, j)) { yo = T(0); ddy = T(0); }
  x_out[n] = xo;
  x_out[n + N] = yo;
  if (d_out) { d_out[n] = ddx; d_out[n + N] = ddy; }
}

template <bool FA, class T>
__device__ __forceinline__ void resid_node2d(const Grid& g, const Mat& m, const T* __restrict__ coef,
                                             T kell, const T* __restrict__ x, T* __restrict__ r,
                                             const T* __restrict__ b, int i, int j) {
  const int N = g.N, n = i + (g.nx + 1) * j;
  T c[6];
  coef6<FA>(g, coef, kell, i, j, c);
  T fx, fy, dx, dy;
  node_force2d<true, false>(g, m, c, x, x + N, i, j, fx, fy, dx, dy);
  r[n] = fixed_x2(g, i, j) ? T(0) : b[n] - fx;
  r[n + N] = fixed_y2(g, i, j) ? T(0) : b[n + N] - fy;
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
