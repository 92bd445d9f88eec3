// Per-node device code of the 3D operator (Kuhn P1 tetrahedra), shared by the
// stencil kernels and the fused coarse-level kernel.
#pragma once

#include "common.h"

namespace frac {

template <int P> struct Perm3;
template <> struct Perm3<0> { static constexpr int a = 0, b = 1, c = 2; };
template <> struct Perm3<1> { static constexpr int a = 0, b = 2, c = 1; };
template <> struct Perm3<2> { static constexpr int a = 1, b = 0, c = 2; };
template <> struct Perm3<3> { static constexpr int a = 1, b = 2, c = 0; };
template <> struct Perm3<4> { static constexpr int a = 2, b = 0, c = 1; };
template <> struct Perm3<5> { static constexpr int a = 2, b = 1, c = 0; };

// offset of local vertex W of tetrahedron P along axis AX
template <int P, int W, int AX>
struct VOff {
  static constexpr int v = W == 0 ? 0
                           : W == 3 ? 1
                           : W == 1 ? (AX == Perm3<P>::a ? 1 : 0)
                                    : ((AX == Perm3<P>::a || AX == Perm3<P>::b) ? 1 : 0);
};

// slot of the 3x3x3 neighbourhood for a node offset (dx, dy, dz) in {-1,0,1}^3
constexpr int nslot(int dx, int dy, int dz) { return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1); }

template <int HX, int HY, int HZ, int P, int W>
struct VSlot {
  static constexpr int v = nslot(HX + VOff<P, W, 0>::v, HY + VOff<P, W, 1>::v, HZ + VOff<P, W, 2>::v);
};

__device__ __forceinline__ bool fixed3(const Grid& g, int comp, int i, int j, int k) {
  if (g.bc != BC_THERMAL_3D) return false;
  if (i != g.nx) return false;
  if (comp == 0) return true;
  if (comp == 1) return j == 0 && k == 0;
  return k == 0 && (j == 0 || j == g.ny);
}

// Per-node neighbourhood: the 15 nodes the Kuhn stencil touches, loaded once.
template <class T>
struct Hood3 {
  T u[27][3];
  T a[27];
};

__device__ __forceinline__ bool in3(const Grid& g, int i, int j, int k) {
  return i >= 0 && j >= 0 && k >= 0 && i <= g.nx && j <= g.ny && k <= g.nz;
}

// the 15 stencil offsets (0, +-e_a, +-(e_a+e_b), +-(1,1,1))
#define FOR_STENCIL3(X)                                                                 \
  X(0, 0, 0) X(1, 0, 0) X(-1, 0, 0) X(0, 1, 0) X(0, -1, 0) X(0, 0, 1) X(0, 0, -1)       \
  X(1, 1, 0) X(-1, -1, 0) X(1, 0, 1) X(-1, 0, -1) X(0, 1, 1) X(0, -1, -1) X(1, 1, 1)    \
  X(-1, -1, -1)

// The 24 (hex offset, tetrahedron, local vertex) incidences of a node.
#define FOR_TETS3(X)                                                                     \
  X(-1, -1, -1, 0, 3) X(-1, -1, -1, 1, 3) X(-1, -1, -1, 2, 3) X(-1, -1, -1, 3, 3)       \
  X(-1, -1, -1, 4, 3) X(-1, -1, -1, 5, 3) X(-1, -1, 0, 0, 2) X(-1, -1, 0, 2, 2)         \
  X(-1, 0, -1, 1, 2) X(-1, 0, -1, 4, 2) X(-1, 0, 0, 0, 1) X(-1, 0, 0, 1, 1)             \
  X(0, -1, -1, 3, 2) X(0, -1, -1, 5, 2) X(0, -1, 0, 2, 1) X(0, -1, 0, 3, 1)             \
  X(0, 0, -1, 4, 1) X(0, 0, -1, 5, 1) X(0, 0, 0, 0, 0) X(0, 0, 0, 1, 0) X(0, 0, 0, 2, 0) \
  X(0, 0, 0, 3, 0) X(0, 0, 0, 4, 0) X(0, 0, 0, 5, 0)

template <class T>
__device__ __forceinline__ T abar4(T a0, T a1, T a2, T a3, T k) {
  const T b0 = T(1) - a0, b1 = T(1) - a1, b2 = T(1) - a2, b3 = T(1) - a3;
  const T s = b0 + b1 + b2 + b3;
  return k + (b0 * b0 + b1 * b1 + b2 * b2 + b3 * b3 + s * s) * (T(1) / T(20));
}

// Gradient of local vertex W of tetrahedron P (axis components).
template <int P, int W, class T>
__device__ __forceinline__ void grad3(const T ih[3], T g[3]) {
  constexpr int A = Perm3<P>::a, B = Perm3<P>::b, C = Perm3<P>::c;
  g[0] = g[1] = g[2] = T(0);
  if (W == 0) g[A] = -ih[A];
  if (W == 1) { g[A] = ih[A]; g[B] = -ih[B]; }
  if (W == 2) { g[B] = ih[B]; g[C] = -ih[C]; }
  if (W == 3) g[C] = ih[C];
}

// Voigt-free strain of a tetrahedron: displacement gradient G[comp][axis].
template <int HX, int HY, int HZ, int P, class T>
__device__ __forceinline__ void tet_grad(const T (&u)[27][3], const T ih[3], T G[3][3]) {
  constexpr int A = Perm3<P>::a, B = Perm3<P>::b, C = Perm3<P>::c;
  constexpr int s0 = VSlot<HX, HY, HZ, P, 0>::v, s1 = VSlot<HX, HY, HZ, P, 1>::v;
  constexpr int s2 = VSlot<HX, HY, HZ, P, 2>::v, s3 = VSlot<HX, HY, HZ, P, 3>::v;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    G[c][A] = (u[s1][c] - u[s0][c]) * ih[A];
    G[c][B] = (u[s2][c] - u[s1][c]) * ih[B];
    G[c][C] = (u[s3][c] - u[s2][c]) * ih[C];
  }
}

// x coordinate of the tetrahedron's centroid, in cells from the hex corner
template <int P>
__device__ __forceinline__ double tet_xc() {
  return 0.25 * (VOff<P, 1, 0>::v + VOff<P, 2, 0>::v + 1.0);
}

template <int HX, int HY, int HZ, int P, int V, bool FA, bool HASX, bool DIAG, bool EIG, class T>
__device__ __forceinline__ void tet_force(const Grid& g, const Mat& m, const Hood3<T>& hd,
                                          const T* __restrict__ abar, T kell, int i, int j, int k,
                                          const T ih[3], T vol, T f[3], T d[3]) {
  const int ci = i + HX, cj = j + HY, ck = k + HZ;
  if (ci < 0 || cj < 0 || ck < 0 || ci >= g.nx || cj >= g.ny || ck >= g.nz) return;
  T c;
  if (FA) {
    c = abar4(hd.a[VSlot<HX, HY, HZ, P, 0>::v], hd.a[VSlot<HX, HY, HZ, P, 1>::v],
              hd.a[VSlot<HX, HY, HZ, P, 2>::v], hd.a[VSlot<HX, HY, HZ, P, 3>::v], kell);
  } else {
    c = abar[6 * (ci + g.nx * (cj + g.ny * ck)) + P];
  }
  const T w = c * vol;
  T gv[3];
  grad3<P, V>(ih, gv);
  const T lam = T(m.lam), mu = T(m.mu);
  if (HASX) {
    T G[3][3];
    tet_grad<HX, HY, HZ, P>(hd.u, ih, G);
    T e0 = G[0][0], e1 = G[1][1], e2 = G[2][2];
    if (EIG) {
      const double xc = (ci + tet_xc<P>()) * g.hx;
      const T s = T(-g.eig_dT * exp(-xc / g.eig_depth));
      e0 -= s; e1 -= s; e2 -= s;
    }
    const T tr = e0 + e1 + e2;
    T S[3][3];
    S[0][0] = lam * tr + T(2) * mu * e0;
    S[1][1] = lam * tr + T(2) * mu * e1;
    S[2][2] = lam * tr + T(2) * mu * e2;
    S[0][1] = S[1][0] = mu * (G[0][1] + G[1][0]);
    S[0][2] = S[2][0] = mu * (G[0][2] + G[2][0]);
    S[1][2] = S[2][1] = mu * (G[1][2] + G[2][1]);
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] += w * (S[a][0] * gv[0] + S[a][1] * gv[1] + S[a][2] * gv[2]);
  }
  if (DIAG) {
    const T gg = gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] += w * ((lam + mu) * gv[a] * gv[a] + mu * gg);
  }
}

template <bool FA, bool HASX, bool DIAG, bool EIG, class T>
__device__ __forceinline__ void node_force3d(const Grid& g, const Mat& m, const T* __restrict__ coef,
                                             T kell, const T* __restrict__ x, int i, int j, int k,
                                             T f[3], T d[3]) {
  const int W = g.nx + 1, H = g.ny + 1, N = g.N;
  const int n = i + W * (j + H * k);
  Hood3<T> hd;
#define LOAD3(DX, DY, DZ)                                                                   \
  {                                                                                         \
    constexpr int sl = nslot(DX, DY, DZ);                                                   \
    const bool ok = in3(g, i + DX, j + DY, k + DZ);                                         \
    const int nn = n + DX + W * (DY + H * DZ);                                              \
    if (HASX) {                                                                             \
      hd.u[sl][0] = ok ? x[nn] : T(0);                                                      \
      hd.u[sl][1] = ok ? x[nn + N] : T(0);                                                  \
      hd.u[sl][2] = ok ? x[nn + 2 * N] : T(0);                                              \
    }                                                                                       \
    if (FA) hd.a[sl] = ok ? coef[nn] : T(0);                                                \
  }
  FOR_STENCIL3(LOAD3)
#undef LOAD3
  const T ih[3] = {T(1.0 / g.hx), T(1.0 / g.hy), T(1.0 / g.hz)};
  const T vol = T(g.hx * g.hy * g.hz / 6.0);
  f[0] = f[1] = f[2] = d[0] = d[1] = d[2] = T(0);
#define TET3(HX, HY, HZ, P, V) \
  tet_force<HX, HY, HZ, P, V, FA, HASX, DIAG, EIG>(g, m, hd, coef, kell, i, j, k, ih, vol, f, d);
  FOR_TETS3(TET3)
#undef TET3
}

// positive edge directions of the Kuhn mesh (the interpolation stencil)
static __device__ __constant__ int c_kuhn_dir[7][3] = {{1,0,0},{0,1,0},{0,0,1},{1,1,0},{1,0,1},{0,1,1},{1,1,1}};

// ---------------------------------------------------------------------------
// per-node transfers between levels (node of the coarse or the fine level)
// ---------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ void restrict_node3d(const Grid& gf, const Grid& gc,
                                                const T* __restrict__ rf, T* __restrict__ bc,
                                                int I, int J, int K) {
  const int Wf = gf.nx + 1, Hf = gf.ny + 1, fi = 2 * I, fj = 2 * J, fk = 2 * K;
  const int f = fi + Wf * (fj + Hf * fk);
  const int nc = I + (gc.nx + 1) * (J + (gc.ny + 1) * K);
  for (int comp = 0; comp < 3; ++comp) {
    const T* r = rf + comp * gf.N;
    T s = r[f], h = 0;
    for (int q = 0; q < 7; ++q) {
      const int dx = c_kuhn_dir[q][0], dy = c_kuhn_dir[q][1], dz = c_kuhn_dir[q][2];
      const int off = dx + Wf * (dy + Hf * dz);
      if (in3(gf, fi + dx, fj + dy, fk + dz)) h += r[f + off];
      if (in3(gf, fi - dx, fj - dy, fk - dz)) h += r[f - off];
    }
    s += T(0.5) * h;
    bc[comp * gc.N + nc] = fixed3(gc, comp, I, J, K) ? T(0) : s;
  }
}

template <class T>
__device__ __forceinline__ void prolong_node3d(const Grid& gf, const Grid& gc,
                                               const T* __restrict__ xc, T* __restrict__ xf,
                                               int i, int j, int k) {
  const int Wc = gc.nx + 1, Hc = gc.ny + 1;
  const int n = i + (gf.nx + 1) * (j + (gf.ny + 1) * k);
  const int c0 = (i >> 1) + Wc * ((j >> 1) + Hc * (k >> 1));
  const int c1 = ((i + 1) >> 1) + Wc * (((j + 1) >> 1) + Hc * ((k + 1) >> 1));
  for (int comp = 0; comp < 3; ++comp) {
    const T* c = xc + comp * gc.N;
    if (!fixed3(gf, comp, i, j, k)) xf[comp * gf.N + n] += T(0.5) * (c[c0] + c[c1]);
  }
}

}  // namespace frac
