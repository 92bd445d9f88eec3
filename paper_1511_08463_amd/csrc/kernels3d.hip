// 3D kernels: P1 Kuhn tetrahedra on a structured grid of hexahedra.
//
// Hexahedron (ci, cj, ck) holds six tetrahedra, one per permutation
// (a, b, c) of the axes (order 012, 021, 102, 120, 201, 210): vertices
// o0 = 0, o1 = e_a, o2 = e_a + e_b, o3 = (1,1,1).  Barycentric gradients are
// g0 = -e_a/h_a, g1 = e_a/h_a - e_b/h_b, g2 = e_b/h_b - e_c/h_c, g3 = e_c/h_c,
// so the displacement gradient along axis a is a difference along the path
// o0 -> o1, along b along o1 -> o2 and along c along o2 -> o3.  Volume
// hx hy hz / 6.  Element e = 6 (ci + nx (cj + ny ck)) + p.
//
// A node lies in 24 tetrahedra; the node kernels sum their forces, enumerated
// at compile time (template parameters) so every stencil index is a
// constant.  The eigenstrain of the thermal load enters as
// eps_eff = eps(u) - s I with s = -DT exp(-x_c/depth) at the element centroid.
#include "common.h"
#include "launch.h"
#include "ops3d.h"

namespace frac {

// ---------------------------------------------------------------------------
// node kernels (apply / residual / Chebyshev step), value type T
// ---------------------------------------------------------------------------

enum { M3_APPLY = 0, M3_RESID = 1, M3_SMOOTH = 2 };
enum { R3_NONE = 0, R3_DOT = 1, R3_FREE2 = 2 };

template <int MODE, bool FA, bool HASX, int RED, bool EIG, class T>
__global__ __launch_bounds__(NB) void k_node3d(Grid g, Mat m, const T* __restrict__ coef, T kell,
                                               const T* __restrict__ x, T* __restrict__ y,
                                               const T* __restrict__ b, const T* __restrict__ din,
                                               T* __restrict__ dout, T cd, T cr, int mask, Red red) {
  const int i = blockIdx.x * NB_X + threadIdx.x;
  const int j = blockIdx.y * NB_Y + threadIdx.y;
  const int k = blockIdx.z;
  double acc = 0.0;
  if (i <= g.nx && j <= g.ny) {
    const int N = g.N, n = i + (g.nx + 1) * (j + (g.ny + 1) * k);
    T f[3], d[3];
    node_force3d<FA, HASX, MODE == M3_SMOOTH, EIG>(g, m, coef, kell, x, i, j, k, f, d);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fx = fixed3(g, c, i, j, k);
      const int q = n + c * N;
      if (MODE == M3_APPLY) {
        const T yv = (mask && fx) ? T(0) : f[c];
        y[q] = yv;
        if (RED == R3_DOT) acc += (double)x[q] * yv;
        if (RED == R3_FREE2) {
          const double r = (double)f[c] - (b ? (double)b[q] : 0.0);
          acc += fx ? 0.0 : r * r;
        }
      } else if (MODE == M3_RESID) {
        const T r = fx ? T(0) : (b ? b[q] : T(0)) - f[c];
        y[q] = r;
        if (RED == R3_DOT) acc += (double)r * r;
      } else {
        const T r = (b ? b[q] : T(0)) - f[c];
        T dd = cr * r / d[c];
        if (din) dd += cd * din[q];
        T xo = (HASX ? x[q] : T(0)) + dd;
        if (fx) { xo = T(0); dd = T(0); }
        y[q] = xo;
        if (dout) dout[q] = dd;
      }
    }
  }
  if (RED != R3_NONE)
    block_reduce<NB, false>(acc, red, gridDim.x * gridDim.y * gridDim.z,
                            blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                            threadIdx.x + NB_X * threadIdx.y);
}

static dim3 node_grid3(const Grid& g) {
  return dim3((g.nx + 1 + NB_X - 1) / NB_X, (g.ny + 1 + NB_Y - 1) / NB_Y, g.nz + 1);
}

int node_blocks3(const Grid& g) {
  dim3 gr = node_grid3(g);
  return (int)(gr.x * gr.y * gr.z);
}

template <class T>
void launch_apply3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* y, const ND<T>* b, int mask, int red, Red r) {
  dim3 gr = node_grid3(g), bl(NB_X, NB_Y);
  const T k = T(kell);
  const bool eig = fine && g.eig_dT != 0.0;
#define A3(FA, RD, EG) \
  hipLaunchKernelGGL((k_node3d<M3_APPLY, FA, true, RD, EG, T>), gr, bl, 0, st, g, m, coef, k, x, y, b, \
                     (const T*)nullptr, (T*)nullptr, T(0), T(0), mask, r)
  if (fine && eig) {
    if (red == R3_NONE) A3(true, R3_NONE, true);
    else if (red == R3_DOT) A3(true, R3_DOT, true);
    else A3(true, R3_FREE2, true);
  } else if (fine) {
    if (red == R3_NONE) A3(true, R3_NONE, false);
    else if (red == R3_DOT) A3(true, R3_DOT, false);
    else A3(true, R3_FREE2, false);
  } else {
    if (red == R3_NONE) A3(false, R3_NONE, false);
    else if (red == R3_DOT) A3(false, R3_DOT, false);
    else A3(false, R3_FREE2, false);
  }
#undef A3
  if (red != R3_NONE) launch_finish(st, r, (int)(gr.x * gr.y * gr.z), false);
}

template <class T>
void launch_resid3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* r, const ND<T>* b, bool red, Red rr) {
  dim3 gr = node_grid3(g), bl(NB_X, NB_Y);
  const T k = T(kell);
  const bool eig = fine && g.eig_dT != 0.0;
#define R3(FA, RD, EG) \
  hipLaunchKernelGGL((k_node3d<M3_RESID, FA, true, RD, EG, T>), gr, bl, 0, st, g, m, coef, k, x, r, b, \
                     (const T*)nullptr, (T*)nullptr, T(0), T(0), 1, rr)
  if (fine) {
    if (eig) { if (red) R3(true, R3_DOT, true); else R3(true, R3_NONE, true); }
    else { if (red) R3(true, R3_DOT, false); else R3(true, R3_NONE, false); }
  } else {
    if (red) R3(false, R3_DOT, false); else R3(false, R3_NONE, false);
  }
#undef R3
  if (red) launch_finish(st, rr, (int)(gr.x * gr.y * gr.z), false);
}

template <class T>
void launch_smooth3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                     double kell, const ND<T>* x_in, T* x_out, const T* b, const ND<T>* d_in,
                     ND<T>* d_out, double cd, double cr) {
  dim3 gr = node_grid3(g), bl(NB_X, NB_Y);
  Red none{};
  const T k = T(kell);
#define S3(FA, HX) \
  hipLaunchKernelGGL((k_node3d<M3_SMOOTH, FA, HX, R3_NONE, false, T>), gr, bl, 0, st, g, m, coef, k, \
                     x_in, x_out, b, d_in, d_out, T(cd), T(cr), 1, none)
  if (fine) { if (x_in) S3(true, true); else S3(true, false); }
  else { if (x_in) S3(false, true); else S3(false, false); }
#undef S3
}

// ---------------------------------------------------------------------------
// transfers
// ---------------------------------------------------------------------------

// The Kuhn triangulation of the half-size grid refines that of the coarse
// grid: each coarse tetrahedron is the union of 8 fine ones.  Children of
// coarse tetrahedron p: (fine hex offset x, y, z in {0,1}, fine permutation).
__device__ __constant__ int c_kuhn_kids[6][8][4] = {
  {{0,0,0,0}, {1,0,0,0}, {1,0,0,2}, {1,0,0,3}, {1,1,0,0}, {1,1,0,1}, {1,1,0,4}, {1,1,1,0}},
  {{0,0,0,1}, {1,0,0,1}, {1,0,0,4}, {1,0,0,5}, {1,0,1,0}, {1,0,1,1}, {1,0,1,2}, {1,1,1,1}},
  {{0,0,0,2}, {0,1,0,0}, {0,1,0,1}, {0,1,0,2}, {1,1,0,2}, {1,1,0,3}, {1,1,0,5}, {1,1,1,2}},
  {{0,0,0,3}, {0,1,0,3}, {0,1,0,4}, {0,1,0,5}, {0,1,1,0}, {0,1,1,2}, {0,1,1,3}, {1,1,1,3}},
  {{0,0,0,4}, {0,0,1,0}, {0,0,1,1}, {0,0,1,4}, {1,0,1,3}, {1,0,1,4}, {1,0,1,5}, {1,1,1,4}},
  {{0,0,0,5}, {0,0,1,2}, {0,0,1,3}, {0,0,1,5}, {0,1,1,1}, {0,1,1,4}, {0,1,1,5}, {1,1,1,5}},
};
// vertex offsets of the 6 tetrahedra: [perm][vertex][axis]
__device__ __constant__ int c_kuhn_off[6][4][3] = {
  {{0,0,0},{1,0,0},{1,1,0},{1,1,1}}, {{0,0,0},{1,0,0},{1,0,1},{1,1,1}},
  {{0,0,0},{0,1,0},{1,1,0},{1,1,1}}, {{0,0,0},{0,1,0},{0,1,1},{1,1,1}},
  {{0,0,0},{0,0,1},{1,0,1},{1,1,1}}, {{0,0,0},{0,0,1},{0,1,1},{1,1,1}},
};

template <bool FA>
__global__ __launch_bounds__(VB) void k_coarsen3d(Grid gf, const double* __restrict__ fine,
                                                  double kell, Grid gc, double* __restrict__ c64,
                                                  float* __restrict__ c32) {
  const int e = blockIdx.x * VB + threadIdx.x;
  const int ne = 6 * gc.nx * gc.ny * gc.nz;
  if (e >= ne) return;
  const int p = e % 6, hex = e / 6;
  const int I = hex % gc.nx, J = (hex / gc.nx) % gc.ny, K = hex / (gc.nx * gc.ny);
  const int W = gf.nx + 1, H = gf.ny + 1;
  double s = 0.0;
  for (int q = 0; q < 8; ++q) {
    const int fi = 2 * I + c_kuhn_kids[p][q][0], fj = 2 * J + c_kuhn_kids[p][q][1];
    const int fk = 2 * K + c_kuhn_kids[p][q][2], fp = c_kuhn_kids[p][q][3];
    if (FA) {
      double a[4];
      for (int v = 0; v < 4; ++v)
        a[v] = fine[(fi + c_kuhn_off[fp][v][0]) + W * ((fj + c_kuhn_off[fp][v][1]) + H * (fk + c_kuhn_off[fp][v][2]))];
      s += abar4(a[0], a[1], a[2], a[3], kell);
    } else {
      s += fine[6 * (fi + gf.nx * (fj + gf.ny * fk)) + fp];
    }
  }
  s *= 0.125;
  c64[e] = s;
  if (c32) c32[e] = (float)s;
}

void launch_coarsen3d(hipStream_t st, const Grid& gf, bool fine_is_alpha, const double* fine,
                      double kell, const Grid& gc, double* c64, float* c32) {
  const int ne = 6 * gc.nx * gc.ny * gc.nz;
  dim3 gr((ne + VB - 1) / VB), bl(VB);
  if (fine_is_alpha) hipLaunchKernelGGL((k_coarsen3d<true>), gr, bl, 0, st, gf, fine, kell, gc, c64, c32);
  else hipLaunchKernelGGL((k_coarsen3d<false>), gr, bl, 0, st, gf, fine, kell, gc, c64, c32);
}


template <class T>
__global__ __launch_bounds__(NB) void k_restrict3d(Grid gf, Grid gc, const T* __restrict__ rf,
                                                   T* __restrict__ bc) {
  const int I = blockIdx.x * NB_X + threadIdx.x, J = blockIdx.y * NB_Y + threadIdx.y, K = blockIdx.z;
  if (I > gc.nx || J > gc.ny) return;
  restrict_node3d(gf, gc, rf, bc, I, J, K);
}

template <class T>
void launch_restrict3d(hipStream_t st, const Grid& gf, const Grid& gc, const T* rf, T* bc) {
  hipLaunchKernelGGL((k_restrict3d<T>), node_grid3(gc), dim3(NB_X, NB_Y), 0, st, gf, gc, rf, bc);
}

template <class T>
__global__ __launch_bounds__(NB) void k_prolong3d(Grid gf, Grid gc, const T* __restrict__ xc,
                                                  T* __restrict__ xf) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y, k = blockIdx.z;
  if (i > gf.nx || j > gf.ny) return;
  prolong_node3d(gf, gc, xc, xf, i, j, k);
}

template <class T>
void launch_prolong3d(hipStream_t st, const Grid& gf, const Grid& gc, const T* xc, T* xf) {
  hipLaunchKernelGGL((k_prolong3d<T>), node_grid3(gf), dim3(NB_X, NB_Y), 0, st, gf, gc, xc, xf);
}

// Dirichlet values of the thermal problem are all zero.
__global__ __launch_bounds__(NB) void k_lift3d(Grid g, double* __restrict__ u) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y, k = blockIdx.z;
  if (i > g.nx || j > g.ny) return;
  const int n = i + (g.nx + 1) * (j + (g.ny + 1) * k);
  for (int c = 0; c < 3; ++c)
    if (fixed3(g, c, i, j, k)) u[c * g.N + n] = 0.0;
}

void launch_lift3d(hipStream_t st, const Grid& g, double* u) {
  hipLaunchKernelGGL(k_lift3d, node_grid3(g), dim3(NB_X, NB_Y), 0, st, g, u);
}

// ---------------------------------------------------------------------------
// damage side: W2 per tetrahedron, Helmholtz node operator, VI evaluation
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(VB) void k_w2_3d(Grid g, Mat m, const double* __restrict__ u,
                                              double* __restrict__ w2) {
  const int e = blockIdx.x * VB + threadIdx.x;
  if (e >= 6 * g.nx * g.ny * g.nz) return;
  const int p = e % 6, hex = e / 6;
  const int ci = hex % g.nx, cj = (hex / g.nx) % g.ny, ck = hex / (g.nx * g.ny);
  const int W = g.nx + 1, H = g.ny + 1, N = g.N;
  const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
  int nd[4];
  for (int v = 0; v < 4; ++v)
    nd[v] = (ci + c_kuhn_off[p][v][0]) + W * ((cj + c_kuhn_off[p][v][1]) + H * (ck + c_kuhn_off[p][v][2]));
  // axis visited by each path step o_v -> o_{v+1}
  int ax[3];
  for (int s = 0; s < 3; ++s)
    for (int a = 0; a < 3; ++a)
      if (c_kuhn_off[p][s + 1][a] != c_kuhn_off[p][s][a]) ax[s] = a;
  double G[3][3];
  for (int c = 0; c < 3; ++c)
    for (int s = 0; s < 3; ++s) G[c][ax[s]] = (u[nd[s + 1] + c * N] - u[nd[s] + c * N]) * ih[ax[s]];
  double e0 = G[0][0], e1 = G[1][1], e2 = G[2][2];
  if (g.eig_dT != 0.0) {
    const double xc = (ci + 0.25 * (c_kuhn_off[p][1][0] + c_kuhn_off[p][2][0] + 1)) * g.hx;
    const double s = -g.eig_dT * exp(-xc / g.eig_depth);
    e0 -= s; e1 -= s; e2 -= s;
  }
  const double g01 = G[0][1] + G[1][0], g02 = G[0][2] + G[2][0], g12 = G[1][2] + G[2][1];
  const double tr = e0 + e1 + e2;
  w2[e] = m.lam * tr * tr + 2.0 * m.mu * (e0 * e0 + e1 * e1 + e2 * e2) +
          m.mu * (g01 * g01 + g02 * g02 + g12 * g12);
}

void launch_w2_3d(hipStream_t st, const Grid& g, const Mat& m, const double* u, double* w2) {
  const int ne = 6 * g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_w2_3d, dim3((ne + VB - 1) / VB), dim3(VB), 0, st, g, m, u, w2);
}

struct Helm3 {
  double cL, cM, cm;
};

// the 24 tetrahedra around a node as runtime data (damage kernels)
__device__ __constant__ int c_tets3[24][5] = {
  {-1,-1,-1,0,3},{-1,-1,-1,1,3},{-1,-1,-1,2,3},{-1,-1,-1,3,3},{-1,-1,-1,4,3},{-1,-1,-1,5,3},
  {-1,-1,0,0,2},{-1,-1,0,2,2},{-1,0,-1,1,2},{-1,0,-1,4,2},{-1,0,0,0,1},{-1,0,0,1,1},
  {0,-1,-1,3,2},{0,-1,-1,5,2},{0,-1,0,2,1},{0,-1,0,3,1},{0,0,-1,4,1},{0,0,-1,5,1},
  {0,0,0,0,0},{0,0,0,1,0},{0,0,0,2,0},{0,0,0,3,0},{0,0,0,4,0},{0,0,0,5,0}};

__device__ __forceinline__ void kuhn_grad(int p, int v, const double ih[3], double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  // gradient of vertex v: difference of the path steps entering and leaving it
  if (v < 3) {
    for (int a = 0; a < 3; ++a)
      if (c_kuhn_off[p][v + 1][a] != c_kuhn_off[p][v][a]) g[a] -= ih[a];
  }
  if (v > 0) {
    for (int a = 0; a < 3; ++a)
      if (c_kuhn_off[p][v][a] != c_kuhn_off[p][v - 1][a]) g[a] += ih[a];
  }
}

// One tetrahedron's part of (H a)_v, g_v and H_vv for node v = (i, j, k): hex
// offset (HX, HY, HZ), tetrahedron P, the node as local vertex V (all known
// at compile time); av holds the field on the node's 15-point stencil.
template <int HX, int HY, int HZ, int P, int V>
__device__ __forceinline__ void tet_helm(const Grid& g, const Helm3& hp,
                                         const double* __restrict__ w2, const double (&av)[27],
                                         int i, int j, int k, const double ih[3], double vol,
                                         double& Ha, double& gv, double& Hd) {
  const int ci = i + HX, cj = j + HY, ck = k + HZ;
  if (ci < 0 || cj < 0 || ck < 0 || ci >= g.nx || cj >= g.ny || ck >= g.nz) return;
  constexpr int A = Perm3<P>::a, B = Perm3<P>::b, C = Perm3<P>::c;
  const double a0 = av[VSlot<HX, HY, HZ, P, 0>::v], a1 = av[VSlot<HX, HY, HZ, P, 1>::v];
  const double a2 = av[VSlot<HX, HY, HZ, P, 2>::v], a3 = av[VSlot<HX, HY, HZ, P, 3>::v];
  // gradient of the P1 field: differences along the path o0 -> o1 -> o2 -> o3
  double grad[3];
  grad[A] = (a1 - a0) * ih[A];
  grad[B] = (a2 - a1) * ih[B];
  grad[C] = (a3 - a2) * ih[C];
  double gvv[3];
  grad3<P, V>(ih, gvv);
  const double we = w2[6 * (ci + g.nx * (cj + g.ny * ck)) + P];
  const double aV = V == 0 ? a0 : (V == 1 ? a1 : (V == 2 ? a2 : a3));
  const double mass = vol / 20.0 * (aV + a0 + a1 + a2 + a3);   // (M_e a)_v
  const double lap = vol * (gvv[0] * grad[0] + gvv[1] * grad[1] + gvv[2] * grad[2]);
  Ha += (we + hp.cM) * mass + hp.cL * lap;
  gv += (we - hp.cm) * vol / 4.0;
  Hd += (we + hp.cM) * vol / 10.0 + hp.cL * vol * (gvv[0] * gvv[0] + gvv[1] * gvv[1] + gvv[2] * gvv[2]);
}

// (H a)_v, g_v and H_vv at node (i,j,k) over its 24 tetrahedra, enumerated
// at compile time; when TRIAL the field is clip(a + mu*d, lo, 1), with MASKIN
// it is read as zero on active nodes, and with XPBY as a + mu*d there.
template <bool TRIAL, bool MASKIN, bool XPBY = false>
__device__ __forceinline__ void helm_node3d(const Grid& g, const Helm3& hp,
                                            const double* __restrict__ w2,
                                            const double* __restrict__ a,
                                            const double* __restrict__ d,
                                            const double* __restrict__ lo, double mu,
                                            const uint8_t* __restrict__ mask, int i, int j, int k,
                                            double& Ha, double& gv, double& Hd) {
  const int W = g.nx + 1, H = g.ny + 1;
  const int n = i + W * (j + H * k);
  const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
  const double vol = g.hx * g.hy * g.hz / 6.0;
  Ha = gv = Hd = 0.0;
  auto val = [&](int q) -> double {
    if (TRIAL) return fmin(fmax(a[q] + mu * d[q], lo[q]), 1.0);
    if (MASKIN && XPBY) return mask[q] ? 0.0 : a[q] + mu * d[q];
    if (MASKIN) return mask[q] ? 0.0 : a[q];
    return a[q];
  };
  double av[27];
#define LOADH3(DX, DY, DZ)                                                     \
  {                                                                            \
    constexpr int sl = nslot(DX, DY, DZ);                                      \
    av[sl] = in3(g, i + DX, j + DY, k + DZ) ? val(n + DX + W * (DY + H * DZ)) : 0.0; \
  }
  FOR_STENCIL3(LOADH3)
#undef LOADH3
#define HELM3(HX, HY, HZ, P, V) tet_helm<HX, HY, HZ, P, V>(g, hp, w2, av, i, j, k, ih, vol, Ha, gv, Hd);
  FOR_TETS3(HELM3)
#undef HELM3
}

template <bool TRIAL>
__global__ __launch_bounds__(NB) void k_vi_eval3d(Grid g, Helm3 hp, const double* __restrict__ w2,
                                                  const double* __restrict__ a,
                                                  const double* __restrict__ d,
                                                  const double* __restrict__ lo,
                                                  const double* __restrict__ S, int mu_slot,
                                                  double zeta, double* __restrict__ F,
                                                  double* __restrict__ phi,
                                                  uint8_t* __restrict__ mask,
                                                  double* __restrict__ hdinv, Red r2, Red rm,
                                                  Red rlo, Red rhi) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y, k = blockIdx.z;
  double p2 = 0.0, pm = 0.0, jlo = -INFINITY, jhi = -INFINITY;
  if (i <= g.nx && j <= g.ny) {
    const int n = i + (g.nx + 1) * (j + (g.ny + 1) * k);
    const double mu = TRIAL ? S[mu_slot] : 0.0;
    double Ha, gv, Hd;
    helm_node3d<TRIAL, false>(g, hp, w2, a, d, lo, mu, nullptr, i, j, k, Ha, gv, Hd);
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
      // row index (j, k) of an inactive node, for the reduced CG range
      const double row = (double)(j + (g.ny + 1) * k);
      if (!act) { jlo = -row; jhi = row; }
    }
  }
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int tid = threadIdx.x + NB_X * threadIdx.y;
  block_reduce<NB, false>(p2, r2, nb, bid, tid);
  block_reduce<NB, true>(pm, rm, nb, bid, tid);
  if (!TRIAL) {
    block_reduce<NB, true>(jlo, rlo, nb, bid, tid);
    block_reduce<NB, true>(jhi, rhi, nb, bid, tid);
  }
}

void launch_vi_eval3d(hipStream_t st, const Grid& g, double cL, double cM, double cm,
                      const double* w2, const double* a, const double* d, const double* lo,
                      const double* S, int mu_slot, double zeta, double* F, double* phi,
                      uint8_t* mask, double* hdinv, Red r2, Red rm, Red rlo, Red rhi, bool trial) {
  Helm3 hp{cL, cM, cm};
  dim3 gr = node_grid3(g), bl(NB_X, NB_Y);
  if (trial)
    hipLaunchKernelGGL((k_vi_eval3d<true>), gr, bl, 0, st, g, hp, w2, a, d, lo, S, mu_slot, zeta, F,
                       phi, mask, hdinv, r2, rm, rlo, rhi);
  else
    hipLaunchKernelGGL((k_vi_eval3d<false>), gr, bl, 0, st, g, hp, w2, a, d, lo, S, mu_slot, zeta,
                       F, phi, mask, hdinv, r2, rm, rlo, rhi);
  const FinishSet fs{{r2, rm, rlo, rhi}, 0b1110, trial ? 2 : 4};
  launch_finish_multi(st, fs, (int)(gr.x * gr.y * gr.z));
}

// y = H x on rows (j, k) whose row index lies in [r0, r1] (MASKED: reduced).
template <bool MASKED, bool DOT>
__global__ __launch_bounds__(NB) void k_helm_apply3d(Grid g, Helm3 hp, const double* __restrict__ w2,
                                                     const double* __restrict__ x,
                                                     const uint8_t* __restrict__ mask,
                                                     double* __restrict__ y, int r0, int r1, Red r) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y, k = blockIdx.z;
  double acc = 0.0;
  const int row = j + (g.ny + 1) * k;
  if (i <= g.nx && j <= g.ny && row >= r0 && row <= r1) {
    const int n = i + (g.nx + 1) * row;
    double Hx, gv, Hd;
    helm_node3d<false, MASKED>(g, hp, w2, x, nullptr, nullptr, 0.0, mask, i, j, k, Hx, gv, Hd);
    if (MASKED && mask[n]) Hx = 0.0;
    y[n] = Hx;
    if (DOT) acc = (MASKED && mask[n]) ? 0.0 : x[n] * Hx;
  }
  if (DOT)
    block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y * gridDim.z,
                            blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                            threadIdx.x + NB_X * threadIdx.y);
}

void launch_helm_apply3d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                         const double* x, const uint8_t* mask, double* y, bool dot, Red r, int r0,
                         int r1) {
  Helm3 hp{cL, cM, 0.0};
  const int rows = (g.ny + 1) * (g.nz + 1);
  if (r0 < 0) r0 = 0;
  if (r1 < 0 || r1 >= rows) r1 = rows - 1;
  dim3 gr = node_grid3(g), bl(NB_X, NB_Y);
#define H3(M, D) hipLaunchKernelGGL((k_helm_apply3d<M, D>), gr, bl, 0, st, g, hp, w2, x, mask, y, r0, r1, r)
  if (mask) { if (dot) H3(true, true); else H3(true, false); }
  else { if (dot) H3(false, true); else H3(false, false); }
#undef H3
  if (dot) launch_finish(st, r, (int)(gr.x * gr.y * gr.z), false);
}

// The 3D form of k_helm_cg2d: p_new = z + beta p_old formed on the fly
// (FIRST: p_new = z), q = H_NN p_new and the partial sums of p_new.q, on
// rows (j, k) whose row index lies in [r0, r1].
template <bool FIRST>
__global__ __launch_bounds__(NB) void k_helm_cg3d(Grid g, Helm3 hp, const double* __restrict__ w2,
                                                  const double* __restrict__ z,
                                                  const double* __restrict__ p_old,
                                                  const uint8_t* __restrict__ mask,
                                                  double* __restrict__ p_new,
                                                  double* __restrict__ q, int r0, int r1,
                                                  int i0, int i1, const double* __restrict__ S,
                                                  Red r) {
  const int i = i0 + blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y;
  const int k = blockIdx.z;
  const double beta = FIRST ? 0.0 : S[S_BETA];
  double acc = 0.0;
  const int row = j + (g.ny + 1) * k;
  if (i <= i1 && j <= g.ny && row >= r0 && row <= r1) {
    const int n = i + (g.nx + 1) * row;
    double Hx, gv, Hd;
    if (FIRST)
      helm_node3d<false, true>(g, hp, w2, z, nullptr, nullptr, 0.0, mask, i, j, k, Hx, gv, Hd);
    else
      helm_node3d<false, true, true>(g, hp, w2, z, p_old, nullptr, beta, mask, i, j, k, Hx, gv, Hd);
    const bool act = mask[n] != 0;
    const double pn = act ? 0.0 : (FIRST ? z[n] : z[n] + beta * p_old[n]);
    if (act) Hx = 0.0;
    p_new[n] = pn;
    q[n] = Hx;
    acc = pn * Hx;
  }
  block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y * gridDim.z,
                          blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                          threadIdx.x + NB_X * threadIdx.y);
}

void launch_helm_cg3d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                      const double* z, const double* p_old, const uint8_t* mask, double* p_new,
                      double* q, int r0, int r1, int i0, int i1, const double* S, bool first,
                      Red r) {
  Helm3 hp{cL, cM, 0.0};
  const int rows = (g.ny + 1) * (g.nz + 1);
  if (r0 < 0) r0 = 0;
  if (r1 < 0 || r1 >= rows) r1 = rows - 1;
  if (i0 < 0) i0 = 0;
  if (i1 < 0 || i1 > g.nx) i1 = g.nx;
  if (i1 < i0) return;
  dim3 gr = node_grid3(g), bl(NB_X, NB_Y);
  gr.x = (i1 - i0 + 1 + NB_X - 1) / NB_X;
  if (first)
    hipLaunchKernelGGL((k_helm_cg3d<true>), gr, bl, 0, st, g, hp, w2, z, p_old, mask, p_new, q, r0,
                       r1, i0, i1, S, r);
  else
    hipLaunchKernelGGL((k_helm_cg3d<false>), gr, bl, 0, st, g, hp, w2, z, p_old, mask, p_new, q, r0,
                       r1, i0, i1, S, r);
  launch_finish(st, r, (int)(gr.x * gr.y * gr.z), false);
}

// -(smallest) and largest column index i of an inactive node (no inactive
// node: -inf), which bound the damage CG's box in x.
__global__ __launch_bounds__(VB) void k_irange3d(Grid g, const uint8_t* __restrict__ mask, Red rlo,
                                                 Red rhi) {
  const int W = g.nx + 1;
  double lo = -INFINITY, hi = -INFINITY;
  for (int n = blockIdx.x * VB + threadIdx.x; n < g.N; n += gridDim.x * VB) {
    if (!mask[n]) {
      const double i = (double)(n % W);
      lo = fmax(lo, -i);
      hi = fmax(hi, i);
    }
  }
  block_reduce<VB, true>(lo, rlo, gridDim.x, blockIdx.x, threadIdx.x);
  block_reduce<VB, true>(hi, rhi, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_irange3d(hipStream_t st, const Grid& g, const uint8_t* mask, Red rlo, Red rhi) {
  int nb = (g.N + VB - 1) / VB;
  if (nb > VGRID) nb = VGRID;
  hipLaunchKernelGGL(k_irange3d, dim3(nb), dim3(VB), 0, st, g, mask, rlo, rhi);
  const FinishSet fs{{rlo, rhi, Red{}, Red{}}, 0b11, 2};
  launch_finish_multi(st, fs, nb);
}

__global__ __launch_bounds__(VB) void k_energy3d(Grid g, Mat m, double kell, double gc_cw, double ell,
                                                 int at2, const double* __restrict__ w2,
                                                 const double* __restrict__ a, Red rel, Red rsu) {
  const int ne = 6 * g.nx * g.ny * g.nz;
  const int W = g.nx + 1, H = g.ny + 1;
  const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
  const double vol = g.hx * g.hy * g.hz / 6.0;
  double el = 0.0, su = 0.0;
  for (int e = blockIdx.x * VB + threadIdx.x; e < ne; e += gridDim.x * VB) {
    const int p = e % 6, hex = e / 6;
    const int ci = hex % g.nx, cj = (hex / g.nx) % g.ny, ck = hex / (g.nx * g.ny);
    double av[4], grad[3] = {0, 0, 0}, s = 0, s2 = 0;
    for (int q = 0; q < 4; ++q) {
      av[q] = a[(ci + c_kuhn_off[p][q][0]) + W * ((cj + c_kuhn_off[p][q][1]) + H * (ck + c_kuhn_off[p][q][2]))];
      s += av[q];
      s2 += av[q] * av[q];
      double gq[3];
      kuhn_grad(p, q, ih, gq);
      for (int c = 0; c < 3; ++c) grad[c] += av[q] * gq[c];
    }
    el += 0.5 * abar4(av[0], av[1], av[2], av[3], kell) * vol * w2[e];
    const double wint = at2 ? vol / 20.0 * (s2 + s * s) : vol / 4.0 * s;
    su += gc_cw * (wint / ell + ell * vol * (grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]));
  }
  block_reduce<VB, false>(el, rel, gridDim.x, blockIdx.x, threadIdx.x);
  block_reduce<VB, false>(su, rsu, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_energy3d(hipStream_t st, const Grid& g, const Mat& m, double kell, double gc_cw,
                     double ell, int at2, const double* w2, const double* a, Red rel, Red rsu) {
  const int ne = 6 * g.nx * g.ny * g.nz;
  int nb = (ne + VB - 1) / VB;
  if (nb > VGRID) nb = VGRID;
  hipLaunchKernelGGL(k_energy3d, dim3(nb), dim3(VB), 0, st, g, m, kell, gc_cw, ell, at2, w2, a, rel, rsu);
  const FinishSet fs{{rel, rsu, Red{}, Red{}}, 0, 2};
  launch_finish_multi(st, fs, nb);
}

// Dense assembly of the coarsest 3D level (one thread per node row).
__global__ __launch_bounds__(1024) void k_dense_assemble3d(Grid g, Mat m, const double* __restrict__ abar,
                                                           double* __restrict__ A,
                                                           const double* __restrict__ S) {
  if (S[S_COARSE_REFRESH] == 0.0) return;   // uniform: the whole block keeps the old system
  const int N = g.N, n3 = 3 * N, W = g.nx + 1, H = g.ny + 1;
  for (int q = threadIdx.x; q < n3 * n3; q += 1024) A[q] = 0.0;
  __syncthreads();
  const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
  const double vol = g.hx * g.hy * g.hz / 6.0;
  for (int n = threadIdx.x; n < N; n += 1024) {
    const int i = n % W, j = (n / W) % H, k = n / (W * H);
    for (int t = 0; t < 24; ++t) {
      const int ci = i + c_tets3[t][0], cj = j + c_tets3[t][1], ck = k + c_tets3[t][2];
      if (ci < 0 || cj < 0 || ck < 0 || ci >= g.nx || cj >= g.ny || ck >= g.nz) continue;
      const int p = c_tets3[t][3], v = c_tets3[t][4];
      const double w = abar[6 * (ci + g.nx * (cj + g.ny * ck)) + p] * vol;
      double gv[3];
      kuhn_grad(p, v, ih, gv);
      for (int q = 0; q < 4; ++q) {
        const int nb = (ci + c_kuhn_off[p][q][0]) + W * ((cj + c_kuhn_off[p][q][1]) + H * (ck + c_kuhn_off[p][q][2]));
        double gw[3];
        kuhn_grad(p, q, ih, gw);
        const double gg = gv[0] * gw[0] + gv[1] * gw[1] + gv[2] * gw[2];
        for (int c = 0; c < 3; ++c)
          for (int d = 0; d < 3; ++d)
            A[(size_t)(c * N + n) * n3 + d * N + nb] +=
                w * (m.lam * gv[c] * gw[d] + m.mu * gv[d] * gw[c] + (c == d ? m.mu * gg : 0.0));
      }
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < n3; r += 1024) {
    const int comp = r / N, n = r % N;
    if (fixed3(g, comp, n % W, (n / W) % H, n / (W * H))) {
      for (int c = 0; c < n3; ++c) {
        A[(size_t)r * n3 + c] = (c == r) ? 1.0 : 0.0;
        A[(size_t)c * n3 + r] = (c == r) ? 1.0 : 0.0;
      }
    }
  }
}

void launch_dense_assemble3d(hipStream_t st, const Grid& g, const Mat& m, const double* abar, double* A,
                             const double* S) {
  hipLaunchKernelGGL(k_dense_assemble3d, dim3(1), dim3(1024), 0, st, g, m, abar, A, S);
}

// ---------------------------------------------------------------------------
// coupled Jacobian blocks (Newton step of Algorithm 3 / 4), 3D
// ---------------------------------------------------------------------------
//
// E_ualpha of eq. (offdiag) with a'(alpha) = -2 (1 - alpha), integrated
// exactly with P1 alpha on a tetrahedron:
//   B[v, j] = sum_e -2 |T| (B_e^T D eps_e(u))_v (M_ref b_e)_j,
// b = 1 - alpha, M_ref = (1 + delta_ab)/20 (the consistent P1 mass of a
// tetrahedron over |T|).  u's strain is its effective strain (eps(u) - eps0)
// under the thermal load.
//
// k_jac_u3d:  y_u = A x_u + B x_a   (A = K(alpha), Dirichlet rows zero)
// k_jac_a3d:  y_a = B^T x_u + C x_a (C = H, rows and columns of active nodes removed)
// The 24 (hex offset, tetrahedron, local vertex) incidences of a node are
// walked from the runtime table c_tets3.

// w^T M_ref b over a tetrahedron's four vertices.
__device__ __forceinline__ double mref_pair4(const double w[4], const double b[4]) {
  double wb = 0.0, sw = 0.0, sb = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    wb += w[q] * b[q];
    sw += w[q];
    sb += b[q];
  }
  return (wb + sw * sb) * (1.0 / 20.0);
}

// Node indices of tetrahedron p of hex (ci, cj, ck) and the axis of each path
// step o_s -> o_{s+1}.
__device__ __forceinline__ void tet_nodes3(const Grid& g, int ci, int cj, int ck, int p, int nd[4],
                                           int ax[3]) {
  const int W = g.nx + 1, H = g.ny + 1;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    nd[v] = (ci + c_kuhn_off[p][v][0]) + W * ((cj + c_kuhn_off[p][v][1]) + H * (ck + c_kuhn_off[p][v][2]));
#pragma unroll
  for (int s = 0; s < 3; ++s)
    for (int a = 0; a < 3; ++a)
      if (c_kuhn_off[p][s + 1][a] != c_kuhn_off[p][s][a]) ax[s] = a;
}

// Displacement gradient G[comp][axis] of the blocked field x on the tetrahedron.
__device__ __forceinline__ void tet_gradient3(const Grid& g, const double* __restrict__ x,
                                              const int nd[4], const int ax[3], const double ih[3],
                                              double G[3][3]) {
  const int N = g.N;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int s = 0; s < 3; ++s) G[c][ax[s]] = (x[nd[s + 1] + c * N] - x[nd[s] + c * N]) * ih[ax[s]];
}

// Stress of u on tetrahedron p of hex (ci, cj, ck): sigma = D (eps(u) - eps0).
template <bool EIG>
__device__ __forceinline__ void tet_stress3(const Grid& g, const Mat& m, const double* __restrict__ u,
                                            const int nd[4], const int ax[3], const double ih[3],
                                            int ci, int p, double S[3][3]) {
  double G[3][3];
  tet_gradient3(g, u, nd, ax, ih, G);
  double e0 = G[0][0], e1 = G[1][1], e2 = G[2][2];
  if (EIG) {
    const double xc = (ci + 0.25 * (c_kuhn_off[p][1][0] + c_kuhn_off[p][2][0] + 1)) * g.hx;
    const double s = -g.eig_dT * exp(-xc / g.eig_depth);
    e0 -= s; e1 -= s; e2 -= s;
  }
  const double tr = e0 + e1 + e2;
  S[0][0] = m.lam * tr + 2.0 * m.mu * e0;
  S[1][1] = m.lam * tr + 2.0 * m.mu * e1;
  S[2][2] = m.lam * tr + 2.0 * m.mu * e2;
  S[0][1] = S[1][0] = m.mu * (G[0][1] + G[1][0]);
  S[0][2] = S[2][0] = m.mu * (G[0][2] + G[2][0]);
  S[1][2] = S[2][1] = m.mu * (G[1][2] + G[2][1]);
}

// (B x_a) at node (i, j, k): per incident tetrahedron the coefficient
// -2 w^T M_ref b (w = x_a on inactive nodes, zero on active ones) times the
// tetrahedron's force sigma(u) grad(phi_v) |T|.
template <bool EIG>
__device__ __forceinline__ void coupling_force3d(const Grid& g, const Mat& m,
                                                 const double* __restrict__ alpha,
                                                 const double* __restrict__ u,
                                                 const double* __restrict__ xa,
                                                 const uint8_t* __restrict__ mask, int i, int j,
                                                 int k, double f[3]) {
  const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
  const double vol = g.hx * g.hy * g.hz / 6.0;
  f[0] = f[1] = f[2] = 0.0;
  for (int t = 0; t < 24; ++t) {
    const int ci = i + c_tets3[t][0], cj = j + c_tets3[t][1], ck = k + c_tets3[t][2];
    if (ci < 0 || cj < 0 || ck < 0 || ci >= g.nx || cj >= g.ny || ck >= g.nz) continue;
    const int p = c_tets3[t][3], v = c_tets3[t][4];
    int nd[4], ax[3];
    tet_nodes3(g, ci, cj, ck, p, nd, ax);
    double w[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      w[q] = mask[nd[q]] ? 0.0 : xa[nd[q]];
      b[q] = 1.0 - alpha[nd[q]];
    }
    const double c = -2.0 * mref_pair4(w, b) * vol;
    if (c == 0.0) continue;
    double S[3][3], gv[3];
    tet_stress3<EIG>(g, m, u, nd, ax, ih, ci, p, S);
    kuhn_grad(p, v, ih, gv);
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] += c * (S[a][0] * gv[0] + S[a][1] * gv[1] + S[a][2] * gv[2]);
  }
}

template <bool HAS_XU, bool HAS_XA, bool DOT, bool EIG>
__global__ __launch_bounds__(NB) void k_jac_u3d(Grid g, Mat m, double kell,
                                                const double* __restrict__ alpha,
                                                const double* __restrict__ u,
                                                const double* __restrict__ xu,
                                                const double* __restrict__ xa,
                                                const uint8_t* __restrict__ mask,
                                                double* __restrict__ yu, Red r,
                                                const double* __restrict__ band) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y, k = blockIdx.z;
  double acc = 0.0;
  // B x_a reaches only rows (j, k) within one cell of an inactive node: with
  // band = (-r_lo, r_hi) of the inactive row indices j + (ny + 1) k, the rows
  // r_lo - (ny + 2) .. r_hi + (ny + 2) (band == nullptr: every row)
  bool couple = HAS_XA;
  if (HAS_XA && band) {
    const double rlo = -band[0], rhi = band[1], row = (double)(j + (g.ny + 1) * k);
    const double pad = (double)(g.ny + 2);
    couple = rlo <= rhi && row >= rlo - pad && row <= rhi + pad;
  }
  if (i <= g.nx && j <= g.ny) {
    const int N = g.N, n = i + (g.nx + 1) * (j + (g.ny + 1) * k);
    double f[3] = {0.0, 0.0, 0.0}, d[3];
    if (HAS_XU) node_force3d<true, true, false, false>(g, m, alpha, kell, xu, i, j, k, f, d);
    if (couple) {
      double gc[3];
      coupling_force3d<EIG>(g, m, alpha, u, xa, mask, i, j, k, gc);
      f[0] += gc[0]; f[1] += gc[1]; f[2] += gc[2];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double yv = fixed3(g, c, i, j, k) ? 0.0 : f[c];
      yu[n + c * N] = yv;
      if (DOT) acc += xu[n + c * N] * yv;
    }
  }
  if (DOT)
    block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y * gridDim.z,
                            blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                            threadIdx.x + NB_X * threadIdx.y);
}

template <bool HAS_XU, bool HAS_XA, bool DOT, bool EIG>
__global__ __launch_bounds__(NB) void k_jac_a3d(Grid g, Mat m, Helm3 hp,
                                                const double* __restrict__ alpha,
                                                const double* __restrict__ u,
                                                const double* __restrict__ w2,
                                                const double* __restrict__ xu,
                                                const double* __restrict__ xa,
                                                const uint8_t* __restrict__ mask,
                                                double* __restrict__ ya, Red r) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y, k = blockIdx.z;
  double acc = 0.0;
  if (i <= g.nx && j <= g.ny) {
    const int n = i + (g.nx + 1) * (j + (g.ny + 1) * k);
    double y = 0.0;
    if (!mask[n]) {
      if (HAS_XA) {
        double Hx, gv, Hd;
        helm_node3d<false, true>(g, hp, w2, xa, nullptr, nullptr, 0.0, mask, i, j, k, Hx, gv, Hd);
        y += Hx;
      }
      if (HAS_XU) {
        const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
        const double vol = g.hx * g.hy * g.hz / 6.0;
        for (int t = 0; t < 24; ++t) {
          const int ci = i + c_tets3[t][0], cj = j + c_tets3[t][1], ck = k + c_tets3[t][2];
          if (ci < 0 || cj < 0 || ck < 0 || ci >= g.nx || cj >= g.ny || ck >= g.nz) continue;
          const int p = c_tets3[t][3], v = c_tets3[t][4];
          int nd[4], ax[3];
          tet_nodes3(g, ci, cj, ck, p, nd, ax);
          double S[3][3], G[3][3];
          tet_stress3<EIG>(g, m, u, nd, ax, ih, ci, p, S);
          tet_gradient3(g, xu, nd, ax, ih, G);
          // sigma(u) : eps(x_u), eps the symmetric part of G
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) s += S[a][c] * 0.5 * (G[a][c] + G[c][a]);
          double bs = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) bs += 1.0 - alpha[nd[q]];
          const double mb = ((1.0 - alpha[nd[v]]) + bs) * (1.0 / 20.0);
          y += -2.0 * vol * s * mb;
        }
      }
    }
    ya[n] = y;
    if (DOT) acc = (HAS_XA && !mask[n]) ? xa[n] * y : 0.0;
  }
  if (DOT)
    block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y * gridDim.z,
                            blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                            threadIdx.x + NB_X * threadIdx.y);
}

void launch_jac3d(hipStream_t st, const Grid& g, const Mat& m, double kell, double cL, double cM,
                  const double* alpha, const double* u, const double* w2, const uint8_t* mask,
                  const double* xu, const double* xa, double* yu, double* ya, bool dot, Red ru,
                  Red ra, const double* band) {
  dim3 gr = node_grid3(g), bl(NB_X, NB_Y);
  Helm3 hp{cL, cM, 0.0};
  const bool eig = g.eig_dT != 0.0;
  if (yu) {
#define JU3(A, B, D)                                                                                \
  do {                                                                                              \
    if (eig && B)                                                                                   \
      hipLaunchKernelGGL((k_jac_u3d<A, B, D, true>), gr, bl, 0, st, g, m, kell, alpha, u, xu, xa,   \
                         mask, yu, ru, band);                                                       \
    else                                                                                            \
      hipLaunchKernelGGL((k_jac_u3d<A, B, D, false>), gr, bl, 0, st, g, m, kell, alpha, u, xu, xa,  \
                         mask, yu, ru, band);                                                       \
  } while (0)
    if (xu && xa) { if (dot) JU3(true, true, true); else JU3(true, true, false); }
    else if (xu) { if (dot) JU3(true, false, true); else JU3(true, false, false); }
    else JU3(false, true, false);
#undef JU3
    if (dot && xu) launch_finish(st, ru, (int)(gr.x * gr.y * gr.z), false);
  }
  if (ya) {
#define JA3(A, B, D)                                                                                \
  do {                                                                                              \
    if (eig && A)                                                                                   \
      hipLaunchKernelGGL((k_jac_a3d<A, B, D, true>), gr, bl, 0, st, g, m, hp, alpha, u, w2, xu, xa, \
                         mask, ya, ra);                                                             \
    else                                                                                            \
      hipLaunchKernelGGL((k_jac_a3d<A, B, D, false>), gr, bl, 0, st, g, m, hp, alpha, u, w2, xu,    \
                         xa, mask, ya, ra);                                                         \
  } while (0)
    if (xu && xa) { if (dot) JA3(true, true, true); else JA3(true, true, false); }
    else if (xa) { if (dot) JA3(false, true, true); else JA3(false, true, false); }
    else JA3(true, false, false);
#undef JA3
    if (dot && xa) launch_finish(st, ra, (int)(gr.x * gr.y * gr.z), false);
  }
}

// y_u += B x_a on the rows (j, k) whose index j + (ny + 1) k lies in r0..r1,
// Dirichlet DOFs left alone; partial sums of x_u . B x_a.
template <bool EIG>
__global__ __launch_bounds__(NB) void k_couple_u3d(Grid g, Mat m, const double* __restrict__ alpha,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ xu,
                                                   const double* __restrict__ xa,
                                                   const uint8_t* __restrict__ mask,
                                                   double* __restrict__ yu, int r0, int r1, Red r) {
  const int i = blockIdx.x * NB_X + threadIdx.x;
  const int row = r0 + blockIdx.y * NB_Y + threadIdx.y;
  double acc = 0.0;
  if (i <= g.nx && row <= r1) {
    const int j = row % (g.ny + 1), k = row / (g.ny + 1);
    const int N = g.N, n = i + (g.nx + 1) * row;
    double f[3];
    coupling_force3d<EIG>(g, m, alpha, u, xa, mask, i, j, k, f);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double gc = fixed3(g, c, i, j, k) ? 0.0 : f[c];
      yu[n + c * N] += gc;
      acc += xu[n + c * N] * gc;
    }
  }
  block_reduce<NB, false>(acc, r, gridDim.x * gridDim.y, blockIdx.x + gridDim.x * blockIdx.y,
                          threadIdx.x + NB_X * threadIdx.y);
}

void launch_couple_u3d(hipStream_t st, const Grid& g, const Mat& m, const double* alpha,
                       const double* u, const double* xu, const double* xa, const uint8_t* mask,
                       double* yu, int r0, int r1, Red r) {
  const int rows = (g.ny + 1) * (g.nz + 1);
  if (r0 < 0) r0 = 0;
  if (r1 >= rows) r1 = rows - 1;
  if (r1 < r0) return;
  dim3 gr((g.nx + 1 + NB_X - 1) / NB_X, (r1 - r0 + 1 + NB_Y - 1) / NB_Y), bl(NB_X, NB_Y);
  if (g.eig_dT != 0.0)
    hipLaunchKernelGGL((k_couple_u3d<true>), gr, bl, 0, st, g, m, alpha, u, xu, xa, mask, yu, r0,
                       r1, r);
  else
    hipLaunchKernelGGL((k_couple_u3d<false>), gr, bl, 0, st, g, m, alpha, u, xu, xa, mask, yu, r0,
                       r1, r);
  launch_finish(st, r, (int)(gr.x * gr.y), false);
}

// Jacobi-preconditioned Chebyshev step on C = H_NN in 3D:
// d_new = cd d_in + cr D^{-1} (b - C x_in); x_out = x_in + d_new.
__global__ __launch_bounds__(NB) void k_cheb_helm3d(Grid g, Helm3 hp, const double* __restrict__ w2,
                                                    const uint8_t* __restrict__ mask,
                                                    const double* __restrict__ x_in,
                                                    double* __restrict__ x_out,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ d_in,
                                                    double* __restrict__ d_out, double cd,
                                                    double cr) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y, k = blockIdx.z;
  if (i > g.nx || j > g.ny) return;
  const int n = i + (g.nx + 1) * (j + (g.ny + 1) * k);
  if (mask[n]) {
    x_out[n] = 0.0;
    if (d_out) d_out[n] = 0.0;
    return;
  }
  double Hx = 0.0, gv, Hd;
  helm_node3d<false, true>(g, hp, w2, x_in ? x_in : b, nullptr, nullptr, 0.0, mask, i, j, k, Hx, gv,
                           Hd);
  if (!x_in) Hx = 0.0;
  double dn = cr * (b[n] - Hx) / Hd;
  if (d_in) dn += cd * d_in[n];
  x_out[n] = (x_in ? x_in[n] : 0.0) + dn;
  if (d_out) d_out[n] = dn;
}

void launch_cheb_helm3d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                        const uint8_t* mask, const double* x_in, double* x_out, const double* b,
                        const double* d_in, double* d_out, double cd, double cr) {
  Helm3 hp{cL, cM, 0.0};
  hipLaunchKernelGGL(k_cheb_helm3d, node_grid3(g), dim3(NB_X, NB_Y), 0, st, g, hp, w2, mask, x_in,
                     x_out, b, d_in, d_out, cd, cr);
}

#define INST3(T)                                                                                \
  template void launch_apply3d<T>(hipStream_t, const Grid&, const Mat&, bool, const T*, double,  \
                                  const T*, T*, const ND<T>*, int, int, Red);                    \
  template void launch_resid3d<T>(hipStream_t, const Grid&, const Mat&, bool, const T*, double,  \
                                  const T*, T*, const ND<T>*, bool, Red);                        \
  template void launch_smooth3d<T>(hipStream_t, const Grid&, const Mat&, bool, const T*, double, \
                                   const ND<T>*, T*, const T*, const ND<T>*, ND<T>*, double,     \
                                   double);                                                      \
  template void launch_restrict3d<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);       \
  template void launch_prolong3d<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);
INST3(float)
INST3(double)
#undef INST3

}  // namespace frac
