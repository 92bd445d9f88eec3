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
#include <algorithm>

#include "common.h"
#include "launch.h"
#include "ops3d.h"

namespace frac {

// ---------------------------------------------------------------------------
// element-centric operator kernels (apply / residual / Chebyshev step)
// ---------------------------------------------------------------------------
//
// A block owns a 15 x 15 x E3_KZ box of nodes.  Each of its 16 x 16 threads
// takes one column of hexahedra (the box's columns and one more on the low
// side in x and y, so every owned node has all eight of its hexahedra) and
// walks the hexahedron layers from one below the box to its top plane.  Per
// layer a thread forms the six tetrahedra of its hexahedron once and adds
// their nodal forces (or, for the diagonal pass, their diagonal entries of K)
// into LDS sums of the layer's two node planes.  A node receives from the four hexahedra of
// a layer that share it in four phases, one per vertex position in the x-y
// plane, so no two threads write one sum at once and the order of every sum
// is fixed: the result is bitwise reproducible.  Three node planes of u and
// alpha and two planes of sums are resident; every node is read from HBM once
// apart from the tile halo.  Each tetrahedron is formed once per layer walk
// (1.14 x 1.25 times on average with the halos) instead of once for each of
// its four vertices by a node-centric kernel.
//
// The diagonal of K depends on the coefficients alone, so it is formed once
// per coefficient update (M3_DIAG) and the Chebyshev steps read it (three
// more reads per node instead of a second set of sums and the registers to
// form it in every step).

enum { M3_APPLY = 0, M3_RESID = 1, M3_SMOOTH = 2, M3_DIAG = 3 };
enum { R3_NONE = 0, R3_DOT = 1, R3_FREE2 = 2 };

constexpr int E3_T = 16;             // hexahedron columns per block edge (16 x 16 threads)
constexpr int E3_O = E3_T - 1;       // owned nodes per block edge
constexpr int E3_P = E3_T + 1;       // node tile edge: the owned nodes and a halo on each side
constexpr int E3_PN = E3_P * E3_P;   // nodes of one tile plane
constexpr int E3_KZ = 4;             // owned node planes per block
static_assert(E3_T * E3_T == NB, "one thread per hexahedron column");

// local vertex (dx + 2 dy + 4 dz) of vertex W of tetrahedron P
template <int P, int W>
struct HexV {
  static constexpr int v = VOff<P, W, 0>::v + 2 * VOff<P, W, 1>::v + 4 * VOff<P, W, 2>::v;
};

// Forces (HASX) and diagonal entries (DIAG) of tetrahedron P of a hexahedron
// added to its vertices.  u, a: the hexahedron's eight vertices; c: the
// degradation coefficient (FA: from a, else given); seig: the eigenstrain
// offset of the tetrahedron (EIG).
template <int P, bool FA, bool HASX, bool DIAG, bool EIG, class T>
__device__ __forceinline__ void hex_tet3(const Mat& m, const T (&u)[8][3], const T (&a)[8], T cgiven,
                                         T kell, T seig, const T ih[3], T vol, T (&fv)[8][3],
                                         T (&dv)[8][3]) {
  constexpr int A = Perm3<P>::a, B = Perm3<P>::b, C = Perm3<P>::c;
  constexpr int v0 = HexV<P, 0>::v, v1 = HexV<P, 1>::v, v2 = HexV<P, 2>::v, v3 = HexV<P, 3>::v;
  const T c = FA ? abar4(a[v0], a[v1], a[v2], a[v3], kell) : cgiven;
  const T w = c * vol;
  const T lam = T(m.lam), mu = T(m.mu);
  if (HASX) {
    T G[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      G[q][A] = (u[v1][q] - u[v0][q]) * ih[A];
      G[q][B] = (u[v2][q] - u[v1][q]) * ih[B];
      G[q][C] = (u[v3][q] - u[v2][q]) * ih[C];
    }
    T e0 = G[0][0], e1 = G[1][1], e2 = G[2][2];
    if (EIG) { e0 -= seig; e1 -= seig; e2 -= seig; }
    const T tr = e0 + e1 + e2;
    T S[3][3];
    S[0][0] = lam * tr + T(2) * mu * e0;
    S[1][1] = lam * tr + T(2) * mu * e1;
    S[2][2] = lam * tr + T(2) * mu * e2;
    S[0][1] = S[1][0] = mu * (G[0][1] + G[1][0]);
    S[0][2] = S[2][0] = mu * (G[0][2] + G[2][0]);
    S[1][2] = S[2][1] = mu * (G[1][2] + G[2][1]);
    // vertex gradients: g0 = -e_A/h_A, g1 = e_A/h_A - e_B/h_B, g2 = e_B/h_B - e_C/h_C, g3 = e_C/h_C
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const T tA = w * S[q][A] * ih[A], tB = w * S[q][B] * ih[B], tC = w * S[q][C] * ih[C];
      fv[v0][q] -= tA;
      fv[v1][q] += tA - tB;
      fv[v2][q] += tB - tC;
      fv[v3][q] += tC;
    }
  }
  if (DIAG) {
    const T lm = lam + mu;
    const T gA = ih[A] * ih[A], gB = ih[B] * ih[B], gC = ih[C] * ih[C];
    // |g_W|^2 and its per-axis squares, as above
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const T s0 = q == A ? gA : T(0);
      const T s1 = q == A ? gA : (q == B ? gB : T(0));
      const T s2 = q == B ? gB : (q == C ? gC : T(0));
      const T s3 = q == C ? gC : T(0);
      dv[v0][q] += w * (lm * s0 + mu * gA);
      dv[v1][q] += w * (lm * s1 + mu * (gA + gB));
      dv[v2][q] += w * (lm * s2 + mu * (gB + gC));
      dv[v3][q] += w * (lm * s3 + mu * gC);
    }
  }
}

template <int MODE, bool FA, bool HASX, int RED, bool EIG, class T>
__global__ __launch_bounds__(NB) void k_elem3d(Grid g, Mat m, const T* __restrict__ coef, T kell,
                                               const T* __restrict__ x, T* __restrict__ y,
                                               const T* __restrict__ b, const T* __restrict__ dg,
                                               const T* __restrict__ din, T* __restrict__ dout,
                                               T cd, T cr, int mask, Red red) {
  constexpr bool DIAG = MODE == M3_DIAG;
  constexpr bool NEED_A = FA;
  __shared__ T su[HASX ? 3 : 1][3][HASX ? E3_PN : 1];   // u: planes p % 3, components
  __shared__ T sa[NEED_A ? 3 : 1][NEED_A ? E3_PN : 1];  // alpha: planes p % 3
  __shared__ T sf[HASX ? 2 : 1][3][HASX ? E3_PN : 1];   // force sums: planes p & 1
  __shared__ T sd[DIAG ? 2 : 1][3][DIAG ? E3_PN : 1];   // diagonal sums: planes p & 1
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + E3_T * ty;
  const int i0 = blockIdx.x * E3_O, j0 = blockIdx.y * E3_O, k0 = blockIdx.z * E3_KZ;
  const int W = g.nx + 1, H = g.ny + 1, N = g.N;
  const int ke = min(k0 + E3_KZ - 1, g.nz);
  const int ci = i0 - 1 + tx, cj = j0 - 1 + ty;
  const bool col_ok = ci >= 0 && cj >= 0 && ci < g.nx && cj < g.ny;
  const bool owner = tx < E3_O && ty < E3_O && i0 + tx <= g.nx && j0 + ty <= g.ny;
  const int own = (tx + 1) + E3_P * (ty + 1);
  const T ih[3] = {T(1.0 / g.hx), T(1.0 / g.hy), T(1.0 / g.hz)};
  const T vol = T(g.hx * g.hy * g.hz / 6.0);
  // eigenstrain offsets of the column's six tetrahedra (they depend on x only)
  T seig[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  if (EIG && col_ok) {
#define SEIG(P) seig[P] = T(-g.eig_dT * exp(-((ci + tet_xc<P>()) * g.hx) / g.eig_depth));
    SEIG(0) SEIG(1) SEIG(2) SEIG(3) SEIG(4) SEIG(5)
#undef SEIG
  }
  // A node plane is fetched into registers one layer ahead (this thread's
  // tile entries tid and tid + NB) and written to LDS after the layer's
  // arithmetic, so no layer waits on its own global loads.
  constexpr int PE = (E3_PN + NB - 1) / NB;
  T pu[PE][3], pa[PE];
  auto fetch_plane = [&](int p) {
#pragma unroll
    for (int r = 0; r < PE; ++r) {
      const int e = tid + r * NB;
      pu[r][0] = pu[r][1] = pu[r][2] = pa[r] = T(0);
      const int lx = e % E3_P, ly = e / E3_P;
      const int gi = i0 - 1 + lx, gj = j0 - 1 + ly;
      if (e < E3_PN && p >= 0 && p <= g.nz && gi >= 0 && gj >= 0 && gi <= g.nx && gj <= g.ny) {
        const int n = gi + W * (gj + H * p);
        if constexpr (HASX) {
          pu[r][0] = x[n];
          pu[r][1] = x[n + N];
          pu[r][2] = x[n + 2 * N];
        }
        if constexpr (NEED_A) pa[r] = coef[n];
      }
    }
  };
  auto store_plane = [&](int p) {
    if (p < 0 || p > g.nz) return;
    const int sl = p % 3;
#pragma unroll
    for (int r = 0; r < PE; ++r) {
      const int e = tid + r * NB;
      if (e < E3_PN) {
        if constexpr (HASX) {
          su[sl][0][e] = pu[r][0];
          su[sl][1][e] = pu[r][1];
          su[sl][2][e] = pu[r][2];
        }
        if constexpr (NEED_A) sa[sl][e] = pa[r];
      }
    }
  };
  for (int e = tid; e < E3_PN; e += NB) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if constexpr (HASX) { sf[0][q][e] = T(0); sf[1][q][e] = T(0); }
      if constexpr (DIAG) { sd[0][q][e] = T(0); sd[1][q][e] = T(0); }
    }
  }
  fetch_plane(k0 - 1);
  store_plane(k0 - 1);
  fetch_plane(k0);
  store_plane(k0);
  double acc = 0.0;
  for (int ck = k0 - 1; ck <= ke; ++ck) {
    // next layer's upper plane, and the owned node's inputs of this layer's
    // finishing step, are in flight during the layer
    if (ck < ke) fetch_plane(ck + 2);   // the upper plane of layer ck + 1
    const bool bot = ck >= k0, top = ck + 1 <= ke;
    T eb[3] = {T(0), T(0), T(0)}, ed[3] = {T(0), T(0), T(0)}, eg[3] = {T(1), T(1), T(1)};
    if (bot && owner) {
      const int n = (i0 + tx) + W * ((j0 + ty) + H * ck);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int q = n + c * N;
        if (MODE != M3_DIAG && b) eb[c] = b[q];
        if (MODE == M3_SMOOTH) {
          eg[c] = dg[q];
          if (din) ed[c] = din[q];
        }
      }
    }
    __syncthreads();
    T fv[8][3], dv[8][3];
#pragma unroll
    for (int v = 0; v < 8; ++v)
#pragma unroll
      for (int q = 0; q < 3; ++q) fv[v][q] = dv[v][q] = T(0);
    const bool hex_ok = col_ok && ck >= 0 && ck < g.nz;
    if (hex_ok) {
      T u[8][3], a[8];
      const int s0 = ck % 3, s1 = (ck + 1) % 3;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int sl = (v & 4) ? s1 : s0;
        const int e = (tx + (v & 1)) + E3_P * (ty + ((v >> 1) & 1));
        if constexpr (HASX) {
#pragma unroll
          for (int q = 0; q < 3; ++q) u[v][q] = su[sl][q][e];
        } else {
#pragma unroll
          for (int q = 0; q < 3; ++q) u[v][q] = T(0);
        }
        a[v] = T(0);
        if constexpr (NEED_A) a[v] = sa[sl][e];
      }
      T cg[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
      if (!FA) {
        const T* ab = coef + 6 * ((int64_t)ci + (int64_t)g.nx * (cj + (int64_t)g.ny * ck));
#pragma unroll
        for (int p = 0; p < 6; ++p) cg[p] = ab[p];
      }
#define HT(P) hex_tet3<P, FA, HASX, DIAG, EIG>(m, u, a, cg[P], kell, seig[P], ih, vol, fv, dv);
      HT(0) HT(1) HT(2) HT(3) HT(4) HT(5)
#undef HT
    }
    // the four vertex positions in the x-y plane, one phase each: bottom
    // vertices into the sums of plane ck, top vertices into those of ck + 1
    const int fb0 = (ck + 2) & 1, fb1 = (ck + 3) & 1;
#pragma unroll
    for (int ph = 0; ph < 4; ++ph) {
      if (hex_ok) {
        const int e = (tx + (ph & 1)) + E3_P * (ty + (ph >> 1));
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if constexpr (HASX) {
            if (bot) sf[fb0][q][e] += fv[ph][q];
            if (top) sf[fb1][q][e] += fv[ph + 4][q];
          }
          if constexpr (DIAG) {
            if (bot) sd[fb0][q][e] += dv[ph][q];
            if (top) sd[fb1][q][e] += dv[ph + 4][q];
          }
        }
      }
      __syncthreads();
    }
    if (bot) {
      // plane ck is complete: the owned nodes finish the operator
      if (owner) {
        const int n = (i0 + tx) + W * ((j0 + ty) + H * ck);
        const int sl = ck % 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const bool fx = fixed3(g, c, i0 + tx, j0 + ty, ck);
          const int q = n + c * N;
          T f = T(0), xv = T(0);
          if constexpr (HASX) {
            f = sf[fb0][c][own];
            xv = su[sl][c][own];
          }
          if (MODE == M3_APPLY) {
            const T yv = (mask && fx) ? T(0) : f;
            y[q] = yv;
            if (RED == R3_DOT) acc += (double)xv * yv;
            if (RED == R3_FREE2) {
              const double r = (double)f - (double)eb[c];
              acc += fx ? 0.0 : r * r;
            }
          } else if (MODE == M3_RESID) {
            const T r = fx ? T(0) : eb[c] - f;
            y[q] = r;
            if (RED == R3_DOT) acc += (double)r * r;
          } else if (MODE == M3_SMOOTH) {
            const T r = eb[c] - f;
            T dd = cr * r / eg[c];
            if (din) dd += cd * ed[c];
            T xo = xv + dd;
            if (fx) { xo = T(0); dd = T(0); }
            y[q] = xo;
            if (dout) dout[q] = dd;
          } else {
            if constexpr (DIAG) y[q] = sd[fb0][c][own];
          }
        }
      }
      // the sums of plane ck are cleared for plane ck + 2: owners clear their
      // own entries (read just above), the first threads the tile halo
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (tx < E3_O && ty < E3_O) {
          if constexpr (HASX) sf[fb0][c][own] = T(0);
          if constexpr (DIAG) sd[fb0][c][own] = T(0);
        }
      }
      if (tid < 4 * E3_P - 4) {
        // the 64 halo entries of the 17 x 17 plane (rows 0 and 16, columns 0 and 16)
        int e;
        if (tid < E3_P) e = tid;
        else if (tid < 2 * E3_P) e = (E3_P - 1) * E3_P + (tid - E3_P);
        else if (tid < 2 * E3_P + (E3_P - 2)) e = E3_P * (1 + tid - 2 * E3_P);
        else e = E3_P * (1 + tid - 2 * E3_P - (E3_P - 2)) + E3_P - 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if constexpr (HASX) sf[fb0][c][e] = T(0);
          if constexpr (DIAG) sd[fb0][c][e] = T(0);
        }
      }
    }
    if (ck < ke) store_plane(ck + 2);
  }
  if (RED != R3_NONE)
    block_reduce<NB, false>(acc, red, gridDim.x * gridDim.y * gridDim.z,
                            blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), tid);
}

// Node of this thread in a one-dimensional launch of 256-thread blocks over
// the N nodes of g (false past the last node).  Rows of the coarse levels are
// 5 to 65 nodes long; walking the nodes flat keeps every lane of a wavefront
// busy where 64-wide row tiles would leave up to half of them idle.
__device__ __forceinline__ bool flat_node3(const Grid& g, int& i, int& j, int& k) {
  const int n = blockIdx.x * NB + threadIdx.x + NB_X * threadIdx.y;
  if (n >= g.N) return false;
  const int W = g.nx + 1, H = g.ny + 1, r = n / W;
  i = n - r * W;
  j = r % H;
  k = r / H;
  return true;
}

static dim3 flat_grid3(const Grid& g) { return dim3((unsigned)((g.N + NB - 1) / NB)); }

// One thread per node, walked flat: the coarser levels, where the element
// kernel's 15 x 15 x 4 tiles would give too few workgroups.  The node sums
// the forces (or diagonal entries) of its 24 tetrahedra.
template <int MODE, bool FA, bool HASX, int RED, bool EIG, class T>
__global__ __launch_bounds__(NB) void k_node3d(Grid g, Mat m, const T* __restrict__ coef, T kell,
                                               const T* __restrict__ x, T* __restrict__ y,
                                               const T* __restrict__ b, const T* __restrict__ dg,
                                               const T* __restrict__ din, T* __restrict__ dout,
                                               T cd, T cr, int mask, Red red) {
  int i = 0, j = 0, k = 0;
  const bool in = flat_node3(g, i, j, k);
  double acc = 0.0;
  if (in) {
    const int N = g.N, n = i + (g.nx + 1) * (j + (g.ny + 1) * k);
    T f[3], d[3];
    node_force3d<FA, HASX, MODE == M3_DIAG, EIG>(g, m, coef, kell, x, i, j, k, f, d);
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
      } else if (MODE == M3_SMOOTH) {
        const T r = (b ? b[q] : T(0)) - f[c];
        T dd = cr * r / dg[q];
        if (din) dd += cd * din[q];
        T xo = (HASX ? x[q] : T(0)) + dd;
        if (fx) { xo = T(0); dd = T(0); }
        y[q] = xo;
        if (dout) dout[q] = dd;
      } else {
        y[q] = d[c];
      }
    }
  }
  if (RED != R3_NONE)
    block_reduce<NB, false>(acc, red, gridDim.x * gridDim.y * gridDim.z,
                            blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                            threadIdx.x + NB_X * threadIdx.y);
}

// Levels with at least g.elem_min nodes use the element kernels.
static bool use_elem3d(const Grid& g) { return g.N >= g.elem_min; }

static dim3 node_grid3(const Grid& g) {
  return dim3((g.nx + 1 + NB_X - 1) / NB_X, (g.ny + 1 + NB_Y - 1) / NB_Y, g.nz + 1);
}

static dim3 elem_grid3(const Grid& g) {
  return dim3((g.nx + 1 + E3_O - 1) / E3_O, (g.ny + 1 + E3_O - 1) / E3_O,
              (g.nz + 1 + E3_KZ - 1) / E3_KZ);
}

// the most blocks a reducing 3D launch on g uses (node and element grids)
int node_blocks3(const Grid& g) {
  const dim3 ge = elem_grid3(g), gn = node_grid3(g);
  const int ne = (int)(ge.x * ge.y * ge.z), nn = (int)(gn.x * gn.y * gn.z);
  return ne > nn ? ne : nn;
}

template <class T>
void launch_apply3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* y, const ND<T>* b, int mask, int red, Red r) {
  const bool el = use_elem3d(g);
  const dim3 gr = el ? elem_grid3(g) : flat_grid3(g);
  const dim3 bl = el ? dim3(E3_T, E3_T) : dim3(NB_X, NB_Y);
  const T k = T(kell);
  const bool eig = fine && g.eig_dT != 0.0;
#define A3(FA, RD, EG)                                                                          \
  do {                                                                                          \
    if (el)                                                                                     \
      hipLaunchKernelGGL((k_elem3d<M3_APPLY, FA, true, RD, EG, T>), gr, bl, 0, st, g, m, coef, k, x, \
                         y, b, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, T(0), T(0), mask, r); \
    else                                                                                        \
      hipLaunchKernelGGL((k_node3d<M3_APPLY, FA, true, RD, EG, T>), gr, bl, 0, st, g, m, coef, k, x, \
                         y, b, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, T(0), T(0), mask, r); \
  } while (0)
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
  const bool el = use_elem3d(g);
  const dim3 gr = el ? elem_grid3(g) : flat_grid3(g);
  const dim3 bl = el ? dim3(E3_T, E3_T) : dim3(NB_X, NB_Y);
  const T k = T(kell);
  const bool eig = fine && g.eig_dT != 0.0;
#define R3(FA, RD, EG)                                                                          \
  do {                                                                                          \
    if (el)                                                                                     \
      hipLaunchKernelGGL((k_elem3d<M3_RESID, FA, true, RD, EG, T>), gr, bl, 0, st, g, m, coef, k, x, \
                         r, b, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, T(0), T(0), 1, rr); \
    else                                                                                        \
      hipLaunchKernelGGL((k_node3d<M3_RESID, FA, true, RD, EG, T>), gr, bl, 0, st, g, m, coef, k, x, \
                         r, b, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, T(0), T(0), 1, rr); \
  } while (0)
  if (fine) {
    if (eig) { if (red) R3(true, R3_DOT, true); else R3(true, R3_NONE, true); }
    else { if (red) R3(true, R3_DOT, false); else R3(true, R3_NONE, false); }
  } else {
    if (red) R3(false, R3_DOT, false); else R3(false, R3_NONE, false);
  }
#undef R3
  if (red) launch_finish(st, rr, (int)(gr.x * gr.y * gr.z), false);
}

// First Chebyshev step from x = 0: d = cd d_in + cr D^{-1} b, x_out = d
// (no stencil); fixed DOFs zero.
template <class T>
__global__ __launch_bounds__(VB) void k_smooth0_3d(Grid g, const T* __restrict__ dg,
                                                   const T* __restrict__ b,
                                                   const T* __restrict__ din, T* __restrict__ x_out,
                                                   T* __restrict__ dout, T cd, T cr) {
  const int64_t N = g.N, W = g.nx + 1, H = g.ny + 1;
  for (int64_t q = blockIdx.x * (int64_t)VB + threadIdx.x; q < 3 * N; q += (int64_t)gridDim.x * VB) {
    const int c = (int)(q / N);
    const int64_t n = q - c * N;
    const int i = (int)(n % W), j = (int)((n / W) % H), k = (int)(n / (W * H));
    T dd = cr * b[q] / dg[q];
    if (din) dd += cd * din[q];
    if (fixed3(g, c, i, j, k)) dd = T(0);
    x_out[q] = dd;
    if (dout) dout[q] = dd;
  }
}

// One Jacobi-preconditioned Chebyshev step with the level's stored diagonal dg
// (launch_diag3d): d_new = cd d_in + cr D^{-1} (b - K x_in), x_out = x_in + d_new.
template <class T>
void launch_smooth3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                     const T* dg, double kell, const ND<T>* x_in, T* x_out, const T* b,
                     const ND<T>* d_in, ND<T>* d_out, double cd, double cr) {
  if (!x_in) {
    const int64_t n = 3 * (int64_t)g.N;
    const int nb = (int)std::min<int64_t>((n + VB - 1) / VB, VGRID);
    hipLaunchKernelGGL((k_smooth0_3d<T>), dim3(nb), dim3(VB), 0, st, g, dg, b, d_in, x_out, d_out,
                       T(cd), T(cr));
    return;
  }
  const bool el = use_elem3d(g);
  const dim3 gr = el ? elem_grid3(g) : flat_grid3(g);
  const dim3 bl = el ? dim3(E3_T, E3_T) : dim3(NB_X, NB_Y);
  Red none{};
  const T k = T(kell);
#define S3(FA)                                                                                  \
  do {                                                                                          \
    if (el)                                                                                     \
      hipLaunchKernelGGL((k_elem3d<M3_SMOOTH, FA, true, R3_NONE, false, T>), gr, bl, 0, st, g, m, \
                         coef, k, x_in, x_out, b, dg, d_in, d_out, T(cd), T(cr), 1, none);     \
    else                                                                                        \
      hipLaunchKernelGGL((k_node3d<M3_SMOOTH, FA, true, R3_NONE, false, T>), gr, bl, 0, st, g, m, \
                         coef, k, x_in, x_out, b, dg, d_in, d_out, T(cd), T(cr), 1, none);     \
  } while (0)
  if (fine) S3(true);
  else S3(false);
#undef S3
}

// dg = diag K on level g (fine: coefficients from nodal alpha; else the
// per-element array)
template <class T>
void launch_diag3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                   double kell, T* dg) {
  const bool el = use_elem3d(g);
  const dim3 gr = el ? elem_grid3(g) : flat_grid3(g);
  const dim3 bl = el ? dim3(E3_T, E3_T) : dim3(NB_X, NB_Y);
  Red none{};
  const T k = T(kell);
#define D3(FA)                                                                                  \
  do {                                                                                          \
    if (el)                                                                                     \
      hipLaunchKernelGGL((k_elem3d<M3_DIAG, FA, false, R3_NONE, false, T>), gr, bl, 0, st, g, m,  \
                         coef, k, (const T*)nullptr, dg, (const T*)nullptr, (const T*)nullptr,  \
                         (const T*)nullptr, (T*)nullptr, T(0), T(0), 0, none);                  \
    else                                                                                        \
      hipLaunchKernelGGL((k_node3d<M3_DIAG, FA, false, R3_NONE, false, T>), gr, bl, 0, st, g, m,  \
                         coef, k, (const T*)nullptr, dg, (const T*)nullptr, (const T*)nullptr,  \
                         (const T*)nullptr, (T*)nullptr, T(0), T(0), 0, none);                  \
  } while (0)
  if (fine) D3(true);
  else D3(false);
#undef D3
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

// Restriction with the coarse level's first Chebyshev step from zero
// (pointwise in 3D: x = d = cr D^{-1} b_c, fixed DOFs zero), one launch.
template <class T>
__global__ __launch_bounds__(NB) void k_restrict_smooth3d(Grid gf, Grid gc, const T* __restrict__ rf,
                                                          T* __restrict__ bc,
                                                          const T* __restrict__ dgc,
                                                          T* __restrict__ xc, T* __restrict__ dc,
                                                          T cr) {
  int I = 0, J = 0, K = 0;
  if (!flat_node3(gc, I, J, K)) return;
  restrict_node3d(gf, gc, rf, bc, I, J, K);
  const int nc = I + (gc.nx + 1) * (J + (gc.ny + 1) * K);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int q = nc + c * gc.N;
    T dd = cr * bc[q] / dgc[q];   // bc[q]: the value this thread has just written
    if (fixed3(gc, c, I, J, K)) dd = T(0);
    xc[q] = dd;
    if (dc) dc[q] = dd;
  }
}

template <class T>
void launch_restrict_smooth3d(hipStream_t st, const Grid& gf, const Grid& gc, const T* rf, T* bc,
                              const T* dgc, T* xc, T* dc, double cr) {
  hipLaunchKernelGGL((k_restrict_smooth3d<T>), flat_grid3(gc), dim3(NB_X, NB_Y), 0, st, gf, gc, rf,
                     bc, dgc, xc, dc, T(cr));
}

template <class T>
__global__ __launch_bounds__(NB) void k_prolong3d(Grid gf, Grid gc, const T* __restrict__ xc,
                                                  T* __restrict__ xf) {
  int i = 0, j = 0, k = 0;
  if (!flat_node3(gf, i, j, k)) return;
  prolong_node3d(gf, gc, xc, xf, i, j, k);
}

template <class T>
void launch_prolong3d(hipStream_t st, const Grid& gf, const Grid& gc, const T* xc, T* xf) {
  hipLaunchKernelGGL((k_prolong3d<T>), flat_grid3(gf), dim3(NB_X, NB_Y), 0, st, gf, gc, xc, xf);
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
// Per-thread constants of tet_helm: the tetrahedron volume and its mass and
// load factors, formed once (not once per tetrahedron).
struct TetK {
  double vol, m20, m4, m10;   // |T|, |T|/20, |T|/4, |T|/10
};

template <int HX, int HY, int HZ, int P, int V>
__device__ __forceinline__ void tet_helm(const Grid& g, const Helm3& hp,
                                         const double* __restrict__ w2, const double (&av)[27],
                                         int i, int j, int k, const double ih[3], const TetK& tk,
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
  const double mass = tk.m20 * (aV + a0 + a1 + a2 + a3);   // (M_e a)_v
  const double lap = tk.vol * (gvv[0] * grad[0] + gvv[1] * grad[1] + gvv[2] * grad[2]);
  Ha += (we + hp.cM) * mass + hp.cL * lap;
  gv += (we - hp.cm) * tk.m4;
  Hd += (we + hp.cM) * tk.m10 + hp.cL * tk.vol * (gvv[0] * gvv[0] + gvv[1] * gvv[1] + gvv[2] * gvv[2]);
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
  const TetK tk{vol, vol / 20.0, vol / 4.0, vol / 10.0};
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
#define HELM3(HX, HY, HZ, P, V) tet_helm<HX, HY, HZ, P, V>(g, hp, w2, av, i, j, k, ih, tk, Ha, gv, Hd);
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
  // nodes walked flat: rows of 129 nodes would leave a third of the
  // wavefronts of 64-wide row tiles with one busy lane
  int i = 0, j = 0, k = 0;
  const bool in = flat_node3(g, i, j, k);
  double p2 = 0.0, pm = 0.0, jlo = -INFINITY, jhi = -INFINITY;
  if (in) {
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
  dim3 gr = flat_grid3(g), bl(NB_X, NB_Y);
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
                                                  double* __restrict__ q, Box bx,
                                                  const double* __restrict__ S, Red r) {
  // one node of the box per thread: the inactive set of a thermal crack is a
  // layer a few nodes thick in x spanning every (j, k) row, so the box is
  // walked as one flat range rather than in 64-wide x tiles
  const int64_t qq = blockIdx.x * (int64_t)NB + threadIdx.x;
  const double beta = FIRST ? 0.0 : S[S_BETA];
  double acc = 0.0;
  if (qq < bx.n) {
    const int64_t n = box_index(bx, qq);
    const int W = g.nx + 1, H = g.ny + 1;
    const int i = (int)(n % W);
    const int64_t row = n / W;
    const int j = (int)(row % H), k = (int)(row / H);
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
  block_reduce<NB, false>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

// One damage-CG direction update and Hessian apply over the box of columns
// [i0, i1] and (j, k) rows [r0, r1] (row = j + (ny+1) k); p.q goes to the
// partials of r.  finish: reduce them here (returns 0), else return their
// count for the CG update to reduce.
int launch_helm_cg3d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                     const double* z, const double* p_old, const uint8_t* mask, double* p_new,
                     double* q, int r0, int r1, int i0, int i1, const double* S, bool first,
                     Red r, bool finish) {
  Helm3 hp{cL, cM, 0.0};
  const int rows = (g.ny + 1) * (g.nz + 1);
  if (r0 < 0) r0 = 0;
  if (r1 < 0 || r1 >= rows) r1 = rows - 1;
  if (i0 < 0) i0 = 0;
  if (i1 < 0 || i1 > g.nx) i1 = g.nx;
  if (i1 < i0 || r1 < r0) return 0;
  const int64_t W = g.nx + 1, w = i1 - i0 + 1;
  const Box bx{(int64_t)r0 * W + i0, W, w, (int64_t)(r1 - r0 + 1) * w};
  const int nb = (int)((bx.n + NB - 1) / NB);
  if (first)
    hipLaunchKernelGGL((k_helm_cg3d<true>), dim3(nb), dim3(NB), 0, st, g, hp, w2, z, p_old, mask,
                       p_new, q, bx, S, r);
  else
    hipLaunchKernelGGL((k_helm_cg3d<false>), dim3(nb), dim3(NB), 0, st, g, hp, w2, z, p_old, mask,
                       p_new, q, bx, S, r);
  if (!finish) return nb;
  launch_finish(st, r, nb, false);
  return 0;
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
  template void launch_smooth3d<T>(hipStream_t, const Grid&, const Mat&, bool, const T*, const T*, \
                                   double, const ND<T>*, T*, const T*, const ND<T>*, ND<T>*,     \
                                   double, double);                                              \
  template void launch_diag3d<T>(hipStream_t, const Grid&, const Mat&, bool, const T*, double,   \
                                 T*);                                                            \
  template void launch_restrict3d<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);       \
  template void launch_restrict_smooth3d<T>(hipStream_t, const Grid&, const Grid&, const T*, T*,  \
                                            const T*, T*, T*, double);                          \
  template void launch_prolong3d<T>(hipStream_t, const Grid&, const Grid&, const T*, T*);
INST3(float)
INST3(double)
#undef INST3

}  // namespace frac
