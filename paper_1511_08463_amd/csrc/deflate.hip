// Crack-aware deflation of the elastic CG (2D): the per-fragment rigid modes
// that Sec. 3.1 names as a possible improvement of the elastic solve.
//
// Fragments are the connected components of the undamaged nodes
// {alpha < theta} in the graph of the element edges (horizontal, vertical and
// the (i, j)-(i+1, j+1) diagonal of the right-diagonal triangles).  They are
// found by a lock-free union-find over the grid:
//   k_cc_init     parent[n] = -1 on damaged nodes; runs of undamaged nodes
//                 along a row within one wavefront become one tree each;
//   k_cc_link     the unions left (across wavefront segments, and between
//                 rows): the larger of two roots is linked under the smaller
//                 by compare-and-swap, so parent indices only decrease along
//                 a path and the root of every final tree is its component's
//                 smallest node index -- the same labels whatever the order
//                 in which threads run;
//   k_cc_flatten  label[n] = root of n;
//   k_cc_count    component sizes (atomic adds: one for the lanes of a
//                 wavefront that share lane 0's label, one per other lane);
//                 the add that takes a component to min_nodes records its
//                 root in a candidate list;
//   k_cc_select   keeps at most max_fragments candidates, the largest first,
//                 ties by the smaller root;
//   k_cc_fid      fid[n] = fragment of node n, -1 when none.
// The coarse space W holds three modes per fragment, the x and y translations
// and the rotation (-(y - yc), x - xc) s about the domain centre,
// s = 2 / max(lx, ly), zero off the fragment and on Dirichlet DOFs.  Its
// columns are never stored: every kernel evaluates them from fid and the
// node's coordinates.  W^T v is a deterministic two-pass reduction (per-block
// partials of all DFL_M modes, summed in a fixed order by one block).
// E = W^T K W is formed column by column from K applied to each mode, and
// inverted by a Cholesky factorisation that drops a mode whose pivot falls
// below a relative threshold (a mode dependent on the others).
#include "common.h"
#include "launch.h"
#include "ops2d.h"

namespace frac {

namespace {

__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, halving the path on the way (every write stores an ancestor, and
// only into a node that is no longer a root, so no link is lost).
__device__ int uf_find(int* parent, int x) {
  for (;;) {
    const int p = ld_agent(parent + x);
    if (p == x) return x;
    const int gp = ld_agent(parent + p);
    if (gp == p) return p;
    __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = gp;
  }
}

// Each failed compare-and-swap means another thread linked that root, so the
// number of roots falls and the loop ends.
__device__ void uf_union(int* parent, int a, int b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) { const int t = a; a = b; b = t; }
    int expect = a;
    if (__hip_atomic_compare_exchange_strong(parent + a, &expect, b, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

// Value of rigid mode t (0: x translation, 1: y translation, 2: rotation) of
// a fragment at node (i, j), before the Dirichlet mask.
__device__ __forceinline__ void rigid2d(const Grid& g, int t, int i, int j, double& vx,
                                        double& vy) {
  const double lx = g.nx * g.hx, ly = g.ny * g.hy;
  const double s = 2.0 / fmax(lx, ly);
  if (t == 0) { vx = 1.0; vy = 0.0; }
  else if (t == 1) { vx = 0.0; vy = 1.0; }
  else { vx = -(j * g.hy - 0.5 * ly) * s; vy = (i * g.hx - 0.5 * lx) * s; }
}

// parent[n] = -1 on damaged nodes; on undamaged ones, the first node of its
// run of undamaged nodes in the same grid row within the same 64-node
// wavefront (runs break at damaged nodes, row starts and wavefront edges),
// so every run is one tree whose root is its smallest index.
__global__ __launch_bounds__(VB) void k_cc_init(Grid g, const double* __restrict__ alpha,
                                                double theta, int* __restrict__ parent,
                                                int* __restrict__ meta) {
  static_assert(VB % WAVE == 0, "wavefronts cover aligned 64-node segments");
  const int n = blockIdx.x * VB + threadIdx.x, N = g.N, W = g.nx + 1;
  if (n == 0) meta[DFL_META_NCAND] = 0;
  const int lane = threadIdx.x & (WAVE - 1);
  const bool solid = n < N && alpha[n] < theta;
  const unsigned long long sm = __ballot(solid);
  const bool prev = lane > 0 && ((sm >> (lane - 1)) & 1ull);
  const unsigned long long st = __ballot(solid && (!prev || n % W == 0));
  if (n >= N) return;
  if (!solid) {
    parent[n] = -1;
    return;
  }
  const unsigned long long upto = lane == WAVE - 1 ? ~0ull : ((2ull << lane) - 1);
  parent[n] = n - (lane - (WAVE - 1 - __builtin_clzll(st & upto)));
}

// The unions the runs of k_cc_init leave: horizontal edges across 64-node
// segments; vertical edges once per stretch of columns where both rows are
// undamaged (the rest of the stretch is joined through the two runs);
// diagonal edges (i, j)-(i+1, j+1) only where neither (i+1, j) nor (i, j+1)
// is undamaged (otherwise a horizontal and a vertical edge join them).  The
// components, hence the labels, are those of all element edges.  A node is
// undamaged exactly when its parent entry is not negative.
__global__ __launch_bounds__(NB) void k_cc_link(Grid g, int* parent) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y;
  if (i > g.nx || j > g.ny) return;
  const int W = g.nx + 1, n = i + W * j;
  if (ld_agent(parent + n) < 0) return;           // damaged: never linked
  const bool right = i < g.nx && ld_agent(parent + n + 1) >= 0;
  if (right && ((n + 1) & (WAVE - 1)) == 0) uf_union(parent, n, n + 1);
  if (j == g.ny) return;
  const bool up = ld_agent(parent + n + W) >= 0;
  if (up && !(i > 0 && ld_agent(parent + n - 1) >= 0 && ld_agent(parent + n + W - 1) >= 0))
    uf_union(parent, n, n + W);
  if (i < g.nx && !up && !right && ld_agent(parent + n + W + 1) >= 0)
    uf_union(parent, n, n + W + 1);
}

// The forest is final here: plain reads follow each path to its root.
__global__ __launch_bounds__(VB) void k_cc_flatten(int N, const int* __restrict__ parent,
                                                   int* __restrict__ label) {
  const int n = blockIdx.x * VB + threadIdx.x;
  if (n >= N) return;
  int x = parent[n];
  if (x >= 0)
    while (parent[x] != x) x = parent[x];
  label[n] = x;
}

__global__ __launch_bounds__(VB) void k_fill_int(int N, int* __restrict__ a, int v) {
  const int n = blockIdx.x * VB + threadIdx.x;
  if (n < N) a[n] = v;
}

__global__ __launch_bounds__(VB) void k_cc_count(int N, const int* __restrict__ label,
                                                 int* cnt, int min_nodes, int* meta) {
  const int n = blockIdx.x * VB + threadIdx.x;
  const int r = n < N ? label[n] : -1;
  const int lane = threadIdx.x & (WAVE - 1);
  const int r0 = __shfl(r, 0, WAVE);
  const unsigned long long same = __ballot(r == r0);
  if (r < 0) return;
  int add = 1;
  bool leader = true;
  if (r == r0) {
    add = __popcll(same);
    leader = lane == __builtin_ctzll(same);
  }
  if (!leader) return;
  const int old = atomicAdd(cnt + r, add);
  if (old < min_nodes && old + add >= min_nodes) {
    const int k = atomicAdd(meta + DFL_META_NCAND, 1);
    if (k < DFL_LIST) meta[DFL_META_LIST + k] = r;
  }
}

// One thread: the max_fragments largest candidates, ties by the smaller root.
__global__ void k_cc_select(const int* __restrict__ cnt, int* __restrict__ meta, int fmax) {
  if (threadIdx.x != 0) return;
  const int nc = min(meta[DFL_META_NCAND], DFL_LIST);
  int nf = 0;
  for (; nf < fmax; ++nf) {
    int best = -1, bs = -1;
    for (int k = 0; k < nc; ++k) {
      const int r = meta[DFL_META_LIST + k];
      bool taken = false;
      for (int q = 0; q < nf; ++q) taken |= meta[DFL_META_ROOTS + q] == r;
      if (taken) continue;
      const int s = cnt[r];
      if (s > bs || (s == bs && r < best)) { best = r; bs = s; }
    }
    if (best < 0) break;
    meta[DFL_META_ROOTS + nf] = best;
  }
  meta[DFL_META_NFRAG] = nf;
}

__global__ __launch_bounds__(VB) void k_cc_fid(int N, const int* __restrict__ label,
                                               const int* __restrict__ meta,
                                               int* __restrict__ fid) {
  const int n = blockIdx.x * VB + threadIdx.x;
  if (n >= N) return;
  const int r = label[n], nf = meta[DFL_META_NFRAG];
  int f = -1;
  if (r >= 0)
    for (int k = 0; k < nf; ++k)
      if (meta[DFL_META_ROOTS + k] == r) f = k;
  fid[n] = f;
}

// Per-block partials of W^T v (DFL_M values per block, grid-stride order).
__global__ __launch_bounds__(VB) void k_dfl_wtv(Grid g, const int* __restrict__ fid,
                                                const double* __restrict__ v,
                                                double* __restrict__ part) {
  __shared__ double sh[VB / WAVE][DFL_M];
  double acc[DFL_M];
#pragma unroll
  for (int k = 0; k < DFL_M; ++k) acc[k] = 0.0;
  const int N = g.N, W = g.nx + 1;
  for (int n = blockIdx.x * VB + threadIdx.x; n < N; n += gridDim.x * VB) {
    const int f = fid[n];
    if (f < 0) continue;
    const int i = n % W, j = n / W;
    const double vx = fixed_x2(g, i, j) ? 0.0 : v[n];
    const double vy = fixed_y2(g, i, j) ? 0.0 : v[n + N];
    double rx, ry;
    rigid2d(g, 2, i, j, rx, ry);
#pragma unroll
    for (int q = 0; q < DFL_FMAX; ++q)
      if (q == f) {
        acc[3 * q] += vx;
        acc[3 * q + 1] += vy;
        acc[3 * q + 2] += vx * rx + vy * ry;
      }
  }
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
  for (int k = 0; k < DFL_M; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) sh[w][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < DFL_M) {
    double s = 0.0;
    for (int q = 0; q < VB / WAVE; ++q) s += sh[q][threadIdx.x];
    part[(size_t)blockIdx.x * DFL_M + threadIdx.x] = s;
  }
}

// Sums the partials: c = W^T v.  Thread t adds the entries t, t + FINT, ...
// of the [nblocks][DFL_M] partials (FINT a multiple of DFL_M, so all of
// them belong to mode t % DFL_M), then thread k < DFL_M adds its mode's FINT /
// DFL_M thread sums in thread order: a fixed order, whatever the schedule.
// col >= 0 stores c as column col of E; otherwise mu = E^{-1} c.
constexpr int FINT = 40 * DFL_M;
__global__ __launch_bounds__(FINT) void k_dfl_finish(const double* __restrict__ part, int nblocks,
                                                     int col, double* __restrict__ E,
                                                     const double* __restrict__ Einv,
                                                     double* __restrict__ mu) {
  __shared__ double sh[FINT];
  __shared__ double c[DFL_M];
  const int t = threadIdx.x, total = nblocks * DFL_M;
  double s = 0.0;
  for (int e = t; e < total; e += FINT) s += part[e];
  sh[t] = s;
  __syncthreads();
  if (t < DFL_M) {
    double a = 0.0;
    for (int q = t; q < FINT; q += DFL_M) a += sh[q];
    c[t] = a;
    if (col >= 0) E[t * DFL_M + col] = a;
  }
  __syncthreads();
  if (col < 0 && t < DFL_M) {
    double a = 0.0;
    for (int l = 0; l < DFL_M; ++l) a += Einv[t * DFL_M + l] * c[l];
    mu[t] = a;
  }
}

// One thread: Einv = (L L^T)^+ over the modes kept by the factorisation,
// zero rows and columns for the rest and for modes beyond 3 nfrag.
__global__ void k_dfl_invert(const double* __restrict__ E, double* __restrict__ Einv,
                             const int* __restrict__ meta) {
  __shared__ double L[DFL_M * DFL_M], Li[DFL_M * DFL_M];
  __shared__ int keep[DFL_M];
  if (threadIdx.x != 0) return;
  const int m = 3 * meta[DFL_META_NFRAG];
  double dmax = 0.0;
  for (int j = 0; j < m; ++j) dmax = fmax(dmax, fabs(E[j * DFL_M + j]));
  for (int a = 0; a < DFL_M * DFL_M; ++a) { L[a] = 0.0; Li[a] = 0.0; }
  for (int j = 0; j < m; ++j) {
    double d = E[j * DFL_M + j];
    for (int k = 0; k < j; ++k) d -= L[j * DFL_M + k] * L[j * DFL_M + k];
    keep[j] = d > DFL_PIVOT * dmax;
    if (!keep[j]) continue;
    const double ljj = sqrt(d);
    L[j * DFL_M + j] = ljj;
    for (int i = j + 1; i < m; ++i) {
      double s = 0.5 * (E[i * DFL_M + j] + E[j * DFL_M + i]);
      for (int k = 0; k < j; ++k) s -= L[i * DFL_M + k] * L[j * DFL_M + k];
      L[i * DFL_M + j] = s / ljj;
    }
  }
  // Li = L^{-1} on the kept indices (forward substitution per column)
  for (int c = 0; c < m; ++c) {
    if (!keep[c]) continue;
    for (int i = c; i < m; ++i) {
      if (!keep[i]) continue;
      double s = i == c ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= L[i * DFL_M + k] * Li[k * DFL_M + c];
      Li[i * DFL_M + c] = s / L[i * DFL_M + i];
    }
  }
  for (int i = 0; i < DFL_M; ++i)
    for (int j = 0; j < DFL_M; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += Li[k * DFL_M + i] * Li[k * DFL_M + j];
      Einv[i * DFL_M + j] = s;
    }
}

// x += sign W mu (mode_k < 0), or x = column mode_k of W.
__global__ __launch_bounds__(NB) void k_dfl_add(Grid g, const int* __restrict__ fid,
                                                const double* __restrict__ mu, double* x,
                                                double sign, int mode_k) {
  const int i = blockIdx.x * NB_X + threadIdx.x, j = blockIdx.y * NB_Y + threadIdx.y;
  if (i > g.nx || j > g.ny) return;
  const int N = g.N, n = i + (g.nx + 1) * j;
  const int f = fid[n];
  const bool fx = fixed_x2(g, i, j), fy = fixed_y2(g, i, j);
  if (mode_k >= 0) {
    double vx = 0.0, vy = 0.0;
    if (f == mode_k / 3) rigid2d(g, mode_k % 3, i, j, vx, vy);
    x[n] = fx ? 0.0 : vx;
    x[n + N] = fy ? 0.0 : vy;
    return;
  }
  if (f < 0) return;
  double rx, ry;
  rigid2d(g, 2, i, j, rx, ry);
  const double m0 = mu[3 * f], m1 = mu[3 * f + 1], m2 = mu[3 * f + 2];
  if (!fx) x[n] += sign * (m0 + m2 * rx);
  if (!fy) x[n + N] += sign * (m1 + m2 * ry);
}

dim3 nodes2(const Grid& g) { return dim3((g.nx + NB_X) / NB_X, (g.ny + NB_Y) / NB_Y); }
int vblocks(int64_t n) { return (int)((n + VB - 1) / VB); }

}  // namespace

int dfl_part_blocks(int64_t N) {
  const int64_t b = (N + VB - 1) / VB;
  return (int)(b < VGRID ? (b < 1 ? 1 : b) : VGRID);
}

void launch_fragments2d(hipStream_t st, const Grid& g, const double* alpha, double theta,
                        int min_nodes, int fmax, int* parent, int* label, int* fid, int* meta) {
  const int N = g.N;
  hipLaunchKernelGGL(k_cc_init, dim3(vblocks(N)), dim3(VB), 0, st, g, alpha, theta, parent, meta);
  hipLaunchKernelGGL(k_cc_link, nodes2(g), dim3(NB_X, NB_Y), 0, st, g, parent);
  hipLaunchKernelGGL(k_cc_flatten, dim3(vblocks(N)), dim3(VB), 0, st, N, parent, label);
  hipLaunchKernelGGL(k_fill_int, dim3(vblocks(N)), dim3(VB), 0, st, N, parent, 0);
  hipLaunchKernelGGL(k_cc_count, dim3(vblocks(N)), dim3(VB), 0, st, N, label, parent, min_nodes,
                     meta);
  hipLaunchKernelGGL(k_cc_select, dim3(1), dim3(WAVE), 0, st, parent, meta, fmax);
  hipLaunchKernelGGL(k_cc_fid, dim3(vblocks(N)), dim3(VB), 0, st, N, label, meta, fid);
}

void launch_dfl_mode(hipStream_t st, const Grid& g, const int* fid, int k, double* w) {
  hipLaunchKernelGGL(k_dfl_add, nodes2(g), dim3(NB_X, NB_Y), 0, st, g, fid, nullptr, w, 0.0, k);
}

void launch_dfl_add(hipStream_t st, const Grid& g, const int* fid, const double* mu, double* x,
                    double sign) {
  hipLaunchKernelGGL(k_dfl_add, nodes2(g), dim3(NB_X, NB_Y), 0, st, g, fid, mu, x, sign, -1);
}

void launch_dfl_wtv(hipStream_t st, const Grid& g, const int* fid, const double* v, double* part,
                    int col, double* E, const double* Einv, double* mu) {
  const int nb = dfl_part_blocks(g.N);
  hipLaunchKernelGGL(k_dfl_wtv, dim3(nb), dim3(VB), 0, st, g, fid, v, part);
  hipLaunchKernelGGL(k_dfl_finish, dim3(1), dim3(FINT), 0, st, part, nb, col, E, Einv, mu);
}

void launch_dfl_invert(hipStream_t st, const double* E, double* Einv, const int* meta) {
  hipLaunchKernelGGL(k_dfl_invert, dim3(1), dim3(WAVE), 0, st, E, Einv, meta);
}

}  // namespace frac
