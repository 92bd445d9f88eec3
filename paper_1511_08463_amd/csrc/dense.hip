// Coarsest multigrid level: assemble the (small) Galerkin operator densely,
// invert it once per coefficient update in a single workgroup (symmetric
// sweeps in registers for the usual small sizes, Gauss-Jordan in global
// memory otherwise), and apply the symmetric inverse as a dense
// matrix-vector product.  Dirichlet rows and columns are replaced by the
// identity, so the inverse leaves them at zero when the right-hand side is.
#include "common.h"
#include "launch.h"

namespace frac {

constexpr int DB = 1024;

__device__ __forceinline__ bool fixed_dof2(const Grid& g, int comp, int i, int j) {
  if (g.bc == BC_SURFING_2D) return i == 0 || i == g.nx || j == 0 || j == g.ny;
  if (g.bc == BC_TSHOCK_2D) return comp == 0 ? (i == 0 || i == g.nx) : (j == g.ny);
  if (g.bc != BC_TENSION_2D) return false;
  return comp == 0 ? (i == 0 && j == 0) : (j == 0 || j == g.ny);
}

// Dense 2D assembly: each thread owns one node and writes its two rows, summing
// the 6x6 element matrices abar |T| B^T D B of the triangles around it.
__global__ __launch_bounds__(DB) void k_dense_assemble2d(Grid g, Mat m, const double* __restrict__ abar,
                                                         double* __restrict__ A,
                                                         const double* __restrict__ S) {
  if (S[S_COARSE_REFRESH] == 0.0) return;   // uniform: the whole block keeps the old system
  const int N = g.N, n2 = 2 * N, W = g.nx + 1;
  for (int k = threadIdx.x; k < n2 * n2; k += DB) A[k] = 0.0;
  __syncthreads();
  const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy, area = 0.5 * g.hx * g.hy;
  for (int n = threadIdx.x; n < N; n += DB) {
    const int i = n % W, j = n / W;
    // six triangles around the node: (cell di, dj, type, local vertex)
    const int tdi[6] = {0, 0, -1, -1, -1, 0}, tdj[6] = {0, 0, 0, -1, -1, -1};
    const int tt[6] = {0, 1, 0, 0, 1, 1}, tv[6] = {0, 0, 1, 2, 1, 2};
    for (int k = 0; k < 6; ++k) {
      const int ci = i + tdi[k], cj = j + tdj[k];
      if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
      const int t = tt[k], v = tv[k];
      double gx[3], gy[3];
      int vi[3], vj[3];
      vi[0] = 0; vj[0] = 0;
      if (t == 0) {
        gx[0] = -ihx; gy[0] = 0.0; gx[1] = ihx; gy[1] = -ihy; gx[2] = 0.0; gy[2] = ihy;
        vi[1] = 1; vj[1] = 0; vi[2] = 1; vj[2] = 1;
      } else {
        gx[0] = 0.0; gy[0] = -ihy; gx[1] = ihx; gy[1] = 0.0; gx[2] = -ihx; gy[2] = ihy;
        vi[1] = 1; vj[1] = 1; vi[2] = 0; vj[2] = 1;
      }
      const double w = abar[2 * (ci + g.nx * cj) + t] * area;
      for (int b = 0; b < 3; ++b) {
        const int nb = (ci + vi[b]) + W * (cj + vj[b]);
        const double kxx = w * (m.l2m * gx[v] * gx[b] + m.mu * gy[v] * gy[b]);
        const double kxy = w * (m.lam * gx[v] * gy[b] + m.mu * gy[v] * gx[b]);
        const double kyx = w * (m.lam * gy[v] * gx[b] + m.mu * gx[v] * gy[b]);
        const double kyy = w * (m.l2m * gy[v] * gy[b] + m.mu * gx[v] * gx[b]);
        A[(size_t)n * n2 + nb] += kxx;
        A[(size_t)n * n2 + N + nb] += kxy;
        A[(size_t)(N + n) * n2 + nb] += kyx;
        A[(size_t)(N + n) * n2 + N + nb] += kyy;
      }
    }
  }
  __syncthreads();
  // Dirichlet rows/columns -> identity
  for (int r = threadIdx.x; r < n2; r += DB) {
    const int comp = r / N, n = r % N;
    if (fixed_dof2(g, comp, n % W, n / W)) {
      for (int c = 0; c < n2; ++c) {
        A[(size_t)r * n2 + c] = (c == r) ? 1.0 : 0.0;
        A[(size_t)c * n2 + r] = (c == r) ? 1.0 : 0.0;
      }
    }
  }
}

// In-place Gauss-Jordan inverse of an SPD matrix (no pivoting) in global
// memory, then symmetrisation into Ainv (any n up to DENSE_MAX).
__global__ __launch_bounds__(DB) void k_gauss_jordan(int n, double* __restrict__ A,
                                                     double* __restrict__ Ainv,
                                                     const double* __restrict__ S) {
  if (S[S_COARSE_REFRESH] == 0.0) return;
  extern __shared__ double sm[];
  double* colk = sm;
  double* rowk = sm + n;
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += DB) colk[i] = A[(size_t)i * n + k];
    __syncthreads();
    const double piv = 1.0 / colk[k];
    for (int j = threadIdx.x; j < n; j += DB) {
      const double v = ((j == k) ? 1.0 : A[(size_t)k * n + j]) * piv;
      rowk[j] = v;
      A[(size_t)k * n + j] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += DB) {
      const int i = e / n, j = e % n;
      if (i == k) continue;
      const double base = (j == k) ? 0.0 : A[e];
      A[e] = base - colk[i] * rowk[j];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += DB) {
    const int i = e / n, j = e % n;
    Ainv[e] = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
  }
}

// Small coarsest levels (n <= GJ_NMAX): the symmetric sweep operator on the
// lower triangle, held in registers.  Sweeping pivot k with d = A_kk maps
//   A_ij -> A_ij - A_ik A_jk / d  (i, j != k),  A_ik -> A_ik / d,  A_kk -> -1/d,
// which keeps the matrix symmetric; after all n pivots it holds -A^{-1}.
// Thread t owns the lower-triangle entries e = t + q DB (row-major packed);
// at step k the owners of column k publish it through LDS and every thread
// updates its own entries: two workgroup barriers per step and no global
// memory traffic.
constexpr int GJ_Q = 14;
constexpr int GJ_NMAX = 168;   // n (n + 1) / 2 <= DB * GJ_Q

__global__ __launch_bounds__(DB) void k_sweep_inverse(int n, const double* __restrict__ A,
                                                      double* __restrict__ Ainv,
                                                      const double* __restrict__ S) {
  if (S[S_COARSE_REFRESH] == 0.0) return;
  extern __shared__ double colk[];
  const int ne = n * (n + 1) / 2, t = threadIdx.x;
  double a[GJ_Q];
  int ij[GJ_Q];   // (row << 16) | column with row >= column, or -1 past the end
#pragma unroll
  for (int q = 0; q < GJ_Q; ++q) {
    const int e = t + q * DB;
    int r = -1, c = 0;
    if (e < ne) {
      r = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while (r * (r + 1) / 2 > e) --r;
      while ((r + 1) * (r + 2) / 2 <= e) ++r;
      c = e - r * (r + 1) / 2;
    }
    ij[q] = r < 0 ? -1 : (r << 16) | c;
    a[q] = r < 0 ? 0.0 : A[(size_t)r * n + c];
  }
  for (int k = 0; k < n; ++k) {
    // column k of the symmetric matrix: entries (i, k) for i >= k, (k, j) for j < k
#pragma unroll
    for (int q = 0; q < GJ_Q; ++q) {
      if (ij[q] < 0) continue;
      const int i = ij[q] >> 16, j = ij[q] & 0xffff;
      if (j == k) colk[i] = a[q];
      else if (i == k) colk[j] = a[q];
    }
    __syncthreads();
    const double d = colk[k], inv = 1.0 / d;
#pragma unroll
    for (int q = 0; q < GJ_Q; ++q) {
      if (ij[q] < 0) continue;
      const int i = ij[q] >> 16, j = ij[q] & 0xffff;
      if (i == k && j == k) a[q] = -inv;
      else if (i == k) a[q] = colk[j] * inv;
      else if (j == k) a[q] = colk[i] * inv;
      else a[q] -= colk[i] * colk[j] * inv;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < GJ_Q; ++q) {
    if (ij[q] < 0) continue;
    const int i = ij[q] >> 16, j = ij[q] & 0xffff;
    Ainv[(size_t)i * n + j] = -a[q];
    Ainv[(size_t)j * n + i] = -a[q];
  }
}

// Whether the coarsest coefficients abar (ne elements) have drifted from ref,
// those the current inverse was formed from, by more than a relative tol
// anywhere (ref not finite or not positive counts as drifted).  On drift
// S[S_COARSE_REFRESH] = 1 and ref <- abar, else 0.  A coarse correction from
// a slightly older but still symmetric positive definite coarse operator
// keeps the V-cycle a fixed SPD preconditioner; only its quality changes.
__global__ __launch_bounds__(DB) void k_coarse_drift(int ne, const double* __restrict__ abar,
                                                     double* __restrict__ ref,
                                                     double* __restrict__ S, double tol) {
  __shared__ double sh[DB / WAVE];
  __shared__ int refresh;
  double m = 0.0;
  for (int e = threadIdx.x; e < ne; e += DB) {
    const double r = ref[e];
    const double rel = (r > 0.0 && isfinite(r)) ? fabs(abar[e] - r) / r : INFINITY;
    m = fmax(m, isnan(rel) ? INFINITY : rel);
  }
  m = wave_max(m);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (lane == 0) sh[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = sh[0];
    for (int k = 1; k < DB / WAVE; ++k) a = fmax(a, sh[k]);
    refresh = !(a <= tol);
    S[S_COARSE_REFRESH] = refresh ? 1.0 : 0.0;
  }
  __syncthreads();
  if (refresh)
    for (int e = threadIdx.x; e < ne; e += DB) ref[e] = abar[e];
}

void launch_dense_setup(hipStream_t st, const Grid& g, const Mat& m, const double* abar,
                        double* A, double* Ainv, double* ref, double* S, double tol) {
  const int n = g.dim * g.N;
  const int ne = g.dim == 3 ? 6 * g.nx * g.ny * g.nz : 2 * g.nx * g.ny;
  hipLaunchKernelGGL(k_coarse_drift, dim3(1), dim3(DB), 0, st, ne, abar, ref, S, tol);
  if (g.dim == 3) launch_dense_assemble3d(st, g, m, abar, A, S);
  else hipLaunchKernelGGL(k_dense_assemble2d, dim3(1), dim3(DB), 0, st, g, m, abar, A, S);
  if (n <= GJ_NMAX)
    hipLaunchKernelGGL(k_sweep_inverse, dim3(1), dim3(DB), n * sizeof(double), st, n, A, Ainv, S);
  else
    hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(DB), 2 * n * sizeof(double), st, n, A, Ainv, S);
}

// x = Ainv b (dense, one block, b in LDS; float64 accumulation for either
// value type of b and x): wave w forms rows w, w + 16, ...; its lanes read a
// row with consecutive addresses and the partial sums meet in a wave
// reduction.
template <class T>
__global__ __launch_bounds__(DB) void k_dense_solve(int n, const double* __restrict__ Ainv,
                                                    const T* __restrict__ b, T* __restrict__ x) {
  extern __shared__ double sb[];
  for (int i = threadIdx.x; i < n; i += DB) sb[i] = (double)b[i];
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  for (int i = w; i < n; i += DB / WAVE) {
    const double* row = Ainv + (size_t)i * n;
    double s = 0.0;
    for (int j = lane; j < n; j += WAVE) s += row[j] * sb[j];
    s = wave_sum(s);
    if (lane == 0) x[i] = T(s);
  }
}

template <class T>
void launch_dense_solve(hipStream_t st, int n, const double* Ainv, const T* b, T* x) {
  hipLaunchKernelGGL((k_dense_solve<T>), dim3(1), dim3(DB), n * sizeof(double), st, n, Ainv, b, x);
}
template void launch_dense_solve<float>(hipStream_t, int, const double*, const float*, float*);
template void launch_dense_solve<double>(hipStream_t, int, const double*, const double*, double*);

}  // namespace frac
