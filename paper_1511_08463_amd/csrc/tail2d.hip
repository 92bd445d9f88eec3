// Bottom of the 2D multigrid V-cycle in one workgroup.
//
// On the smallest levels every kernel of a V-cycle costs a few microseconds
// of launch and memory latency while doing almost no work.  This kernel runs
// the last few smoothed levels (pre-smoothing, residual, restriction), the
// dense coarsest solve and the way back up (prolongation, post-smoothing)
// in a single workgroup, with all vectors and element coefficients of those
// levels resident in LDS and a workgroup barrier between the steps.  Every
// step applies the same per-node arithmetic, in the same order, as the
// per-level kernels, so the result equals the kernel-per-step V-cycle.
#include "common.h"
#include "launch.h"
#include "ops2d.h"

namespace frac {

constexpr int TB = 1024;

static size_t level_words(const Grid& g) {
  return (size_t)2 * g.nx * g.ny + (size_t)5 * 2 * g.N;
}

size_t tail_lds_bytes(const Grid* g, int nl, int n, size_t elem) {
  size_t w = 2 * (size_t)n;
  for (int l = 0; l < nl; ++l) w += level_words(g[l]);
  return w * elem;
}

// One Jacobi-Chebyshev step on level g over LDS vectors (see launch_smooth2d).
template <bool HASX, class T>
__device__ __forceinline__ void tail_smooth(const Grid& g, const Mat& m, const T* coef, T kell,
                                            const T* x_in, T* x_out, const T* b, const T* d_in,
                                            T* d_out, T cd, T cr) {
  const int W = g.nx + 1, N = g.N;
  double acc = 0.0;
  for (int n = threadIdx.x; n < N; n += TB) {
    const int i = n % W, j = n / W;
    T c[6];
    coef6<false>(g, coef, kell, i, j, c);
    T fx, fy, dx, dy;
    node_force2d<HASX, true>(g, m, c, x_in, x_in + N, i, j, fx, fy, dx, dy);
    const T xc = HASX ? x_in[n] : T(0), yc = HASX ? x_in[n + N] : T(0);
    node_out2d<M_SMOOTH, R_NONE>(g, i, j, fx, fy, dx, dy, xc, yc, x_out, b, d_in, d_out, cd, cr,
                                 1, acc);
  }
}

template <class T>
__global__ __launch_bounds__(TB) void k_vtail2d(TailArgs<T> a) {
  __shared__ T lds[TAIL_LDS_BYTES / sizeof(T)];
  T *coef[TAIL_MAX_LEVELS], *b[TAIL_MAX_LEVELS + 1], *xa[TAIL_MAX_LEVELS + 1];
  T *xb[TAIL_MAX_LEVELS], *d[TAIL_MAX_LEVELS], *r[TAIL_MAX_LEVELS], *res[TAIL_MAX_LEVELS + 1];
  const int nl = a.nl, t = threadIdx.x;
  {
    size_t off = 0;
    for (int l = 0; l < nl; ++l) {
      const Grid& g = a.g[l];
      const int n2 = 2 * g.N;
      coef[l] = lds + off; off += (size_t)2 * g.nx * g.ny;
      b[l] = lds + off; off += n2;
      xa[l] = lds + off; off += n2;
      xb[l] = lds + off; off += n2;
      d[l] = lds + off; off += n2;
      r[l] = lds + off; off += n2;
    }
    b[nl] = lds + off; off += a.dense_n;
    xa[nl] = lds + off;
  }
  for (int l = 0; l < nl; ++l)
    for (int e = t; e < 2 * a.g[l].nx * a.g[l].ny; e += TB) coef[l][e] = a.coef[l][e];
  for (int e = t; e < 2 * a.g[0].N; e += TB) b[0][e] = a.b[e];
  __syncthreads();
  const T kell = T(a.kell);
  const int k = a.k;
  double acc = 0.0;
  // down: pre-smoothing from zero, residual, restriction
  for (int l = 0; l < nl; ++l) {
    const Grid& g = a.g[l];
    T* cur = nullptr;
    for (int s = 0; s < k; ++s) {
      T* out = (s % 2 == 0) ? xa[l] : xb[l];
      const T* din = s == 0 ? nullptr : (s == 1 ? cur : d[l]);
      T* dout = (s < k - 1) ? d[l] : nullptr;
      if (cur) tail_smooth<true>(g, a.m, coef[l], kell, cur, out, b[l], din, dout, T(a.cd[s]), T(a.cr[s]));
      else tail_smooth<false>(g, a.m, coef[l], kell, cur, out, b[l], din, dout, T(a.cd[s]), T(a.cr[s]));
      __syncthreads();
      cur = out;
    }
    res[l] = cur;
    const int W = g.nx + 1, N = g.N;
    for (int n = t; n < N; n += TB) {
      const int i = n % W, j = n / W;
      T c[6];
      coef6<false>(g, coef[l], kell, i, j, c);
      T fx, fy, dx, dy;
      node_force2d<true, false>(g, a.m, c, cur, cur + N, i, j, fx, fy, dx, dy);
      node_out2d<M_RESID, R_NONE>(g, i, j, fx, fy, dx, dy, cur[n], cur[n + N], r[l], b[l],
                                  (const T*)nullptr, (T*)nullptr, T(0), T(0), 1, acc);
    }
    __syncthreads();
    const Grid& gc = a.g[l + 1];
    const int Wc = gc.nx + 1;
    for (int n = t; n < gc.N; n += TB) restrict_node2d(g, gc, r[l], b[l + 1], n % Wc, n / Wc);
    __syncthreads();
  }
  // coarsest level: x = Ainv b, one wave per row (as k_dense_solve)
  {
    const int n = a.dense_n, lane = t & (WAVE - 1), w = t / WAVE;
    for (int i = w; i < n; i += TB / WAVE) {
      const double* row = a.Ainv + (size_t)i * n;
      double s = 0.0;
      for (int j = lane; j < n; j += WAVE) s += row[j] * (double)b[nl][j];
      s = wave_sum(s);
      if (lane == 0) xa[nl][i] = T(s);
    }
    res[nl] = xa[nl];
  }
  __syncthreads();
  // up: prolongation, post-smoothing
  for (int l = nl - 1; l >= 0; --l) {
    const Grid& g = a.g[l];
    const Grid& gc = a.g[l + 1];
    const int W = g.nx + 1;
    T* cur = res[l];
    for (int n = t; n < g.N; n += TB) prolong_node2d(g, gc, res[l + 1], cur, n % W, n / W);
    __syncthreads();
    for (int s = 0; s < k; ++s) {
      T* out = (cur == xa[l]) ? xb[l] : xa[l];
      const T* din = s == 0 ? nullptr : d[l];
      T* dout = (s < k - 1) ? d[l] : nullptr;
      tail_smooth<true>(g, a.m, coef[l], kell, cur, out, b[l], din, dout, T(a.cd[s]), T(a.cr[s]));
      __syncthreads();
      cur = out;
    }
    res[l] = cur;
  }
  for (int e = t; e < 2 * a.g[0].N; e += TB) a.x[e] = res[0][e];
}

template <class T>
void launch_vtail2d(hipStream_t st, const TailArgs<T>& a) {
  hipLaunchKernelGGL((k_vtail2d<T>), dim3(1), dim3(TB), 0, st, a);
}

template void launch_vtail2d<float>(hipStream_t, const TailArgs<float>&);
template void launch_vtail2d<double>(hipStream_t, const TailArgs<double>&);

}  // namespace frac
