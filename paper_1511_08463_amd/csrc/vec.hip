// 1D vector kernels: Krylov updates with fused deterministic reductions,
// the over-relaxed updates of Algorithm 2 and the projected steps of
// Algorithm 4.  Scalars that depend on earlier reductions (CG alpha/beta,
// line-search mu) are read from the device scalar array, so no host round
// trip sits between dependent kernels.
#include "common.h"
#include "launch.h"

namespace frac {

static int vgrid(int64_t n) {
  int64_t b = (n + VB - 1) / VB;
  if (b > VGRID) b = VGRID;
  if (b < 1) b = 1;
  return (int)b;
}

int vec_blocks(int64_t n) { return vgrid(n); }

// Second pass of every reduction: one block sums (or maxes) the partials in a
// fixed order and applies the scalar post-operation.
constexpr int FB = 1024;
template <bool MAX>
__global__ __launch_bounds__(FB) void k_finish(Red r, int nblocks) {
  __shared__ double sh[FB / WAVE];
  double acc = MAX ? -INFINITY : 0.0;
  for (int k = threadIdx.x; k < nblocks; k += FB) acc = MAX ? fmax(acc, r.part[k]) : acc + r.part[k];
  acc = MAX ? wave_max(acc) : wave_sum(acc);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (lane == 0) sh[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = sh[0];
    for (int k = 1; k < FB / WAVE; ++k) s = MAX ? fmax(s, sh[k]) : s + sh[k];
    post_scalar(s, r);
  }
}

// Two independent sums finished at once, one block each.
__global__ __launch_bounds__(FB) void k_finish2(Red r0, Red r1, int nblocks) {
  __shared__ double sh[FB / WAVE];
  const Red& r = blockIdx.x == 0 ? r0 : r1;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += FB) acc += r.part[k];
  acc = wave_sum(acc);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (lane == 0) sh[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = sh[0];
    for (int k = 1; k < FB / WAVE; ++k) s += sh[k];
    post_scalar(s, r);
  }
}

// Up to four independent reductions of one launch finished at once, one
// block each (bit q of maxmask: reduction q is a max).
__global__ __launch_bounds__(FB) void k_finish_multi(FinishSet fs, int nblocks) {
  __shared__ double sh[FB / WAVE];
  const Red& r = fs.r[blockIdx.x];
  const bool mx = (fs.maxmask >> blockIdx.x) & 1;
  double acc = mx ? -INFINITY : 0.0;
  for (int k = threadIdx.x; k < nblocks; k += FB) acc = mx ? fmax(acc, r.part[k]) : acc + r.part[k];
  acc = mx ? wave_max(acc) : wave_sum(acc);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (lane == 0) sh[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = sh[0];
    for (int k = 1; k < FB / WAVE; ++k) s = mx ? fmax(s, sh[k]) : s + sh[k];
    post_scalar(s, r);
  }
}

void launch_finish_multi(hipStream_t st, const FinishSet& fs, int nblocks) {
  hipLaunchKernelGGL(k_finish_multi, dim3(fs.count), dim3(FB), 0, st, fs, nblocks);
}

void launch_finish(hipStream_t st, const Red& r, int nblocks, bool is_max) {
  if (is_max)
    hipLaunchKernelGGL((k_finish<true>), dim3(1), dim3(FB), 0, st, r, nblocks);
  else
    hipLaunchKernelGGL((k_finish<false>), dim3(1), dim3(FB), 0, st, r, nblocks);
}

#define GRID_STRIDE(k, n) for (int64_t k = (int64_t)blockIdx.x * VB + threadIdx.x; k < (n); k += (int64_t)gridDim.x * VB)

// x += a p; r -= a q; S[slot] = r.r   (a = S[S_ALPHA])
__global__ __launch_bounds__(VB) void k_cg_update(int64_t n, double* __restrict__ x,
                                                  double* __restrict__ r,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ q,
                                                  const double* __restrict__ S, Red rr) {
  const double a = S[S_ALPHA];
  double acc = 0.0;
  GRID_STRIDE(k, n) {
    x[k] += a * p[k];
    const double rv = r[k] - a * q[k];
    r[k] = rv;
    acc += rv * rv;
  }
  block_reduce<VB, false>(acc, rr, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_cg_update(hipStream_t st, int64_t n, double* x, double* r, const double* p,
                      const double* q, const double* S, Red rr) {
  hipLaunchKernelGGL(k_cg_update, dim3(vgrid(n)), dim3(VB), 0, st, n, x, r, p, q, S, rr);
  launch_finish(st, rr, vgrid(n), false);
}

// The CG step length alpha = rz / pq from the per-block partials of pq, summed
// in k_finish's order (FB threads striding the partials, then their wave sums
// in wave order), so every block forms the same value and the result equals
// the separate finishing launch bit for bit.
__device__ __forceinline__ double cg_alpha_from_parts(const double* __restrict__ part, int nb,
                                                      const double* __restrict__ S) {
  static_assert(FB % VB == 0 && VB % WAVE == 0, "virtual finishing threads");
  constexpr int M = FB / VB;
  __shared__ double sh[FB / WAVE];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double acc = 0.0;
    for (int k = threadIdx.x + m * VB; k < nb; k += FB) acc += part[k];
    acc = wave_sum(acc);
    if (lane == 0) sh[w + m * (VB / WAVE)] = acc;
  }
  __syncthreads();
  double pq = sh[0];
  for (int k = 1; k < FB / WAVE; ++k) pq += sh[k];
  return (pq != 0.0) ? S[S_RZ] / pq : 0.0;
}

// x += a p; r -= a q; z = dinv .* r; S[rr.slot] = r.r, S[rz.slot] = r.z over
// the entries of a box (both sums finished by one launch); a = S[S_ALPHA], or
// (pq_part) formed by every block from the partials of p.q.  The two
// reductions must not touch each other's scalars: rz's post-operation reads
// S_RZ only.
__global__ __launch_bounds__(VB) void k_cg_update_jac(Box bx, double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      const double* __restrict__ dinv,
                                                      double* __restrict__ z,
                                                      const double* __restrict__ S,
                                                      const double* __restrict__ pq_part,
                                                      int pq_nb, Red rr, Red rz) {
  const double a = pq_part ? cg_alpha_from_parts(pq_part, pq_nb, S) : S[S_ALPHA];
  double arr = 0.0, arz = 0.0;
  GRID_STRIDE(qq, bx.n) {
    const int64_t k = box_index(bx, qq);
    x[k] += a * p[k];
    const double rv = r[k] - a * q[k];
    r[k] = rv;
    const double zv = dinv[k] * rv;
    z[k] = zv;
    arr += rv * rv;
    arz += rv * zv;
  }
  block_reduce<VB, false>(arr, rr, gridDim.x, blockIdx.x, threadIdx.x);
  block_reduce<VB, false>(arz, rz, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_cg_update_jac(hipStream_t st, const Box& bx, double* x, double* r, const double* p,
                          const double* q, const double* dinv, double* z, const double* S, Red rr,
                          Red rz, const double* pq_part, int pq_nb) {
  hipLaunchKernelGGL(k_cg_update_jac, dim3(vgrid(bx.n)), dim3(VB), 0, st, bx, x, r, p, q, dinv, z,
                     S, pq_part, pq_nb, rr, rz);
  hipLaunchKernelGGL(k_finish2, dim3(2), dim3(FB), 0, st, rr, rz, vgrid(bx.n));
}

// p = z + beta p   (beta = S[S_BETA])
__global__ __launch_bounds__(VB) void k_xpby(int64_t n, const double* __restrict__ z,
                                             double* __restrict__ p, const double* __restrict__ S) {
  const double b = S[S_BETA];
  GRID_STRIDE(k, n) p[k] = z[k] + b * p[k];
}

void launch_xpby(hipStream_t st, int64_t n, const double* z, double* p, const double* S) {
  hipLaunchKernelGGL(k_xpby, dim3(vgrid(n)), dim3(VB), 0, st, n, z, p, S);
}

// S[slot] = a.b (with the Red post-operation)
__global__ __launch_bounds__(VB) void k_dot(int64_t n, const double* __restrict__ a,
                                            const double* __restrict__ b, Red r) {
  double acc = 0.0;
  GRID_STRIDE(k, n) acc += a[k] * b[k];
  block_reduce<VB, false>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_dot(hipStream_t st, int64_t n, const double* a, const double* b, Red r) {
  hipLaunchKernelGGL(k_dot, dim3(vgrid(n)), dim3(VB), 0, st, n, a, b, r);
  launch_finish(st, r, vgrid(n), false);
}

// z = dinv .* r; S = r.z (post), over the entries of a box
__global__ __launch_bounds__(VB) void k_jacobi_dot(Box bx, const double* __restrict__ r,
                                                   const double* __restrict__ dinv,
                                                   double* __restrict__ z, Red red) {
  double acc = 0.0;
  GRID_STRIDE(q, bx.n) {
    const int64_t k = box_index(bx, q);
    const double zv = dinv[k] * r[k];
    z[k] = zv;
    acc += r[k] * zv;
  }
  block_reduce<VB, false>(acc, red, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_jacobi_dot(hipStream_t st, const Box& bx, const double* r, const double* dinv, double* z,
                       Red red) {
  hipLaunchKernelGGL(k_jacobi_dot, dim3(vgrid(bx.n)), dim3(VB), 0, st, bx, r, dinv, z, red);
  launch_finish(st, red, vgrid(bx.n), false);
}

// S = ||x||^2 over the entries of a box
__global__ __launch_bounds__(VB) void k_norm2_box(Box bx, const double* __restrict__ x, Red r) {
  double acc = 0.0;
  GRID_STRIDE(q, bx.n) {
    const double v = x[box_index(bx, q)];
    acc += v * v;
  }
  block_reduce<VB, false>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_norm2_box(hipStream_t st, const Box& bx, const double* x, Red r) {
  hipLaunchKernelGGL(k_norm2_box, dim3(vgrid(bx.n)), dim3(VB), 0, st, bx, x, r);
  launch_finish(st, r, vgrid(bx.n), false);
}

// y = a x + b y (host scalars)
__global__ __launch_bounds__(VB) void k_axpby(int64_t n, double a, const double* __restrict__ x,
                                              double b, double* __restrict__ y) {
  // b == 0 overwrites y without reading it (y may hold anything, NaN included)
  if (b == 0.0) {
    GRID_STRIDE(k, n) y[k] = a * x[k];
  } else {
    GRID_STRIDE(k, n) y[k] = a * x[k] + b * y[k];
  }
}

void launch_axpby(hipStream_t st, int64_t n, double a, const double* x, double b, double* y) {
  hipLaunchKernelGGL(k_axpby, dim3(vgrid(n)), dim3(VB), 0, st, n, a, x, b, y);
}

// y = x (a plain streaming copy)
__global__ __launch_bounds__(VB) void k_copy(int64_t n, const double* __restrict__ x,
                                             double* __restrict__ y) {
  GRID_STRIDE(k, n) y[k] = x[k];
}

// The scalar array into pinned host memory, written by the kernel itself (one
// small launch instead of a runtime copy).
__global__ __launch_bounds__(WAVE) void k_scalars_out(const double* __restrict__ S,
                                                      double* __restrict__ out) {
  for (int q = threadIdx.x; q < S_COUNT; q += WAVE) out[q] = S[q];
}

void launch_scalars_out(hipStream_t st, const double* S, double* host) {
  hipLaunchKernelGGL(k_scalars_out, dim3(1), dim3(WAVE), 0, st, S, host);
}

void launch_copy(hipStream_t st, int64_t n, const double* x, double* y) {
  hipLaunchKernelGGL(k_copy, dim3(vgrid(n)), dim3(VB), 0, st, n, x, y);
}

// ---------------------------------------------------------------------------
// MINRES on the device: the scalar recurrence (preconditioned Lanczos with
// Givens rotations, as in the host form it replaces) runs in one-thread
// kernels between the vector kernels, which read their coefficients from S.
// ---------------------------------------------------------------------------

// gamma_1 = sqrt(z_1 . v_1) from S_TMP2; rotations and eta initialised.
__global__ void k_minres_init(double* S) {
  if (threadIdx.x != 0) return;
  const double gg = S[S_TMP2];
  const double g = gg > 0.0 ? sqrt(gg) : 0.0;
  S[S_MN_G] = g;
  S[S_MN_G1] = g;
  S[S_MN_GP] = 1.0;
  S[S_MN_ETA] = g;
  S[S_MN_ABSETA] = g;
  S[S_MN_GN] = g;
  S[S_MN_C] = 1.0;
  S[S_MN_CP] = 1.0;
  S[S_MN_S] = 0.0;
  S[S_MN_SP] = 0.0;
  S[S_MN_BAD] = isfinite(gg) ? 0.0 : 1.0;
}

// after J z_j (z_j unnormalised; S_TMP0 + S_TMP1 = z_j . J z_j):
// delta = z.Jz / gamma^2 and the coefficients of
// v_{j+1} = J z_j / gamma - (delta / gamma) v_j - (gamma / gamma_prev) v_{j-1}
__global__ void k_minres_a(double* S) {
  if (threadIdx.x != 0) return;
  const double g = S[S_MN_G], gp = S[S_MN_GP];
  const double d = (S[S_TMP0] + S[S_TMP1]) / (g * g);
  S[S_MN_D] = d;
  S[S_MN_L0] = 1.0 / g;
  S[S_MN_L1] = -d / g;
  S[S_MN_L2] = -g / gp;
  if (!isfinite(d)) S[S_MN_BAD] = 1.0;
}

// after z_{j+1} = P v_{j+1} and S_TMP2 = z_{j+1} . v_{j+1}: the next Givens
// rotation, the coefficients of w_{j+1} = (z_j / gamma - a3 w_{j-1} - a2 w_j) / a1
// and of x += c_{j+1} eta w_{j+1}, then eta and the scalars shift by one.
__global__ void k_minres_b(double* S, double* host) {
  if (threadIdx.x != 0) return;
  const double g = S[S_MN_G], d = S[S_MN_D], c = S[S_MN_C], cp = S[S_MN_CP];
  const double s = S[S_MN_S], sp = S[S_MN_SP], eta = S[S_MN_ETA], gn2 = S[S_TMP2];
  const double gn = sqrt(gn2 > 0.0 ? gn2 : 0.0);
  const double a0 = c * d - cp * s * g;
  const double a1 = sqrt(a0 * a0 + gn * gn);
  const double a2 = s * d + cp * c * g;
  const double a3 = sp * g;
  const double cn = a0 / a1, sn = gn / a1;
  S[S_MN_U0] = 1.0 / (a1 * g);
  S[S_MN_U1] = -a3 / a1;
  S[S_MN_U2] = -a2 / a1;
  S[S_MN_U3] = cn * eta;
  const double etan = -sn * eta;
  S[S_MN_ETA] = etan;
  S[S_MN_ABSETA] = fabs(etan);
  S[S_MN_GN] = gn;
  S[S_MN_GP] = g;
  S[S_MN_G] = gn;
  S[S_MN_CP] = c;
  S[S_MN_C] = cn;
  S[S_MN_SP] = s;
  S[S_MN_S] = sn;
  if (!isfinite(gn2)) S[S_MN_BAD] = 1.0;
  if (host) {   // |eta|, gamma_{j+1}, the non-finite flag for the host's lagged test
    host[0] = S[S_MN_ABSETA];
    host[1] = S[S_MN_GN];
    host[2] = S[S_MN_BAD];
  }
}

void launch_minres_init(hipStream_t st, double* S) {
  hipLaunchKernelGGL(k_minres_init, dim3(1), dim3(WAVE), 0, st, S);
}
void launch_minres_a(hipStream_t st, double* S) {
  hipLaunchKernelGGL(k_minres_a, dim3(1), dim3(WAVE), 0, st, S);
}
void launch_minres_b(hipStream_t st, double* S, double* host) {
  hipLaunchKernelGGL(k_minres_b, dim3(1), dim3(WAVE), 0, st, S, host);
}

// z = L0 z + L1 x + L2 y with the coefficients in S, on the entries of sg
__global__ __launch_bounds__(VB) void k_lincomb3_s(Seg sg, const double* __restrict__ S,
                                                   double* __restrict__ z,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ y) {
  const double a = S[S_MN_L0], b = S[S_MN_L1], c = S[S_MN_L2];
  GRID_STRIDE(q, sg.n) {
    const int64_t k = seg_index(sg, q);
    z[k] = a * z[k] + b * x[k] + c * y[k];
  }
}

void launch_lincomb3_s(hipStream_t st, const Seg& sg, const double* S, double* z, const double* x,
                       const double* y) {
  hipLaunchKernelGGL(k_lincomb3_s, dim3(vgrid(sg.n)), dim3(VB), 0, st, sg, S, z, x, y);
}

// w2 = U0 z + U1 w2 + U2 w1; x += U3 w2 with the coefficients in S, on the
// entries of sg
__global__ __launch_bounds__(VB) void k_minres_update_s(Seg sg, const double* __restrict__ S,
                                                        const double* __restrict__ z,
                                                        double* __restrict__ w2,
                                                        const double* __restrict__ w1,
                                                        double* __restrict__ x) {
  const double a = S[S_MN_U0], b = S[S_MN_U1], c = S[S_MN_U2], e = S[S_MN_U3];
  GRID_STRIDE(q, sg.n) {
    const int64_t k = seg_index(sg, q);
    const double wn = a * z[k] + b * w2[k] + c * w1[k];
    w2[k] = wn;
    x[k] += e * wn;
  }
}

void launch_minres_update_s(hipStream_t st, const Seg& sg, const double* S, const double* z,
                            double* w2, const double* w1, double* x) {
  hipLaunchKernelGGL(k_minres_update_s, dim3(vgrid(sg.n)), dim3(VB), 0, st, sg, S, z, w2, w1, x);
}

// S = a.b over the entries of sg (with the Red post-operation)
__global__ __launch_bounds__(VB) void k_dot_seg(Seg sg, const double* __restrict__ a,
                                                const double* __restrict__ b, Red r) {
  double acc = 0.0;
  GRID_STRIDE(q, sg.n) {
    const int64_t k = seg_index(sg, q);
    acc += a[k] * b[k];
  }
  block_reduce<VB, false>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_dot_seg(hipStream_t st, const Seg& sg, const double* a, const double* b, Red r) {
  hipLaunchKernelGGL(k_dot_seg, dim3(vgrid(sg.n)), dim3(VB), 0, st, sg, a, b, r);
  launch_finish(st, r, vgrid(sg.n), false);
}

// S[slot] = ||x||^2 or max|x| (NaN -> inf)
template <bool MAX>
__global__ __launch_bounds__(VB) void k_norm(int64_t n, const double* __restrict__ x, Red r) {
  double acc = MAX ? 0.0 : 0.0;
  GRID_STRIDE(k, n) {
    const double v = x[k];
    acc = MAX ? fmax(acc, nan_to_inf(fabs(v))) : acc + v * v;
  }
  block_reduce<VB, MAX>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_norm2(hipStream_t st, int64_t n, const double* x, Red r) {
  hipLaunchKernelGGL((k_norm<false>), dim3(vgrid(n)), dim3(VB), 0, st, n, x, r);
  launch_finish(st, r, vgrid(n), false);
}
void launch_normmax(hipStream_t st, int64_t n, const double* x, Red r) {
  hipLaunchKernelGGL((k_norm<true>), dim3(vgrid(n)), dim3(VB), 0, st, n, x, r);
  launch_finish(st, r, vgrid(n), true);
}

// Reduced damage CG set-up: r = -F on inactive nodes (0 on active), x = 0.
__global__ __launch_bounds__(VB) void k_neg_masked(int64_t n, const double* __restrict__ F,
                                                   const uint8_t* __restrict__ mask,
                                                   double* __restrict__ r,
                                                   double* __restrict__ x) {
  GRID_STRIDE(k, n) {
    r[k] = mask[k] ? 0.0 : -F[k];
    x[k] = 0.0;
  }
}

void launch_neg_masked(hipStream_t st, int64_t n, const double* F, const uint8_t* mask, double* r,
                       double* x) {
  hipLaunchKernelGGL(k_neg_masked, dim3(vgrid(n)), dim3(VB), 0, st, n, F, mask, r, x);
}

// u += omega (ut - u)   (Algorithm 2, displacement relaxation)
__global__ __launch_bounds__(VB) void k_relax_u(int64_t n, double* __restrict__ u,
                                                const double* __restrict__ ut, double omega) {
  GRID_STRIDE(k, n) u[k] += omega * (ut[k] - u[k]);
}

void launch_relax_u(hipStream_t st, int64_t n, double* u, const double* ut, double omega) {
  hipLaunchKernelGGL(k_relax_u, dim3(vgrid(n)), dim3(VB), 0, st, n, u, ut, omega);
}

// alpha <- clip(alpha + w (at - alpha), lo, 1) with w = omega (projection) or
// w = S[wslot] (a common factor); S[dslot] = max |alpha_new - alpha|.
__global__ __launch_bounds__(VB) void k_relax_alpha(int64_t n, double* __restrict__ a,
                                                    const double* __restrict__ at,
                                                    const double* __restrict__ lo, double omega,
                                                    const double* __restrict__ S, int wslot,
                                                    Red rd) {
  const double w = wslot >= 0 ? S[wslot] : omega;
  double acc = 0.0;
  GRID_STRIDE(k, n) {
    const double old = a[k];
    // at omega = 1 the damage iterate itself (feasible by construction), so
    // that the new alpha is exactly the point the damage solve evaluated
    const double nv = w == 1.0 ? at[k] : fmin(fmax(old + w * (at[k] - old), lo[k]), 1.0);
    a[k] = nv;
    acc = fmax(acc, nan_to_inf(fabs(nv - old)));
  }
  block_reduce<VB, true>(acc, rd, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_relax_alpha(hipStream_t st, int64_t n, double* a, const double* at, const double* lo,
                        double omega, const double* S, int wslot, Red rd) {
  hipLaunchKernelGGL(k_relax_alpha, dim3(vgrid(n)), dim3(VB), 0, st, n, a, at, lo, omega, S, wslot,
                     rd);
  launch_finish(st, rd, vgrid(n), true);
}

// Exact ratio test: S[slot] = -(largest feasible common factor), reduced as a
// max of negated ratios so that the max-reduction machinery serves.
__global__ __launch_bounds__(VB) void k_ratio(int64_t n, const double* __restrict__ a,
                                              const double* __restrict__ at,
                                              const double* __restrict__ lo, double omega, Red r) {
  double acc = -omega;
  GRID_STRIDE(k, n) {
    const double d = at[k] - a[k];
    double lim = omega;
    if (d > 0.0) lim = (1.0 - a[k]) / d;
    else if (d < 0.0) lim = (lo[k] - a[k]) / d;
    acc = fmax(acc, -lim);
  }
  block_reduce<VB, true>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_ratio(hipStream_t st, int64_t n, const double* a, const double* at, const double* lo,
                  double omega, Red r) {
  hipLaunchKernelGGL(k_ratio, dim3(vgrid(n)), dim3(VB), 0, st, n, a, at, lo, omega, r);
  launch_finish(st, r, vgrid(n), true);
}

// S[slot] = max violation of the bounds by alpha + w (at - alpha) (0 when feasible).
__global__ __launch_bounds__(VB) void k_violation(int64_t n, const double* __restrict__ a,
                                                  const double* __restrict__ at,
                                                  const double* __restrict__ lo, double w, Red r) {
  double acc = 0.0;
  GRID_STRIDE(k, n) {
    const double v = a[k] + w * (at[k] - a[k]);
    acc = fmax(acc, fmax(v - 1.0, lo[k] - v));
  }
  block_reduce<VB, true>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_violation(hipStream_t st, int64_t n, const double* a, const double* at,
                      const double* lo, double w, Red r) {
  hipLaunchKernelGGL(k_violation, dim3(vgrid(n)), dim3(VB), 0, st, n, a, at, lo, w, r);
  launch_finish(st, r, vgrid(n), true);
}

// alpha <- clip(alpha + mu d, lo, 1), mu = S[S_MU]   (projected step, Algorithm 4)
__global__ __launch_bounds__(VB) void k_proj_step(int64_t n, double* __restrict__ a,
                                                  const double* __restrict__ d,
                                                  const double* __restrict__ lo,
                                                  const double* __restrict__ S) {
  const double mu = S[S_MU];
  GRID_STRIDE(k, n) a[k] = fmin(fmax(a[k] + mu * d[k], lo[k]), 1.0);
}

void launch_proj_step(hipStream_t st, int64_t n, double* a, const double* d, const double* lo,
                      const double* S) {
  hipLaunchKernelGGL(k_proj_step, dim3(vgrid(n)), dim3(VB), 0, st, n, a, d, lo, S);
}

// Steepest-descent fallback of Algorithm 4 for the box QP: the generalised
// Jacobian of Phi gives grad psi = ca*Phi + H (cf*Phi); this kernel writes
// w = cf*Phi and g = ca*Phi (the H product is added by the caller).
__global__ __launch_bounds__(VB) void k_merit_parts(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ F,
                                                    const double* __restrict__ lo,
                                                    double* __restrict__ w,
                                                    double* __restrict__ g) {
  GRID_STRIDE(k, n) {
    const double l = lo[k], u = 1.0, xv = x[k], Fv = F[k];
    const double p = u - xv, q = -Fv;
    const double c = fb(p, q);
    const double a = xv - l;
    const double ph = fb(a, c);
    const double ro = hypot(a, c), ri = hypot(p, q);
    const double s2 = 0.70710678118654752440;
    const double dao = (ro > 0 ? a / ro : s2) - 1.0, dbo = (ro > 0 ? c / ro : s2) - 1.0;
    const double dai = (ri > 0 ? p / ri : s2) - 1.0, dbi = (ri > 0 ? q / ri : s2) - 1.0;
    const double ca = dao - dbo * dai, cf = -dbo * dbi;
    w[k] = cf * ph;
    g[k] = ca * ph;
  }
}

void launch_merit_parts(hipStream_t st, int64_t n, const double* x, const double* F,
                        const double* lo, double* w, double* g) {
  hipLaunchKernelGGL(k_merit_parts, dim3(vgrid(n)), dim3(VB), 0, st, n, x, F, lo, w, g);
}

// d = -(g + Hw) : the descent direction from the two parts; S[slot] = |d|^2
__global__ __launch_bounds__(VB) void k_neg_sum(int64_t n, const double* __restrict__ g,
                                                const double* __restrict__ hw,
                                                double* __restrict__ d, Red r) {
  double acc = 0.0;
  GRID_STRIDE(k, n) {
    const double v = -(g[k] + hw[k]);
    d[k] = v;
    acc += v * v;
  }
  block_reduce<VB, false>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_neg_sum(hipStream_t st, int64_t n, const double* g, const double* hw, double* d, Red r) {
  hipLaunchKernelGGL(k_neg_sum, dim3(vgrid(n)), dim3(VB), 0, st, n, g, hw, d, r);
  launch_finish(st, r, vgrid(n), false);
}

// Scalar store on the device (S[slot] = v) without a host-to-device copy.
__global__ void k_set_scalar(double* S, int slot, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) S[slot] = v;
}

void launch_set_scalar(hipStream_t st, double* S, int slot, double v) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(WAVE), 0, st, S, slot, v);
}

// ---- float32 vectors of the mixed-precision inner solver (float64 sums) ----

// x += a p; r -= a q; S[slot] = r.r  (a = S[S_ALPHA])
__global__ __launch_bounds__(VB) void k_cg_update_f(int64_t n, float* __restrict__ x,
                                                    float* __restrict__ r,
                                                    const float* __restrict__ p,
                                                    const float* __restrict__ q,
                                                    const double* __restrict__ S, Red rr) {
  const float a = (float)S[S_ALPHA];
  double acc = 0.0;
  GRID_STRIDE(k, n) {
    x[k] += a * p[k];
    const float rv = r[k] - a * q[k];
    r[k] = rv;
    acc += (double)rv * rv;
  }
  block_reduce<VB, false>(acc, rr, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_cg_update_f(hipStream_t st, int64_t n, float* x, float* r, const float* p,
                        const float* q, const double* S, Red rr) {
  hipLaunchKernelGGL(k_cg_update_f, dim3(vgrid(n)), dim3(VB), 0, st, n, x, r, p, q, S, rr);
  launch_finish(st, rr, vgrid(n), false);
}

// p = z + beta p (beta = S[S_BETA])
__global__ __launch_bounds__(VB) void k_xpby_f(int64_t n, const float* __restrict__ z,
                                               float* __restrict__ p, const double* __restrict__ S) {
  const float b = (float)S[S_BETA];
  GRID_STRIDE(k, n) p[k] = z[k] + b * p[k];
}

void launch_xpby_f(hipStream_t st, int64_t n, const float* z, float* p, const double* S) {
  hipLaunchKernelGGL(k_xpby_f, dim3(vgrid(n)), dim3(VB), 0, st, n, z, p, S);
}

__global__ __launch_bounds__(VB) void k_dot_f(int64_t n, const float* __restrict__ a,
                                              const float* __restrict__ b, Red r) {
  double acc = 0.0;
  GRID_STRIDE(k, n) acc += (double)a[k] * b[k];
  block_reduce<VB, false>(acc, r, gridDim.x, blockIdx.x, threadIdx.x);
}

void launch_dot_f(hipStream_t st, int64_t n, const float* a, const float* b, Red r) {
  hipLaunchKernelGGL(k_dot_f, dim3(vgrid(n)), dim3(VB), 0, st, n, a, b, r);
  launch_finish(st, r, vgrid(n), false);
}

// y = float(x * scale)
__global__ __launch_bounds__(VB) void k_to_float(int64_t n, const double* __restrict__ x,
                                                 float* __restrict__ y, double scale) {
  GRID_STRIDE(k, n) y[k] = (float)(x[k] * scale);
}

void launch_to_float(hipStream_t st, int64_t n, const double* x, float* y, double scale) {
  hipLaunchKernelGGL(k_to_float, dim3(vgrid(n)), dim3(VB), 0, st, n, x, y, scale);
}

// x += scale * e  (float64 accumulation of a float32 correction)
__global__ __launch_bounds__(VB) void k_add_scaled_f(int64_t n, double* __restrict__ x,
                                                     const float* __restrict__ e, double scale) {
  GRID_STRIDE(k, n) x[k] += scale * (double)e[k];
}

void launch_add_scaled_f(hipStream_t st, int64_t n, double* x, const float* e, double scale) {
  hipLaunchKernelGGL(k_add_scaled_f, dim3(vgrid(n)), dim3(VB), 0, st, n, x, e, scale);
}

// x = scale * e
__global__ __launch_bounds__(VB) void k_from_float(int64_t n, const float* __restrict__ e,
                                                   double* __restrict__ x, double scale) {
  GRID_STRIDE(k, n) x[k] = scale * (double)e[k];
}

void launch_from_float(hipStream_t st, int64_t n, const float* e, double* x, double scale) {
  hipLaunchKernelGGL(k_from_float, dim3(vgrid(n)), dim3(VB), 0, st, n, e, x, scale);
}

}  // namespace frac
