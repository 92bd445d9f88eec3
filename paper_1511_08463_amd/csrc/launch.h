// Host-side launchers of the device kernels (one declaration per kernel
// family).  All launches are asynchronous on the given stream.
#pragma once

#include "common.h"

namespace frac {

// ---- 2D operator kernels (kernels2d.hip) -----------------------------------
int node_blocks2(const Grid& g);
int node_blocks(const Grid& g);
template <class T>
void launch_apply2d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* y, const ND<T>* b, int mask, int red, Red r);
template <class T>
void launch_resid2d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* r, const ND<T>* b, bool red, Red rr);
template <class T>
void launch_smooth2d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                     double kell, const ND<T>* x_in, T* x_out, const T* b, const ND<T>* d_in, ND<T>* d_out,
                     double cd, double cr);
void launch_coarsen2d(hipStream_t st, const Grid& gf, bool fine_is_alpha, const double* fine,
                      double kell, const Grid& gc, double* coarse64, float* coarse32);
template <class T>
void launch_restrict2d(hipStream_t st, const Grid& gf, const Grid& gc, const T* rf, T* bc);
template <class T>
void launch_restrict_smooth2d(hipStream_t st, const Grid& gf, const Grid& gc, const Mat& m,
                              const T* coef, double kell, const T* rf, T* bc, T* xout, T* dout,
                              double cr);
template <class T>
void launch_prol_smooth2d(hipStream_t st, const Grid& g, const Grid& gc, const Mat& m, bool fine,
                          const T* coef, double kell, const T* x, const T* xc, T* y, const T* b,
                          T* dout, double cr);

void launch_lift2d(hipStream_t st, const Grid& g, double* u, double t, const Load2D& ld);
void launch_w2_2d(hipStream_t st, const Grid& g, const Mat& m, const double* u, double* w2);
void launch_vi_eval2d(hipStream_t st, const Grid& g, double cL, double cM, double cm,
                      const double* w2, const double* a, const double* d, const double* lo,
                      const double* S, int mu_slot, double zeta, double* F, double* phi,
                      uint8_t* mask, double* hdinv, Red r2, Red rm, Red rlo, Red rhi,
                      bool trial);
// rows j0..j1 only (j1 < 0: all rows)
void launch_helm_apply2d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                         const double* x, const uint8_t* mask, double* y, bool dot, Red r,
                         int j0 = 0, int j1 = -1);
void launch_energy2d(hipStream_t st, const Grid& g, const Mat& m, double kell, double gc_cw,
                     double ell, int at2, const double* u, const double* a, Red rel, Red rsu);

void launch_jac2d(hipStream_t st, const Grid& g, const Mat& m, double kell, double cL, double cM,
                  const double* alpha, const double* u, const double* w2, const uint8_t* mask,
                  const double* xu, const double* xa, double* yu, double* ya, bool dot, Red ru,
                  Red ra, const double* band);
void launch_irange3d(hipStream_t st, const Grid& g, const uint8_t* mask, Red rlo, Red rhi);
// 3D forms of the coupled Jacobian blocks (kernels3d.hip); the 2D launchers
// dispatch to them.  Rows of a 3D band are the indices j + (ny + 1) k.
void launch_jac3d(hipStream_t st, const Grid& g, const Mat& m, double kell, double cL, double cM,
                  const double* alpha, const double* u, const double* w2, const uint8_t* mask,
                  const double* xu, const double* xa, double* yu, double* ya, bool dot, Red ru,
                  Red ra, const double* band);
void launch_couple_u3d(hipStream_t st, const Grid& g, const Mat& m, const double* alpha,
                       const double* u, const double* xu, const double* xa, const uint8_t* mask,
                       double* yu, int r0, int r1, Red r);
void launch_cheb_helm3d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                        const uint8_t* mask, const double* x_in, double* x_out, const double* b,
                        const double* d_in, double* d_out, double cd, double cr);
void launch_couple_u2d(hipStream_t st, const Grid& g, const Mat& m, const double* alpha,
                       const double* u, const double* xu, const double* xa, const uint8_t* mask,
                       double* yu, int r0, int r1, Red r);
void launch_cheb_helm2d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                        const uint8_t* mask, const double* x_in, double* x_out, const double* b,
                        const double* d_in, double* d_out, double cd, double cr);
void launch_trial_state(hipStream_t st, int64_t n2, int64_t N, const double* u, const double* a,
                        const double* du, const double* da, const double* lo, const double* S,
                        double* ut, double* at);

// ---- 3D operator kernels (kernels3d.hip); the 2D launchers forward to these
// when g.dim == 3 ----------------------------------------------------------
int node_blocks3(const Grid& g);
template <class T>
void launch_apply3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* y, const ND<T>* b, int mask, int red, Red r);
template <class T>
void launch_resid3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                    double kell, const T* x, T* r, const ND<T>* b, bool red, Red rr);
template <class T>
void launch_smooth3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                     const T* dg, double kell, const ND<T>* x_in, T* x_out, const T* b,
                     const ND<T>* d_in, ND<T>* d_out, double cd, double cr);
template <class T>
void launch_diag3d(hipStream_t st, const Grid& g, const Mat& m, bool fine, const T* coef,
                   double kell, T* dg);
void launch_coarsen3d(hipStream_t st, const Grid& gf, bool fine_is_alpha, const double* fine,
                      double kell, const Grid& gc, double* c64, float* c32);
template <class T>
void launch_restrict3d(hipStream_t st, const Grid& gf, const Grid& gc, const T* rf, T* bc);
template <class T>
void launch_restrict_smooth3d(hipStream_t st, const Grid& gf, const Grid& gc, const T* rf, T* bc,
                              const T* dgc, T* xc, T* dc, double cr);
template <class T>
void launch_prolong3d(hipStream_t st, const Grid& gf, const Grid& gc, const T* xc, T* xf);
void launch_lift3d(hipStream_t st, const Grid& g, double* u);
void launch_w2_3d(hipStream_t st, const Grid& g, const Mat& m, const double* u, double* w2);
void launch_vi_eval3d(hipStream_t st, const Grid& g, double cL, double cM, double cm,
                      const double* w2, const double* a, const double* d, const double* lo,
                      const double* S, int mu_slot, double zeta, double* F, double* phi,
                      uint8_t* mask, double* hdinv, Red r2, Red rm, Red rlo, Red rhi, bool trial);
void launch_helm_apply3d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                         const double* x, const uint8_t* mask, double* y, bool dot, Red r, int r0,
                         int r1);
void launch_energy3d(hipStream_t st, const Grid& g, const Mat& m, double kell, double gc_cw,
                     double ell, int at2, const double* w2, const double* a, Red rel, Red rsu);
void launch_dense_assemble3d(hipStream_t st, const Grid& g, const Mat& m, const double* abar,
                             double* A, const double* S);

// ---- coarse dense solve (dense.hip) ----------------------------------------
void launch_dense_setup(hipStream_t st, const Grid& g, const Mat& m, const double* abar,
                        double* A, double* Ainv, double* ref, double* S, double tol);
template <class T>
void launch_dense_solve(hipStream_t st, int n, const double* Ainv, const T* b, T* x);

// ---- bottom of the 2D V-cycle in one workgroup (tail2d.hip) -----------------
constexpr int TAIL_MAX_LEVELS = 3;
constexpr int TAIL_LDS_BYTES = 160 * 1024;

template <class T>
struct TailArgs {
  int nl;                          // smoothed levels in the tail, 1 .. TAIL_MAX_LEVELS
  Grid g[TAIL_MAX_LEVELS + 1];     // those levels (finest first), then the coarsest level
  const T* coef[TAIL_MAX_LEVELS];  // their element coefficients
  Mat m;
  double kell;
  int k;                           // Chebyshev steps per V-cycle side
  double cd[8], cr[8];
  const double* Ainv;              // inverse of the coarsest operator, dense_n^2
  int dense_n;
  const T* b;                      // right-hand side on the first tail level
  T* x;                            // V-cycle result on the first tail level
};

// LDS bytes of a tail over levels g[0 .. nl-1] and a coarsest system of n DOFs.
size_t tail_lds_bytes(const Grid* g, int nl, int n, size_t elem);
template <class T>
void launch_vtail2d(hipStream_t st, const TailArgs<T>& a);

// ---- vector kernels (vec.hip) -----------------------------------------------
int vec_blocks(int64_t n);
void launch_finish(hipStream_t st, const Red& r, int nblocks, bool is_max);
void launch_finish_multi(hipStream_t st, const FinishSet& fs, int nblocks);
void launch_cg_update(hipStream_t st, int64_t n, double* x, double* r, const double* p,
                      const double* q, const double* S, Red rr);
void launch_xpby(hipStream_t st, int64_t n, const double* z, double* p, const double* S);
// pq_part (optional): the unfinished partials of p.q (pq_nb of them), from
// which each block forms alpha itself
void launch_cg_update_jac(hipStream_t st, const Box& bx, double* x, double* r, const double* p,
                          const double* q, const double* dinv, double* z, const double* S, Red rr,
                          Red rz, const double* pq_part = nullptr, int pq_nb = 0);
int launch_helm_cg3d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                     const double* z, const double* p_old, const uint8_t* mask, double* p_new,
                     double* q, int r0, int r1, int i0, int i1, const double* S, bool first, Red r,
                     bool finish);
// Returns 0 after finishing the p.q reduction into S (finish set), else the
// number of partials left for the consumer (the CG update forms alpha).
int launch_helm_cg2d(hipStream_t st, const Grid& g, double cL, double cM, const double* w2,
                     const double* z, const double* p_old, const uint8_t* mask, double* p_new,
                     double* q, int r0, int r1, int i0, int i1, const double* S, bool first, Red r,
                     bool finish = true);
void launch_dot(hipStream_t st, int64_t n, const double* a, const double* b, Red r);
void launch_jacobi_dot(hipStream_t st, const Box& bx, const double* r, const double* dinv, double* z,
                       Red red);
void launch_norm2_box(hipStream_t st, const Box& bx, const double* x, Red r);
void launch_axpby(hipStream_t st, int64_t n, double a, const double* x, double b, double* y);
void launch_norm2(hipStream_t st, int64_t n, const double* x, Red r);
void launch_normmax(hipStream_t st, int64_t n, const double* x, Red r);
void launch_neg_masked(hipStream_t st, int64_t n, const double* F, const uint8_t* mask, double* r,
                       double* x);
void launch_relax_u(hipStream_t st, int64_t n, double* u, const double* ut, double omega);
void launch_relax_alpha(hipStream_t st, int64_t n, double* a, const double* at, const double* lo,
                        double omega, const double* S, int wslot, Red rd);
void launch_ratio(hipStream_t st, int64_t n, const double* a, const double* at, const double* lo,
                  double omega, Red r);
void launch_violation(hipStream_t st, int64_t n, const double* a, const double* at,
                      const double* lo, double w, Red r);
void launch_proj_step(hipStream_t st, int64_t n, double* a, const double* d, const double* lo,
                      const double* S);
void launch_merit_parts(hipStream_t st, int64_t n, const double* x, const double* F,
                        const double* lo, double* w, double* g);
void launch_neg_sum(hipStream_t st, int64_t n, const double* g, const double* hw, double* d, Red r);
void launch_set_scalar(hipStream_t st, double* S, int slot, double v);
// float32 vectors (mixed-precision inner solver)
void launch_cg_update_f(hipStream_t st, int64_t n, float* x, float* r, const float* p,
                        const float* q, const double* S, Red rr);
void launch_xpby_f(hipStream_t st, int64_t n, const float* z, float* p, const double* S);
void launch_dot_f(hipStream_t st, int64_t n, const float* a, const float* b, Red r);
void launch_to_float(hipStream_t st, int64_t n, const double* x, float* y, double scale);
void launch_add_scaled_f(hipStream_t st, int64_t n, double* x, const float* e, double scale);
void launch_copy(hipStream_t st, int64_t n, const double* x, double* y);
void launch_scalars_out(hipStream_t st, const double* S, double* host);
void launch_minres_init(hipStream_t st, double* S);
void launch_minres_a(hipStream_t st, double* S);
void launch_minres_b(hipStream_t st, double* S, double* host);
void launch_lincomb3_s(hipStream_t st, const Seg& sg, const double* S, double* z, const double* x,
                       const double* y);
void launch_minres_update_s(hipStream_t st, const Seg& sg, const double* S, const double* z,
                            double* w2, const double* w1, double* x);
void launch_dot_seg(hipStream_t st, const Seg& sg, const double* a, const double* b, Red r);
void launch_from_float(hipStream_t st, int64_t n, const float* e, double* x, double scale);


// crack-aware deflation of the elastic CG (deflate.hip)
int dfl_part_blocks(int64_t N);
void launch_fragments2d(hipStream_t st, const Grid& g, const double* alpha, double theta,
                        int min_nodes, int fmax, int* parent, int* label, int* fid, int* meta);
void launch_dfl_mode(hipStream_t st, const Grid& g, const int* fid, int k, double* w);
void launch_dfl_add(hipStream_t st, const Grid& g, const int* fid, const double* mu, double* x,
                    double sign);
void launch_dfl_wtv(hipStream_t st, const Grid& g, const int* fid, const double* v, double* part,
                    int col, double* E, const double* Einv, double* mu);
void launch_dfl_invert(hipStream_t st, const double* E, double* Einv, const int* meta);

}  // namespace frac
