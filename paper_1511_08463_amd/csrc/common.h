// Shared device helpers and plain-data structs of the fracture library.
//
// Reductions are deterministic: each block reduces in a fixed order
// (wavefront shuffles, then LDS) and writes one partial; a one-block finishing
// kernel sums the partials in a fixed order and applies the scalar
// post-operation.  The result does not depend on block scheduling, so a run
// is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace frac {

// Non-deduced type alias: lets nullptr stand for an optional T* argument of a
// function template whose T is fixed by the other arguments.
template <class T> struct NonDeduced { using type = T; };
template <class T> using ND = typename NonDeduced<T>::type;

constexpr int WAVE = 64;
constexpr int NB_X = 64;          // 2D node kernels: 64 x 4 threads per block
constexpr int NB_Y = 4;
constexpr int NB = NB_X * NB_Y;
constexpr int VB = 256;           // 1D vector kernels
constexpr int VGRID = 2048;       // fixed grid of 1D reductions (8 blocks per CU)

// Boundary-condition families (mirrors FRACTURE_LOAD_* of the C ABI).
enum { BC_TENSION_2D = 0, BC_THERMAL_3D = 1, BC_SURFING_2D = 2, BC_TSHOCK_2D = 3 };

// Parameters of the 2D Dirichlet lifting: for the surfing load, the boundary
// carries K_I/(2 mu) sqrt(r/2pi) (kappa - cos theta) (cos(theta/2), sin(theta/2))
// about the tip (lc + v t, ly/2).
struct Load2D {
  int kind;          // BC_TENSION_2D, BC_SURFING_2D or BC_TSHOCK_2D
  double ki2mu;      // K_I / (2 mu)
  double kappa;      // (3 - nu) / (1 + nu)
  double lc, v;      // initial tip abscissa and speed
};

// Indices of device-resident scalars (an array of doubles in the workspace).
enum {
  S_RZ = 0, S_PQ, S_ALPHA, S_RR, S_BETA, S_RZNEW, S_MU,
  S_PHI2, S_PHIMAX, S_DAMAX, S_EL, S_SURF, S_EU2, S_TMP0, S_TMP1, S_TMP2,
  S_RATIO, S_INFEAS, S_GG, S_JLO, S_JHI,
  // MINRES recurrence (Lanczos scalars, Givens rotations, vector coefficients)
  S_MN_G, S_MN_GP, S_MN_G1, S_MN_C, S_MN_CP, S_MN_S, S_MN_SP, S_MN_ETA, S_MN_D,
  S_MN_L0, S_MN_L1, S_MN_L2, S_MN_U0, S_MN_U1, S_MN_U2, S_MN_U3,
  S_MN_ABSETA, S_MN_GN, S_MN_BAD,
  S_COARSE_REFRESH,   // 1: the coarsest dense system is re-assembled and re-inverted
  S_ILO, S_IHI,       // 3D: -(smallest) and largest column i of an inactive damage node
  S_COUNT = 64
};
static_assert(S_IHI < S_COUNT, "scalar slots");
// the host reads |eta|, gamma_{j+1} and the non-finite flag of MINRES as one block
static_assert(S_MN_GN == S_MN_ABSETA + 1 && S_MN_BAD == S_MN_ABSETA + 2, "MINRES status slots");
// kernels read the inactive row band as the pair (S[S_JLO], S[S_JHI])
static_assert(S_JHI == S_JLO + 1, "band slots must be adjacent");
// Partial-sum slots: one per reduction that may be pending at the same time.
enum { C_SLOTS = 18 };

// A structured level: (nx+1)(ny+1)[(nz+1)] nodes.
// Crack-aware deflation of the elastic CG (2D): at most DFL_FMAX fragments,
// three rigid modes each; the int metadata array holds the fragment count,
// the candidate count, the kept roots and the candidate list.
constexpr int DFL_FMAX = 8;
constexpr int DFL_M = 3 * DFL_FMAX;
constexpr int DFL_LIST = 256;
enum { DFL_META_NFRAG = 0, DFL_META_NCAND = 1, DFL_META_ROOTS = 2, DFL_META_LIST = 16,
       DFL_META_INTS = DFL_META_LIST + DFL_LIST };
static_assert(DFL_META_ROOTS + DFL_FMAX <= DFL_META_LIST, "deflation metadata layout");
// a mode whose Cholesky pivot falls below this fraction of E's largest
// diagonal entry is dropped
constexpr double DFL_PIVOT = 1e-12;

struct Grid {
  int nx, ny, nz;
  double hx, hy, hz;
  int N;
  int bc;
  int dim;
  // thermal eigenstrain per element: eps0 = -eig_dT exp(-x_c / eig_depth) I
  // (3D thermal load) or -eig_dT erfc(y_c / eig_depth) I (2D thermal shock,
  // bc == BC_TSHOCK_2D); eig_dT is zero for operator actions on error
  // equations
  double eig_dT, eig_depth;
  int elem_min;   // 3D: levels of at least this many nodes use the element kernels
};

// Isotropic A0 in the form the element kernels use: sigma_xx = l2m e_xx +
// lam e_yy (+ lam e_zz), sigma_xy = mu gamma_xy.
struct Mat {
  double l2m, lam, mu;
};

// What the finishing block does with a reduced sum s (see post_scalar).
enum Post { P_STORE = 0, P_CG_ALPHA, P_CG_BETA, P_SQRT, P_NEG, P_FCG_BETA, P_FCG_ALPHA, P_ADD };

struct Red {
  double* part;       // >= number of blocks of the launch
  double* S;          // scalar array
  int slot;           // S[slot] receives the result
  int post;           // Post
  double* host = nullptr;   // optional: pinned host memory that also receives S[slot]
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_down(v, off, WAVE);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, WAVE));
  return v;
}

__device__ __forceinline__ void post_scalar(double s, const Red& r) {
  switch (r.post) {
    case P_CG_ALPHA: {  // alpha = rz / pq
      r.S[r.slot] = s;
      r.S[S_ALPHA] = (s != 0.0) ? r.S[S_RZ] / s : 0.0;
    } break;
    case P_CG_BETA: {   // beta = rz_new / rz; rz = rz_new
      double rz = r.S[S_RZ];
      r.S[S_BETA] = (rz != 0.0) ? s / rz : 0.0;
      r.S[S_RZ] = s;
      r.S[r.slot] = s;
    } break;
    case P_SQRT:
      r.S[r.slot] = sqrt(s);
      break;
    case P_NEG:
      r.S[r.slot] = -s;
      break;
    case P_FCG_BETA: {  // beta = -(z.q_prev) / (p_prev.q_prev)
      const double pq = r.S[S_PQ];
      r.S[S_BETA] = (pq != 0.0) ? -s / pq : 0.0;
      r.S[r.slot] = s;
    } break;
    case P_FCG_ALPHA: {  // alpha = (p.r) / (p.q)
      const double pq = r.S[S_PQ];
      r.S[S_ALPHA] = (pq != 0.0) ? s / pq : 0.0;
      r.S[r.slot] = s;
    } break;
    case P_ADD:   // a second part of a sum stored earlier in the same slot
      r.S[r.slot] += s;
      break;
    default:
      r.S[r.slot] = s;
  }
  if (r.host) r.host[0] = r.S[r.slot];   // the host reads it behind an event, no copy
}

// Entries [0, n0) and [b0, b0 + n - n0) of a vector, walked as one index
// range 0..n-1: the displacement block and the damage rows that can be
// nonzero (the inactive band) of the coupled Newton vectors.
struct Seg {
  int64_t n0, b0, n;
};

__device__ __forceinline__ int64_t seg_index(const Seg& s, int64_t q) {
  return q < s.n0 ? q : s.b0 + (q - s.n0);
}

// The nodes of a box in a row-major grid: rows of stride W starting at base,
// w consecutive entries taken per row (w == W: one contiguous range), n
// entries in all, walked as one index range 0..n-1.
struct Box {
  int64_t base, W, w, n;
};

__device__ __forceinline__ int64_t box_index(const Box& b, int64_t q) {
  if (b.w == b.W) return b.base + q;
  const int64_t r = q / b.w;
  return b.base + r * b.W + (q - r * b.w);
}

// Independent reductions of one launch, finished together (launch_finish_multi):
// their post-operations must not read each other's results.
struct FinishSet {
  Red r[4];
  int maxmask;   // bit q set: r[q] is a max
  int count;     // 1..4
};

// Block-wide deterministic sum (MAX = false) or max (MAX = true) of v, stored
// as the block's partial r.part[bid].  A finishing kernel (launch_finish)
// then reduces the partials in a fixed order.  Every thread of the block must
// call it.  No fences or atomics: the kernel boundary orders the two passes.
template <int NT, bool MAX>
__device__ __forceinline__ void block_reduce(double v, const Red& r, int nblocks, int bid,
                                              int tid) {
  __shared__ double sh[NT / WAVE];
  (void)nblocks;
  __syncthreads();
  v = MAX ? wave_max(v) : wave_sum(v);
  const int lane = tid & (WAVE - 1), w = tid / WAVE;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (tid == 0) {
    double s = sh[0];
    for (int k = 1; k < NT / WAVE; ++k) s = MAX ? fmax(s, sh[k]) : s + sh[k];
    r.part[bid] = s;
  }
}

// XCD-aware tile order.  The dispatcher deals consecutive workgroups to the
// eight XCDs in turn, and each XCD has its own L2; remapping the dispatch
// index p so that XCD x receives one contiguous range of tiles keeps a
// tile's neighbours (which share its halo rows) in the same L2.
constexpr int NUM_XCD = 8;

__device__ __forceinline__ int xcd_tile(int p, int total) {
  const int x = p % NUM_XCD, slot = p / NUM_XCD;
  const int per = total / NUM_XCD, rem = total % NUM_XCD;
  return x * per + (x < rem ? x : rem) + slot;
}

// Map NaN to +inf so that max-reductions report non-finite values.
__device__ __forceinline__ double nan_to_inf(double x) { return (x != x) ? INFINITY : x; }

// Fischer--Burmeister NCP function phi(a, b) = sqrt(a^2 + b^2) - a - b.
__device__ __forceinline__ double fb(double a, double b) { return hypot(a, b) - a - b; }

// Box residual of MCP(F, l, u) for one component: phi(x - l, phi(u - x, -F)).
__device__ __forceinline__ double mcp_fb(double x, double F, double l, double u) {
  return fb(x - l, fb(u - x, -F));
}

}  // namespace frac
