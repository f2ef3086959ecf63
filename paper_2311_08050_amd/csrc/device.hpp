// Shared device-side definitions of the dense-INLA HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace inla {

// Tile geometry of the blocked Cholesky.
constexpr int NBI = 64;      // diagonal block / inner panel width
constexpr int PADN = 128;    // matrix orders and border heights are padded to this
constexpr int KC = 16;       // K chunk staged through LDS by the MFMA kernels

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Global-address-space views.  Pointers read out of descriptor structs are
// generic; without the cast the compiler emits flat loads, which also count
// against the LDS wait counter and so serialise prefetch with LDS reads.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) d2 gd2;
typedef __attribute__((address_space(1))) const d2 gcd2;
template <typename T> __device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// One matrix being factored by the bordered blocked Cholesky.  Columns [0, nf)
// are factored; rows [nf, nrows) are border rows carried along (they end up as
// G L^{-T}); the trailing update also maintains the Schur block of the border
// for columns [nf, ncols).  Column-major, leading dimension ld >= nrows.
struct FactorDesc {
  void *A;         // double or float elements (the factorisation's storage type)
  void *linv;      // (nf / NBI) x NBI x NBI: inverse of every diagonal block (col-major)
  int *info;       // first failing pivot (1-based), 0 if none
  int ld;
  int nf;          // columns to factor (multiple of PADN)
  int nrows;       // multiple of PADN
  int ncols;       // nf <= ncols <= nrows, multiple of PADN
  int id_row0;     // first row of an identity border block (INT_MAX if none)
  int pad_;
  // BF16 copies of the current panel for the BF16 trailing update, two slots
  // (panel parity): slot s holds entry (k-group g, row r) = the eight panel
  // values of row r at k = p0 + 8g .. p0 + 8g + 7 as 16 bytes at
  // pbf[s * pbf_slot + g * nf + r]; rows [p0 + nb, nf) are written
  void *pbf;
  int64_t pbf_slot;  // entries per slot
};

// Likelihood / prior kinds (values match the C header).
enum { LIK_GAUSSIAN = 0, LIK_POISSON = 1 };
enum { PRIOR_DENSE = 0, PRIOR_EXPCOV = 1, PRIOR_KRON = 2 };

// Per-theta model and workspace description used by the assembly, solve and
// reduction kernels.
struct ThetaDesc {
  // model (device pointers owned by the caller)
  const double *y, *E, *C, *e, *coords, *Quser;
  int n, k, lik, prior, n_s, n_t, ldquser;
  int n_pad;       // round_up(n, PADN)
  double tau, rho, delta, lpar;   // prior parameters; lpar = sigma^2 or beta0
  // workspace (owned by the library)
  double *Qp; int ldqp;           // prior precision, n_pad x n_pad, lower, identity padded
  void *W; int ldw; int Nw; int Ncw;    // big working matrix (double or float): Nw rows, Ncw columns
  double *S; int lds; int Ns; int k_pad;   // small (kriging) system working matrix
  double *P; int ldp; int Np; int ns_pad;  // prior-build working matrix
  double *x;       // current iterate / linearisation point [n_pad]
  double *r;       // right-hand side / new iterate [n_pad]
  double *xn;      // refined new iterate [n_pad] (mixed precision)
  double *z;       // residual / forward-solve vector [n_pad] (mixed precision)
  double *lam;     // [k_pad] kriging multipliers
  double *dlam;    // [k_pad] multiplier correction (mixed precision)
  double *rtwo;    // [k_pad] constraint residual e - C x (mixed precision)
  double *part;    // [2 * ldw] per-column partial sums (loglik, x'Qx)
  double *dres;    // [16] per-theta device results (see DRES_*)
  void *linv;      // inverses of the big factor's 64 x 64 diagonal blocks (factor storage type)
  double *u;       // forward-solve output / refinement correction [n_pad]
  double *symv;    // partial sums of Q_prior v from its lower triangle: P
                   // ((n_pad / 64) x n_pad, block column J's part of row i at
                   // J n_pad + i), then D [n_pad] (the transposed part)
  double *out;     // caller's output vector (mode or variances), device
  // variational-Bayes mean correction: with vb_var set, the likelihood terms
  // are expectations over eta ~ N(eta(x), vb_var[i]) by ngh-point Gauss-Hermite
  // quadrature (gh: nodes, then weights divided by sqrt(pi))
  const double *vb_var;
  const double *gh;
  int ngh;
  // general design matrix (m > 0; m == 0 means A = I): the caller's CSR, its
  // CSC and the lower pattern of A^T A (column c: entries patp[c] .. patp[c+1],
  // entry e in row patr[e] with terms patt[e] .. patt[e+1] of coefficient
  // tcoef[q] = A_{i r} A_{i c} for observation tobs[q]); per-observation
  // workspace: A x, the likelihood terms g, W and log pi(y_i | eta_i)
  int m;
  const int *A_rowptr, *A_col;
  const double *A_val;
  const int *cscp, *csci;
  const double *cscv;
  const int *patp, *patr, *patt, *tobs;
  const double *tcoef;
  double *obs_ax, *obs_g, *obs_W, *obs_ll;
};

// Per-theta device result slots.
enum {
  DRES_LOGDET_L = 0,   // 2 sum log L_ii of the big factor (first n pivots)
  DRES_LOGDET_S = 1,   // 2 sum log of the kriging factor (first k pivots)
  DRES_WNORM2 = 2,     // ||L_S^{-1} (C x_u - e)||^2
  DRES_STEP = 3,       // ||x_new - x||_inf
  DRES_SCALE = 4,      // max(1, ||x_new||_inf)
  DRES_XQX = 5,
  DRES_LOGLIK = 6,
  DRES_NONFINITE = 7,  // 1 if a non-finite value was met
  DRES_RANK = 8,       // 1 if the kriging system is numerically singular
  DRES_IR_DX = 9,      // last refinement correction ||dx||_inf
  DRES_IR_X = 10,      // max(1, ||x||_inf) of the refined iterate
  DRES_COUNT = 16
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Deterministic sum over a 256-thread block (fixed pairing order).
__device__ __forceinline__ double block_sum256(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}
__device__ __forceinline__ double block_max256(double v, double *sh) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  __syncthreads();
  return t;
}

}  // namespace inla
