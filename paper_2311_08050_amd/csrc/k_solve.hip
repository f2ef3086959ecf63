// Triangular solves, the kriging solve, Newton control, mixed-precision
// refinement steps and fixed-order reductions.  One workgroup per theta unless
// stated otherwise.  Factors may be stored in FP64 or FP32 (template T); every
// solve accumulates in FP64.
#include <cmath>

#include "device.hpp"
#include "host.hpp"
#include "model.hpp"

namespace inla {

// Solve L^T x = x in place for a lower-triangular L (column-major, order np, a
// multiple of 64) in 64-row blocks from the bottom.  For each block: the 64
// dot products with the already solved tail (coalesced column reads, 16 columns
// per wave), then a 64-step substitution in wave 0 against the block staged in
// LDS (D, 64 x 65 doubles).  Global writes to x are made visible to the other
// waves of the workgroup by the barriers.
template <typename T>
__device__ void trsv_lt_block(const T *__restrict__ L, int ld, int np, double *x, double *sred, double (*D)[65]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i0 = np - 64; i0 >= 0; i0 -= 64) {
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    const T *Lc = L + (size_t)(i0 + 16 * w) * ld;
    for (int j = i0 + 64 + lane; j < np; j += 64) {
      const double xj = x[j];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += (double)Lc[(size_t)q * ld + j] * xj;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double s = wave_sum(acc[q]);
      if (lane == 0) sred[16 * w + q] = s;
    }
    for (int e = tid; e < 64 * 64; e += 256) {
      const int r = e & 63, c = e >> 6;
      D[r][c] = (double)L[(size_t)(i0 + c) * ld + i0 + r];
    }
    __syncthreads();
    if (w == 0) {
      double rhs = x[i0 + lane] - sred[lane];
      double xm = 0.0;
      for (int i = 63; i >= 0; --i) {
        const double xi = __shfl(rhs, i, 64) / D[i][i];
        if (lane == i) xm = xi;
        if (lane < i) rhs -= D[i][lane] * xi;
      }
      x[i0 + lane] = xm;
    }
    __syncthreads();
  }
}

// Solve L x = x in place (forward substitution), same blocking from the top.
// The block's rows against the solved head: thread (row i, column phase p)
// sums columns j = p, p+4, ... (each column read is 64 contiguous values).
template <typename T>
__device__ void trsv_l_block(const T *__restrict__ L, int ld, int np, double *x, double *sred4, double (*D)[65]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i0 = 0; i0 < np; i0 += 64) {
    double s = 0.0;
#pragma unroll 8
    for (int j = w; j < i0; j += 4) s += (double)L[(size_t)j * ld + i0 + lane] * x[j];
    sred4[w * 64 + lane] = s;
    for (int e = tid; e < 64 * 64; e += 256) {
      const int r = e & 63, c = e >> 6;
      D[r][c] = (double)L[(size_t)(i0 + c) * ld + i0 + r];
    }
    __syncthreads();
    if (w == 0) {
      double rhs = x[i0 + lane] - ((sred4[lane] + sred4[64 + lane]) + (sred4[128 + lane] + sred4[192 + lane]));
      double xm = 0.0;
      for (int c = 0; c < 64; ++c) {
        const double xc = __shfl(rhs, c, 64) / D[c][c];
        if (lane == c) xm = xc;
        if (lane > c) rhs -= D[lane][c] * xc;
      }
      x[i0 + lane] = xm;
    }
    __syncthreads();
  }
}

// Vector selectors for the step-wise triangular solves (V_* in model.hpp).
__device__ __forceinline__ double *vsel(const ThetaDesc &t, int v) {
  return v == V_X ? t.x : v == V_R ? t.r : v == V_XN ? t.xn : v == V_Z ? t.z : t.u;
}

// y = M v or y = M^T v for a 64 x 64 block M stored column-major at Mg
// (element (m, c) at Mg[c * 64 + m]).  block64_load reads the block into
// registers, lane m of wave w holding row m of columns 16w .. 16w + 15 (each
// load 64 contiguous elements of one column), so that the caller can issue it
// ahead of other work; neither product stages the block in LDS, which keeps
// the solve steps' LDS at a few KB.
template <typename T>
__device__ __forceinline__ void block64_load(const T *__restrict__ Mg, T (&e)[16]) {
  const auto *g = gptr(Mg);
  const int m = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 16; ++q) e[q] = g[(16 * w + q) * 64 + m];
}

// Sums a[0..15] over the 64 lanes of a wave: lane l returns the total of
// a[l >> 2].  A butterfly that halves the values it carries at each of the
// first four exchanges (lane bits 5, 4, 3, 2 pick the half kept), then adds
// across lane bits 1 and 0: 17 exchanges in place of 16 full reductions.
// a is overwritten.
template <int HALF>
__device__ __forceinline__ void fold_half(double (&a)[16], int l) {
  const bool up = (l & (4 * HALF)) != 0;
#pragma unroll
  for (int h = 0; h < HALF; ++h) {
    const double keep = up ? a[h + HALF] : a[h], send = up ? a[h] : a[h + HALF];
    a[h] = keep + __shfl_xor(send, 4 * HALF, 64);
  }
}
__device__ __forceinline__ double wave_sum16(double (&a)[16]) {
  const int l = threadIdx.x & 63;
  fold_half<8>(a, l);
  fold_half<4>(a, l);
  fold_half<2>(a, l);
  fold_half<1>(a, l);
  double s = a[0];
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 1, 64);
  return s;
}

// y = M v for the block whose elements block64_load read into e: each wave
// sums its 16 columns, the four partial sums meet in `part` (4 x 64 doubles of
// LDS).  v and y live in LDS.  All 256 threads take part; returns after a
// barrier.
template <typename T>
__device__ __forceinline__ void block64_mv(const T (&e)[16], const double *v, double *y, double (*part)[64]) {
  const int tid = threadIdx.x, m = tid & 63, w = tid >> 6;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) s += (double)e[q] * v[16 * w + q];
  part[w][m] = s;
  __syncthreads();
  if (tid < 64) y[tid] = (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
  __syncthreads();
}

// y = M^T v for the block in e: y[16w + q] = sum over the rows m (the lanes)
// of M[m][16w + q] v[m], formed whole by wave w.  v and y live in LDS; returns
// after a barrier.
template <typename T>
__device__ __forceinline__ void block64_mtv(const T (&e)[16], const double *v, double *y) {
  const int m = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double vm = v[m];
  double a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) a[q] = (double)e[q] * vm;
  const double s = wave_sum16(a);
  if ((m & 3) == 0) y[16 * w + (m >> 2)] = s;
  __syncthreads();
}

// One 64-row block step of the forward solve L z = r for every theta (a launch
// per block, blocks from the top).  On entry z_b = L_bb^{-1} r_b is already in
// z (written by the previous step; the first step forms it from the stored
// inverse of the diagonal block).  The rows below are updated,
// r_j -= sum_c L[j][i0 + c] z_b[c], 256 rows per workgroup (one thread per row,
// each column read contiguous across the threads).  The workgroup holding the
// next block's rows finalises them and forms z_{b+1} for the next launch.
template <typename T>
__global__ __launch_bounds__(256) void trsv_fwd_step_kernel(const ThetaDesc *__restrict__ td, int i0, int src, int dst) {
  const ThetaDesc t = td[blockIdx.y];
  const int np = t.n_pad;
  if (i0 >= np) return;
  const int tid = threadIdx.x;
  const auto *L = gptr((const T *)t.W);
  const T *linv = (const T *)t.linv;
  auto *r = gptr(vsel(t, src));
  auto *z = gptr(vsel(t, dst));
  __shared__ double part[4][64];
  __shared__ double zb[64], rb[64], zn[64];
  const bool next = blockIdx.x == 0 && i0 + 64 < np;   // this workgroup forms z_{b+1}
  T e[16];
  if (i0 == 0) {
    block64_load(linv, e);
    if (tid < 64) rb[tid] = r[tid];
    __syncthreads();
    block64_mv(e, rb, zb, part);
    if (blockIdx.x == 0 && tid < 64) z[tid] = zb[tid];
  } else {
    if (tid < 64) zb[tid] = z[i0 + tid];
    __syncthreads();
  }
  // the next diagonal block's inverse is read while the rows are updated
  if (next) block64_load(linv + (size_t)(i0 / 64 + 1) * 4096, e);
  const int j = i0 + 64 + blockIdx.x * 256 + tid;
  double nv = 0.0;
  if (j < np) {
    T lv[64];   // all 64 loads in flight before the first product
#pragma unroll
    for (int c = 0; c < 64; ++c) lv[c] = L[(size_t)(i0 + c) * t.ldw + j];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 64; ++c) s += (double)lv[c] * zb[c];
    nv = r[j] - s;
    r[j] = nv;
  }
  if (next) {
    if (tid < 64) rb[tid] = nv;
    __syncthreads();
    block64_mv(e, rb, zn, part);
    if (tid < 64) z[i0 + 64 + tid] = zn[tid];
  }
}

// One 64-row block step of the back solve L^T x = r (blocks from the bottom).
// On entry x_b = L_bb^{-T} r_b is already in x (the bottom block of a theta
// forms it from the stored inverse).  The columns above are updated,
// r_j -= sum_m L[i0 + m][j] x_b[m]: a workgroup takes 64 columns, a wave 16 of
// them with its lanes on the 64 contiguous rows of each, and the wave's 16 x 64
// products are summed per column across its lanes (wave_sum16).  The workgroup
// holding the columns just above the block finalises them and forms x_{b-1}
// for the next launch.
template <typename T>
__global__ __launch_bounds__(256) void trsv_bwd_step_kernel(const ThetaDesc *__restrict__ td, int i0, int src, int dst) {
  const ThetaDesc t = td[blockIdx.y];
  const int np = t.n_pad;
  if (i0 >= np) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const auto *L = gptr((const T *)t.W);
  const T *linv = (const T *)t.linv;
  auto *r = gptr(vsel(t, src));
  auto *x = gptr(vsel(t, dst));
  __shared__ double xb[64], rb[64], xn[64];
  T e[16];
  if (i0 + 64 == np) {
    block64_load(linv + (size_t)(i0 / 64) * 4096, e);
    if (tid < 64) rb[tid] = r[i0 + tid];
    __syncthreads();
    block64_mtv(e, rb, xb);
    if (blockIdx.x == 0 && tid < 64) x[i0 + tid] = xb[tid];
  } else {
    if (tid < 64) xb[tid] = x[i0 + tid];
    __syncthreads();
  }
  const int g = blockIdx.x;
  if (64 * g >= i0) return;
  // the workgroup holding the columns just above the block forms x_{b-1}:
  // its diagonal block's inverse is read while the columns are updated
  const bool prev = 64 * g + 64 == i0;
  if (prev) block64_load(linv + (size_t)(i0 / 64 - 1) * 4096, e);
  const double xm = xb[lane];
  const int j0 = 64 * g + 16 * w;
  T v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = L[(size_t)(j0 + q) * t.ldw + i0 + lane];
  double a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) a[q] = (double)v[q] * xm;
  const double s = wave_sum16(a);
  const int jc = j0 + (lane >> 2);
  double nv = 0.0;
  if ((lane & 3) == 0) {
    nv = r[jc] - s;
    r[jc] = nv;
  }
  if (prev) {
    if ((lane & 3) == 0) rb[16 * w + (lane >> 2)] = nv;
    __syncthreads();
    block64_mtv(e, rb, xn);
    if (tid < 64) x[i0 - 64 + tid] = xn[tid];
  }
}

// A Newton step taken in correction form starts its new iterate at the current
// one (xn <- x); one refinement step then adds the constrained correction.
__global__ __launch_bounds__(256) void restart_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < t.n_pad) t.xn[i] = t.x[i];
}

// Accept the refined iterate: Newton stopping quantities and x <- xn.
__global__ __launch_bounds__(256) void newton_accept_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.x];
  __shared__ double sh[4];
  double st = 0.0, sc = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < t.n; i += 256) {
    const double xn = t.xn[i], xo = t.x[i];
    if (!isfinite(xn)) bad = 1.0;
    st = fmax(st, fabs(xn - xo));
    sc = fmax(sc, fabs(xn));
  }
  st = block_max256(st, sh);
  sc = block_max256(sc, sh);
  bad = block_sum256(bad, sh);
  for (int i = threadIdx.x; i < t.n_pad; i += 256) t.x[i] = i < t.n ? t.xn[i] : 0.0;
  if (threadIdx.x == 0) {
    t.dres[DRES_STEP] = st;
    t.dres[DRES_SCALE] = fmax(1.0, sc);
    if (bad > 0.0) t.dres[DRES_NONFINITE] = 1.0;
  }
}

// Kriging solve after the small (FP64) factorisation: w from the border row,
// then lambda = L_S^{-T} w; also log|S| = 2 sum log (L_S)_ii, ||w||^2 and the
// numerical-rank flag.
__global__ __launch_bounds__(256) void kriging_solve_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.x];
  __shared__ double sred[64];
  __shared__ double sh[4];
  __shared__ double D[64][65];
  const int kp = t.k_pad, k = t.k;
  double lds_ = 0.0, w2 = 0.0, dmin = INFINITY, dmax = 0.0;
  for (int i = threadIdx.x; i < kp; i += 256) {
    const double wv = i < k ? t.S[(size_t)i * t.lds + kp] : 0.0;
    t.lam[i] = wv;
    w2 += wv * wv;
    if (i < k) {
      const double d = t.S[(size_t)i * t.lds + i];
      lds_ += log(d);
      dmin = fmin(dmin, d * d);
      dmax = fmax(dmax, d * d);
    }
  }
  lds_ = block_sum256(lds_, sh);
  w2 = block_sum256(w2, sh);
  dmin = -block_max256(-dmin, sh);
  dmax = block_max256(dmax, sh);
  trsv_lt_block<double>(t.S, t.lds, kp, t.lam, sred, D);
  if (threadIdx.x == 0) {
    t.dres[DRES_LOGDET_S] = 2.0 * lds_;
    t.dres[DRES_WNORM2] = w2;
    // squared pivot below 1e-13 of the largest: numerically dependent constraints
    t.dres[DRES_RANK] = (k > 0 && !(dmin >= 1e-13 * dmax)) ? 1.0 : 0.0;
  }
}

// r_c = z_c - sum_a lambda_a (G L^{-T})_{a,c}.  Newton (from_z = 0): z is the
// factored b row and lambda the kriging multipliers, giving the corrected
// right-hand side of x = L^{-T}(L^{-1} b - L^{-1} C^T lambda).  Refinement
// (from_z = 1): u = L^{-1} r1 and lambda = dlambda.
template <typename T>
__global__ __launch_bounds__(256) void rhs_kernel(const ThetaDesc *__restrict__ td, int from_z) {
  const ThetaDesc t = td[blockIdx.y];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c0 = blockIdx.x * 64 + w * 16;
  if (c0 >= t.n_pad) return;
  const int k = t.k, np = t.n_pad;
  const double *lam = from_z ? t.dlam : t.lam;
  for (int q = 0; q < 16; ++q) {
    const int c = c0 + q;
    const T *col = (const T *)t.W + (size_t)c * t.ldw + np;
    double s = 0.0;
    for (int a = lane; a < k; a += 64) s += lam[a] * (double)col[a];
    s = wave_sum(s);
    if (lane == 0) t.r[c] = (from_z ? t.u[c] : (double)col[k]) - s;
  }
}

// Refinement, constrained part 1: t = (L^{-1} C^T)^T u - r2 = C Q~^{-1} r1 - r2 with
// u = L^{-1} r1, into dlam.  A workgroup per 64 border rows; the four waves split
// the columns, each column read is 64 contiguous border values.
template <typename T>
__global__ __launch_bounds__(256) void border_gemv_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int a = blockIdx.x * 64 + (threadIdx.x & 63), w = threadIdx.x >> 6;
  __shared__ double part[4][64];
  if ((int)blockIdx.x * 64 >= t.k_pad) return;
  const int np = t.n_pad;
  double s = 0.0;
  if (a < t.k) {
    const T *row = (const T *)t.W + np + a;
#pragma unroll 8
    for (int c = w; c < np; c += 4) s += (double)row[(size_t)c * t.ldw] * t.u[c];
  }
  part[w][threadIdx.x & 63] = s;
  __syncthreads();
  if (w == 0) {
    const int l = threadIdx.x;
    t.dlam[a] = a < t.k ? ((part[0][l] + part[1][l]) + (part[2][l] + part[3][l])) - t.rtwo[a] : 0.0;
  }
}

// Refinement, constrained part 2: dlambda = S~^{-1} t with the FP64 kriging factor.
__global__ __launch_bounds__(256) void kriging_correct_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.x];
  __shared__ double sred4[256];
  __shared__ double D[64][65];
  if (t.k_pad > 0) {
    trsv_l_block<double>(t.S, t.lds, t.k_pad, t.dlam, sred4, D);
    trsv_lt_block<double>(t.S, t.lds, t.k_pad, t.dlam, sred4, D);
  }
}

// Refinement, update: xn += dx (dx in u), lambda += dlambda, and the
// quantities of the refinement stopping test.
__global__ __launch_bounds__(256) void ir_update_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.x];
  __shared__ double sh[4];
  double dm = 0.0, xm = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < t.n_pad; i += 256) {
    double v = 0.0;
    if (i < t.n) {
      const double dx = t.u[i];
      v = t.xn[i] + dx;
      if (!isfinite(v)) bad = 1.0;
      dm = fmax(dm, fabs(dx));
      xm = fmax(xm, fabs(v));
    }
    t.xn[i] = v;
  }
  for (int a = threadIdx.x; a < t.k; a += 256) t.lam[a] += t.dlam[a];
  dm = block_max256(dm, sh);
  xm = block_max256(xm, sh);
  bad = block_sum256(bad, sh);
  if (threadIdx.x == 0) {
    t.dres[DRES_IR_DX] = bad > 0.0 ? INFINITY : dm;
    t.dres[DRES_IR_X] = fmax(1.0, xm);
  }
}

// log|Q| = 2 sum_{i<n} log L_ii of the big factor, and the fixed-order sums of
// the per-column partials (log-likelihood, x^T Q_prior x).
template <typename T>
__global__ __launch_bounds__(256) void finish_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.x];
  __shared__ double sh[4];
  double ld = 0.0, ll = 0.0, xq = 0.0;
  const T *W = (const T *)t.W;
  for (int i = threadIdx.x; i < t.n; i += 256) {
    ld += log((double)W[(size_t)i * t.ldw + i]);
    ll += t.part[i];
    xq += t.part[t.ldw + i];
  }
  for (int i = threadIdx.x; i < t.m; i += 256) ll += t.obs_ll[i];   // general design matrix
  ld = block_sum256(ld, sh);
  ll = block_sum256(ll, sh);
  xq = block_sum256(xq, sh);
  if (threadIdx.x == 0) {
    t.dres[DRES_LOGDET_L] = 2.0 * ld;
    t.dres[DRES_LOGLIK] = ll;
    t.dres[DRES_XQX] = xq;
  }
}

// Caller matrix (t.Quser, ld t.ldquser, order n) -> working matrix (storage T),
// identity padded.
template <typename T>
__global__ __launch_bounds__(256) void copy_in_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= t.Nw) return;
  T *col = (T *)t.W + (size_t)c * t.ldw;
  const double *src = t.Quser + (size_t)c * t.ldquser;
  for (int r = c + threadIdx.x; r < t.Nw; r += 256) col[r] = (T)((r < t.n && c < t.n) ? src[r] : (r == c ? 1.0 : 0.0));
}
// Factor -> caller matrix (lower triangle only, as FP64).
template <typename T>
__global__ __launch_bounds__(256) void copy_out_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= t.n) return;
  const T *col = (const T *)t.W + (size_t)c * t.ldw;
  double *dst = (double *)t.Quser + (size_t)c * t.ldquser;
  for (int r = c + threadIdx.x; r < t.n; r += 256) dst[r] = (double)col[r];
}

// Marginal variances, small system: S = -Schur(C, C) with the border rows
// V_i = -Schur(I_i, C) (V = Q^{-1} C^T) below it, k_pad columns to factor.
__global__ __launch_bounds__(256) void var_small_build_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  const int kp = t.k_pad, k = t.k, np = t.n_pad;
  if (c >= kp) return;
  double *col = t.S + (size_t)c * t.lds;
  const double *sch = (const double *)t.W + (size_t)(np + c) * t.ldw + np;   // column np + c, from row np
  for (int r = c + threadIdx.x; r < t.Ns; r += 256) {
    double v = 0.0;
    if (r < kp) {
      if (r < k && c < k) v = -sch[r];
      else if (r == c) v = 1.0;
    } else if (c < k) {
      v = -sch[kp + (r - kp)];     // row np + kp + i of the big matrix: identity-border row i
    }
    col[r] = v;
  }
}

// var_i = ||row i of L^{-T}||^2 - ||row i of V L_S^{-T}||^2 (i < n), written to t.out.
__global__ __launch_bounds__(256) void var_norms_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= t.n) return;
  const int np = t.n_pad, kp = t.k_pad;
  const double *row = (const double *)t.W + np + kp + i;
  double s = 0.0;
  for (int c = 0; c < np; ++c) { const double v = row[(size_t)c * t.ldw]; s += v * v; }
  double s2 = 0.0;
  if (t.k > 0) {
    const double *row2 = t.S + kp + i;
    for (int c = 0; c < t.k; ++c) { const double v = row2[(size_t)c * t.lds]; s2 += v * v; }
  }
  t.out[i] = s - s2;
}

// ------------------------------------------------------------------ launchers
#define INLA_DISPATCH_T(prec, KERNEL, ...)                                        \
  do {                                                                            \
    if ((prec) != INLA_PREC_FP64) hipLaunchKernelGGL(KERNEL<float>, __VA_ARGS__); \
    else hipLaunchKernelGGL(KERNEL<double>, __VA_ARGS__);                        \
  } while (0)

void launch_kriging_solve(Ctx &ctx, const ThetaDesc *dtd, int B) {
  if (B <= 0) return;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] { hipLaunchKernelGGL(kriging_solve_kernel, dim3(B), dim3(256), 0, ctx.stream, dtd); });
}
void launch_rhs(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, int from_z, int prec) {
  if (B <= 0 || np_max <= 0) return;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
    INLA_DISPATCH_T(prec, rhs_kernel, dim3((np_max + 63) / 64, B), dim3(256), 0, ctx.stream, dtd, from_z);
  });
}
void launch_trsv_fwd(Ctx &ctx, const std::vector<ThetaDesc> &htd, int np_max, int src, int dst, double bytes,
                     int prec) {
  const int B = (int)htd.size();
  if (B <= 0 || np_max <= 0) return;
  const std::vector<int64_t> key = {0x54525346, prec != INLA_PREC_FP64, B, np_max, src, dst,
                                    (int64_t)std::llround(bytes)};
  (void)ctx.sequence(INLA_K_SOLVE, key, htd.data(), sizeof(ThetaDesc) * B, [&](const void *dv) {
    const ThetaDesc *dtd = (const ThetaDesc *)dv;
    for (int i0 = 0; i0 < np_max; i0 += 64) {
      const int gx = std::max(1, (np_max - i0 - 64 + 255) / 256);
      ctx.launch(INLA_K_SOLVE, 0.0, bytes * (double)(np_max - i0) / np_max * 2.0 / np_max, [&] {
        INLA_DISPATCH_T(prec, trsv_fwd_step_kernel, dim3(gx, B), dim3(256), 0, ctx.stream, dtd, i0, src, dst);
      });
    }
  });
}
void launch_trsv_bwd(Ctx &ctx, const std::vector<ThetaDesc> &htd, int np_max, int src, int dst, double bytes,
                     int prec) {
  const int B = (int)htd.size();
  if (B <= 0 || np_max <= 0) return;
  const std::vector<int64_t> key = {0x54525342, prec != INLA_PREC_FP64, B, np_max, src, dst,
                                    (int64_t)std::llround(bytes)};
  (void)ctx.sequence(INLA_K_SOLVE, key, htd.data(), sizeof(ThetaDesc) * B, [&](const void *dv) {
    const ThetaDesc *dtd = (const ThetaDesc *)dv;
    for (int i0 = np_max - 64; i0 >= 0; i0 -= 64) {
      const int gx = std::max(1, (i0 + 63) / 64);
      ctx.launch(INLA_K_SOLVE, 0.0, bytes * (double)(i0 + 64) / np_max * 2.0 / np_max, [&] {
        INLA_DISPATCH_T(prec, trsv_bwd_step_kernel, dim3(gx, B), dim3(256), 0, ctx.stream, dtd, i0, src, dst);
      });
    }
  });
}
void launch_restart(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max) {
  if (B <= 0 || np_max <= 0) return;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(restart_kernel, dim3((np_max + 255) / 256, B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_newton_accept(Ctx &ctx, const ThetaDesc *dtd, int B) {
  if (B <= 0) return;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] { hipLaunchKernelGGL(newton_accept_kernel, dim3(B), dim3(256), 0, ctx.stream, dtd); });
}
void launch_ir_correct(Ctx &ctx, const ThetaDesc *dtd, int B, int kp_max, int prec) {
  if (B <= 0) return;
  if (kp_max > 0)
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      INLA_DISPATCH_T(prec, border_gemv_kernel, dim3(kp_max / 64, B), dim3(256), 0, ctx.stream, dtd);
    });
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] { hipLaunchKernelGGL(kriging_correct_kernel, dim3(B), dim3(256), 0, ctx.stream, dtd); });
}
void launch_ir_update(Ctx &ctx, const ThetaDesc *dtd, int B) {
  if (B <= 0) return;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] { hipLaunchKernelGGL(ir_update_kernel, dim3(B), dim3(256), 0, ctx.stream, dtd); });
}
void launch_finish(Ctx &ctx, const ThetaDesc *dtd, int B, int prec) {
  if (B <= 0) return;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
    INLA_DISPATCH_T(prec, finish_kernel, dim3(B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_copy_in(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, int prec) {
  if (B <= 0 || np_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    INLA_DISPATCH_T(prec, copy_in_kernel, dim3(np_max, B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_copy_out(Ctx &ctx, const ThetaDesc *dtd, int B, int n_max, int prec) {
  if (B <= 0 || n_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    INLA_DISPATCH_T(prec, copy_out_kernel, dim3(n_max, B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_var_small_build(Ctx &ctx, const ThetaDesc *dtd, int B, int kp_max) {
  if (B <= 0 || kp_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(var_small_build_kernel, dim3(kp_max, B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_var_norms(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max) {
  if (B <= 0 || np_max <= 0) return;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(var_norms_kernel, dim3((np_max + 255) / 256, B), dim3(256), 0, ctx.stream, dtd);
  });
}

}  // namespace inla
