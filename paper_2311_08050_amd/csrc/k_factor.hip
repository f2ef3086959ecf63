// Bordered, batched, blocked Cholesky for gfx950.
//
// Dense Cholesky is the step the paper names as the bottleneck of every
// hyperparameter evaluation (section "Implementation of INLA+: OpenMP and MPI
// parallelization"; 3-5 factorisations per evaluation in section "Running INLA+
// on multiple nodes").  Here each theta of a batch owns one column-major matrix;
// every launch processes the same step of all of them.
//
// A matrix is [[Q, .], [G, D]] with G the border rows; factoring the first nf
// columns leaves L (Q = L L^T), G L^{-T} in the border rows and D - G Q^{-1} G^T
// in the Schur block.  Border rows carry the constraint rows C and the Newton
// right-hand side b, so C Q^{-1} C^T, C Q^{-1} b and L^{-1} b fall out of the
// factorisation's own MFMA updates.
//
// Per outer panel [p0, pend = p0 + nb), left-looking inside the panel and
// right-looking across panels:
//   potf2_inv  : L_pp = chol(A_pp) and X = L_pp^{-1} in FP64 in LDS for the first
//                diagonal block (one workgroup per theta)
//   panel step : per 64-wide block column j, per 64-row tile I below it
//                L[I,j] = (A[I,j] - L[I,p0:j] L[j,p0:j]^T) X_j^T, the SYRK of the
//                in-panel diagonal block A[I,I], and chol / inverse of the next
//                diagonal block by the tile just below (MFMA, one launch per j)
//   TRAIL      : A[pend:, pend:ncols] -= A[pend:, p0:pend] A[pend:ncols, p0:pend]^T
// Blocked right-looking Cholesky is the textbook form; the left-looking panel
// and the fused diagonal factorisation are this implementation's choice.
//
// Storage and MFMA precision are template parameters: FP64 storage with
// v_mfma_f64_16x16x4f64, or FP32 storage with v_mfma_f32_16x16x4f32 (FP32
// accumulate).  Operands are LDS-staged in double-buffered K chunks.
#include <limits>
#include <type_traits>

#include "device.hpp"
#include "host.hpp"

namespace inla {

// TRAIL updates everything right of the panel; with lookahead it is split into
// TRAIL_A (the next panel's columns) and TRAIL_B (the columns after it), so
// that the next panel can be factored while TRAIL_B runs.
enum { KIND_TRAIL = 0, KIND_TRAIL_A = 1, KIND_TRAIL_B = 2 };

typedef float f4 __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------------------
// Diagonal block: Cholesky of the 64 x 64 block A_jj and its inverse in one
// LDS-resident FP64 pass of 34 KB: L_jj overwrites the lower triangle and
// X = L_jj^{-1} (lower triangular) is built in the strict upper triangle,
// transposed, with its diagonal 1 / L_cc kept apart.
// Cholesky by sub-panels of width 16: an unblocked 16 x 16 Cholesky held in
// registers of wave 0 (lane r owns row r, pivots and columns broadcast with
// readlane), a forward-substitution TRSM of the rows below (one thread per
// row, reciprocal pivots), and the rank-16 update of the rest (row in
// registers, column values broadcast from LDS).  Inverse by 16 x 16 blocks:
// X_ii = L_ii^{-1} (one wave per block, one lane per column), then
// X_ij = -X_ii (L_ij X_jj + ... + L_i,i-1 X_i-1,j) by distance i - j.
// --------------------------------------------------------------------------
struct Potf2Lds {
  double M[NBI][NBI + 1];   // lower: the block, then L; strict upper: X[a][b] at M[b][a] (a > b)
  double rd[NBI];           // reciprocal pivots 1 / L_cc = X[c][c]
  int fail;
};

__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __hiloint2double(hi, lo);
}

// X = L^{-1} element (a, b), a >= b, from its packed place.
__device__ __forceinline__ double xinv(const Potf2Lds &S, int a, int b) {
  return a == b ? S.rd[a] : S.M[b][a];
}

// sqrt(x) and 1 / sqrt(x) for x > 0 by Goldschmidt's coupled iteration
// (g -> sqrt(x), h -> 1 / (2 sqrt(x)), each step squaring the relative error
// r = 1/2 - g h) from the hardware reciprocal square root estimate; two steps
// take the estimate's error below the FP64 rounding level.
__device__ __forceinline__ void sqrt_rsqrt(double x, double &sq, double &rs) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
  }
  sq = g;
  rs = 2.0 * h;
}

// S.M's lower triangle holds the block (upper triangle ignored), S.fail = 0;
// all of it visible to the block.  On return the lower triangle holds L_jj,
// S.rd its reciprocal pivots, S.fail the first failing pivot (1-based) or 0.
__device__ __forceinline__ void potf2_factor(Potf2Lds &S, int tid) {
  constexpr int W = 16;
  for (int jb = 0; jb < NBI; jb += W) {
    // 1. 16 x 16 diagonal Cholesky in wave 0
    if (tid < 64) {
      const int r = tid & (W - 1);
      double a[W];
#pragma unroll
      for (int cc = 0; cc < W; ++cc) a[cc] = cc <= r ? S.M[jb + r][jb + cc] : 0.0;
      int bad = 0;
#pragma unroll
      for (int c = 0; c < W; ++c) {
        double dcc = lane_bcast(a[c], c);
        if (!(dcc > 0.0)) {
          if (bad == 0) bad = jb + c + 1;
          dcc = __builtin_nan("");
        }
        double sd, rs;
        sqrt_rsqrt(dcc, sd, rs);
        const double l = (r == c) ? sd : a[c] * rs;
        a[c] = l;
        if (tid == 0) S.rd[jb + c] = rs;
#pragma unroll
        for (int cc = c + 1; cc < W; ++cc) a[cc] -= l * lane_bcast(l, cc);
      }
      if (tid < W) {
#pragma unroll
        for (int cc = 0; cc < W; ++cc)
          if (cc <= r) S.M[jb + r][jb + cc] = a[cc];
      }
      if (tid == 0 && bad != 0 && S.fail == 0) S.fail = bad;
    }
    __syncthreads();
    // 2. TRSM of the block rows below the sub-panel
    const int R = NBI - (jb + W);
    if (tid < R) {
      const int r = jb + W + tid;
      double x[W];
#pragma unroll
      for (int c = 0; c < W; ++c) x[c] = S.M[r][jb + c];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        double s = x[c];
#pragma unroll
        for (int m = 0; m < c; ++m) s -= x[m] * S.M[jb + c][jb + m];
        x[c] = s * S.rd[jb + c];
      }
#pragma unroll
      for (int c = 0; c < W; ++c) S.M[r][jb + c] = x[c];
    }
    __syncthreads();
    // 3. rank-16 update of the lower triangle of columns [jb + 16, 64)
    if (R > 0) {
      const int nsplit = 256 / R;
      const int rr = tid % R, part = tid / R;
      if (part < nsplit) {
        const int r = jb + W + rr;
        double p[W];
#pragma unroll
        for (int m = 0; m < W; ++m) p[m] = S.M[r][jb + m];
        const int per = (R + nsplit - 1) / nsplit;
        const int cb = jb + W + part * per;
        const int ce = min(cb + per, r + 1);
        for (int c = cb; c < ce; ++c) {
          double s = S.M[r][c];
#pragma unroll
          for (int m = 0; m < W; ++m) s -= p[m] * S.M[c][jb + m];
          S.M[r][c] = s;
        }
      }
    }
    __syncthreads();
  }
}

// X = L^{-1} into the strict upper triangle (transposed) after potf2_factor.
__device__ __forceinline__ void potf2_invert(Potf2Lds &S, int tid) {
  constexpr int W = 16;
  // X_ii: wave i, lane c < 16 solves L_ii x = e_c by forward substitution
  {
    const int o = W * (tid >> 6), c = tid & 63;
    if (c < W) {
      double x[W];
#pragma unroll
      for (int r = 0; r < W; ++r) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < r; ++m) s += S.M[o + r][o + m] * x[m];
        x[r] = r < c ? 0.0 : (r == c ? S.rd[o + r] : -S.rd[o + r] * s);
      }
#pragma unroll
      for (int r = 1; r < W; ++r)
        if (r > c) S.M[o + c][o + r] = x[r];
    }
  }
  __syncthreads();
  // X_ij (i > j) by distance: T = sum_{k=j}^{i-1} L_ik X_kj, then X_ij = -X_ii T;
  // thread (r, c) = (tid / 16, tid % 16) of each block at that distance
  const int r = tid >> 4, c = tid & 15;
#pragma unroll
  for (int dist = 1; dist < NBI / W; ++dist) {
    const int nblk = NBI / W - dist;
    double t[NBI / W - 1];
#pragma unroll
    for (int q = 0; q < nblk; ++q) {
      const int i = q + dist, j = q, ar = W * i + r, bc = W * j + c;
      double s = 0.0;
      for (int k = j; k < i; ++k)
        for (int m = (k == j ? c : 0); m < W; ++m) s += S.M[ar][W * k + m] * xinv(S, W * k + m, bc);
      t[q] = s;
    }
    // T goes to X_ij's place, so that every thread can read all of it
#pragma unroll
    for (int q = 0; q < nblk; ++q) S.M[W * q + c][W * (q + dist) + r] = t[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < nblk; ++q) {
      const int i = q + dist, j = q;
      double s = 0.0;
      for (int m = 0; m <= r; ++m) s += xinv(S, W * i + r, W * i + m) * S.M[W * j + c][W * i + m];
      t[q] = -s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < nblk; ++q) S.M[W * q + c][W * (q + dist) + r] = t[q];
    __syncthreads();
  }
}

// Writes L_jj over the block's lower triangle at Ad (column-major, ld) and its
// inverse into slot j / 64 of d.linv; records a failing pivot in d.info.
template <typename T>
__device__ __forceinline__ void potf2_store(const Potf2Lds &S, const FactorDesc &d, int j,
                                            __attribute__((address_space(1))) T *Ad, int tid) {
  __attribute__((address_space(1))) T *Li = gptr((T *)d.linv) + (size_t)(j / NBI) * NBI * NBI;
#pragma unroll 4
  for (int i = 0; i < NBI * NBI / 256; ++i) {
    const int e = tid + 256 * i, r = e & (NBI - 1), c = e >> 6;
    if (r >= c) Ad[(size_t)c * d.ld + r] = (T)S.M[r][c];
    Li[c * NBI + r] = (T)(r >= c ? xinv(S, r, c) : 0.0);   // column-major (L^{-1})[r][c]
  }
  if (tid == 0 && S.fail != 0 && *d.info == 0) *d.info = j + S.fail;
}

template <typename T>
__global__ __launch_bounds__(256) void potf2_inv_kernel(const FactorDesc *__restrict__ descs, int j) {
  const FactorDesc d = descs[blockIdx.x];
  if (j >= d.nf) return;
  __shared__ Potf2Lds S;
  const int tid = threadIdx.x;
  __attribute__((address_space(1))) T *Ad = gptr((T *)d.A) + (size_t)j * d.ld + j;
  // all 16 loads in flight before the first LDS store
  T v[NBI * NBI / 256];
#pragma unroll
  for (int i = 0; i < NBI * NBI / 256; ++i) {
    const int e = tid + 256 * i;
    v[i] = Ad[(size_t)(e >> 6) * d.ld + (e & (NBI - 1))];
  }
#pragma unroll
  for (int i = 0; i < NBI * NBI / 256; ++i) {
    const int e = tid + 256 * i, r = e & (NBI - 1), c = e >> 6;
    S.M[r][c] = (r >= c) ? (double)v[i] : 0.0;
  }
  if (tid == 0) S.fail = 0;
  __syncthreads();
  potf2_factor(S, tid);
  potf2_invert(S, tid);
  potf2_store<T>(S, d, j, Ad, tid);
}

// XCD-aware workgroup order.  The hardware hands the workgroup with linear id
// L to XCD L % 8, and each XCD has its own L2; remapped, XCD k walks the
// contiguous range [k N/8, (k+1) N/8) of (theta, tile) pairs, so workgroups
// that run side by side on one XCD work on neighbouring tiles of one theta and
// share panel blocks in its L2.  The grid size N must be a multiple of 8.
__device__ __forceinline__ void xcd_order(int &bx, int &by) {
  const int N = gridDim.x * gridDim.y;
  const int L = blockIdx.y * gridDim.x + blockIdx.x;
  const int G = (L & 7) * (N >> 3) + (L >> 3);
  by = G / gridDim.x;
  bx = G - by * gridDim.x;
}

// Tile t of a lower trapezoid of nr tile rows and nc <= nr tile columns (tile
// (I, J) present when J <= I), in groups of GR tile rows, column by column
// within a group: consecutive tiles share their column block, and a group's GR
// row blocks stay in L2 while its columns go by.  Returns false past the end.
__device__ __forceinline__ bool trap_grouped(int t, int nr, int nc, int &I, int &J) {
  constexpr int GR = 8;
  auto before = [&](int r) {   // tiles in rows [0, r)
    const int m = min(r, nc);
    return m * (m + 1) / 2 + max(0, r - nc) * nc;
  };
  if (t >= before(nr)) return false;
  int lo = 0, hi = (nr + GR - 1) / GR - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (before(mid * GR) <= t) lo = mid;
    else hi = mid - 1;
  }
  const int r0 = lo * GR, gh = min(GR, nr - r0);
  int u = t - before(r0);
  const int full = min(r0, nc);   // columns left of the group's diagonal: gh tiles each
  if (u < full * gh) {
    J = u / gh;
    I = r0 + u % gh;
    return true;
  }
  u -= full * gh;
  J = r0;                         // column J >= r0 holds rows J .. r0 + gh - 1
  while (u >= r0 + gh - J) {
    u -= r0 + gh - J;
    ++J;
  }
  I = J + u;
  return true;
}

// Tile bx of one trailing-update launch: rows/columns of the C tile and the K
// range [ks, ke) = [p0, pend), the lower-triangular tiles of the updated block
// in the grouped order of trap_grouped.  Returns false when the workgroup has
// no tile, its tile reads identity border rows (or columns) that are still
// zero over [ks, ke), or the row selection excludes it (sel: 0 every tile,
// 1 tiles of the factored rows (row < nf), 2 tiles of the border rows
// (row >= nf)).
__device__ __forceinline__ bool update_tile(const FactorDesc &d, int kind, int p0, int nb, int TM, int TN, int sel,
                                            int bx, int &row0, int &col0, int &ks, int &ke) {
  if (p0 >= d.nf) return false;
  const int pend = min(p0 + nb, d.nf);
  int r0, c0, cend;
  ks = p0; ke = pend;
  if (kind == KIND_TRAIL) {
    r0 = pend; c0 = pend; cend = d.ncols;
  } else if (kind == KIND_TRAIL_A) {
    r0 = pend; c0 = pend; cend = min(pend + nb, d.nf);
  } else {
    c0 = min(pend + nb, d.nf); r0 = c0; cend = d.ncols;
  }
  if (r0 >= d.nrows || c0 >= cend) return false;
  const int nr = (d.nrows - r0) / TM;
  int I, J;
  if (!trap_grouped(bx, nr, (cend - c0) / TN, I, J)) return false;
  row0 = r0 + I * TM;
  col0 = c0 + J * TN;
  if ((sel == 1 && row0 >= d.nf) || (sel == 2 && row0 < d.nf)) return false;
  if (row0 >= d.id_row0 && row0 - d.id_row0 >= ke) return false;
  if (col0 >= d.id_row0 && col0 - d.id_row0 >= ke) return false;
  return true;
}

// C -= acc for one wave's BM x BN accumulator blocks (tile coordinates from rl,
// cl).  A tile that straddles the diagonal touches only its lower triangle.
template <typename T, int BM, int BN, typename Acc, typename RL, typename CL>
__device__ __forceinline__ void subtract_tile(__attribute__((address_space(1))) T *Cg, int ld, Acc (&acc)[BM][BN],
                                              RL rl, CL cl, bool diag_tile, int row0, int col0) {
  if (!diag_tile) {
#pragma unroll
    for (int a = 0; a < BM; ++a) {
      T cv[BN][4];
#pragma unroll
      for (int b = 0; b < BN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) cv[b][v] = Cg[(size_t)cl(b, v) * ld + rl(a, v)];
#pragma unroll
      for (int b = 0; b < BN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) Cg[(size_t)cl(b, v) * ld + rl(a, v)] = cv[b][v] - acc[a][b][v];
    }
  } else {
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (row0 + rl(a, v) >= col0 + cl(b, v)) {
            __attribute__((address_space(1))) T *p = Cg + (size_t)cl(b, v) * ld + rl(a, v);
            *p = *p - acc[a][b][v];
          }
        }
  }
}

// --------------------------------------------------------------------------
// MFMA tile update.  C(TM x TN) = or -= A(TM x K) B(TN x K)^T, A and B read from
// column-major storage (element (r, k) at base[k*ld + r]).
//
// FP64: v_mfma_f64_16x16x4f64 puts D row (l/16 + 4v), column (l%16) in lane l;
// the operands are swapped (x from B, y from A) so that a lane's four results
// are C row (l%16) of columns (l/16 + 4v) and every store covers four whole
// 128-byte column segments.
// FP32: v_mfma_f32_16x16x4f32 puts D rows (4(l/16) + v), column (l%16) in lane
// l; operands are not swapped, so a lane's four results are four consecutive
// rows of one column.
// Lane group g = l/16 supplies k = 4g + s at MFMA step s of each 16-deep
// sub-chunk.  LDS rows are padded by 4 elements so that each read is free of
// bank conflicts.
// --------------------------------------------------------------------------
// SEL (row selection of update_tile) is a template parameter so that the
// border-row launch beside a BF16 trailing update is a kernel of its own; the
// trailing update of every row is trail_update_kernel (below), so that each
// launch class has its own kernel symbol.
template <typename T, int TM, int TN, int SEL, int NBUF>
__device__ __forceinline__ void gemm_update_body(const FactorDesc *__restrict__ descs, int kind, int p0, int nb) {
  constexpr bool F64 = sizeof(T) == 8;
  // K chunk staged per LDS buffer: 16 deep in both precisions, which keeps a
  // 128 x 128 FP32 tile's buffers at 34 KB (up to four workgroups per CU)
  constexpr int KCH = 16;
  constexpr int VEC = 16 / sizeof(T);           // elements per 16-byte global load
  constexpr int WM = 2, WN = 2;                 // 2 x 2 waves
  constexpr int WTM = TM / WM, WTN = TN / WN;   // wave tile
  constexpr int BM = WTM / 16, BN = WTN / 16;   // MFMA blocks per wave
  constexpr int PAD = 4;
  constexpr int LA = KCH * TM / VEC / 256, LB = KCH * TN / VEC / 256;
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  typedef __attribute__((address_space(1))) T gT;
  typedef __attribute__((address_space(1))) const T gcT;
  typedef __attribute__((address_space(1))) const vec_t gcvec;
  typedef typename std::conditional<F64, d4, f4>::type acc_t;
  static_assert(NBUF == 1 || NBUF == 2, "one or two LDS buffers");
  __shared__ __attribute__((aligned(16))) T As[NBUF][KCH][TM + PAD];
  __shared__ __attribute__((aligned(16))) T Bs[NBUF][KCH][TN + PAD];

  int bx, by;
  xcd_order(bx, by);
  const FactorDesc d = descs[by];
  int row0, col0, ks, ke;
  if (!update_tile(d, kind, p0, nb, TM, TN, SEL, bx, row0, col0, ks, ke)) return;

  const int ld = d.ld, ldb = ld;
  gcT *Ag = gptr((const T *)d.A) + (size_t)ks * ld + row0;
  gcT *Bg = gptr((const T *)d.A) + (size_t)ks * ld + col0;
  gT *Cg = gptr((T *)d.A) + (size_t)col0 * ld + row0;
  const int K = ke - ks;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WN, wn = w % WN;
  const int g = lane >> 4, li = lane & 15;

  acc_t acc[BM][BN];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  vec_t ra[LA], rb[LB];
  auto gload = [&](int kc) {
#pragma unroll
    for (int it = 0; it < LA; ++it) {
      const int lin = it * 256 + tid, kk = lin / (TM / VEC), rp = lin % (TM / VEC);
      ra[it] = *reinterpret_cast<gcvec *>(Ag + (size_t)(kc + kk) * ld + VEC * rp);
    }
#pragma unroll
    for (int it = 0; it < LB; ++it) {
      const int lin = it * 256 + tid, kk = lin / (TN / VEC), rp = lin % (TN / VEC);
      rb[it] = *reinterpret_cast<gcvec *>(Bg + (size_t)(kc + kk) * ldb + VEC * rp);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int it = 0; it < LA; ++it) {
      const int lin = it * 256 + tid, kk = lin / (TM / VEC), rp = lin % (TM / VEC);
      *reinterpret_cast<vec_t *>(&As[buf][kk][VEC * rp]) = ra[it];
    }
#pragma unroll
    for (int it = 0; it < LB; ++it) {
      const int lin = it * 256 + tid, kk = lin / (TN / VEC), rp = lin % (TN / VEC);
      *reinterpret_cast<vec_t *>(&Bs[buf][kk][VEC * rp]) = rb[it];
    }
  };

  gload(0);
  lstore(0);
  __syncthreads();
  int buf = 0;
  for (int kc = 0; kc < K; kc += KCH) {
    const bool more = kc + KCH < K;
    if (more) gload(kc + KCH);
    // FP32 128 x 128 tiles: the compiler's interleaving of LDS reads with the
    // MFMA steps (scheduling only; 2% faster at four workgroups per CU, where
    // the FP64 tiles lose occupancy to it)
    if constexpr (!F64 && TM == 128) __builtin_amdgcn_iglp_opt(0);
#pragma unroll
    for (int s = 0; s < KCH / 4; ++s) {
      const int kk = 16 * (s >> 2) + 4 * g + (s & 3);
      T ya[BM], xb[BN];
#pragma unroll
      for (int a = 0; a < BM; ++a) ya[a] = As[buf][kk][wm * WTM + a * 16 + li];
#pragma unroll
      for (int b = 0; b < BN; ++b) xb[b] = Bs[buf][kk][wn * WTN + b * 16 + li];
#pragma unroll
      for (int a = 0; a < BM; ++a)
#pragma unroll
        for (int b = 0; b < BN; ++b) {
          if constexpr (F64) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], acc[a][b], 0, 0, 0);
          else acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[a], xb[b], acc[a][b], 0, 0, 0);
        }
    }
    if constexpr (NBUF == 2) {
      if (more) lstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    } else {
      __syncthreads();   // every wave is done reading the buffer
      if (more) {
        lstore(0);
        __syncthreads();
      }
    }
  }

  // Epilogue: tile element (rl(a, v), cl(b, v)) for accumulator component v.
  auto rl = [&](int a, int v) { return wm * WTM + a * 16 + (F64 ? li : 4 * g + v); };
  auto cl = [&](int b, int v) { return wn * WTN + b * 16 + (F64 ? g + 4 * v : li); };
  subtract_tile<T, BM, BN>(Cg, ld, acc, rl, cl, row0 < col0 + TN, row0, col0);
}

// The border rows' trailing update beside a BF16 trailing update (SEL 2).
template <typename T, int TM, int TN, int SEL>
__global__ __launch_bounds__(256, 2) void gemm_update_kernel(const FactorDesc *__restrict__ descs, int kind,
                                                             int p0, int nb) {
  gemm_update_body<T, TM, TN, SEL, 2>(descs, kind, p0, nb);
}

// The trailing update of the blocked Cholesky (kinds TRAIL, TRAIL_A, TRAIL_B).
// The FP64 64 x 64 tile stages its operands through one LDS buffer (17 KB, six
// workgroups per CU, 7% faster than two buffers at four); the others through
// two.
template <typename T, int TM, int TN>
__global__ __launch_bounds__(256, 2) void trail_update_kernel(const FactorDesc *__restrict__ descs, int kind, int p0,
                                                              int nb) {
  gemm_update_body<T, TM, TN, 0, (sizeof(T) == 8 && TM == 64) ? 1 : 2>(descs, kind, p0, nb);
}

// The same update for a factorisation on the handle's aux stream (the
// concurrent prior pass), always with two LDS buffers: the FP64 64 x 64 tile
// then holds four workgroups per CU rather than six, which leaves every CU
// room for the caller's stream's panel steps and solves beside it.
template <typename T, int TM, int TN>
__global__ __launch_bounds__(256, 2) void trail_update_aux_kernel(const FactorDesc *__restrict__ descs, int kind,
                                                                  int p0, int nb) {
  gemm_update_body<T, TM, TN, 0, 2>(descs, kind, p0, nb);
}

// --------------------------------------------------------------------------
// One step of the left-looking panel: block column j of the panel [p0, pend),
// one 64-row tile I (rows r0 = j + 64 (t + 1) .. r0 + 63) per workgroup:
//   C      = A[I, j] - A[I, p0:j] A[j, p0:j]^T     (the panel's earlier columns,
//                                                  MFMA from global via LDS)
//   L[I,j] = C L_jj^{-T}                           (MFMA, C from registers and
//                                                  L_jj^{-1} staged in 16-deep chunks)
//   A[I,I] -= L[I,j] L[I,j]^T                      (tiles with r0 < pend: the
//                                                  diagonal block's update)
// The tile just below the diagonal block (t = 0) then holds the next diagonal
// block fully updated and factors and inverts it (potf2_factor, potf2_invert)
// in the same launch, so a panel takes one potf2_inv launch and one launch per
// block column.  Each tile reads its own rows of the panel's earlier columns
// and writes one 64 x 64 block, in place of the right-looking rank-64 updates
// that read and wrote the panel's whole trailing part once per block column.
// Every phase fits in about 34 KB of LDS, so four workgroups can share a CU.
//
// Identity border rows (rows id_row0 + s hold e_s) are zero left of column s,
// so a tile of them starts its K range at r0 - id_row0 and is skipped when
// that is past the block column.
//
// Grid: act + 8 Q workgroups.  The first act (one per theta) take tile 0, so
// the diagonal factorisations start first; the rest take tiles 1 .. gx - 1 of
// every theta in the XCD-aware order of xcd_order (Q = ceil(act (gx - 1) / 8)).
// --------------------------------------------------------------------------
template <typename T>
struct PanelLds {
  static constexpr int LDC = NBI + 4;          // LDS row length (elements): conflict-free MFMA operand reads
  static constexpr int PKC = sizeof(T) == 4 ? 32 : 16;   // K chunk of the left-looking product
  union {
    struct { T As[2][PKC][LDC]; T Bs[2][PKC][LDC]; } g;   // K chunks ([k][row]); chunk 0 also stages
                                                           // the TRSM and SYRK operands
    Potf2Lds f;                                            // the next diagonal block's factorisation
  };
};

// Four workgroups per CU in FP32; three in FP64, whose registers would
// otherwise spill at the 128-register budget of four.
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 3) void panel_step_kernel(const FactorDesc *__restrict__ descs, int p0, int nb,
                                                            int j, int act, int gx, int Q) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int VEC = 16 / sizeof(T);
  constexpr int LDC = PanelLds<T>::LDC, PKC = PanelLds<T>::PKC;
  constexpr int WTM = 32, WTN = 32, BM = 2, BN = 2;   // 2 x 2 waves, 32 x 32 wave tiles
  constexpr int LA = PKC * NBI / VEC / 256;           // 16-byte loads per thread per operand chunk
  constexpr int LX = KC * NBI / VEC / 256;            // ... per 16-deep chunk of L_jj^{-1}
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  typedef __attribute__((address_space(1))) T gT;
  typedef __attribute__((address_space(1))) const vec_t gcvec;
  typedef typename std::conditional<F64, d4, f4>::type acc_t;
  __shared__ __attribute__((aligned(16))) PanelLds<T> S;

  int th, t;
  {
    const int L = blockIdx.x;
    if (L < act) {
      th = L; t = 0;
    } else {
      const int L2 = L - act, G = (L2 & 7) * Q + (L2 >> 3);
      if (gx <= 1 || G >= act * (gx - 1)) return;
      th = G / (gx - 1);
      t = 1 + G % (gx - 1);
    }
  }
  const FactorDesc d = descs[th];
  if (j >= d.nf) return;
  const int r0 = j + NBI * (t + 1);
  if (r0 >= d.nrows) return;
  const int pend = min(p0 + nb, d.nf);
  int ks = p0;
  if (r0 >= d.id_row0) {
    if (r0 - d.id_row0 >= j + NBI) return;   // zero in block column j: nothing to do
    ks = max(ks, r0 - d.id_row0);
  }
  const int ld = d.ld, K = j - ks;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int g = lane >> 4, li = lane & 15;
  // tile element (rl(a, v), cl(b, v)) of accumulator component v
  auto rl = [&](int a, int v) { return wm * WTM + a * 16 + (F64 ? li : 4 * g + v); };
  auto cl = [&](int b, int v) { return wn * WTN + b * 16 + (F64 ? g + 4 * v : li); };
  auto zero = [&](acc_t (&c)[BM][BN]) {
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b) c[a][b] = acc_t{0, 0, 0, 0};
  };
  // c += X(64 x 16) Y(64 x 16)^T for one 16-deep chunk held [k][row] in LDS
  auto mfma_chunk = [&](acc_t (&c)[BM][BN], const T (*X)[LDC], const T (*Y)[LDC], int k0) {
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kk = k0 + 4 * g + s;
      T ya[BM], xb[BN];
#pragma unroll
      for (int a = 0; a < BM; ++a) ya[a] = X[kk][wm * WTM + a * 16 + li];
#pragma unroll
      for (int b = 0; b < BN; ++b) xb[b] = Y[kk][wn * WTN + b * 16 + li];
#pragma unroll
      for (int a = 0; a < BM; ++a)
#pragma unroll
        for (int b = 0; b < BN; ++b) {
          if constexpr (F64) c[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], c[a][b], 0, 0, 0);
          else c[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[a], xb[b], c[a][b], 0, 0, 0);
        }
    }
  };
  // columns [k0, k0 + 16) of the tile held in accumulator layout, into LDS as [k][row]
  auto stage_cols = [&](const acc_t (&c)[BM][BN], T (*dst)[LDC], int k0) {
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = cl(b, v) - k0;
          if (col >= 0 && col < KC) dst[col][rl(a, v)] = c[a][b][v];
        }
  };

  // 1. acc = A[I, ks:j] A[j, ks:j]^T, double-buffered PKC-deep chunks
  acc_t acc[BM][BN];
  zero(acc);
  if (K > 0) {
    const __attribute__((address_space(1))) T *Ag = gptr((const T *)d.A) + (size_t)ks * ld + r0;
    const __attribute__((address_space(1))) T *Bg = gptr((const T *)d.A) + (size_t)ks * ld + j;
    vec_t ra[LA], rb[LA];
    auto gload = [&](int kc) {
#pragma unroll
      for (int it = 0; it < LA; ++it) {
        const int lin = it * 256 + tid, kk = lin / (NBI / VEC), rp = lin % (NBI / VEC);
        ra[it] = *reinterpret_cast<gcvec *>(Ag + (size_t)(kc + kk) * ld + VEC * rp);
        rb[it] = *reinterpret_cast<gcvec *>(Bg + (size_t)(kc + kk) * ld + VEC * rp);
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int it = 0; it < LA; ++it) {
        const int lin = it * 256 + tid, kk = lin / (NBI / VEC), rp = lin % (NBI / VEC);
        *reinterpret_cast<vec_t *>(&S.g.As[buf][kk][VEC * rp]) = ra[it];
        *reinterpret_cast<vec_t *>(&S.g.Bs[buf][kk][VEC * rp]) = rb[it];
      }
    };
    gload(0);
    lstore(0);
    __syncthreads();
    int buf = 0;
    for (int kc = 0; kc < K; kc += PKC) {   // K is a multiple of 64
      const bool more = kc + PKC < K;
      if (more) gload(kc + PKC);
#pragma unroll
      for (int k0 = 0; k0 < PKC; k0 += KC) mfma_chunk(acc, S.g.As[buf], S.g.Bs[buf], k0);
      if (more) lstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // 2. C = A[I, j] - acc (in acc), then L[I, j] = C L_jj^{-T} into lacc over
  //    16-deep chunks of k (columns of block j): C's columns and rows of
  //    L_jj^{-1} (column-major: X[n][k] at k * 64 + n) staged in LDS chunk 0
  gT *Cg = gptr((T *)d.A) + (size_t)j * ld + r0;
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = Cg[cl(b, v) * ld + rl(a, v)] - acc[a][b][v];
  const __attribute__((address_space(1))) T *Li = gptr((const T *)d.linv) + (size_t)(j / NBI) * NBI * NBI;
  acc_t lacc[BM][BN];
  zero(lacc);
#pragma unroll
  for (int k0 = 0; k0 < NBI; k0 += KC) {
    vec_t xv[LX];
#pragma unroll
    for (int it = 0; it < LX; ++it)
      xv[it] = *reinterpret_cast<gcvec *>(Li + (size_t)k0 * NBI + (size_t)VEC * (it * 256 + tid));
    stage_cols(acc, S.g.As[0], k0);
#pragma unroll
    for (int it = 0; it < LX; ++it) {
      const int lin = it * 256 + tid, kk = lin / (NBI / VEC), rp = lin % (NBI / VEC);
      *reinterpret_cast<vec_t *>(&S.g.Bs[0][kk][VEC * rp]) = xv[it];
    }
    __syncthreads();
    mfma_chunk(lacc, S.g.As[0], S.g.Bs[0], 0);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) Cg[cl(b, v) * ld + rl(a, v)] = lacc[a][b][v];
  if (r0 >= pend) return;

  // 3. diagonal block of the tile's rows: D = L[I, j] L[I, j]^T (into acc)
  zero(acc);
#pragma unroll
  for (int k0 = 0; k0 < NBI; k0 += KC) {
    stage_cols(lacc, S.g.As[0], k0);
    __syncthreads();
    mfma_chunk(acc, S.g.As[0], S.g.As[0], 0);
    __syncthreads();
  }
  gT *Dg = gptr((T *)d.A) + (size_t)r0 * ld + r0;
  if (t != 0) {
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = rl(a, v), c = cl(b, v);
          if (r >= c) Dg[c * ld + r] = Dg[c * ld + r] - acc[a][b][v];
        }
    return;
  }

  // 4. tile 0: the block at r0 = j + 64 has had every update of the panel's
  //    earlier columns; factor and invert it in LDS, store L and its inverse
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rl(a, v), c = cl(b, v);
        S.f.M[r][c] = (r >= c) ? (double)(T)(Dg[c * ld + r] - acc[a][b][v]) : 0.0;
      }
  if (tid == 0) S.f.fail = 0;
  __syncthreads();
  potf2_factor(S.f, tid);
  potf2_invert(S.f, tid);
  potf2_store<T>(S.f, d, r0, Dg, tid);
}

// --------------------------------------------------------------------------
// Trailing update with BF16 operands (factored rows only): FP32 storage, the
// panel rounded once to BF16 (round to nearest even) into a packed copy,
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation, FP32 read-modify-write of
// C.  That instruction takes in lane l the row (l%16) of A and the column
// (l%16) of B^T at the eight k values 8(l/16) .. 8(l/16)+7, and returns D rows
// 4(l/16)+v of column (l%16) (the FP32 layout, so the epilogue is shared).
//
// The packed copy holds, per group of eight k values, one 16-byte entry per
// row, which is exactly an MFMA operand: a K chunk of 32 is 4 groups x 128
// rows of entries, loaded with 16-byte loads (a wave covers 1 KB contiguous)
// and stored unchanged into LDS.  LDS holds entry [g][row] at slot
// row ^ ((row >> 4) & 3), so that the sixteen rows a quarter-wave reads fall
// into distinct 16-byte slots of a 256-byte bank window.
// --------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(1))) const bf8 gcbf8;

__device__ __forceinline__ int bf_slot(int r) { return r ^ ((r >> 4) & 3); }

// Packed BF16 copy of the panel [p0, pend) for rows [pend, nf): one thread per
// (row, group of eight k), slot (p0 / nb) & 1.
__global__ __launch_bounds__(256) void panel_bf16_kernel(const FactorDesc *__restrict__ descs, int p0, int nb) {
  const FactorDesc d = descs[blockIdx.z];
  const int pend = min(p0 + nb, d.nf);
  const int r = pend + blockIdx.x * 256 + threadIdx.x, gk = blockIdx.y;
  if (r >= d.nf || p0 + 8 * gk >= pend) return;
  const __attribute__((address_space(1))) float *src = gptr((const float *)d.A) + (size_t)(p0 + 8 * gk) * d.ld + r;
  bf8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = (__bf16)src[(size_t)i * d.ld];
  bf8 *dst = (bf8 *)d.pbf + (size_t)((p0 / nb) & 1) * d.pbf_slot + (size_t)gk * d.nf + r;
  *gptr(dst) = v;
}

template <int TM, int TN>
__global__ __launch_bounds__(256, 2) void trail_bf16_kernel(const FactorDesc *__restrict__ descs, int kind, int p0,
                                                            int nb) {
  constexpr int KCH = 32, KG = KCH / 8;
  constexpr int WM = 2, WN = 2, WTM = TM / WM, WTN = TN / WN, BM = WTM / 16, BN = WTN / 16;
  constexpr int EA = KG * TM / 256, EB = KG * TN / 256;   // entries per thread per chunk
  typedef __attribute__((address_space(1))) float gT;
  __shared__ bf8 As[2][KG][TM];
  __shared__ bf8 Bs[2][KG][TN];

  int bx, by;
  xcd_order(bx, by);
  const FactorDesc d = descs[by];
  int row0, col0, ks, ke;
  if (!update_tile(d, kind, p0, nb, TM, TN, 1, bx, row0, col0, ks, ke)) return;
  const int ld = d.ld;
  // the packed panel: entry (group g, row r) at P[g * nf + r]; k = ks + 8 g
  gcbf8 *P = gptr((const bf8 *)d.pbf + (size_t)((p0 / nb) & 1) * d.pbf_slot);
  gT *Cg = gptr((float *)d.A) + (size_t)col0 * ld + row0;
  const int K = ke - ks, nf = d.nf;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WN, wn = w % WN;
  const int g = lane >> 4, li = lane & 15;

  f4 acc[BM][BN];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b) acc[a][b] = f4{0, 0, 0, 0};

  bf8 ra[EA], rb[EB];
  auto gload = [&](int kc) {
    const int g0 = kc / 8;
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int e = i * 256 + tid, eg = e / TM, er = e % TM;
      ra[i] = P[(size_t)(g0 + eg) * nf + row0 + er];
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int e = i * 256 + tid, eg = e / TN, er = e % TN;
      rb[i] = P[(size_t)(g0 + eg) * nf + col0 + er];
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int e = i * 256 + tid;
      As[buf][e / TM][bf_slot(e % TM)] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int e = i * 256 + tid;
      Bs[buf][e / TN][bf_slot(e % TN)] = rb[i];
    }
  };

  gload(0);
  lstore(0);
  __syncthreads();
  int buf = 0;
  for (int kc = 0; kc < K; kc += KCH) {
    const bool more = kc + KCH < K;
    if (more) gload(kc + KCH);
#pragma unroll
    for (int s = 0; s < KCH / 32; ++s) {
      bf8 ya[BM], xb[BN];
#pragma unroll
      for (int a = 0; a < BM; ++a) ya[a] = As[buf][4 * s + g][bf_slot(wm * WTM + a * 16 + li)];
#pragma unroll
      for (int b = 0; b < BN; ++b) xb[b] = Bs[buf][4 * s + g][bf_slot(wn * WTN + b * 16 + li)];
#pragma unroll
      for (int a = 0; a < BM; ++a)
#pragma unroll
        for (int b = 0; b < BN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[a], xb[b], acc[a][b], 0, 0, 0);
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  auto rl = [&](int a, int v) { return wm * WTM + a * 16 + 4 * g + v; };
  auto cl = [&](int b, int v) { (void)v; return wn * WTN + b * 16 + li; };
  subtract_tile<float, BM, BN>(Cg, ld, acc, rl, cl, row0 < col0 + TN, row0, col0);
}

// --------------------------------------------------------------------------
// Host driver
// --------------------------------------------------------------------------
static int count_rows_real(const HostFactor &h, int a) {
  // real rows in [a, nrows): [a, n_real) U [max(a, nf), nf + kb_real)
  int c = 0;
  if (a < h.n_real) c += h.n_real - a;
  const int b0 = a > h.d.nf ? a : h.d.nf;
  if (b0 < h.d.nf + h.kb_real) c += h.d.nf + h.kb_real - b0;
  return c;
}
static int count_cols_real(const HostFactor &h, int a, int cend) {
  int c = 0;
  const int e1 = cend < h.n_real ? cend : h.n_real;
  if (a < e1) c += e1 - a;
  const int b0 = a > h.d.nf ? a : h.d.nf;
  const int e2 = cend < h.d.nf + h.ks_real ? cend : h.d.nf + h.ks_real;
  if (b0 < e2) c += e2 - b0;
  return c;
}
static double trap_elems(double nr, double nc) { return nc * (nc + 1.0) * 0.5 + (nr - nc) * nc; }
// Real (unpadded) lower-triangle elements of columns [c0, c1), rows at or below
// each column; with only_factored, rows of the factored block only.
static double lower_real(const HostFactor &h, int c0, int c1, bool only_factored) {
  double s = 0.0;
  const int fa = c0, fb = std::min(c1, h.n_real);
  if (fa < fb) {
    const double m = fb - fa;
    s += m * h.n_real - (double)(fa + fb - 1) * m * 0.5;
    if (!only_factored) s += m * h.kb_real;
  }
  if (!only_factored) {
    const int sa = std::max(c0, h.d.nf), sb = std::min(c1, h.d.nf + h.ks_real);
    if (sa < sb) {
      const double m = sb - sa;
      s += m * (h.d.nf + h.kb_real) - (double)(sa + sb - 1) * m * 0.5;
    }
  }
  return s;
}

static int tiles_for(const FactorDesc &d, int kind, int p0, int nb, int TM) {
  if (p0 >= d.nf) return 0;
  const int pend = std::min(p0 + nb, d.nf);
  int r0, c0, cend;
  if (kind == KIND_TRAIL) { r0 = pend; c0 = pend; cend = d.ncols; }
  else if (kind == KIND_TRAIL_A) { r0 = pend; c0 = pend; cend = std::min(pend + nb, d.nf); }
  else { c0 = std::min(pend + nb, d.nf); r0 = c0; cend = d.ncols; }
  if (r0 >= d.nrows || c0 >= cend) return 0;
  const int nr = (d.nrows - r0) / TM;
  const int nc = (cend - c0) / TM;
  return nc * (nc + 1) / 2 + (nr - nc) * nc;
}

// Synthetic symmetric positive definite batch for the autotuner: unit-free
// values, diagonally dominant on the factored columns, small border rows.
template <typename T>
__global__ __launch_bounds__(256) void tune_fill_kernel(const FactorDesc *__restrict__ descs) {
  const FactorDesc d = descs[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= d.ncols) return;
  __attribute__((address_space(1))) T *col = gptr((T *)d.A) + (size_t)c * d.ld;
  for (int r = c + threadIdx.x; r < d.nrows; r += 256) {
    const uint32_t h = (uint32_t)r * 2654435761u ^ (uint32_t)c * 40503u;
    const double off = ((double)(h >> 8) / 16777216.0 - 0.5) / (double)d.nf;
    col[r] = (T)(r == c ? (c < d.nf ? 2.0 : 1.0) : off);
  }
  if (c == 0 && threadIdx.x == 0) *d.info = 0;
}

template <typename T>
static int factor_batch_t(Ctx &ctx, const std::vector<HostFactor> &fs, int nb, int tm, bool look_cfg,
                          bool bf16_trail) {
  const int B = (int)fs.size();
  if (B == 0) return 0;
  const double esz = sizeof(T);
  // device descriptor array, sorted by nf descending so active sets are prefixes
  std::vector<int> order(B);
  for (int i = 0; i < B; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fs[a].d.nf > fs[b].d.nf; });
  std::vector<FactorDesc> hd(B);
  for (int i = 0; i < B; ++i) hd[i] = fs[order[i]].d;
  const bool split = std::is_same<T, float>::value && bf16_trail;
  if (split) {
    // two slots of the packed BF16 panel copy per theta (16-byte entries)
    size_t entries = 0;
    for (int i = 0; i < B; ++i) entries += 2 * (size_t)(nb / 8) * hd[i].nf;
    char *base = ctx.pbf_reserve(16 * entries);
    if (!base) return INLA_ERR_NOMEM;
    size_t off = 0;
    for (int i = 0; i < B; ++i) {
      hd[i].pbf = base + 16 * off;
      hd[i].pbf_slot = (int64_t)(nb / 8) * hd[i].nf;
      off += 2 * (size_t)hd[i].pbf_slot;
    }
  }
  FactorDesc *dd = (FactorDesc *)ctx.upload(hd.data(), sizeof(FactorDesc) * B);
  if (!dd) return INLA_ERR_NOMEM;
  const int nf_max = hd[0].nf;
  auto active = [&](int col) {
    int a = 0;
    while (a < B && hd[a].nf > col) ++a;
    return a;
  };
  // Every grid and scalar argument of a panel's launch sequence follows from
  // these sizes; the pointers travel in the argument block.
  std::vector<int64_t> key0 = {0x46414354, (int64_t)sizeof(T), bf16_trail, nb, B};
  for (int i = 0; i < B; ++i) {
    const HostFactor &h = fs[order[i]];
    key0.insert(key0.end(), {h.d.nf, h.d.nrows, h.d.ncols, h.d.id_row0, h.n_real, h.kb_real, h.ks_real});
  }
  // the panel [p0, p0 + nb): potf2_inv of its first diagonal block, then one
  // left-looking panel step per 64-wide block column (one graph replay),
  // enqueued on ctx.stream
  auto panel_seq = [&](int p0, const std::vector<int64_t> &key) -> int {
    return ctx.sequence(INLA_K_PANEL, key, hd.data(), sizeof(FactorDesc) * B, [&](const void *dv) {
      const FactorDesc *pd = (const FactorDesc *)dv;
      for (int j = p0; j < p0 + nb && j < nf_max; j += NBI) {
        const int act = active(j);
        if (j == p0) {
          double fl = 0;
          for (int i = 0; i < act; ++i) {
            const double kr = std::max(0, std::min(NBI, fs[order[i]].n_real - j));
            fl += 2.0 * kr * kr * kr / 3.0;
          }
          ctx.launch(INLA_K_POTF2, fl, 0.0, [&] {
            hipLaunchKernelGGL(potf2_inv_kernel<T>, dim3(act), dim3(256), 0, ctx.stream, pd, j);
          });
        }
        // algorithmic work per theta (real rows and columns): the left-looking
        // product over [p0, j), the TRSM, the SYRK of each in-panel diagonal
        // block below and the next diagonal block's factorisation
        int gx = 0;
        double fl = 0, by = 0;
        for (int i = 0; i < act; ++i) {
          const HostFactor &h = fs[order[i]];
          gx = std::max(gx, (h.d.nrows - j - NBI) / NBI);
          const int pend = std::min(p0 + nb, h.d.nf);
          const double kr = std::max(0, std::min(NBI, h.n_real - j));
          const double kl = std::max(0, std::min(j, h.n_real) - p0);
          const double m = count_rows_real(h, j + NBI);
          fl += 2.0 * m * kr * kl + m * kr * kr;
          by += esz * m * (kl + 2.0 * kr);
          for (int r = j + NBI; r < pend; r += NBI) {
            const double kd = std::max(0, std::min(NBI, h.n_real - r));
            fl += kd * (kd + 1.0) * kr;
            by += 2.0 * esz * kd * (kd + 1.0) * 0.5;
            if (r == j + NBI) fl += 2.0 * kd * kd * kd / 3.0;
          }
        }
        if (gx == 0) continue;
        const int Q = (act * (gx - 1) + 7) / 8;
        ctx.launch(INLA_K_PANEL, fl, by, [&] {
          hipLaunchKernelGGL(panel_step_kernel<T>, dim3(act + 8 * Q), dim3(256), 0, ctx.stream, pd, p0, nb, j, act,
                             gx, Q);
        });
      }
    });
  };
  // the packed BF16 copy of panel p0 for the BF16 trailing update, on ctx.stream
  auto panel_copy = [&](int p0) {
    const int act = active(p0);
    int rows = 0;
    double by = 0;
    for (int i = 0; i < act; ++i) {
      const HostFactor &h = fs[order[i]];
      const int pend = std::min(p0 + nb, h.d.nf);
      rows = std::max(rows, h.d.nf - pend);
      by += 6.0 * std::max(0, h.n_real - pend) * (double)std::max(0, std::min(pend, h.n_real) - p0);
    }
    if (rows <= 0) return;
    ctx.launch(INLA_K_PANEL, 0.0, by, [&] {
      hipLaunchKernelGGL(panel_bf16_kernel, dim3((rows + 255) / 256, nb / 8, act), dim3(256), 0, ctx.stream, dd, p0,
                         nb);
    });
  };
  auto panel = [&](int p0) -> int {
    std::vector<int64_t> key = key0;
    key.push_back(p0);
    const int rc = panel_seq(p0, key);
    if (!rc && split) panel_copy(p0);
    return rc;
  };
  // the trailing update of kind TRAIL (everything right of the panel), TRAIL_A
  // (the next panel's columns) or TRAIL_B (the columns after the next panel),
  // enqueued on ctx.stream
  auto trail = [&](int p0, int kind) {
    const int act = active(p0);
    const int TT = split ? 128 : tm;   // the BF16 split path has 128 x 128 tiles only
    int gx = 0;
    double fl = 0, by = 0, fl_q = 0, by_q = 0;   // all tiles; tiles of the factored rows only
    bool rows_q = false;                          // some theta has factored rows in the region
    for (int i = 0; i < act; ++i) {
      const HostFactor &h = fs[order[i]];
      gx = std::max(gx, tiles_for(h.d, kind, p0, nb, TT));
      const int pend = std::min(p0 + nb, h.d.nf), pnext = std::min(pend + nb, h.d.nf);
      int c0 = pend, c1 = h.d.ncols;
      if (kind == KIND_TRAIL_A) c1 = pnext;
      else if (kind == KIND_TRAIL_B) c0 = pnext;
      if (c0 >= c1) continue;
      rows_q = rows_q || c0 < h.d.nf;
      const double kr = std::max(0, std::min(pend, h.n_real) - p0);
      const double el = lower_real(h, c0, c1, false), elq = lower_real(h, c0, c1, true);
      const double nr = count_rows_real(h, c0), nc = count_cols_real(h, c0, c1);
      const double nrq = std::max(0, h.n_real - c0), ncq = std::max(0, std::min(c1, h.n_real) - c0);
      fl += 2.0 * el * kr;
      by += 2.0 * esz * el + esz * (nr + nc) * kr;
      fl_q += 2.0 * elq * kr;
      by_q += elq > 0 ? 2.0 * esz * elq + esz * (nrq + ncq) * kr : 0.0;
    }
    if (gx == 0) return;
    gx = round_up(gx, 8);   // xcd_order needs a grid of a multiple of 8 workgroups
    if (split) {
      // BF16 operands for the factored rows only: the border rows carry the
      // constraint rows and the right-hand side, whose Schur block (C Q^{-1}
      // C^T and C Q^{-1} b) arises by cancellation and keeps FP32 operands
      if (rows_q)
        ctx.launch(INLA_K_TRAIL, fl_q, by_q, [&] {
          hipLaunchKernelGGL((trail_bf16_kernel<128, 128>), dim3(gx, act), dim3(256), 0, ctx.stream, dd, kind, p0,
                             nb);
        });
      ctx.launch(INLA_K_BORDER, fl - fl_q, by - by_q, [&] {
        hipLaunchKernelGGL((gemm_update_kernel<T, 128, 128, 2>), dim3(gx, act), dim3(256), 0, ctx.stream, dd, kind,
                           p0, nb);
      });
    } else {
      const bool aux = ctx.lane == 1;
      ctx.launch(INLA_K_TRAIL, fl, by, [&] {
        if (TT == 64 && aux)
          hipLaunchKernelGGL((trail_update_aux_kernel<T, 64, 64>), dim3(gx, act), dim3(256), 0, ctx.stream, dd, kind,
                             p0, nb);
        else if (TT == 64)
          hipLaunchKernelGGL((trail_update_kernel<T, 64, 64>), dim3(gx, act), dim3(256), 0, ctx.stream, dd, kind, p0,
                             nb);
        else if (aux)
          hipLaunchKernelGGL((trail_update_aux_kernel<T, 128, 128>), dim3(gx, act), dim3(256), 0, ctx.stream, dd,
                             kind, p0, nb);
        else
          hipLaunchKernelGGL((trail_update_kernel<T, 128, 128>), dim3(gx, act), dim3(256), 0, ctx.stream, dd, kind,
                             p0, nb);
      });
    }
  };
  // Lookahead: the next panel's columns are updated first (TRAIL_A, on the
  // caller's stream), the rest (TRAIL_B) on the handle's side stream, and the
  // next panel is factored on the caller's stream while TRAIL_B runs.  TRAIL_A
  // of the following panel waits for TRAIL_B, which updated its columns too.
  // (lookahead runs on the caller's lane only: the side stream and its events
  // serve one factorisation at a time)
  // (and not inside a pass graph, which is captured on one stream)
  const bool look = look_cfg && ctx.lookahead && ctx.lane == 0 && ctx.pg_mode == Ctx::PG_OFF && nf_max > nb &&
                    ctx.side_ready() == INLA_OK;
  int rc = 0;
  hipStream_t main_stream = ctx.stream;
  for (int p0 = 0; p0 < nf_max && !rc; p0 += nb) {
    if (!look) {
      if ((rc = panel(p0))) break;
      trail(p0, KIND_TRAIL);
      continue;
    }
    if (p0 == 0 && (rc = panel(p0))) break;
    if (p0 > 0 && hipStreamWaitEvent(main_stream, ctx.ev_b, 0) != hipSuccess) { rc = INLA_ERR_HIP; break; }
    trail(p0, KIND_TRAIL_A);
    if (hipEventRecord(ctx.ev_a, main_stream) != hipSuccess ||
        hipStreamWaitEvent(ctx.side, ctx.ev_a, 0) != hipSuccess) { rc = INLA_ERR_HIP; break; }
    ctx.stream = ctx.side;
    trail(p0, KIND_TRAIL_B);
    ctx.stream = main_stream;
    if (hipEventRecord(ctx.ev_b, ctx.side) != hipSuccess) { rc = INLA_ERR_HIP; break; }
    if (p0 + nb < nf_max && (rc = panel(p0 + nb))) break;
  }
  ctx.stream = main_stream;
  if (look && hipStreamWaitEvent(main_stream, ctx.ev_b, 0) != hipSuccess && !rc) rc = INLA_ERR_HIP;
  if (rc) return rc;
  return ctx.check();
}

// ------------------------------------------------------------------ tuning
static int b_bucket(int B) {
  int b = 1;
  while (b < B) b <<= 1;
  return b;
}

std::vector<int64_t> tune_key(int prec, int nf_max, int B) { return {prec, nf_max, b_bucket(B)}; }

// Untuned configuration: 512-wide panels; 64 x 64 FP64 trailing tiles (at
// 8192 they measure about 4% faster than 128 x 128), 128 x 128 otherwise.
// BF16 batches of padded order 4096 and above take 1024-wide panels: their
// trailing update then reads and writes the FP32 trailing block once per 1024
// of K rather than per 512 (the BF16 evaluation of 64 theta at n = 8192:
// 864 -> 827 ms, its BF16 trailing update 13% -> 17% of the BF16 peak);
// smaller ones keep 512, which leaves them trailing updates at all.
TuneCfg default_config(int prec, int nf_max) {
  TuneCfg c;
  if (prec == INLA_PREC_FP64) c.tm = 64;
  if (prec == INLA_PREC_BF16 && nf_max >= 4096) c.nb = 1024;
  return c;
}

TuneCfg tuned_config(const Ctx &ctx, int prec, int nf_max, int B) {
  auto it = ctx.tune.find(tune_key(prec, nf_max, B));
  if (it != ctx.tune.end()) return it->second;
  return default_config(prec, nf_max);
}

bool tune_valid(int prec, const TuneCfg &c) {
  const bool nbok = c.nb == 128 || c.nb == 256 || c.nb == 512 || c.nb == 1024;
  const bool tmok = c.tm == 128 || (c.tm == 64 && prec != INLA_PREC_BF16);
  return nbok && tmok && (c.look == 0 || c.look == 1);
}

int factor_batch(Ctx &ctx, const std::vector<HostFactor> &fs, int prec, const TuneCfg *cfg) {
  if (fs.empty()) return 0;
  PrecScope tag(ctx, prec);
  TuneCfg c;
  if (cfg) {
    c = *cfg;
  } else {
    int nf_max = 0;
    for (const HostFactor &h : fs) nf_max = std::max(nf_max, h.d.nf);
    c = tuned_config(ctx, prec, nf_max, (int)fs.size());
  }
  if (prec == INLA_PREC_FP64) return factor_batch_t<double>(ctx, fs, c.nb, c.tm, c.look != 0, false);
  return factor_batch_t<float>(ctx, fs, c.nb, c.tm, c.look != 0, prec == INLA_PREC_BF16);
}

constexpr double LOOKAHEAD_MARGIN = 0.05;
constexpr double DEFAULT_MARGIN = 0.03;

// Candidate (panel width, trailing tile) pairs without lookahead; the BF16 path
// has one tile size.  The fastest is then timed once more with lookahead.
static std::vector<TuneCfg> tune_candidates(int prec) {
  std::vector<TuneCfg> c;
  for (int nb : {128, 256, 512, 1024})
    for (int tm : {64, 128})
      if (prec != INLA_PREC_BF16 || tm == 128) c.push_back({nb, tm, 0});
  return c;
}

int autotune(Ctx &ctx, int B, const int *n, const int *kb, int prec, int reps, TuneCfg *best_out, double *ms_out,
             int *n_cand) {
  const size_t esz = prec == INLA_PREC_FP64 ? 8 : 4;
  std::vector<HostFactor> fs(B);
  std::vector<size_t> offs(B);
  size_t total = 0;
  int nf_max = 0;
  for (int i = 0; i < B; ++i) {
    HostFactor &h = fs[i];
    const int nf = round_up(std::max(n[i], 1), PADN);
    const int kbp = kb[i] > 0 ? round_up(kb[i], PADN) : 0;
    h.d.nf = nf; h.d.nrows = h.d.ncols = h.d.ld = nf + kbp;
    h.d.id_row0 = std::numeric_limits<int>::max();
    h.n_real = n[i]; h.kb_real = kb[i] > 0 ? kb[i] : 0; h.ks_real = h.kb_real;
    nf_max = std::max(nf_max, nf);
    offs[i] = total;
    total += (esz * (size_t)h.d.ld * h.d.ncols + esz * (size_t)nf * NBI + sizeof(int) + 255) & ~size_t(255);
  }
  if (!ctx.reserve(total)) return INLA_ERR_NOMEM;
  for (int i = 0; i < B; ++i) {
    char *base = ctx.ws + offs[i];
    fs[i].d.A = base;
    fs[i].d.linv = base + esz * (size_t)fs[i].d.ld * fs[i].d.ncols;
    fs[i].d.info = (int *)((char *)fs[i].d.linv + esz * (size_t)fs[i].d.nf * NBI);
  }
  std::vector<FactorDesc> hd(B);
  int cmax = 0;
  for (int i = 0; i < B; ++i) { hd[i] = fs[i].d; cmax = std::max(cmax, hd[i].ncols); }
  const FactorDesc *dd = (const FactorDesc *)ctx.upload(hd.data(), sizeof(FactorDesc) * B);
  if (!dd) return INLA_ERR_NOMEM;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return INLA_ERR_HIP;
  const bool prof = ctx.prof;
  ctx.prof = false;
  auto cand = tune_candidates(prec);
  int best = -1, rc = 0;
  double best_ms = 0;
  auto time_cfg = [&](const TuneCfg &cfg) {
    double tot = 0;
    for (int r = 0; r <= reps && !rc; ++r) {   // one untimed run, then `reps` timed ones
      if (prec == INLA_PREC_FP64)
        hipLaunchKernelGGL(tune_fill_kernel<double>, dim3(cmax, B), dim3(256), 0, ctx.stream, dd);
      else
        hipLaunchKernelGGL(tune_fill_kernel<float>, dim3(cmax, B), dim3(256), 0, ctx.stream, dd);
      (void)hipEventRecord(a, ctx.stream);
      rc = factor_batch(ctx, fs, prec, &cfg);
      (void)hipEventRecord(b, ctx.stream);
      if (hipEventSynchronize(b) != hipSuccess) rc = INLA_ERR_HIP;
      float ms = 0;
      if (!rc && r > 0 && hipEventElapsedTime(&ms, a, b) == hipSuccess) tot += ms;
    }
    return tot / std::max(1, reps);
  };
  const size_t nbase = cand.size();
  int dflt = -1;
  double dflt_ms = 0;
  for (size_t c = 0; c < nbase && !rc; ++c) {
    const double avg = time_cfg(cand[c]);
    if (ms_out) ms_out[c] = avg;
    if (!rc && (best < 0 || avg < best_ms)) { best = (int)c; best_ms = avg; }
    if (cand[c].nb == default_config(prec, nf_max).nb && cand[c].tm == default_config(prec, nf_max).tm) { dflt = (int)c; dflt_ms = avg; }
  }
  // the default configuration stays unless another is clearly faster, so that
  // timing noise between near-equal candidates does not change the choice
  if (!rc && dflt >= 0 && best_ms > (1.0 - DEFAULT_MARGIN) * dflt_ms) { best = dflt; best_ms = dflt_ms; }
  if (!rc && ctx.lookahead) {
    TuneCfg la = cand[best];
    la.look = 1;
    cand.push_back(la);
    const double avg = time_cfg(la);
    if (ms_out) ms_out[nbase] = avg;
    // Lookahead must win clearly: the synthetic timing leaves out the rest of
    // an evaluation (assembly, solves, host decisions between passes), in
    // which the overlap has been seen to gain less than it does here.
    if (!rc && avg < (1.0 - LOOKAHEAD_MARGIN) * best_ms) { best = (int)nbase; best_ms = avg; }
  }
  ctx.prof = prof;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  ctx.tune[tune_key(prec, nf_max, B)] = cand[best];
  ++ctx.tune_epoch;
  if (best_out) *best_out = cand[best];
  if (n_cand) *n_cand = (int)cand.size();
  return ctx.check();
}

}  // namespace inla
