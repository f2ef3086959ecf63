// The Moore-Penrose route for intrinsic (rank-deficient) priors, section
// "Bypassing constraints complexity in disease mapping models using dense
// matrices": the pseudo-inverse Q^+ of the prior precision by a cyclic two-sided
// Jacobi eigen-decomposition (one per evaluation where the prior changes), and
// the Laplace evaluation with the posterior covariance in the Woodbury form of
// Eq. (woodeqn), for A = I or a general sparse design matrix.
//
// Jacobi: a block method.  The indices form blocks of 32; the block pairs of a
// round follow the round-robin (circle) schedule, so their rotations are
// disjoint.  Per round, each pair's 64 x 64 principal submatrix is diagonalised
// in LDS by cyclic Jacobi (rotations accumulated from the identity), then every
// pair's columns of A and V are multiplied by its 64 x 64 rotation and its rows
// of A by the transpose (two passes of 64-wide tile products).  A sweep thus
// passes over A and V n/32 times instead of n times.
//
// Woodbury Newton: with W the likelihood curvature (Q_l = diag(W)) and
// S = diag(sqrt(W)), the symmetric form of Eq. (woodeqn) is
//     Sigma* = Q^+ - Q^+ S M^{-1} S Q^+,   M = I + S Q^+ S  (eigenvalues >= 1),
// so each step factors M with the blocked Cholesky instead of solving the
// non-symmetric system I + Q_l Q^+.  The new iterate is
//     x_new = Sigma* b = Q^+ (b - S M^{-1} S Q^+ b),   b = g + W x,
// the forward substitution L^{-1} r (r = S Q^+ b) comes out of the
// factorisation as its border row, and x_new^T Q_prior x_new = z^T x_new with
// z = b - S M^{-1} r, because Q^+ Q_prior Q^+ = Q^+.  The marginal variances
// diag(Sigma*) factor M once more with the n border rows Q^+ S.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "device.hpp"
#include "host.hpp"
#include "model.hpp"

struct inla_handle;

namespace inla {

Ctx *handle_ctx(inla_handle *h);

// ------------------------------------------------------------------ Jacobi
constexpr int JB = 32;               // block width of the block Jacobi method
constexpr int JP = 2 * JB;           // block-pair width (the inner eigenproblem's order)
constexpr int JAC_MAX_N = 16384;
// One inner sweep per block pair and round: the outer rounds carry the
// convergence, and an inexact inner solve keeps each pair's rotation product
// orthogonal, so the method stays exact while each round costs one inner sweep
// instead of the 2-6 a converged inner solve takes.  Measured at n = 3000 and
// on the order-1000 Kronecker block of the Type IV prior: 35 and 45 outer
// sweeps, 1.8 and 3.8 times faster than converged inner solves.
constexpr int JAC_MAX_SWEEPS = 120;
constexpr int JAC_INNER_SWEEPS = 1;
constexpr double JAC_RTOL_DEFAULT = 1e-9;
constexpr int JAC_NORM_BLOCKS = 256;

struct JacDesc {
  const double *Q;   // input, lower triangle read (ld ldq)
  double *A, *V;     // ne x ne working matrix and eigenvectors (ld ne), ne a multiple of JP
  double *R;         // [nbk / 2][JP * JP] the round's pair rotations, column-major
  double *f;         // [ne] 1/lambda_k or 0
  double *part;      // [2 * JAC_NORM_BLOCKS] per-workgroup partial sums of squares
  double *norms;     // [4] off-diagonal sum of squares, sum of squares, max|lambda|, rank
  double *P;         // output Q^+ (ld ldp), full symmetric
  int n, ne, nbk, ldq, ldp;
};

// Round-robin schedule of np (even) players, round r in [0, np - 2]: slot 0
// holds player 0, the other players rotate through slots 1 .. np - 1; slots s
// and np - 1 - s play each other.  Players are blocks of JB indices in the
// outer iteration and single indices in the inner one.
__host__ __device__ __forceinline__ int rr_pos(int slot, int r, int np) {
  return slot == 0 ? 0 : 1 + (slot - 1 + r) % (np - 1);
}

// The rotation J = [c s; -s c] (rows and columns p, q) with (J^T A J)_pq = 0
// (the symmetric Schur decomposition of the 2 x 2 block).
__device__ __forceinline__ void jac_rot(double app, double aqq, double apq, double &c, double &s) {
  if (apq == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double tau = (aqq - app) / (2.0 * apq);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// Global index of local index l (0 .. JP-1) of the pair of blocks (I, K).
__device__ __forceinline__ int pair_idx(int l, int I, int K) { return l < JB ? I * JB + l : K * JB + (l - JB); }

// A = Q (symmetric from its lower triangle, zero padded to ne), V = I.  Grid
// (ne / 256 row blocks, ne columns, B).
__global__ __launch_bounds__(256) void jacobi_init_kernel(const JacDesc *__restrict__ jd) {
  const JacDesc J = jd[blockIdx.z];
  const int c = blockIdx.y, i = blockIdx.x * 256 + threadIdx.x;
  if (c >= J.ne || i >= J.ne) return;
  double a = 0.0;
  if (i < J.n && c < J.n) a = i >= c ? J.Q[(size_t)c * J.ldq + i] : J.Q[(size_t)i * J.ldq + c];
  J.A[(size_t)c * J.ne + i] = a;
  J.V[(size_t)c * J.ne + i] = i == c ? 1.0 : 0.0;
}

// Inner eigenproblem of one block pair: the JP x JP principal submatrix S of A
// on the pair's indices is reduced in LDS by cyclic Jacobi (round-robin over
// its JP indices, rotations accumulated from the identity, so R stays close to
// I, which the outer iteration's convergence needs): JAC_INNER_SWEEPS sweeps,
// none once its off-diagonal part is at the rounding level.  Writes R
// (column-major).  Grid (nbk / 2 pairs, B).
__global__ __launch_bounds__(256) void jacobi_pair_eig_kernel(const JacDesc *__restrict__ jd, int r) {
  const JacDesc J = jd[blockIdx.y];
  const int j = blockIdx.x;
  if (j >= J.nbk / 2) return;
  const int rb = r % (J.nbk - 1);
  const int I = rr_pos(j, rb, J.nbk), K = rr_pos(J.nbk - 1 - j, rb, J.nbk);
  __shared__ double S[JP][JP + 1];    // S[row][col]
  __shared__ double Rt[JP][JP + 1];   // Rt[col][row] = R(row, col)
  __shared__ double cs[JP / 2], sn[JP / 2];
  __shared__ int pp[JP / 2], qq[JP / 2];
  __shared__ double sh[4];
  const int tid = threadIdx.x;
  const auto *A = gptr((const double *)J.A);
  for (int e = tid; e < JP * JP; e += 256) {
    const int l = e % JP, m = e / JP;
    S[l][m] = A[(size_t)pair_idx(m, I, K) * J.ne + pair_idx(l, I, K)];
    Rt[m][l] = l == m ? 1.0 : 0.0;
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  for (int sw = 0; sw < JAC_INNER_SWEEPS; ++sw) {
    double off = 0.0, fro = 0.0;
    for (int e = tid; e < JP * JP; e += 256) {
      const int l = e % JP, m = e / JP;
      const double v = S[l][m];
      fro += v * v;
      if (l != m) off += v * v;
    }
    off = block_sum256(off, sh);
    fro = block_sum256(fro, sh);
    // already diagonal to the rounding level: no rotation
    if (off <= 16.0 * eps * eps * fro) break;
    for (int ri = 0; ri < JP - 1; ++ri) {
      if (tid < JP / 2) {
        const int p = rr_pos(tid, ri, JP), q = rr_pos(JP - 1 - tid, ri, JP);
        double c, s;
        jac_rot(S[p][p], S[q][q], S[q][p], c, s);
        pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
      }
      __syncthreads();
      // Each thread owns row i of the pairs t = tid / JP + 4 u (u < 8): all its
      // loads are issued before any of its stores (the pairs' columns are
      // disjoint, so no thread reads what another writes in the same pass).
      constexpr int NU = (JP / 2) * JP / 256;
      {
        const int i = tid % JP, t0 = tid / JP;
        double a[NU], b[NU], ra[NU], rb2[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {   // columns p, q of S and of R
          const int t = t0 + 4 * u, p = pp[t], q = qq[t];
          a[u] = S[i][p]; b[u] = S[i][q]; ra[u] = Rt[p][i]; rb2[u] = Rt[q][i];
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int t = t0 + 4 * u, p = pp[t], q = qq[t];
          const double c = cs[t], s = sn[t];
          S[i][p] = c * a[u] - s * b[u];
          S[i][q] = s * a[u] + c * b[u];
          Rt[p][i] = c * ra[u] - s * rb2[u];
          Rt[q][i] = s * ra[u] + c * rb2[u];
        }
      }
      __syncthreads();
      {
        const int i = tid % JP, t0 = tid / JP;
        double a[NU], b[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {   // rows p, q of S; the pair's entry is annihilated
          const int t = t0 + 4 * u;
          a[u] = S[pp[t]][i]; b[u] = S[qq[t]][i];
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int t = t0 + 4 * u, p = pp[t], q = qq[t];
          const double c = cs[t], s = sn[t];
          S[p][i] = i == q ? 0.0 : c * a[u] - s * b[u];
          S[q][i] = i == p ? 0.0 : s * a[u] + c * b[u];
        }
      }
      __syncthreads();
    }
  }
  double *Rg = J.R + (size_t)j * JP * JP;
  for (int e = tid; e < JP * JP; e += 256) Rg[e] = Rt[e / JP][e % JP];
}

// Columns of every pair: X[:, pair] <- X[:, pair] R for X = A (z even) and
// X = V (z odd), one 64-row tile per workgroup.  Grid (ne / 64, nbk / 2, 2 B).
__global__ __launch_bounds__(256) void jacobi_pair_cols_kernel(const JacDesc *__restrict__ jd, int r) {
  const JacDesc J = jd[blockIdx.z >> 1];
  double *X = (blockIdx.z & 1) ? J.V : J.A;
  const int j = blockIdx.y, i0 = blockIdx.x * 64;
  if (j >= J.nbk / 2 || i0 >= J.ne) return;
  const int rb = r % (J.nbk - 1);
  const int I = rr_pos(j, rb, J.nbk), K = rr_pos(J.nbk - 1 - j, rb, J.nbk);
  __shared__ double Xt[64][JP + 1];   // Xt[row][l]
  __shared__ double Rs[JP][JP + 1];   // Rs[l][m] = R(l, m)
  const int tid = threadIdx.x;
  const double *Rg = J.R + (size_t)j * JP * JP;
  auto *Xg = gptr(X);
  for (int e = tid; e < 64 * JP; e += 256) {
    const int row = e % 64, l = e / 64;
    Xt[row][l] = Xg[(size_t)pair_idx(l, I, K) * J.ne + i0 + row];
    Rs[e % JP][e / JP] = Rg[e];
  }
  __syncthreads();
  // 64 x 64 x 64 product on FP64 MFMA: wave w owns the 32 x 32 quadrant
  // (rows wr.., columns wc..) as 2 x 2 blocks of 16 x 16.  Operands are
  // swapped as in the factorisation's trailing update, so lane l's four
  // results are output row li of columns g + 4v and each store covers whole
  // 128-byte column segments.
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, g = lane >> 4;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < JP; k0 += 4) {
    const int k = k0 + g;
    double x[2], q[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) x[a] = Xt[wr + 16 * a + li][k];
#pragma unroll
    for (int b = 0; b < 2; ++b) q[b] = Rs[k][wc + 16 * b + li];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(q[b], x[a], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const size_t col = (size_t)pair_idx(wc + 16 * b + g + 4 * v, I, K) * J.ne + i0;
#pragma unroll
      for (int a = 0; a < 2; ++a) Xg[col + wr + 16 * a + li] = acc[a][b][v];
    }
}

// Rows of every pair: A[pair, :] <- R^T A[pair, :], one 64-column tile per
// workgroup.  The pair's own block keeps the computed R^T S R: the inner
// iteration's rounding-level residual stays in A for later rounds (writing
// diag(lambda) there instead discards it, which a CPU model measured as about
// 20 times less accurate).  Grid (ne / 64, nbk / 2, B).
__global__ __launch_bounds__(256) void jacobi_pair_rows_kernel(const JacDesc *__restrict__ jd, int r) {
  const JacDesc J = jd[blockIdx.z];
  const int j = blockIdx.y, c0 = blockIdx.x * 64;
  if (j >= J.nbk / 2 || c0 >= J.ne) return;
  const int rb = r % (J.nbk - 1);
  const int I = rr_pos(j, rb, J.nbk), K = rr_pos(J.nbk - 1 - j, rb, J.nbk);
  __shared__ double At[JP][64 + 1];   // At[l][col]
  __shared__ double Rs[JP][JP + 1];   // Rs[l][m] = R(l, m)
  const int tid = threadIdx.x;
  const double *Rg = J.R + (size_t)j * JP * JP;
  auto *Ag = gptr(J.A);
  for (int e = tid; e < JP * 64; e += 256) {
    const int l = e % JP, col = e / JP;
    At[l][col] = Ag[(size_t)(c0 + col) * J.ne + pair_idx(l, I, K)];
    Rs[e % JP][e / JP] = Rg[e];
  }
  __syncthreads();
  // R^T At on FP64 MFMA, laid out as in the column pass: lane l's four
  // results are pair row wr + 16 a + li of columns g + 4v (16 consecutive pair
  // rows lie in one 32-row block, so each store covers 128-byte segments).
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, g = lane >> 4;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < JP; k0 += 4) {
    const int k = k0 + g;
    double p[2], q[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) p[a] = Rs[k][wr + 16 * a + li];
#pragma unroll
    for (int b = 0; b < 2; ++b) q[b] = At[k][wc + 16 * b + li];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(q[b], p[a], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const size_t col = (size_t)(c0 + wc + 16 * b + g + 4 * v) * J.ne;
#pragma unroll
      for (int a = 0; a < 2; ++a) Ag[col + pair_idx(wr + 16 * a + li, I, K)] = acc[a][b][v];
    }
}

// Sums of squares of the off-diagonal and of all entries: workgroup g sums
// columns g, g + JAC_NORM_BLOCKS, ... (grid (JAC_NORM_BLOCKS, B)); the second
// kernel adds the partials in a fixed order (grid B).
__global__ __launch_bounds__(256) void jacobi_norms_kernel(const JacDesc *__restrict__ jd) {
  const JacDesc J = jd[blockIdx.y];
  __shared__ double sh[4];
  double off = 0.0, fro = 0.0;
  const auto *A = gptr((const double *)J.A);
  for (int c = blockIdx.x; c < J.ne; c += JAC_NORM_BLOCKS) {
    for (int i = threadIdx.x; i < J.ne; i += 256) {
      const double a = A[(size_t)c * J.ne + i];
      fro += a * a;
      if (i != c) off += a * a;
    }
  }
  off = block_sum256(off, sh);
  fro = block_sum256(fro, sh);
  if (threadIdx.x == 0) {
    J.part[2 * blockIdx.x] = off;
    J.part[2 * blockIdx.x + 1] = fro;
  }
}
__global__ __launch_bounds__(256) void jacobi_norms_sum_kernel(const JacDesc *__restrict__ jd) {
  const JacDesc J = jd[blockIdx.x];
  __shared__ double sh[4];
  const double off = block_sum256(J.part[2 * threadIdx.x], sh);
  const double fro = block_sum256(J.part[2 * threadIdx.x + 1], sh);
  if (threadIdx.x == 0) {
    J.norms[0] = off;
    J.norms[1] = fro;
  }
}
static_assert(JAC_NORM_BLOCKS == 256, "jacobi_norms_sum_kernel adds one partial per thread");

// f_k = 1 / lambda_k for |lambda_k| > rtol * max|lambda|, else 0; the rank.
// One workgroup per matrix (grid B).
__global__ __launch_bounds__(256) void pinv_spectrum_kernel(const JacDesc *__restrict__ jd, double rtol) {
  const JacDesc J = jd[blockIdx.x];
  __shared__ double sh[4];
  double mx = 0.0;
  for (int k = threadIdx.x; k < J.ne; k += 256) mx = fmax(mx, fabs(J.A[(size_t)k * J.ne + k]));
  mx = block_max256(mx, sh);
  const double cut = rtol * mx;
  double cnt = 0.0;
  for (int k = threadIdx.x; k < J.ne; k += 256) {
    const double l = J.A[(size_t)k * J.ne + k];
    const bool keep = fabs(l) > cut;
    J.f[k] = keep ? 1.0 / l : 0.0;
    cnt += keep ? 1.0 : 0.0;
  }
  cnt = block_sum256(cnt, sh);
  if (threadIdx.x == 0) {
    J.norms[2] = mx;
    J.norms[3] = cnt;
  }
}

// Q^+ = V diag(f) V^T, one 64 x 64 output tile per workgroup (4 x 4 per
// thread, K staged through LDS in chunks of 16).  Grid (n / 64, n / 64, B).
__global__ __launch_bounds__(256) void pinv_form_kernel(const JacDesc *__restrict__ jd) {
  const JacDesc J = jd[blockIdx.z];
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (i0 >= J.n || j0 >= J.n) return;
  __shared__ double Vi[16][65], Vj[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const auto *V = gptr((const double *)J.V);
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k0 = 0; k0 < J.ne; k0 += 16) {
    for (int e = tid; e < 1024; e += 256) {
      const int r = e & 63, kk = e >> 6, k = k0 + kk;
      double vi = 0.0, vj = 0.0;
      if (k < J.ne) {
        const double fk = J.f[k];
        if (i0 + r < J.ne) vi = V[(size_t)k * J.ne + i0 + r] * fk;
        if (j0 + r < J.ne) vj = V[(size_t)k * J.ne + j0 + r];
      }
      Vi[kk][r] = vi;
      Vj[kk][r] = vj;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = Vi[kk][tx + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Vj[kk][ty + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int jj = j0 + ty + 16 * v;
    if (jj >= J.n) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ii = i0 + tx + 16 * u;
      if (ii < J.n) J.P[(size_t)jj * J.ldp + ii] = acc[u][v];
    }
  }
}

static size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

// Batched pseudo-inverse; see inla_pinv in the header.
static int pinv_batch(Ctx &ctx, int B, const int *n, const double *const *Q, const int *ldq, double *const *P,
                      const int *ldp, double rtol, int *rank, int *sweeps, int *info) {
  if (rtol <= 0) rtol = JAC_RTOL_DEFAULT;
  std::vector<JacDesc> hd(B);
  std::vector<size_t> off(B);
  size_t total = 0;
  int ne_max = 0;
  auto sizes = [&](int ne) {
    const int nbk = ne / JB;
    return 2 * a256(sizeof(double) * (size_t)ne * ne) + a256(sizeof(double) * (size_t)(nbk / 2) * JP * JP) +
           a256(sizeof(double) * ((size_t)ne + 2 * JAC_NORM_BLOCKS)) + a256(sizeof(double) * 4);
  };
  for (int b = 0; b < B; ++b) {
    const int ne = round_up(n[b], JP);
    off[b] = total;
    total += sizes(ne);
    ne_max = std::max(ne_max, ne);
  }
  if (!ctx.reserve(total)) return INLA_ERR_NOMEM;
  for (int b = 0; b < B; ++b) {
    const int ne = round_up(n[b], JP);
    char *base = ctx.ws + off[b];
    JacDesc &J = hd[b];
    J.Q = Q[b]; J.ldq = ldq[b]; J.P = P[b]; J.ldp = ldp[b]; J.n = n[b]; J.ne = ne; J.nbk = ne / JB;
    J.A = (double *)base;
    base += a256(sizeof(double) * (size_t)ne * ne);
    J.V = (double *)base;
    base += a256(sizeof(double) * (size_t)ne * ne);
    J.R = (double *)base;
    base += a256(sizeof(double) * (size_t)(J.nbk / 2) * JP * JP);
    J.f = (double *)base;
    J.part = J.f + ne;
    base += a256(sizeof(double) * ((size_t)ne + 2 * JAC_NORM_BLOCKS));
    J.norms = (double *)base;
  }
  const JacDesc *dall = (const JacDesc *)ctx.upload(hd.data(), sizeof(JacDesc) * B);
  if (!dall) return INLA_ERR_NOMEM;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 16.0 * ne_max * ne_max * B, [&] {
    hipLaunchKernelGGL(jacobi_init_kernel, dim3((ne_max + 255) / 256, ne_max, B), dim3(256), 0, ctx.stream, dall);
  });
  std::vector<int> act(B);
  for (int b = 0; b < B; ++b) { act[b] = b; sweeps[b] = 0; info[b] = INLA_INFO_OK; }
  std::vector<double> prev(B, std::numeric_limits<double>::infinity());
  std::vector<double> hn(4 * (size_t)B);
  // Global round counter: every matrix takes its own rounds in order (r mod
  // (nbk - 1)).  An outer sweep is nbk - 1 rounds of the largest active matrix;
  // a smaller one completes (nbk_max - 1) / (nbk - 1) of its own sweeps in it,
  // and its convergence is checked, and its sweeps counted, at the outer sweep
  // boundaries.
  int r = 0;
  for (int sw = 0; sw < JAC_MAX_SWEEPS && !act.empty(); ++sw) {
    std::vector<JacDesc> ha;
    int ne_act = 0;
    for (int b : act) { ha.push_back(hd[b]); ne_act = std::max(ne_act, hd[b].ne); }
    const JacDesc *da = (const JacDesc *)ctx.upload(ha.data(), sizeof(JacDesc) * ha.size());
    if (!da) return INLA_ERR_NOMEM;
    const int nb = (int)ha.size(), nbk = ne_act / JB, tiles = ne_act / 64;
    // per round: columns of A and V (2 JP flops and 16 bytes per element each),
    // then rows of A
    const double round_flops = 6.0 * JP * (double)ne_act * ne_act * nb;
    const double round_bytes = 48.0 * (double)ne_act * ne_act * nb;
    for (int k = 0; k < nbk - 1; ++k, ++r) {
      const int rr = r;
      ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
        hipLaunchKernelGGL(jacobi_pair_eig_kernel, dim3(nbk / 2, nb), dim3(256), 0, ctx.stream, da, rr);
      });
      ctx.launch(INLA_K_SOLVE, round_flops * 2.0 / 3.0, round_bytes * 2.0 / 3.0, [&] {
        hipLaunchKernelGGL(jacobi_pair_cols_kernel, dim3(tiles, nbk / 2, 2 * nb), dim3(256), 0, ctx.stream, da, rr);
      });
      ctx.launch(INLA_K_SOLVE, round_flops / 3.0, round_bytes / 3.0, [&] {
        hipLaunchKernelGGL(jacobi_pair_rows_kernel, dim3(tiles, nbk / 2, nb), dim3(256), 0, ctx.stream, da, rr);
      });
    }
    ctx.launch(INLA_K_SOLVE, 0.0, 8.0 * ne_act * ne_act * nb, [&] {
      hipLaunchKernelGGL(jacobi_norms_kernel, dim3(JAC_NORM_BLOCKS, nb), dim3(256), 0, ctx.stream, da);
    });
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(jacobi_norms_sum_kernel, dim3(nb), dim3(256), 0, ctx.stream, da);
    });
    for (int q = 0; q < nb; ++q)
      if (hipMemcpyAsync(hn.data() + 4 * q, ha[q].norms, sizeof(double) * 2, hipMemcpyDeviceToHost, ctx.stream) !=
          hipSuccess)
        return INLA_ERR_HIP;
    if (hipStreamSynchronize(ctx.stream) != hipSuccess) return INLA_ERR_HIP;
    std::vector<int> keep;
    for (int q = 0; q < nb; ++q) {
      const int b = act[q];
      sweeps[b] = sw + 1;
      const double off_ = std::sqrt(hn[4 * q]), fro = std::sqrt(hn[4 * q + 1]);
      if (!std::isfinite(off_) || !std::isfinite(fro)) { info[b] = INLA_INFO_NONFINITE; continue; }
      const double eps = std::numeric_limits<double>::epsilon();
      // converged: the off-diagonal part at the rounding level.  Clustered
      // spectra pass through plateaus well above it, so a sweep that no longer
      // shrinks it ends the iteration only once it is already below 1e-14 of
      // the matrix.
      const bool done = off_ <= 4.0 * eps * fro || (off_ <= 1e-14 * fro && off_ >= 0.9 * prev[b]);
      prev[b] = off_;
      if (!done) keep.push_back(b);
    }
    act.swap(keep);
  }
  for (int b : act) info[b] = INLA_INFO_EIG_MAXIT;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(pinv_spectrum_kernel, dim3(B), dim3(256), 0, ctx.stream, dall, rtol);
  });
  int n_max = 0;
  for (int b = 0; b < B; ++b) n_max = std::max(n_max, n[b]);
  const int tiles = (n_max + 63) / 64;
  double fl = 0;
  for (int b = 0; b < B; ++b) fl += 2.0 * n[b] * (double)n[b] * hd[b].ne;
  ctx.launch(INLA_K_ASSEMBLE, fl, 0.0, [&] {
    hipLaunchKernelGGL(pinv_form_kernel, dim3(tiles, tiles, B), dim3(256), 0, ctx.stream, dall);
  });
  for (int b = 0; b < B; ++b)
    if (hipMemcpyAsync(hn.data() + 4 * b, hd[b].norms, sizeof(double) * 4, hipMemcpyDeviceToHost, ctx.stream) !=
        hipSuccess)
      return INLA_ERR_HIP;
  if (hipStreamSynchronize(ctx.stream) != hipSuccess) return INLA_ERR_HIP;
  for (int b = 0; b < B; ++b) rank[b] = (int)std::llround(hn[4 * b + 3]);
  return ctx.check();
}

// ------------------------------------------------------------------ Woodbury Newton
// A general design matrix A (m observations, eta = offset + A x) reduces to the
// A = I iteration in observation space: eta has the prior covariance
// K = A Q^+ A^T, the Newton step of eta is the A = I step with Q^+ replaced by
// K (b = g + W eta, M = I + S K S), and the latent step is x_new = HT z with
// HT = Q^+ A^T and the same z = b - S t, so that x_new^T Q_prior x_new =
// z^T (A x_new) and log|M| = log|I + Q^+ A^T W A|.  HT and K are formed once per
// call from the CSR rows of A.
constexpr int WB_CH = 32;   // column chunks of the matrix-vector products
// The covariance form settles on a rounding floor set by the condition of M
// (weak priors make Q^+ large); below this relative step, a step that is no
// longer at most half the previous one ends the iteration there.
constexpr double WB_FLOOR_TOL = 1e-7;
enum { WR_STEP = 0, WR_SCALE = 1, WR_ZTX = 2, WR_LOGDET = 3, WR_LOGLIK = 4, WR_NONFINITE = 5, WR_COUNT = 8 };
enum { WV_X = 0, WV_B = 1, WV_U = 2, WV_T = 3, WV_W = 4 };

struct WbDesc {
  const double *Pq;    // observation-space covariance: Q^+ (A = I, caller's) or K (workspace); ld ldq
  const double *y, *E;
  double *xext;        // caller's start / mode [n_lat]
  double *vext;        // caller's variances [n_lat] (inla_woodbury_var)
  double *M;           // factor storage: ldm rows (border rows from n_pad), n_pad columns
  double *linv;
  double *x, *b, *sw, *u, *s, *t, *w, *z;   // observation-space vectors [n_pad]; x holds A x
  double *part;        // [WB_CH][max(n_pad, n_lat_pad)]
  double *res;         // [WR_COUNT]
  int *info;
  const double *Plat;  // caller's Q^+ (latent space), ld ldlat
  double *HT;          // Q^+ A^T: n_lat_pad x n, ld ldh (general A only)
  double *xl;          // latent iterate [n_lat_pad] (general A only)
  const int *rp, *ci;  // CSR of A (general A only)
  const double *av;
  double lpar;         // Gaussian: sigma^2; Poisson: beta0
  int n, n_pad, ldq, ldm, lik, general;
  int n_lat, n_lat_pad, ldlat, ldh;
};

__device__ __forceinline__ double *wb_vec(const WbDesc &D, int v) {
  return v == WV_X ? D.x : v == WV_B ? D.b : v == WV_U ? D.u : v == WV_T ? D.t : D.w;
}

// HT = Q^+ A^T: column i = sum over row i of A of a_ik Q^+[:, k].  Grid
// (n_lat_pad / 256, n, B).
__global__ __launch_bounds__(256) void wb_ht_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.z];
  const int i = blockIdx.y, j = blockIdx.x * 256 + threadIdx.x;
  if (!D.general || i >= D.n || j >= D.n_lat_pad) return;
  double acc = 0.0;
  if (j < D.n_lat)
    for (int e = D.rp[i]; e < D.rp[i + 1]; ++e) acc = fma(D.av[e], D.Plat[(size_t)D.ci[e] * D.ldlat + j], acc);
  D.HT[(size_t)i * D.ldh + j] = acc;
}

// K = A HT (the observation-space covariance, n x n, ld ldq): column i, row r =
// sum over row r of A of a_rk HT[k, i].  Grid (n_pad / 256, n_pad, B).
__global__ __launch_bounds__(256) void wb_k_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.z];
  const int i = blockIdx.y, r = blockIdx.x * 256 + threadIdx.x;
  if (!D.general || i >= D.n || r >= D.n) return;
  const double *col = D.HT + (size_t)i * D.ldh;
  double acc = 0.0;
  for (int e = D.rp[r]; e < D.rp[r + 1]; ++e) acc = fma(D.av[e], col[D.ci[e]], acc);
  ((double *)D.Pq)[(size_t)i * D.ldq + r] = acc;
}

// Start: A = I: x <- caller's vector (start = 1) or 0.  General A: latent
// iterate from the caller or 0, and x = A x_latent.  Grid (max(n_pad,
// n_lat_pad) / 256, B).
__global__ __launch_bounds__(256) void wb_start_kernel(const WbDesc *__restrict__ wd, int start) {
  const WbDesc D = wd[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (!D.general) {
    if (i < D.n_pad) D.x[i] = (start && i < D.n) ? D.xext[i] : 0.0;
    return;
  }
  if (i < D.n_lat_pad) D.xl[i] = (start && i < D.n_lat) ? D.xext[i] : 0.0;
  if (i < D.n_pad) {
    double acc = 0.0;
    if (start && i < D.n)
      for (int e = D.rp[i]; e < D.rp[i + 1]; ++e) acc = fma(D.av[e], D.xext[D.ci[e]], acc);
    D.x[i] = acc;
  }
}

// b = g + W x and sw = sqrt(W) at the current iterate (Q_l = diag(W), the
// negative second derivative of log pi(y | eta)); clears the factor status.
__global__ __launch_bounds__(256) void wb_lik_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *D.info = 0;
  if (i >= D.n_pad) return;
  double bi = 0.0, si = 0.0;
  if (i < D.n) {
    const double xi = D.x[i];
    double g, W;
    if (D.lik == LIK_POISSON) {
      const double mu = (D.E ? D.E[i] : 1.0) * exp(D.lpar + xi);
      g = D.y[i] - mu;
      W = mu;
    } else {
      W = 1.0 / D.lpar;
      g = (D.y[i] - xi) * W;
    }
    bi = g + W * xi;
    si = sqrt(W);
  }
  D.b[i] = bi;
  D.sw[i] = si;
}

// Partial products of Pq v over WB_CH column chunks (v = src, or sw * src).
// Grid (n_pad / 256, WB_CH, B); the row reads of each column are coalesced.
__global__ __launch_bounds__(256) void wb_symv_part_kernel(const WbDesc *__restrict__ wd, int src, int scaled) {
  const WbDesc D = wd[blockIdx.z];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if ((int)blockIdx.x * 256 >= D.n_pad) return;
  const int cs = (D.n + WB_CH - 1) / WB_CH;
  const int j0 = blockIdx.y * cs, j1 = min(D.n, j0 + cs);
  const double *v = wb_vec(D, src);
  double acc = 0.0;
  if (i < D.n) {
    const auto *col = gptr(D.Pq) + i;
#pragma unroll 8
    for (int j = j0; j < j1; ++j) acc = fma(col[(size_t)j * D.ldq], scaled ? D.sw[j] * v[j] : v[j], acc);
  }
  if (i < D.n_pad) D.part[(size_t)blockIdx.y * D.n_pad + i] = acc;
}

// dst = sum of the partials in chunk order; with `border` also the border row
// of M: r = sw * dst.  Grid (n_pad / 256, B).
__global__ __launch_bounds__(256) void wb_symv_reduce_kernel(const WbDesc *__restrict__ wd, int dst, int border) {
  const WbDesc D = wd[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= D.n_pad) return;
  double s = 0.0;
  for (int c = 0; c < WB_CH; ++c) s += D.part[(size_t)c * D.n_pad + i];
  wb_vec(D, dst)[i] = s;
  if (border) D.M[(size_t)i * D.ldm + D.n_pad] = D.sw[i] * s;
}

// M = I + diag(sw) Pq diag(sw), lower triangle, identity on the padding.
// Border rows (i >= n_pad): Newton (var = 0): zero below row n_pad, whose r is
// written by the reduction; variances (var = 1): row n_pad + a holds
// (Q^+ A^T S)_{a, j} = HT_{a j} sw_j (A = I: Q^+_{a j} sw_j) for a < n_lat,
// zero beyond.  Grid (ldm / 256, n_pad, B).
__global__ __launch_bounds__(256) void wb_assemble_kernel(const WbDesc *__restrict__ wd, int var) {
  const WbDesc D = wd[blockIdx.z];
  const int j = blockIdx.y;
  if (j >= D.n_pad) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= D.ldm || i < j || (!var && i == D.n_pad)) return;
  double v = 0.0;
  if (i < D.n_pad) {
    v = i == j ? 1.0 : 0.0;
    if (i < D.n && j < D.n) v += D.sw[i] * D.Pq[(size_t)j * D.ldq + i] * D.sw[j];
  } else if (var) {
    const int a = i - D.n_pad;
    if (a < D.n_lat && j < D.n)
      v = (D.general ? D.HT[(size_t)j * D.ldh + a] : D.Pq[(size_t)j * D.ldq + a]) * D.sw[j];
  }
  D.M[(size_t)j * D.ldm + i] = v;
}

// var_a = Q^+_aa - ||row a of the factored border||^2 = diag(Sigma*)_a, written
// to the caller's vector.  Grid (n_lat_pad / 256, B); the column reads of the
// border are coalesced across the rows.
__global__ __launch_bounds__(256) void wb_var_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.y];
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= D.n_lat) return;
  const auto *G = gptr((const double *)D.M) + D.n_pad + a;
  double s = 0.0;
  for (int j = 0; j < D.n; ++j) {
    const double g = G[(size_t)j * D.ldm];
    s = fma(g, g, s);
  }
  D.vext[a] = D.Plat[(size_t)a * D.ldlat + a] - s;
}

// s = L^{-1} r from the factored border row.  Grid (n_pad / 256, B).
__global__ __launch_bounds__(256) void wb_border_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= D.n_pad) return;
  D.s[i] = D.M[(size_t)i * D.ldm + D.n_pad];
}

// x_new = u - w, the step, max(1, |x_new|_inf), z = b - sw * t and z^T x_new,
// and log|M| = 2 sum log L_ii.  One workgroup per theta.
__global__ __launch_bounds__(256) void wb_update_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.x];
  __shared__ double sh[4];
  double step = 0.0, xmax = 0.0, ztx = 0.0, ld = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < D.n; i += 256) {
    const double xn = D.u[i] - D.w[i];
    const double zi = D.b[i] - D.sw[i] * D.t[i];
    step = fmax(step, fabs(xn - D.x[i]));
    xmax = fmax(xmax, fabs(xn));
    ztx += zi * xn;
    ld += log(D.M[(size_t)i * D.ldm + i]);
    if (!isfinite(xn)) bad = 1.0;
    D.x[i] = xn;
    D.z[i] = zi;
  }
  step = block_max256(step, sh);
  xmax = block_max256(xmax, sh);
  ztx = block_sum256(ztx, sh);
  ld = block_sum256(ld, sh);
  bad = block_max256(bad, sh);
  if (threadIdx.x == 0) {
    D.res[WR_STEP] = step;
    D.res[WR_SCALE] = fmax(1.0, xmax);
    D.res[WR_ZTX] = ztx;
    D.res[WR_LOGDET] = 2.0 * ld;
    D.res[WR_NONFINITE] = bad;
  }
}

// General A: partial products HT z over WB_CH column chunks.  Grid
// (n_lat_pad / 256, WB_CH, B).
__global__ __launch_bounds__(256) void wb_xl_part_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.z];
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (!D.general || (int)blockIdx.x * 256 >= D.n_lat_pad) return;
  const int cs = (D.n + WB_CH - 1) / WB_CH;
  const int i0 = blockIdx.y * cs, i1 = min(D.n, i0 + cs);
  double acc = 0.0;
  if (j < D.n_lat) {
    const auto *row = gptr((const double *)D.HT) + j;
#pragma unroll 8
    for (int i = i0; i < i1; ++i) acc = fma(row[(size_t)i * D.ldh], D.z[i], acc);
  }
  if (j < D.n_lat_pad) D.part[(size_t)blockIdx.y * D.n_lat_pad + j] = acc;
}

// General A: x_latent = sum of the partials, and the latent step and scale
// (these replace the observation-space ones in the stopping rule).  One
// workgroup per theta.
__global__ __launch_bounds__(256) void wb_xl_update_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.x];
  if (!D.general) return;
  __shared__ double sh[4];
  double step = 0.0, xmax = 0.0, bad = 0.0;
  for (int j = threadIdx.x; j < D.n_lat; j += 256) {
    double xn = 0.0;
    for (int c = 0; c < WB_CH; ++c) xn += D.part[(size_t)c * D.n_lat_pad + j];
    step = fmax(step, fabs(xn - D.xl[j]));
    xmax = fmax(xmax, fabs(xn));
    if (!isfinite(xn)) bad = 1.0;
    D.xl[j] = xn;
  }
  step = block_max256(step, sh);
  xmax = block_max256(xmax, sh);
  bad = block_max256(bad, sh);
  if (threadIdx.x == 0) {
    D.res[WR_STEP] = step;
    D.res[WR_SCALE] = fmax(1.0, xmax);
    if (bad != 0.0) D.res[WR_NONFINITE] = 1.0;
  }
}

// sum_i log pi(y_i | eta_i) at the mode (normalising constants included) and
// the caller's copy of the mode.  One workgroup per theta.
__global__ __launch_bounds__(256) void wb_final_kernel(const WbDesc *__restrict__ wd) {
  const WbDesc D = wd[blockIdx.x];
  __shared__ double sh[4];
  double ll = 0.0;
  for (int i = threadIdx.x; i < D.n; i += 256) {
    const double xi = D.x[i], yi = D.y[i];
    if (D.lik == LIK_POISSON) {
      const double Ei = D.E ? D.E[i] : 1.0;
      const double eta = D.lpar + xi;
      ll += yi * (log(Ei) + eta) - Ei * exp(eta) - lgamma(yi + 1.0);
    } else {
      const double r = yi - xi;
      ll += -0.5 * log(2.0 * M_PI * D.lpar) - r * r / (2.0 * D.lpar);
    }
    if (!D.general) D.xext[i] = xi;
  }
  if (D.general)
    for (int j = threadIdx.x; j < D.n_lat; j += 256) D.xext[j] = D.xl[j];
  ll = block_sum256(ll, sh);
  if (threadIdx.x == 0) D.res[WR_LOGLIK] = ll;
}

static bool wb_model_ok(const inla_model &m) {
  if (m.prior != INLA_PRIOR_PINV || m.n < 1 || m.k != 0 || !m.Qprior || m.ldq < m.n || !m.y ||
      (m.lik != INLA_LIK_GAUSSIAN && m.lik != INLA_LIK_POISSON))
    return false;
  if (m.m < 0 || (m.m > 0 && (m.nnz < 0 || !m.A_rowptr || (m.nnz > 0 && (!m.A_col || !m.A_val))))) return false;
  return true;
}

// The CSR arrays of a general design matrix, copied back once per call: row
// pointers non-decreasing from 0 to nnz, column indices in [0, n).  The kernels
// index the caller's Q^+ and start vector through them.
static bool wb_design_ok(const inla_model &m) {
  if (m.m == 0) return true;
  std::vector<int> rp(m.m + 1), ci(std::max(m.nnz, 0));
  if (hipMemcpy(rp.data(), m.A_rowptr, sizeof(int) * rp.size(), hipMemcpyDeviceToHost) != hipSuccess) return false;
  if (m.nnz > 0 && hipMemcpy(ci.data(), m.A_col, sizeof(int) * ci.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return false;
  if (rp[0] != 0 || rp[m.m] != m.nnz) return false;
  for (int i = 0; i < m.m; ++i)
    if (rp[i + 1] < rp[i]) return false;
  for (int c : ci)
    if (c < 0 || c >= m.n) return false;
  return true;
}

// Workspace of one theta: the factor (Newton: one border block; variances:
// n_lat_pad border rows), diagonal-block inverses, vectors, partials, and for a
// general A the matrices K and HT and the latent iterate.
struct WbLayout {
  std::vector<size_t> off;
  size_t total = 0;
  int np_max = 0, nlp_max = 0, ldm_max = 0, n_max = 0, any_general = 0;
};

static size_t wb_bytes(const inla_model &m, bool var) {
  const bool gen = m.m > 0;
  const int n = gen ? m.m : m.n, np = round_up(n, PADN), nlp = round_up(m.n, PADN);
  const int ldm = var ? np + nlp : np + PADN;
  size_t b = a256(sizeof(double) * (size_t)ldm * np) + a256(sizeof(double) * (size_t)np * NBI) +
             a256(sizeof(double) * 8 * (size_t)np) + a256(sizeof(double) * WB_CH * (size_t)std::max(np, nlp));
  if (gen)
    b += a256(sizeof(double) * (size_t)np * np) + a256(sizeof(double) * (size_t)nlp * n) +
         a256(sizeof(double) * (size_t)nlp);
  return b;
}

static WbLayout wb_layout(int B, const inla_model *models, bool var, size_t head) {
  WbLayout L;
  L.total = head;
  L.off.resize(B);
  for (int b = 0; b < B; ++b) {
    const inla_model &m = models[b];
    const bool gen = m.m > 0;
    const int n = gen ? m.m : m.n, np = round_up(n, PADN), nlp = round_up(m.n, PADN);
    L.off[b] = L.total;
    L.total += wb_bytes(m, var);
    L.np_max = std::max(L.np_max, np);
    L.nlp_max = std::max(L.nlp_max, nlp);
    L.ldm_max = std::max(L.ldm_max, var ? np + nlp : np + PADN);
    L.n_max = std::max(L.n_max, n);
    L.any_general |= gen;
  }
  return L;
}

static WbDesc wb_desc(const inla_model &m, const double *theta, char *base, bool var, double *xext, double *vext,
                      double *res, int *info) {
  WbDesc D{};
  const bool gen = m.m > 0;
  D.general = gen;
  D.n = gen ? m.m : m.n;
  D.n_pad = round_up(D.n, PADN);
  D.n_lat = m.n;
  D.n_lat_pad = round_up(m.n, PADN);
  D.ldm = var ? D.n_pad + D.n_lat_pad : D.n_pad + PADN;
  D.y = m.y; D.E = m.E; D.lik = m.lik; D.xext = xext; D.vext = vext; D.res = res; D.info = info;
  D.Plat = m.Qprior; D.ldlat = m.ldq;
  const double lp = theta[0];
  D.lpar = m.lik == INLA_LIK_GAUSSIAN ? std::exp(lp) : lp;
  D.M = (double *)base;
  base += a256(sizeof(double) * (size_t)D.ldm * D.n_pad);
  D.linv = (double *)base;
  base += a256(sizeof(double) * (size_t)D.n_pad * NBI);
  double *v = (double *)base;
  D.x = v; D.b = v + D.n_pad; D.sw = v + 2 * D.n_pad; D.u = v + 3 * D.n_pad; D.s = v + 4 * D.n_pad;
  D.t = v + 5 * D.n_pad; D.w = v + 6 * D.n_pad; D.z = v + 7 * D.n_pad;
  base += a256(sizeof(double) * 8 * (size_t)D.n_pad);
  D.part = (double *)base;
  base += a256(sizeof(double) * WB_CH * (size_t)std::max(D.n_pad, D.n_lat_pad));
  if (gen) {
    D.Pq = (const double *)base;
    D.ldq = D.n_pad;
    base += a256(sizeof(double) * (size_t)D.n_pad * D.n_pad);
    D.HT = (double *)base;
    D.ldh = D.n_lat_pad;
    base += a256(sizeof(double) * (size_t)D.n_lat_pad * D.n);
    D.xl = (double *)base;
    D.rp = m.A_rowptr; D.ci = m.A_col; D.av = m.A_val;
  } else {
    D.Pq = m.Qprior;
    D.ldq = m.ldq;
  }
  return D;
}

// HT and K of the general-A thetas (no-ops for A = I).
static void wb_prepare(Ctx &ctx, const WbDesc *dd, int B, const WbLayout &L) {
  if (!L.any_general) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(wb_ht_kernel, dim3((L.nlp_max + 255) / 256, L.n_max, B), dim3(256), 0, ctx.stream, dd);
  });
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(wb_k_kernel, dim3((L.np_max + 255) / 256, L.np_max, B), dim3(256), 0, ctx.stream, dd);
  });
}

static HostFactor wb_factor(const WbDesc &D, bool var) {
  HostFactor h{};
  h.d.A = D.M; h.d.linv = D.linv; h.d.info = D.info; h.d.ld = D.ldm; h.d.nf = D.n_pad;
  h.d.nrows = D.ldm; h.d.ncols = D.n_pad; h.d.id_row0 = std::numeric_limits<int>::max();
  h.n_real = D.n; h.kb_real = var ? D.n_lat : 1; h.ks_real = 0;
  return h;
}

static int wb_validate(int B, const inla_model *models, const double *theta, int ldtheta, double *const *x,
                       const inla_opts *opts, inla_result *res) {
  if (B < 0) return -2;
  if (B == 0) return INLA_OK;
  if (!models) return -3;
  if (!theta || ldtheta < 1) return -4;
  if (!x) return -6;
  if (!res) return -8;
  if (opts && opts->prec != INLA_PREC_FP64) return INLA_ERR_UNSUPPORTED;
  for (int b = 0; b < B; ++b) {
    if (!wb_model_ok(models[b])) return -3;
    if (!x[b]) return -6;
  }
  for (int b = 0; b < B; ++b)
    if (!wb_design_ok(models[b])) return -3;
  return INLA_OK;
}

static int woodbury_eval(Ctx &ctx, int B, const inla_model *models, const double *theta, int ldtheta,
                         double *const *x, const inla_opts *opts, inla_result *res) {
  const int max_iter = opts && opts->max_iter > 0 ? opts->max_iter : 50;
  const double tol = opts && opts->tol > 0 ? opts->tol : 1e-11;
  const int start = opts ? opts->start : 0;
  const size_t head = a256(sizeof(double) * WR_COUNT * B) + a256(sizeof(int) * B);
  const WbLayout L = wb_layout(B, models, false, head);
  if (!ctx.reserve(L.total)) return INLA_ERR_NOMEM;
  double *dres = (double *)ctx.ws;
  int *dinfo = (int *)(ctx.ws + a256(sizeof(double) * WR_COUNT * B));
  std::vector<WbDesc> hd(B);
  for (int b = 0; b < B; ++b) {
    hd[b] = wb_desc(models[b], theta + (size_t)b * ldtheta, ctx.ws + L.off[b], false, x[b], nullptr,
                    dres + WR_COUNT * b, dinfo + b);
    res[b] = inla_result{};
    if (!std::isfinite(theta[(size_t)b * ldtheta])) res[b].info = INLA_INFO_NONFINITE;
  }
  std::vector<int> act;
  for (int b = 0; b < B; ++b) if (res[b].info == INLA_INFO_OK) act.push_back(b);
  {
    const WbDesc *dall = (const WbDesc *)ctx.upload(hd.data(), sizeof(WbDesc) * B);
    if (!dall) return INLA_ERR_NOMEM;
    wb_prepare(ctx, dall, B, L);
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(wb_start_kernel, dim3((std::max(L.np_max, L.nlp_max) + 255) / 256, B), dim3(256), 0,
                         ctx.stream, dall, start);
    });
  }
  std::vector<double> hres((size_t)WR_COUNT * B);
  std::vector<double> prev(B, std::numeric_limits<double>::infinity());
  std::vector<int> hinfo(B);
  std::vector<int> done;
  for (int it = 1; it <= max_iter && !act.empty(); ++it) {
    std::vector<WbDesc> ha;
    std::vector<HostFactor> fs;
    std::vector<ThetaDesc> td;
    int np = 0, ldm = 0, nlp = 0, gen = 0;
    double qbytes = 0;
    for (int b : act) {
      const WbDesc &D = hd[b];
      ha.push_back(D);
      np = std::max(np, D.n_pad);
      ldm = std::max(ldm, D.ldm);
      nlp = std::max(nlp, D.n_lat_pad);
      gen |= D.general;
      qbytes += 8.0 * D.n * D.n;
      fs.push_back(wb_factor(D, false));
      ThetaDesc t{};
      t.W = D.M; t.ldw = D.ldm; t.linv = D.linv; t.n_pad = D.n_pad; t.n = D.n; t.r = D.s; t.u = D.t;
      td.push_back(t);
    }
    const int na = (int)ha.size();
    const WbDesc *da = (const WbDesc *)ctx.upload(ha.data(), sizeof(WbDesc) * na);
    if (!da) return INLA_ERR_NOMEM;
    const dim3 gv((np + 255) / 256, na);
    ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(wb_lik_kernel, gv, dim3(256), 0, ctx.stream, da);
    });
    ctx.launch(INLA_K_SOLVE, 2.0 * qbytes / 8.0, qbytes, [&] {
      hipLaunchKernelGGL(wb_symv_part_kernel, dim3((np + 255) / 256, WB_CH, na), dim3(256), 0, ctx.stream, da, WV_B, 0);
    });
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(wb_symv_reduce_kernel, gv, dim3(256), 0, ctx.stream, da, WV_U, 1);
    });
    ctx.launch(INLA_K_ASSEMBLE, 0.0, qbytes, [&] {
      hipLaunchKernelGGL(wb_assemble_kernel, dim3((ldm + 255) / 256, np, na), dim3(256), 0, ctx.stream, da, 0);
    });
    int rc = factor_batch(ctx, fs, INLA_PREC_FP64);
    if (rc) return rc;
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(wb_border_kernel, gv, dim3(256), 0, ctx.stream, da);
    });
    launch_trsv_bwd(ctx, td, np, V_R, V_U, 0.0, INLA_PREC_FP64);
    ctx.launch(INLA_K_SOLVE, 2.0 * qbytes / 8.0, qbytes, [&] {
      hipLaunchKernelGGL(wb_symv_part_kernel, dim3((np + 255) / 256, WB_CH, na), dim3(256), 0, ctx.stream, da, WV_T, 1);
    });
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(wb_symv_reduce_kernel, gv, dim3(256), 0, ctx.stream, da, WV_W, 0);
    });
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(wb_update_kernel, dim3(na), dim3(256), 0, ctx.stream, da);
    });
    if (gen) {
      ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
        hipLaunchKernelGGL(wb_xl_part_kernel, dim3((nlp + 255) / 256, WB_CH, na), dim3(256), 0, ctx.stream, da);
      });
      ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
        hipLaunchKernelGGL(wb_xl_update_kernel, dim3(na), dim3(256), 0, ctx.stream, da);
      });
    }
    if (hipMemcpyAsync(hres.data(), dres, sizeof(double) * WR_COUNT * B, hipMemcpyDeviceToHost, ctx.stream) !=
            hipSuccess ||
        hipMemcpyAsync(hinfo.data(), dinfo, sizeof(int) * B, hipMemcpyDeviceToHost, ctx.stream) != hipSuccess)
      return INLA_ERR_HIP;
    if (hipStreamSynchronize(ctx.stream) != hipSuccess) return INLA_ERR_HIP;
    if ((rc = ctx.check())) return rc;
    std::vector<int> keep;
    for (int b : act) {
      const double *R = hres.data() + WR_COUNT * b;
      inla_result &o = res[b];
      o.iters = it;
      o.step = R[WR_STEP];
      if (hinfo[b] > 0) { o.info = hinfo[b]; continue; }
      if (R[WR_NONFINITE] != 0.0 || !std::isfinite(R[WR_STEP])) { o.info = INLA_INFO_NONFINITE; continue; }
      const bool floor = R[WR_STEP] <= WB_FLOOR_TOL * R[WR_SCALE] && R[WR_STEP] > 0.5 * prev[b];
      prev[b] = R[WR_STEP];
      if (models[b].lik == INLA_LIK_GAUSSIAN || R[WR_STEP] <= tol * R[WR_SCALE] || floor) {
        done.push_back(b);
        continue;
      }
      if (it == max_iter) {
        o.info = INLA_INFO_NEWTON_MAXIT;
        done.push_back(b);
        continue;
      }
      keep.push_back(b);
    }
    act.swap(keep);
  }
  if (!done.empty()) {
    std::vector<WbDesc> ha;
    for (int b : done) ha.push_back(hd[b]);
    const WbDesc *da = (const WbDesc *)ctx.upload(ha.data(), sizeof(WbDesc) * ha.size());
    if (!da) return INLA_ERR_NOMEM;
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(wb_final_kernel, dim3((unsigned)ha.size()), dim3(256), 0, ctx.stream, da);
    });
    if (hipMemcpyAsync(hres.data(), dres, sizeof(double) * WR_COUNT * B, hipMemcpyDeviceToHost, ctx.stream) !=
        hipSuccess)
      return INLA_ERR_HIP;
    if (hipStreamSynchronize(ctx.stream) != hipSuccess) return INLA_ERR_HIP;
    for (int b : done) {
      const double *R = hres.data() + WR_COUNT * b;
      inla_result &o = res[b];
      o.xqx = R[WR_ZTX];
      o.loglik = R[WR_LOGLIK];
      o.logdet_qstar = R[WR_LOGDET];
      o.objective = o.loglik - 0.5 * o.xqx - 0.5 * o.logdet_qstar;
    }
  }
  return ctx.check();
}

// Marginal variances diag(Sigma*) at given modes: M = I + S K S with W at the
// mode, factored with the n_lat border rows (Q^+ A^T S), which come out as
// (L^{-1} S A Q^+)^T.
static int woodbury_var(Ctx &ctx, int B, const inla_model *models, const double *theta, int ldtheta,
                        const double *const *x, double *const *var, int *info) {
  const size_t head = a256(sizeof(int) * B);
  const WbLayout L = wb_layout(B, models, true, head);
  if (!ctx.reserve(L.total)) return INLA_ERR_NOMEM;
  int *dinfo = (int *)ctx.ws;
  std::vector<WbDesc> hd(B);
  std::vector<HostFactor> fs;
  for (int b = 0; b < B; ++b) {
    hd[b] = wb_desc(models[b], theta + (size_t)b * ldtheta, ctx.ws + L.off[b], true, (double *)x[b], var[b],
                    nullptr, dinfo + b);
    fs.push_back(wb_factor(hd[b], true));
  }
  const WbDesc *dd = (const WbDesc *)ctx.upload(hd.data(), sizeof(WbDesc) * B);
  if (!dd) return INLA_ERR_NOMEM;
  wb_prepare(ctx, dd, B, L);
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(wb_start_kernel, dim3((std::max(L.np_max, L.nlp_max) + 255) / 256, B), dim3(256), 0,
                       ctx.stream, dd, 1);
  });
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(wb_lik_kernel, dim3((L.np_max + 255) / 256, B), dim3(256), 0, ctx.stream, dd);
  });
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(wb_assemble_kernel, dim3((L.ldm_max + 255) / 256, L.np_max, B), dim3(256), 0, ctx.stream,
                       dd, 1);
  });
  int rc = factor_batch(ctx, fs, INLA_PREC_FP64);
  if (rc) return rc;
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(wb_var_kernel, dim3((L.nlp_max + 255) / 256, B), dim3(256), 0, ctx.stream, dd);
  });
  std::vector<int> hinfo(B);
  if (hipMemcpyAsync(hinfo.data(), dinfo, sizeof(int) * B, hipMemcpyDeviceToHost, ctx.stream) != hipSuccess)
    return INLA_ERR_HIP;
  if (hipStreamSynchronize(ctx.stream) != hipSuccess) return INLA_ERR_HIP;
  for (int b = 0; b < B; ++b) info[b] = hinfo[b];
  return ctx.check();
}

// ------------------------------------------------------------------ block-structured Q^+(theta)
struct PinvBlock {
  const double *P;
  int off, size, ld, pad_;
};

// out_b = blockdiag_k(scale[b][k] P_k), full n x n (ld n).  Grid (n / 256, n, B).
__global__ __launch_bounds__(256) void pinv_prior_kernel(const PinvBlock *__restrict__ blk, int nblk,
                                                         const double *__restrict__ scale, int n,
                                                         double *const *__restrict__ out) {
  const int j = blockIdx.y, b = blockIdx.z, i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n || j >= n) return;
  double v = 0.0;
  for (int k = 0; k < nblk; ++k) {
    const PinvBlock &B = blk[k];
    if (j >= B.off && j < B.off + B.size) {
      if (i >= B.off && i < B.off + B.size)
        v = scale[(size_t)b * nblk + k] * B.P[(size_t)(j - B.off) * B.ld + (i - B.off)];
      break;
    }
  }
  out[b][(size_t)j * n + i] = v;
}

// 0 if the description is valid for order n and theta dimension t (t < 0: not
// checked), else -3.
int pinv_prior_check(const inla_pinv_prior *pp, int n, int t) {
  if (!pp || pp->n_blocks < 1 || !pp->offset || !pp->size || !pp->P || !pp->ld || !pp->tau_index) return -3;
  std::vector<std::pair<int, int>> iv;
  for (int k = 0; k < pp->n_blocks; ++k) {
    if (pp->size[k] < 1 || pp->offset[k] < 0 || !pp->P[k] || pp->ld[k] < pp->size[k]) return -3;
    if (pp->tau_index[k] < 0 && (!pp->fixed_scale || !std::isfinite(pp->fixed_scale[k]))) return -3;
    if (t >= 0 && pp->tau_index[k] >= t) return -3;
    iv.push_back({pp->offset[k], pp->size[k]});
  }
  std::sort(iv.begin(), iv.end());
  int pos = 0;
  for (auto &q : iv) {
    if (q.first != pos) return -3;
    pos += q.second;
  }
  if (pos != n) return -3;
  if (t >= 0 && pp->lik_index >= t) return -3;
  if (pp->lik_index < 0 && !std::isfinite(pp->lik_value)) return -3;
  return 0;
}

int pinv_prior_assemble(Ctx &ctx, const inla_pinv_prior &pp, int n, int B, const double *theta, int ldtheta,
                        double *const *out) {
  const int nb = pp.n_blocks;
  std::vector<PinvBlock> hb(nb);
  for (int k = 0; k < nb; ++k) hb[k] = PinvBlock{pp.P[k], pp.offset[k], pp.size[k], pp.ld[k], 0};
  std::vector<double> sc((size_t)B * nb);
  for (int b = 0; b < B; ++b)
    for (int k = 0; k < nb; ++k)
      sc[(size_t)b * nb + k] = pp.tau_index[k] >= 0 ? std::exp(-theta[(size_t)b * ldtheta + pp.tau_index[k]])
                                                    : pp.fixed_scale[k];
  const PinvBlock *db = (const PinvBlock *)ctx.upload(hb.data(), sizeof(PinvBlock) * nb);
  const double *ds = (const double *)ctx.upload(sc.data(), sizeof(double) * sc.size());
  double *const *dout = (double *const *)ctx.upload(out, sizeof(double *) * B);
  if (!db || !ds || !dout) return INLA_ERR_NOMEM;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 8.0 * n * (double)n * B, [&] {
    hipLaunchKernelGGL(pinv_prior_kernel, dim3((n + 255) / 256, n, B), dim3(256), 0, ctx.stream, db, nb, ds, n,
                       dout);
  });
  return ctx.check();
}

}  // namespace inla

extern "C" {

int inla_pinv(inla_handle *h, int32_t B, const int32_t *n, const double *const *Q, const int32_t *ldq,
              double *const *Qpinv, const int32_t *ldp, double rtol, int32_t *rank, int32_t *sweeps, int32_t *info) {
  using namespace inla;
  if (!h) return -1;
  if (B < 0) return -2;
  if (B == 0) return INLA_OK;
  if (!n) return -3;
  if (!Q) return -4;
  if (!ldq) return -5;
  if (!Qpinv) return -6;
  if (!ldp) return -7;
  if (!rank) return -9;
  if (!sweeps) return -10;
  if (!info) return -11;
  for (int b = 0; b < B; ++b) {
    if (n[b] < 1 || n[b] > JAC_MAX_N) return -3;
    if (!Q[b]) return -4;
    if (ldq[b] < n[b]) return -5;
    if (!Qpinv[b]) return -6;
    if (ldp[b] < n[b]) return -7;
  }
  if (!(rtol < 1.0)) return -8;
  return pinv_batch(*handle_ctx(h), B, n, Q, ldq, Qpinv, ldp, rtol, rank, sweeps, info);
}

int inla_woodbury_var(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                      const double *const *x_mode, double *const *var, int32_t *info) {
  using namespace inla;
  if (!h) return -1;
  if (B < 0) return -2;
  if (B == 0) return INLA_OK;
  if (!models) return -3;
  if (!theta || ldtheta < 1) return -4;
  if (!x_mode) return -6;
  if (!var) return -7;
  if (!info) return -8;
  for (int b = 0; b < B; ++b) {
    if (!wb_model_ok(models[b])) return -3;
    if (!std::isfinite(theta[(size_t)b * ldtheta])) return -4;
    if (!x_mode[b]) return -6;
    if (!var[b]) return -7;
  }
  for (int b = 0; b < B; ++b)
    if (!wb_design_ok(models[b])) return -3;
  return woodbury_var(*handle_ctx(h), B, models, theta, ldtheta, x_mode, var, info);
}

int inla_pinv_prior_assemble(inla_handle *h, const inla_pinv_prior *prior, int32_t n, int32_t B, const double *theta,
                             int32_t ldtheta, double *const *out) {
  using namespace inla;
  if (!h) return -1;
  if (n < 1) return -3;
  if (B < 0) return -4;
  if (!theta || ldtheta < 1) return -5;
  if (pinv_prior_check(prior, n, ldtheta)) return -2;
  if (B == 0) return INLA_OK;
  if (!out) return -7;
  for (int b = 0; b < B; ++b)
    if (!out[b]) return -7;
  return pinv_prior_assemble(*handle_ctx(h), *prior, n, B, theta, ldtheta, out);
}

int inla_woodbury_eval(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                       double *const *x, const inla_opts *opts, inla_result *res) {
  using namespace inla;
  if (!h) return -1;
  int rc = wb_validate(B, models, theta, ldtheta, x, opts, res);
  if (rc || B == 0) return rc;
  return woodbury_eval(*handle_ctx(h), B, models, theta, ldtheta, x, opts, res);
}

}  // extern "C"
