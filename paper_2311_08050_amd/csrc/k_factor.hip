// Bordered, batched, right-looking blocked Cholesky for gfx950.
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
// Steps per inner block j (width NBI = 64) of an outer panel [p0, p0 + nb):
//   potf2_inv  : L_jj = chol(A_jj) in LDS and X = L_jj^{-1} (one workgroup per theta)
//   TRSM       : A[j+64:, j:j+64] <- A[j+64:, j:j+64] X^T     (MFMA, in place)
//   PANEL      : A[j+64:, j+64:pend] -= A[j+64:, j:j+64] A[j+64:pend, j:j+64]^T
// and per outer panel
//   TRAIL      : A[pend:, pend:ncols] -= A[pend:, p0:pend] A[pend:ncols, p0:pend]^T
// All updates are FP64 MFMA (v_mfma_f64_16x16x4f64) tile kernels with LDS-staged,
// double-buffered K chunks.
#include "device.hpp"
#include "host.hpp"

namespace inla {

enum { KIND_TRSM = 0, KIND_PANEL = 1, KIND_TRAIL = 2 };

// --------------------------------------------------------------------------
// Diagonal block: unblocked right-looking Cholesky of the 64 x 64 block in LDS,
// then its triangular inverse by column-wise forward substitution.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void potf2_inv_kernel(const FactorDesc *__restrict__ descs, int j) {
  const FactorDesc d = descs[blockIdx.x];
  if (j >= d.nf) return;
  __shared__ double L[NBI][NBI + 1];
  __shared__ double X[NBI][NBI + 1];
  __shared__ int fail;
  const int tid = threadIdx.x;
  double *Ad = d.A + (size_t)j * d.ld + j;
  for (int e = tid; e < NBI * NBI; e += 256) {
    const int r = e & (NBI - 1), c = e >> 6;
    L[r][c] = (r >= c) ? Ad[(size_t)c * d.ld + r] : 0.0;
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int c = 0; c < NBI; ++c) {
    if (tid == 0) {
      double v = L[c][c];
      if (!(v > 0.0)) {
        if (fail == 0) fail = c + 1;
        v = __builtin_nan("");
      }
      L[c][c] = sqrt(v);
    }
    __syncthreads();
    if (tid > c && tid < NBI) L[tid][c] /= L[c][c];
    __syncthreads();
    for (int e = tid; e < NBI * NBI; e += 256) {
      const int r = e & (NBI - 1), cc = e >> 6;
      if (cc > c && r >= cc) L[r][cc] -= L[r][c] * L[cc][c];
    }
    __syncthreads();
  }
  // X = L^{-1}: thread c owns column c.
  if (tid < NBI) {
    const int c = tid;
    for (int r = 0; r < c; ++r) X[r][c] = 0.0;
    X[c][c] = 1.0 / L[c][c];
    for (int r = c + 1; r < NBI; ++r) {
      double s = 0.0;
      for (int m = c; m < r; ++m) s += L[r][m] * X[m][c];
      X[r][c] = -s / L[r][r];
    }
  }
  __syncthreads();
  for (int e = tid; e < NBI * NBI; e += 256) {
    const int r = e & (NBI - 1), c = e >> 6;
    if (r >= c) Ad[(size_t)c * d.ld + r] = L[r][c];
    d.linv[c * NBI + r] = X[r][c];
  }
  if (tid == 0 && fail != 0 && *d.info == 0) *d.info = j + fail;
}

// --------------------------------------------------------------------------
// MFMA tile update.  C(TM x TN) = or -= A(TM x K) B(TN x K)^T, A and B read from
// column-major storage (element (r, k) at base[k*ld + r]).
//
// MFMA operands are swapped (x from B, y from A) so that lane l's four results
// are C rows (l % 16) of columns (l / 16 + 4 v): with the f64 16x16x4 output
// layout (D row = l/16 + 4v, D column = l%16) every store covers four whole
// 128-byte column segments.  Lane group g = l/16 supplies k = 4g + s at
// MFMA step s of a 16-deep chunk.
// --------------------------------------------------------------------------
template <int TM, int TN>
__global__ __launch_bounds__(256, 2) void gemm_update_kernel(const FactorDesc *__restrict__ descs, int kind,
                                                             int p0, int nb, int j) {
  constexpr int WM = 2, WN = 2;                 // 2 x 2 waves
  constexpr int WTM = TM / WM, WTN = TN / WN;   // wave tile
  constexpr int BM = WTM / 16, BN = WTN / 16;   // MFMA blocks per wave
  constexpr int PAD = 4;
  constexpr int LA = TM / 32, LB = TN / 32;     // double2 loads per thread per chunk
  __shared__ __attribute__((aligned(16))) double As[2][KC][TM + PAD];
  __shared__ __attribute__((aligned(16))) double Bs[2][KC][TN + PAD];

  const FactorDesc d = descs[blockIdx.y];
  if (j >= d.nf) return;
  const int pend = min(p0 + nb, d.nf);
  int r0, c0, cend, ks, ke;
  if (kind == KIND_TRSM) {
    r0 = j + NBI; c0 = j; cend = j + NBI; ks = j; ke = j + NBI;
  } else if (kind == KIND_PANEL) {
    r0 = j + NBI; c0 = j + NBI; cend = pend; ks = j; ke = j + NBI;
  } else {
    r0 = pend; c0 = pend; cend = d.ncols; ks = p0; ke = pend;
  }
  if (r0 >= d.nrows || c0 >= cend) return;
  const int nr = (d.nrows - r0) / TM;
  int I, J;
  if (kind == KIND_TRSM) {
    if ((int)blockIdx.x >= nr) return;
    I = blockIdx.x; J = 0;
  } else {
    const int nc = (cend - c0) / TN;
    const int tri = nc * (nc + 1) / 2;
    const int t = blockIdx.x;
    if (t >= tri + (nr - nc) * nc) return;
    if (t < tri) {
      int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while (i * (i + 1) / 2 > t) --i;
      while ((i + 1) * (i + 2) / 2 <= t) ++i;
      I = i; J = t - i * (i + 1) / 2;
    } else {
      const int u = t - tri;
      I = nc + u / nc; J = u % nc;
    }
  }
  const int row0 = r0 + I * TM, col0 = c0 + J * TN;
  // identity border rows (or columns) that are still zero over [ks, ke) contribute nothing
  if (row0 >= d.id_row0 && row0 - d.id_row0 >= ke) return;
  if (kind != KIND_TRSM && col0 >= d.id_row0 && col0 - d.id_row0 >= ke) return;

  const int ld = d.ld;
  const double *Ag = d.A + (size_t)ks * ld + row0;
  const double *Bg;
  int ldb;
  if (kind == KIND_TRSM) { Bg = d.linv; ldb = NBI; }
  else { Bg = d.A + (size_t)ks * ld + col0; ldb = ld; }
  double *Cg = d.A + (size_t)col0 * ld + row0;
  const int K = ke - ks;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WN, wn = w % WN;
  const int g = lane >> 4, li = lane & 15;

  d4 acc[BM][BN];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  d2 ra[LA], rb[LB];
  auto gload = [&](int kc) {
#pragma unroll
    for (int it = 0; it < LA; ++it) {
      const int lin = it * 256 + tid, kk = lin / (TM / 2), rp = lin % (TM / 2);
      ra[it] = *reinterpret_cast<const d2 *>(Ag + (size_t)(kc + kk) * ld + 2 * rp);
    }
#pragma unroll
    for (int it = 0; it < LB; ++it) {
      const int lin = it * 256 + tid, kk = lin / (TN / 2), rp = lin % (TN / 2);
      rb[it] = *reinterpret_cast<const d2 *>(Bg + (size_t)(kc + kk) * ldb + 2 * rp);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int it = 0; it < LA; ++it) {
      const int lin = it * 256 + tid, kk = lin / (TM / 2), rp = lin % (TM / 2);
      *reinterpret_cast<d2 *>(&As[buf][kk][2 * rp]) = ra[it];
    }
#pragma unroll
    for (int it = 0; it < LB; ++it) {
      const int lin = it * 256 + tid, kk = lin / (TN / 2), rp = lin % (TN / 2);
      *reinterpret_cast<d2 *>(&Bs[buf][kk][2 * rp]) = rb[it];
    }
  };

  gload(0);
  lstore(0);
  __syncthreads();
  int buf = 0;
  for (int kc = 0; kc < K; kc += KC) {
    const bool more = kc + KC < K;
    if (more) gload(kc + KC);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = 4 * g + s;
      double ya[BM], xb[BN];
#pragma unroll
      for (int a = 0; a < BM; ++a) ya[a] = As[buf][kk][wm * WTM + a * 16 + li];
#pragma unroll
      for (int b = 0; b < BN; ++b) xb[b] = Bs[buf][kk][wn * WTN + b * 16 + li];
#pragma unroll
      for (int a = 0; a < BM; ++a)
#pragma unroll
        for (int b = 0; b < BN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b], ya[a], acc[a][b], 0, 0, 0);
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // Epilogue.  Lane holds C(row = rb + li, col = cb + g + 4 v).
  const bool diag_tile = (kind != KIND_TRSM) && (row0 < col0 + TN);
  const bool sub = kind != KIND_TRSM;
#pragma unroll
  for (int a = 0; a < BM; ++a) {
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      const int rl = wm * WTM + a * 16 + li;
      const int cl = wn * WTN + b * 16 + g;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cc = cl + 4 * v;
        if (diag_tile && row0 + rl < col0 + cc) continue;
        double *p = Cg + (size_t)cc * ld + rl;
        *p = sub ? (*p - acc[a][b][v]) : acc[a][b][v];
      }
    }
  }
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

static int tiles_for(const FactorDesc &d, int kind, int p0, int nb, int j, int TM) {
  if (j >= d.nf) return 0;
  const int pend = std::min(p0 + nb, d.nf);
  int r0, c0, cend;
  if (kind == KIND_TRSM) { r0 = j + NBI; c0 = j; cend = j + NBI; }
  else if (kind == KIND_PANEL) { r0 = j + NBI; c0 = j + NBI; cend = pend; }
  else { r0 = pend; c0 = pend; cend = d.ncols; }
  if (r0 >= d.nrows || c0 >= cend) return 0;
  const int nr = (d.nrows - r0) / TM;
  if (kind == KIND_TRSM) return nr;
  const int nc = (cend - c0) / TM;
  return nc * (nc + 1) / 2 + (nr - nc) * nc;
}

int factor_batch(Ctx &ctx, const std::vector<HostFactor> &fs, int nb) {
  const int B = (int)fs.size();
  if (B == 0) return 0;
  // device descriptor array, sorted by nf descending so active sets are prefixes
  std::vector<int> order(B);
  for (int i = 0; i < B; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fs[a].d.nf > fs[b].d.nf; });
  std::vector<FactorDesc> hd(B);
  for (int i = 0; i < B; ++i) hd[i] = fs[order[i]].d;
  FactorDesc *dd = (FactorDesc *)ctx.upload(hd.data(), sizeof(FactorDesc) * B);
  if (!dd) return INLA_ERR_NOMEM;
  const int nf_max = hd[0].nf;
  auto active = [&](int col) {
    int a = 0;
    while (a < B && hd[a].nf > col) ++a;
    return a;
  };
  for (int p0 = 0; p0 < nf_max; p0 += nb) {
    for (int j = p0; j < p0 + nb && j < nf_max; j += NBI) {
      const int act = active(j);
      // potf2 + inverse
      {
        double fl = 0;
        for (int i = 0; i < act; ++i) {
          const HostFactor &h = fs[order[i]];
          const double kr = std::max(0, std::min(NBI, h.n_real - j));
          fl += 2.0 * kr * kr * kr / 3.0;
        }
        ctx.launch(INLA_K_POTF2, fl, 0.0, [&] { hipLaunchKernelGGL(potf2_inv_kernel, dim3(act), dim3(256), 0, ctx.stream, dd, j); });
      }
      for (int kind : {KIND_TRSM, KIND_PANEL}) {
        int gx = 0;
        double fl = 0, by = 0;
        for (int i = 0; i < act; ++i) {
          const HostFactor &h = fs[order[i]];
          gx = std::max(gx, tiles_for(h.d, kind, p0, nb, j, 64));
          const int pend = std::min(p0 + nb, h.d.nf);
          const double kr = std::max(0, std::min(NBI, h.n_real - j));
          if (kind == KIND_TRSM) {
            const double m = count_rows_real(h, j + NBI);
            fl += m * kr * kr;
            by += 16.0 * m * kr;
          } else if (j + NBI < pend) {
            const double nc = count_cols_real(h, j + NBI, pend), nr = count_rows_real(h, j + NBI);
            fl += 2.0 * trap_elems(nr, nc) * kr;
            by += 16.0 * trap_elems(nr, nc) + 8.0 * (nr + nc) * kr;
          }
        }
        if (gx == 0) continue;
        ctx.launch(INLA_K_GEMM, fl, by, [&] {
          hipLaunchKernelGGL((gemm_update_kernel<64, 64>), dim3(gx, act), dim3(256), 0, ctx.stream, dd, kind, p0, nb, j);
        });
      }
    }
    const int act = active(p0);
    int gx = 0;
    double fl = 0, by = 0;
    for (int i = 0; i < act; ++i) {
      const HostFactor &h = fs[order[i]];
      gx = std::max(gx, tiles_for(h.d, KIND_TRAIL, p0, nb, p0, 128));
      const int pend = std::min(p0 + nb, h.d.nf);
      const double kr = std::max(0, std::min(pend, h.n_real) - p0);
      const double nc = count_cols_real(h, pend, h.d.ncols), nr = count_rows_real(h, pend);
      if (nc > 0) {
        fl += 2.0 * trap_elems(nr, nc) * kr;
        by += 16.0 * trap_elems(nr, nc) + 8.0 * (nr + nc) * kr;
      }
    }
    if (gx > 0)
      ctx.launch(INLA_K_GEMM, fl, by, [&] {
        hipLaunchKernelGGL((gemm_update_kernel<128, 128>), dim3(gx, act), dim3(256), 0, ctx.stream, dd, KIND_TRAIL, p0,
                           nb, p0);
      });
  }
  return ctx.check();
}

}  // namespace inla
