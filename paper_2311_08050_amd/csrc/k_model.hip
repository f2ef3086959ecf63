// Model assembly kernels: prior precision builders, the bordered Q* / b
// assembly with the likelihood terms, the kriging-system build, and the FP64
// residuals of the constrained Newton system used by mixed-precision
// refinement.
#include "device.hpp"
#include "host.hpp"
#include "model.hpp"

namespace inla {

// Sigma_ij = exp(-||p_i - p_j|| / rho) for the first n_s points, identity padded
// to ns_pad, bordered below by the identity (rows ns_pad + i = e_i).  Factoring
// the first ns_pad columns leaves -Sigma^{-1} in the Schur block.  The prior of
// the exponential-covariance models is tau Sigma^{-1}.  Always FP64.
__global__ __launch_bounds__(256) void expcov_bordered_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  const int np = t.ns_pad, N = t.Np;
  if (c >= N) return;
  const int ns = t.prior == PRIOR_EXPCOV ? t.n : t.n_s;
  double *col = t.P + (size_t)c * t.ldp;
  const double inv_rho = 1.0 / t.rho;
  double px = 0.0, py = 0.0;
  if (c < ns) { px = t.coords[2 * c]; py = t.coords[2 * c + 1]; }
  for (int r = c + threadIdx.x; r < N; r += 256) {
    double v = 0.0;
    if (c < np) {
      if (r < np) {
        if (r < ns && c < ns) {
          const double dx = t.coords[2 * r] - px, dy = t.coords[2 * r + 1] - py;
          v = exp(-sqrt(dx * dx + dy * dy) * inv_rho);
        } else if (r == c) {
          v = 1.0;
        }
      } else if (r - np == c) {
        v = 1.0;
      }
    }
    col[r] = v;
  }
}

// Q_prior from -Sigma^{-1} left in the Schur block of P:
//   EXPCOV: Q = tau Sigma^{-1};
//   KRON:   Q[t1 n_s + s1, t2 n_s + s2] = tau (R_t[t1,t2] Sigma_s^{-1}[s1,s2] + delta [i == j]),
//           R_t the unscaled first-order random walk (tridiagonal 1,2,..,2,1 / -1);
//   DENSE:  copy of the caller's matrix (its lower triangle).
// Only the lower triangle (rows r >= c of column c) is written: the assembly
// and the lower-triangle products read no more.  Identity on padded diagonal
// entries; one workgroup per column.
__global__ __launch_bounds__(256) void prior_assemble_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= t.n_pad) return;
  double *col = t.Qp + (size_t)c * t.ldqp;
  const int n = t.n;
  if (c >= n) {
    for (int r = c + threadIdx.x; r < t.n_pad; r += 256) col[r] = (r == c) ? 1.0 : 0.0;
    return;
  }
  if (t.prior == PRIOR_DENSE) {
    for (int r = c + threadIdx.x; r < t.n_pad; r += 256) col[r] = r < n ? t.Quser[(size_t)c * t.ldquser + r] : 0.0;
  } else if (t.prior == PRIOR_EXPCOV) {
    const double *Sn = t.P + (size_t)t.ns_pad * t.ldp + t.ns_pad;  // -Sigma^{-1}, lower
    for (int r = c + threadIdx.x; r < t.n_pad; r += 256) col[r] = r < n ? -t.tau * Sn[(size_t)c * t.ldp + r] : 0.0;
  } else {
    const int ns = t.n_s, nt = t.n_t;
    const int t2 = c / ns, s2 = c % ns;
    const double *Sn = t.P + (size_t)t.ns_pad * t.ldp + t.ns_pad;  // -Sigma_s^{-1}, lower
    for (int r = c + threadIdx.x; r < t.n_pad; r += 256) {
      double v = 0.0;
      if (r < n) {
        const int t1 = r / ns, s1 = r % ns;
        double R = 0.0;
        if (t1 == t2) R = (nt == 1) ? 0.0 : ((t1 == 0 || t1 == nt - 1) ? 1.0 : 2.0);
        else if (t1 - t2 == 1 || t2 - t1 == 1) R = -1.0;
        if (R != 0.0) {
          const int a = s1 > s2 ? s1 : s2, b = s1 > s2 ? s2 : s1;
          v = -R * Sn[(size_t)b * t.ldp + a];
        }
        if (r == c) v += t.delta;
        v *= t.tau;
      }
      col[r] = v;
    }
  }
}

__device__ __forceinline__ void lik_point_at(const ThetaDesc &t, int i, double x, double &g, double &W, double &ll) {
  const double y = t.y[i];
  if (t.lik == LIK_GAUSSIAN) {
    const double s2 = t.lpar;
    const double r = y - x;
    g = r / s2;
    W = 1.0 / s2;
    ll = -0.5 * log(2.0 * M_PI * s2) - r * r / (2.0 * s2);
  } else {
    const double E = t.E ? t.E[i] : 1.0;
    const double eta = t.lpar + x;
    const double mu = E * exp(eta);
    g = y - mu;
    W = mu;
    ll = y * (log(E) + eta) - mu - lgamma(y + 1.0);
  }
}

// g = d log pi(y_i | eta) / d eta and W = -d^2 log pi / d eta^2 at eta(x); in a
// variational-Bayes pass their expectations over eta ~ N(eta(x), vb_var[i])
// (appendix "Variational Bayes approximation strategy": I' = -E g, I'' = E W),
// by Gauss-Hermite quadrature: E h = sum_j w_j / sqrt(pi) h(eta + sqrt(2 var) r_j).
__device__ __forceinline__ void lik_point(const ThetaDesc &t, int i, double x, double &g, double &W, double &ll) {
  lik_point_at(t, i, x, g, W, ll);
  if (!t.vb_var) return;
  const double sd = sqrt(2.0 * t.vb_var[i]);
  double eg = 0.0, ew = 0.0;
  for (int j = 0; j < t.ngh; ++j) {
    double gj, wj, lj;
    lik_point_at(t, i, x + sd * t.gh[j], gj, wj, lj);
    eg += t.gh[t.ngh + j] * gj;
    ew += t.gh[t.ngh + j] * wj;
  }
  g = eg;
  W = ew;
}

// Per observation of a model with a general design matrix: (A x)_i by the CSR
// row, then the likelihood terms at eta_i = offset + (A x)_i.
__global__ __launch_bounds__(256) void obs_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (t.m == 0 || i >= t.m) return;
  double ax = 0.0;
  for (int p = t.A_rowptr[i]; p < t.A_rowptr[i + 1]; ++p) ax += t.A_val[p] * t.x[t.A_col[p]];
  double g, W, ll;
  lik_point_at(t, i, ax, g, W, ll);
  t.obs_ax[i] = ax;
  t.obs_g[i] = g;
  t.obs_W[i] = W;
  t.obs_ll[i] = ll;
}

// The bordered posterior precision of one Newton step (algorithm "Gaussian
// Approximation": Q* = Q_prior + Q_l(x0), b = grad + Q_l x0; A = I so Q_l is the
// diagonal W), written in the factorisation's storage type T:
//   rows [0, n_pad)          Q_prior + diag(W)            (lower)
//   rows n_pad + a, a < k    constraint row C_a
//   row  n_pad + k           b^T                 (border == BORDER_CB)
//   rows n_pad + kc_pad + i  e_i^T               (border == BORDER_CI)
// Schur-block columns start at zero.  `with_lik` = 0 gives the prior pass
// (W = 0, b = 0).  Per-column partial sums of log pi(y|eta) and x^T Q_prior x go
// to t.part for a fixed-order reduction.
template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(const ThetaDesc *__restrict__ td, int with_lik, int want_xqx,
                                                       int border) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  const int N = t.Nw;
  if (c >= t.Ncw) return;
  T *col = (T *)t.W + (size_t)c * t.ldw;
  const int np = t.n_pad, n = t.n, k = t.k;
  __shared__ double sh[4];
  if (c >= np) {
    for (int r = c + threadIdx.x; r < N; r += 256) col[r] = (T)0;
    return;
  }
  double g = 0.0, W = 0.0, ll = 0.0, xc = 0.0, bc = 0.0;
  if (c < n) {
    xc = t.x[c];
    if (with_lik && t.m == 0) lik_point(t, c, xc, g, W, ll);
  }
  if (with_lik && t.m == 0) {
    bc = g + W * xc;
  } else if (with_lik && c < n) {
    // b_c = (A^T (g + W A x))_c over the CSC column, fixed-order block sum
    double s = 0.0;
    for (int p = t.cscp[c] + threadIdx.x; p < t.cscp[c + 1]; p += 256) {
      const int i = t.csci[p];
      s += t.cscv[p] * (t.obs_g[i] + t.obs_W[i] * t.obs_ax[i]);
    }
    bc = block_sum256(s, sh);
  }
  const double *q = t.Qp + (size_t)c * t.ldqp;
  const int kc_pad = round_up_dev(k, PADN);
  double xq = 0.0;
  // Four rows per thread and pass, their loads issued before any store (the
  // stores to the working matrix may alias the prior for the compiler, which
  // would otherwise keep one load in flight per thread).  Each thread still
  // visits its rows in increasing order, so the x^T Q x partial sums keep
  // their order.
  constexpr int U = 4;
  for (int rb = c + threadIdx.x; rb < N; rb += 256 * U) {
    double qv[U], xr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = rb + 256 * u;
      qv[u] = r < np ? q[r] : 0.0;
      xr[u] = (want_xqx && r < n) ? t.x[r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = rb + 256 * u;
      if (r >= N) break;
      double v;
      if (r < np) {
        v = qv[u] + (r == c ? W : 0.0);
        if (want_xqx && r < n) xq += (r == c ? 1.0 : 2.0) * qv[u] * xr[u];
      } else {
        const int a = r - np;
        if (a < k) v = (c < n) ? t.C[(size_t)a * n + c] : 0.0;
        else if (border == BORDER_CB) v = (a == k) ? bc : 0.0;
        else v = (a - kc_pad == c) ? 1.0 : 0.0;
      }
      col[r] = (T)v;
    }
  }
  if (want_xqx) {
    xq = block_sum256(xq, sh);
    if (threadIdx.x == 0) t.part[t.ldw + c] = xq * xc;
  }
  if (with_lik && t.m > 0 && c < n) {
    // + (A^T W A)_{r c} for the lower pattern entries of column c (distinct rows)
    __syncthreads();
    double bad = 0.0;
    for (int e = t.patp[c] + threadIdx.x; e < t.patp[c + 1]; e += 256) {
      double v = 0.0;
      for (int q = t.patt[e]; q < t.patt[e + 1]; ++q) v += t.tcoef[q] * t.obs_W[t.tobs[q]];
      if (!isfinite(v)) bad = 1.0;
      const int r = t.patr[e];
      col[r] = (T)((double)col[r] + v);
    }
    bad = block_sum256(bad, sh);
    if (threadIdx.x == 0 && bad > 0.0) t.dres[DRES_NONFINITE] = 1.0;
  }
  if (threadIdx.x == 0) {
    t.part[c] = ll;
    if (!isfinite(W) || !isfinite(bc)) t.dres[DRES_NONFINITE] = 1.0;
  }
}

// Kriging system from the Schur block -[[S, C x_u], [., b^T x_u]] of the big
// factorisation: S into rows/cols [0, k) (identity padded to k_pad) and the
// border row (C x_u - e)^T at row k_pad, always in FP64.  Factoring it leaves
// L_S and w^T = (C x_u - e)^T L_S^{-T} in the border row.
template <typename T>
__global__ __launch_bounds__(256) void kriging_build_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  const int kp = t.k_pad, N = t.Ns, k = t.k;
  if (c >= kp) return;   // only the k_pad factor columns exist; the border is a row
  double *col = t.S + (size_t)c * t.lds;
  const T *sch = (const T *)t.W + (size_t)(t.n_pad + c) * t.ldw + t.n_pad;
  for (int r = c + threadIdx.x; r < N; r += 256) {
    double v = 0.0;
    if (r < kp) {
      if (r < k && c < k) v = -(double)sch[r];
      else if (r == c) v = 1.0;
    } else if (r == kp && c < k) {
      const double e = t.e ? t.e[c] : 0.0;
      v = -(double)sch[k] - e;   // C x_u - e (Schur holds -C Q^{-1} b = -C x_u)
    }
    col[r] = v;
  }
}

// y = Q_prior v from the lower triangle of Q_prior alone (half the bytes of a
// whole-column product; the consumers below finish it).  Block (J, theta) takes
// the 64 columns [64 J, 64 J + 64) and walks the 64-row tiles at and below the
// diagonal through LDS: row r of a tile receives sum_{c in J, c <= r} Q_rc v_c,
// written to P[J][r]; column c receives sum_{r > c} Q_rc v_r, summed over the
// tiles in registers and written to D[c].  Then (Q v)_i = D[i] + sum over
// J <= i / 64 of P[J][i], in that order (no atomics: fixed summation order).
// src 0: v = xn (refinement residuals); 1: v = x (objective terms).
__global__ __launch_bounds__(256) void symv_lower_part_kernel(const ThetaDesc *__restrict__ td, int src) {
  const ThetaDesc t = td[blockIdx.y];
  const int J = blockIdx.x, c0 = J * 64, np = t.n_pad, n = t.n;
  if (c0 >= np) return;
  const double *v = src ? t.x : t.xn;
  __shared__ double T[64][65];
  __shared__ double vc[64], vr[64];
  __shared__ double red[4][64];
  const int tid = threadIdx.x, lo = tid & 63, part = tid >> 6;
  double *P = t.symv;
  double *D = t.symv + (size_t)(np / 64) * np;
  if (tid < 64) vc[tid] = c0 + tid < n ? v[c0 + tid] : 0.0;
  const double *Qc = t.Qp + (size_t)c0 * t.ldqp;
  double dot = 0.0;
  // the next tile's 16 loads per thread are in flight while this tile is reduced
  double buf[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) buf[q] = Qc[(size_t)(part + 4 * q) * t.ldqp + c0 + lo];
  for (int r0 = c0; r0 < np; r0 += 64) {
    __syncthreads();   // the previous tile and its row sums are consumed
#pragma unroll
    for (int q = 0; q < 16; ++q) T[lo][part + 4 * q] = buf[q];
    if (r0 + 64 < np) {
#pragma unroll
      for (int q = 0; q < 16; ++q) buf[q] = Qc[(size_t)(part + 4 * q) * t.ldqp + r0 + 64 + lo];
    }
    if (tid < 64) vr[tid] = r0 + tid < n ? v[r0 + tid] : 0.0;
    __syncthreads();
    const bool diag = r0 == c0;
    double rs = 0.0;   // row lo, columns 16 part .. 16 part + 15
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = 16 * part + q;
      if (!diag || c <= lo) rs += T[lo][c] * vc[c];
    }
    red[part][lo] = rs;
#pragma unroll
    for (int q = 0; q < 16; ++q) {   // column lo, rows 16 part .. 16 part + 15
      const int r = 16 * part + q;
      if (!diag || r > lo) dot += T[r][lo] * vr[r];
    }
    __syncthreads();
    if (tid < 64) P[(size_t)J * np + r0 + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
  }
  __syncthreads();
  red[part][lo] = dot;
  __syncthreads();
  if (tid < 64) D[c0 + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// (Q_prior v)_i from the partial sums of symv_lower_part_kernel.
__device__ __forceinline__ double symv_row(const ThetaDesc &t, int i) {
  const int np = t.n_pad;
  double y = t.symv[(size_t)(np / 64) * np + i];
  for (int J = 0; J <= i / 64; ++J) y += t.symv[(size_t)J * np + i];
  return y;
}

// FP64 residual of the constrained Newton system at the refined iterate xn:
//   r1 = b - (Q_prior + diag W) xn - C^T lambda,   b = g(x) + W(x) x
// with g, W at the linearisation point x and Q_prior xn from the lower-triangle
// partial sums; one thread per row, the result to t.z.
__global__ __launch_bounds__(256) void kkt_residual_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= t.n_pad) return;
  double r = 0.0;
  if (i < t.n) {
    double s = symv_row(t, i);
    for (int a = 0; a < t.k; ++a) s += t.C[(size_t)a * t.n + i] * t.lam[a];
    double g, W, ll;
    lik_point(t, i, t.x[i], g, W, ll);
    r = (g + W * t.x[i]) - W * t.xn[i] - s;
  }
  t.z[i] = r;
}

// Objective terms at the mode without re-assembling: x^T Q_prior x (from the
// lower-triangle partial sums of Q_prior x) and log pi(y | eta) into the
// per-column partial sums read by the finish kernel.  Used when the last Newton
// factorisation is reused for log|Q*|.
__global__ __launch_bounds__(256) void objective_terms_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= t.n_pad) return;
  double ll = 0.0, xq = 0.0;
  if (i < t.n) {
    double g, W;
    lik_point(t, i, t.x[i], g, W, ll);
    xq = t.x[i] * symv_row(t, i);
  }
  t.part[i] = ll;
  t.part[t.ldw + i] = xq;
}

// r2 = e - C xn, one wave per constraint row (zero on padded rows).
__global__ __launch_bounds__(256) void constraint_residual_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a = blockIdx.x * 4 + w;
  if (a >= t.k_pad) return;
  double s = 0.0;
  if (a < t.k)
    for (int i = lane; i < t.n; i += 64) s += t.C[(size_t)a * t.n + i] * t.xn[i];
  s = wave_sum(s);
  if (lane == 0) t.rtwo[a] = a < t.k ? (t.e ? t.e[a] : 0.0) - s : 0.0;
}

// ------------------------------------------------------------------ launchers
void launch_expcov_bordered(Ctx &ctx, const ThetaDesc *dtd, int B, int Np_max) {
  if (B <= 0 || Np_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(expcov_bordered_kernel, dim3(Np_max, B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_prior_assemble(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, double bytes) {
  if (B <= 0 || np_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, bytes, [&] {
    hipLaunchKernelGGL(prior_assemble_kernel, dim3(np_max, B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_assemble(Ctx &ctx, const ThetaDesc *dtd, int B, int N_max, int with_lik, int want_xqx, int border,
                     double bytes, int prec, int m_max) {
  if (B <= 0 || N_max <= 0) return;
  if (with_lik && m_max > 0)
    ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(obs_kernel, dim3((m_max + 255) / 256, B), dim3(256), 0, ctx.stream, dtd);
    });
  ctx.launch(INLA_K_ASSEMBLE, 0.0, bytes, [&] {
    if (prec != INLA_PREC_FP64)
      hipLaunchKernelGGL(assemble_kernel<float>, dim3(N_max, B), dim3(256), 0, ctx.stream, dtd, with_lik, want_xqx,
                         border);
    else
      hipLaunchKernelGGL(assemble_kernel<double>, dim3(N_max, B), dim3(256), 0, ctx.stream, dtd, with_lik, want_xqx,
                         border);
  });
}
void launch_kriging_build(Ctx &ctx, const ThetaDesc *dtd, int B, int kp_max, int prec) {
  if (B <= 0 || kp_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    if (prec != INLA_PREC_FP64)
      hipLaunchKernelGGL(kriging_build_kernel<float>, dim3(kp_max, B), dim3(256), 0, ctx.stream, dtd);
    else
      hipLaunchKernelGGL(kriging_build_kernel<double>, dim3(kp_max, B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_objective_terms(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, double bytes) {
  if (B <= 0 || np_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, bytes, [&] {
    hipLaunchKernelGGL(symv_lower_part_kernel, dim3(np_max / 64, B), dim3(256), 0, ctx.stream, dtd, 1);
  });
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(objective_terms_kernel, dim3((np_max + 255) / 256, B), dim3(256), 0, ctx.stream, dtd);
  });
}
void launch_kkt_residual(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, int kp_max, double bytes) {
  if (B <= 0 || np_max <= 0) return;
  ctx.launch(INLA_K_SOLVE, 0.0, bytes, [&] {
    hipLaunchKernelGGL(symv_lower_part_kernel, dim3(np_max / 64, B), dim3(256), 0, ctx.stream, dtd, 0);
  });
  ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(kkt_residual_kernel, dim3((np_max + 255) / 256, B), dim3(256), 0, ctx.stream, dtd);
  });
  if (kp_max > 0)
    ctx.launch(INLA_K_SOLVE, 0.0, 0.0, [&] {
      hipLaunchKernelGGL(constraint_residual_kernel, dim3(kp_max / 4, B), dim3(256), 0, ctx.stream, dtd);
    });
}

}  // namespace inla
