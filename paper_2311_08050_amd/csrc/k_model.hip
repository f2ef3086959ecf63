// Model assembly kernels: prior precision builders, the bordered Q* / b
// assembly with the likelihood terms, and the kriging-system build.
#include "device.hpp"
#include "host.hpp"
#include "model.hpp"

namespace inla {

// Sigma_ij = exp(-||p_i - p_j|| / rho) for the first n_s points, identity padded
// to ns_pad, bordered below by the identity (rows ns_pad + i = e_i).  Factoring
// the first ns_pad columns leaves -Sigma^{-1} in the Schur block.  The prior of
// the exponential-covariance models is tau Sigma^{-1} (configurations of the
// Gaussian and space x time models).
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
//   DENSE:  copy of the caller's matrix.
// Lower triangle, identity on padded diagonal entries, one workgroup per column.
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
    const double *src = t.Quser + (size_t)c * t.ldquser;
    for (int r = c + threadIdx.x; r < t.n_pad; r += 256) col[r] = r < n ? src[r] : 0.0;
  } else if (t.prior == PRIOR_EXPCOV) {
    const double *src = t.P + (size_t)(t.ns_pad + c) * t.ldp + t.ns_pad;
    for (int r = c + threadIdx.x; r < t.n_pad; r += 256) col[r] = r < n ? -t.tau * src[r] : 0.0;
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
        else if (t1 - t2 == 1) R = -1.0;
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

__device__ __forceinline__ void lik_point(const ThetaDesc &t, int i, double x, double &g, double &W, double &ll) {
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

// The bordered posterior precision of one Newton step (algorithm "Gaussian
// Approximation": Q* = Q_prior + Q_l(x0), b = grad + Q_l x0; A = I so Q_l is the
// diagonal W):
//   rows [0, n_pad)          Q_prior + diag(W)            (lower)
//   rows n_pad + a, a < k    constraint row C_a
//   row  n_pad + k           b^T                 (border == BORDER_CB)
//   rows n_pad + kc_pad + i  e_i^T               (border == BORDER_CI)
// Schur-block columns start at zero.  `with_lik` = 0 gives the prior pass
// (W = 0, b = 0).  Per-column partial sums of log pi(y|eta) and x^T Q_prior x go
// to t.part for a fixed-order reduction.
__global__ __launch_bounds__(256) void assemble_kernel(const ThetaDesc *__restrict__ td, int with_lik, int want_xqx,
                                                       int border) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  const int N = t.Nw;
  if (c >= t.Ncw) return;
  double *col = t.W + (size_t)c * t.ldw;
  const int np = t.n_pad, n = t.n, k = t.k;
  __shared__ double sh[4];
  if (c >= np) {
    for (int r = c + threadIdx.x; r < N; r += 256) col[r] = 0.0;
    return;
  }
  double g = 0.0, W = 0.0, ll = 0.0, xc = 0.0;
  if (c < n) {
    xc = t.x[c];
    if (with_lik) lik_point(t, c, xc, g, W, ll);
  }
  const double bc = with_lik ? g + W * xc : 0.0;
  const double *q = t.Qp + (size_t)c * t.ldqp;
  const int kc_pad = round_up_dev(k, PADN);
  double xq = 0.0;
  for (int r = c + threadIdx.x; r < N; r += 256) {
    double v;
    if (r < np) {
      const double qv = q[r];
      v = qv + (r == c ? W : 0.0);
      if (want_xqx && r < n) xq += (r == c ? 1.0 : 2.0) * qv * t.x[r];
    } else {
      const int a = r - np;
      if (a < k) v = (c < n) ? t.C[(size_t)a * n + c] : 0.0;
      else if (border == BORDER_CB) v = (a == k) ? bc : 0.0;
      else v = (a - kc_pad == c) ? 1.0 : 0.0;
    }
    col[r] = v;
  }
  if (want_xqx) {
    xq = block_sum256(xq, sh);
    if (threadIdx.x == 0) t.part[t.ldw + c] = xq * xc;
  }
  if (threadIdx.x == 0) {
    t.part[c] = ll;
    if (!isfinite(W) || !isfinite(bc)) t.dres[DRES_NONFINITE] = 1.0;
  }
}

// Kriging system from the Schur block -[[S, C x_u], [., b^T x_u]] of the big
// factorisation: S into rows/cols [0, k) (identity padded to k_pad) and the
// border row (C x_u - e)^T at row k_pad.  Factoring it leaves L_S and
// w^T = (C x_u - e)^T L_S^{-T} in the border row.
__global__ __launch_bounds__(256) void kriging_build_kernel(const ThetaDesc *__restrict__ td) {
  const ThetaDesc t = td[blockIdx.y];
  const int c = blockIdx.x;
  const int kp = t.k_pad, N = t.Ns, k = t.k;
  if (c >= kp) return;   // only the k_pad factor columns exist; the border is a row
  double *col = t.S + (size_t)c * t.lds;
  const double *sch = t.W + (size_t)(t.n_pad + c) * t.ldw + t.n_pad;
  for (int r = c + threadIdx.x; r < N; r += 256) {
    double v = 0.0;
    if (r < kp) {
      if (r < k && c < k) v = -sch[r];
      else if (r == c) v = 1.0;
    } else if (r == kp && c < k) {
      const double e = t.e ? t.e[c] : 0.0;
      v = -sch[k] - e;   // C x_u - e (Schur holds -C Q^{-1} b = -C x_u)
    }
    col[r] = v;
  }
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
                     double bytes) {
  if (B <= 0 || N_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, bytes, [&] {
    hipLaunchKernelGGL(assemble_kernel, dim3(N_max, B), dim3(256), 0, ctx.stream, dtd, with_lik, want_xqx, border);
  });
}
void launch_kriging_build(Ctx &ctx, const ThetaDesc *dtd, int B, int Ns_max) {
  if (B <= 0 || Ns_max <= 0) return;
  ctx.launch(INLA_K_ASSEMBLE, 0.0, 0.0, [&] {
    hipLaunchKernelGGL(kriging_build_kernel, dim3(Ns_max, B), dim3(256), 0, ctx.stream, dtd);
  });
}

}  // namespace inla
