// Stage 1 of the method around the batched Laplace evaluation: the mode theta*
// of log pi~(theta | y) by BFGS with central-difference gradients, the
// finite-difference Hessian at theta*, and the central composite design (CCD)
// points and weights used to explore the hyperparameter space (section
// "Hyperparameter exploration"; appendix "Marginal posteriors of the
// hyperparameters", Eq. (41) and the z-parameterisation that follows it).
//
// Host code only: every objective value comes from inla_laplace_eval (or, on the
// Moore-Penrose route, from inla_woodbury_eval after Q_prior(theta)^+ is
// assembled from the prior's block pseudo-inverses), and every gradient, line
// search and Hessian stencil is one batched call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "../../include/inla_dense.h"
#include "host.hpp"

namespace inla {
hipStream_t handle_stream(inla_handle *h);
}

namespace {

// f(theta) = -(log pi~(y | theta) + log pi(theta)) over batches of theta; each
// batch starts its Newton iterations from the mode at the current centre.
struct Evaluator {
  inla_handle *h;
  const inla_model *model;
  int t, n;
  inla_opts eo;
  inla_log_prior_fn lp;
  void *user;
  double *xbuf = nullptr;   // device [cap + 1][n]: one mode per point, then the centre's
  int cap = 0;
  bool have_centre = false;
  int evals = 0;
  // Moore-Penrose route: the prior's block pseudo-inverses, and device room for
  // Q_prior(theta)^+ of each point of a batch ([qcap][n][n])
  const inla_pinv_prior *pp = nullptr;
  double *qbuf = nullptr;
  int qcap = 0;

  ~Evaluator() {
    if (xbuf || qbuf) (void)hipStreamSynchronize(inla::handle_stream(h));
    if (xbuf) (void)hipFree(xbuf);
    if (qbuf) (void)hipFree(qbuf);
  }
  int ensure_q(int B) {
    if (B <= qcap) return INLA_OK;
    if (qbuf) {
      if (hipStreamSynchronize(inla::handle_stream(h)) != hipSuccess) return INLA_ERR_HIP;
      (void)hipFree(qbuf);
      qbuf = nullptr;
      qcap = 0;
    }
    if (hipMalloc(&qbuf, sizeof(double) * (size_t)B * n * n) != hipSuccess) {
      (void)hipGetLastError();
      qbuf = nullptr;
      return INLA_ERR_NOMEM;
    }
    qcap = B;
    return INLA_OK;
  }
  double *centre() { return xbuf + (size_t)cap * n; }
  int ensure(int B) {
    if (B <= cap) return INLA_OK;
    double *nb = nullptr;
    if (hipMalloc(&nb, sizeof(double) * (size_t)(B + 1) * n) != hipSuccess) {
      (void)hipGetLastError();
      return INLA_ERR_NOMEM;
    }
    hipStream_t s = inla::handle_stream(h);
    if (xbuf) {
      if (have_centre &&
          hipMemcpyAsync(nb + (size_t)B * n, centre(), sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return INLA_ERR_HIP;
      if (hipStreamSynchronize(s) != hipSuccess) return INLA_ERR_HIP;
      (void)hipFree(xbuf);
    }
    xbuf = nb;
    cap = B;
    return INLA_OK;
  }
  // f[b] for the B rows of th (row-major, stride t); +inf where the evaluation failed
  int eval(int B, const double *th, double *f) {
    int rc = ensure(B);
    if (rc) return rc;
    hipStream_t s = inla::handle_stream(h);
    std::vector<double *> xs(B);
    for (int b = 0; b < B; ++b) {
      xs[b] = xbuf + (size_t)b * n;
      if (have_centre &&
          hipMemcpyAsync(xs[b], centre(), sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return INLA_ERR_HIP;
    }
    std::vector<inla_model> ms(B, *model);
    std::vector<inla_result> r(B);
    inla_opts o = eo;
    o.start = have_centre ? 1 : 0;
    if (pp) {
      if ((rc = ensure_q(B))) return rc;
      std::vector<double *> qs(B);
      std::vector<double> lik(B);
      for (int b = 0; b < B; ++b) {
        qs[b] = qbuf + (size_t)b * n * n;
        ms[b].Qprior = qs[b];
        ms[b].ldq = n;
        lik[b] = pp->lik_index >= 0 ? th[(size_t)b * t + pp->lik_index] : pp->lik_value;
      }
      if ((rc = inla::pinv_prior_assemble(*inla::handle_ctx(h), *pp, n, B, th, t, qs.data()))) return rc;
      rc = inla_woodbury_eval(h, B, ms.data(), lik.data(), 1, xs.data(), &o, r.data());
    } else {
      rc = inla_laplace_eval(h, B, ms.data(), th, t, xs.data(), &o, r.data());
    }
    if (rc) return rc;
    for (int b = 0; b < B; ++b) {
      const double prior = lp ? lp(th + (size_t)b * t, t, user) : 0.0;
      f[b] = (r[b].info == 0 && std::isfinite(r[b].objective) && std::isfinite(prior))
                 ? -(r[b].objective + prior)
                 : std::numeric_limits<double>::infinity();
    }
    evals += B;
    return INLA_OK;
  }
  // the mode of point b of the last batch becomes the centre's
  int set_centre(int b) {
    if (hipMemcpyAsync(centre(), xbuf + (size_t)b * n, sizeof(double) * n, hipMemcpyDeviceToDevice,
                       inla::handle_stream(h)) != hipSuccess)
      return INLA_ERR_HIP;
    have_centre = true;
    return INLA_OK;
  }
};

// Central-difference gradient at theta from the 2t points theta +- h e_i.
int gradient(Evaluator &ev, const std::vector<double> &th, double h, std::vector<double> &g) {
  const int t = ev.t;
  std::vector<double> pts(2 * t * t), f(2 * t);
  for (int i = 0; i < t; ++i)
    for (int s = 0; s < 2; ++s) {
      double *p = &pts[(size_t)(2 * i + s) * t];
      std::copy(th.begin(), th.end(), p);
      p[i] += s ? -h : h;
    }
  int rc = ev.eval(2 * t, pts.data(), f.data());
  if (rc) return rc;
  g.assign(t, 0.0);
  for (int i = 0; i < t; ++i) g[i] = (f[2 * i] - f[2 * i + 1]) / (2.0 * h);
  for (double v : g)
    if (!std::isfinite(v)) return 1;
  return INLA_OK;
}

int n_prior_params(int prior) { return prior == INLA_PRIOR_DENSE ? 0 : (prior == INLA_PRIOR_EXPCOV ? 2 : 3); }

}  // namespace

namespace inla {

// Symmetric eigen-decomposition of a small matrix (cyclic Jacobi rotations):
// A (t x t, row-major) = V diag(w) V^T, V's columns the eigenvectors.
void sym_eigen(int t, std::vector<double> A, std::vector<double> &w, std::vector<double> &V) {
  V.assign((size_t)t * t, 0.0);
  for (int i = 0; i < t; ++i) V[(size_t)i * t + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < t; ++i)
      for (int j = 0; j < t; ++j) {
        tot += A[(size_t)i * t + j] * A[(size_t)i * t + j];
        if (i != j) off += A[(size_t)i * t + j] * A[(size_t)i * t + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < t; ++p)
      for (int q = p + 1; q < t; ++q) {
        const double apq = A[(size_t)p * t + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * t + p], aqq = A[(size_t)q * t + q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double tn = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + tn * tn), s = tn * c;
        for (int k = 0; k < t; ++k) {   // A <- J^T A J with the rotation in plane (p, q)
          const double akp = A[(size_t)k * t + p], akq = A[(size_t)k * t + q];
          A[(size_t)k * t + p] = c * akp - s * akq;
          A[(size_t)k * t + q] = s * akp + c * akq;
        }
        for (int k = 0; k < t; ++k) {
          const double apk = A[(size_t)p * t + k], aqk = A[(size_t)q * t + k];
          A[(size_t)p * t + k] = c * apk - s * aqk;
          A[(size_t)q * t + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < t; ++k) {
          const double vkp = V[(size_t)k * t + p], vkq = V[(size_t)k * t + q];
          V[(size_t)k * t + p] = c * vkp - s * vkq;
          V[(size_t)k * t + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(t);
  for (int i = 0; i < t; ++i) w[i] = A[(size_t)i * t + i];
}

// Gauss-Hermite rule of d points for the weight e^{-z^2} (Golub-Welsch: the
// nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix with
// off-diagonal sqrt(k / 2), the weights sqrt(pi) times the squared first
// components of its normalised eigenvectors).  Returns d nodes, then the d
// weights divided by sqrt(pi) (they sum to 1).
std::vector<double> gauss_hermite(int d) {
  std::vector<double> J((size_t)d * d, 0.0), w, V;
  for (int k = 1; k < d; ++k) J[(size_t)(k - 1) * d + k] = J[(size_t)k * d + k - 1] = std::sqrt(0.5 * k);
  sym_eigen(d, J, w, V);
  std::vector<double> out(2 * (size_t)d);
  for (int j = 0; j < d; ++j) {
    out[j] = w[j];
    out[d + j] = V[j] * V[j];   // first row of V
  }
  return out;
}

}  // namespace inla

using inla::sym_eigen;

namespace {

// BFGS for the mode of log pi~(theta | y) with the evaluator's route.
int theta_mode_run(Evaluator &ev, int32_t t, const double *theta0, const inla_theta_opts *opts, double *theta_star,
                   double *f_star, double *grad, int32_t *iters, int32_t *evals, int32_t *info) {
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 100;
  const double hd = (opts && opts->h > 0) ? opts->h : 1e-3;
  const double gtol = (opts && opts->gtol > 0) ? opts->gtol : 1e-3;
  const double ftol = (opts && opts->ftol > 0) ? opts->ftol : 1e-12;
  const double max_step = (opts && opts->max_step > 0) ? opts->max_step : 1.0;
  int status = INLA_THETA_MAXIT, it = 0;
  std::vector<double> th(theta0, theta0 + t), g, gn, Hi((size_t)t * t, 0.0);
  double f = 0.0;
  int rc = ev.eval(1, th.data(), &f);
  if (rc) return rc;
  if (!std::isfinite(f)) {
    status = INLA_THETA_EVAL_FAILED;
  } else {
    if ((rc = ev.set_centre(0))) return rc;
    rc = gradient(ev, th, hd, g);
    if (rc < 0) return rc;
    if (rc) status = INLA_THETA_EVAL_FAILED;
  }
  for (int i = 0; i < t; ++i) Hi[(size_t)i * t + i] = 1.0;
  bool scaled = false;
  while (status == INLA_THETA_MAXIT && it < max_iter) {
    double gn_inf = 0.0;
    for (double v : g) gn_inf = std::max(gn_inf, std::fabs(v));
    if (gn_inf <= gtol) { status = INLA_THETA_OK; break; }
    ++it;
    // quasi-Newton direction; steepest descent if it is not a descent direction
    std::vector<double> p(t, 0.0);
    double gp = 0.0;
    for (int i = 0; i < t; ++i) {
      for (int j = 0; j < t; ++j) p[i] -= Hi[(size_t)i * t + j] * g[j];
      gp += g[i] * p[i];
    }
    if (!(gp < 0.0)) {
      for (int i = 0; i < t; ++i) {
        for (int j = 0; j < t; ++j) Hi[(size_t)i * t + j] = i == j;
        p[i] = -g[i];
      }
      gp = 0.0;
      for (int i = 0; i < t; ++i) gp += g[i] * p[i];
      scaled = false;
    }
    double pinf = 0.0;
    for (double v : p) pinf = std::max(pinf, std::fabs(v));
    if (pinf > max_step)
      for (double &v : p) v *= max_step / pinf;
    if (pinf > max_step) gp *= max_step / pinf;
    // backtracking line search (Armijo, c1 = 1e-4), four step lengths per batch
    constexpr int NA = 4;
    double alpha = 0.0, fa = 0.0;
    int chosen = -1;
    for (int round = 0; round < 3 && chosen < 0; ++round) {
      std::vector<double> pts((size_t)NA * t), fs(NA), al(NA);
      for (int a = 0; a < NA; ++a) {
        al[a] = std::ldexp(1.0, -(round * NA + a));
        for (int i = 0; i < t; ++i) pts[(size_t)a * t + i] = th[i] + al[a] * p[i];
      }
      if ((rc = ev.eval(NA, pts.data(), fs.data()))) return rc;
      for (int a = 0; a < NA && chosen < 0; ++a)
        if (fs[a] <= f + 1e-4 * al[a] * gp) { chosen = a; alpha = al[a]; fa = fs[a]; }
    }
    if (chosen < 0) { status = INLA_THETA_LINESEARCH; break; }
    if ((rc = ev.set_centre(chosen))) return rc;
    std::vector<double> thn(t), s(t), y(t);
    for (int i = 0; i < t; ++i) { thn[i] = th[i] + alpha * p[i]; s[i] = thn[i] - th[i]; }
    rc = gradient(ev, thn, hd, gn);
    if (rc < 0) return rc;
    if (rc) { status = INLA_THETA_EVAL_FAILED; break; }
    double sy = 0.0, yy = 0.0, ss = 0.0;
    for (int i = 0; i < t; ++i) {
      y[i] = gn[i] - g[i];
      sy += s[i] * y[i];
      yy += y[i] * y[i];
      ss += s[i] * s[i];
    }
    if (sy > 1e-12 * std::sqrt(ss * yy)) {
      if (!scaled) {   // initial inverse-Hessian scaling of the first update
        for (int i = 0; i < t; ++i)
          for (int j = 0; j < t; ++j) Hi[(size_t)i * t + j] = i == j ? sy / yy : 0.0;
        scaled = true;
      }
      // Hi <- (I - rho s y^T) Hi (I - rho y s^T) + rho s s^T
      const double rho = 1.0 / sy;
      std::vector<double> Hy(t, 0.0), yH(t, 0.0);
      double yHy = 0.0;
      for (int i = 0; i < t; ++i)
        for (int j = 0; j < t; ++j) {
          Hy[i] += Hi[(size_t)i * t + j] * y[j];
          yH[j] += y[i] * Hi[(size_t)i * t + j];
        }
      for (int i = 0; i < t; ++i) yHy += y[i] * Hy[i];
      for (int i = 0; i < t; ++i)
        for (int j = 0; j < t; ++j)
          Hi[(size_t)i * t + j] += -rho * (Hy[i] * s[j] + s[i] * yH[j]) + (rho * rho * yHy + rho) * s[i] * s[j];
    }
    const double df = f - fa;
    th = thn;
    f = fa;
    g = gn;
    if (df <= ftol * std::max(1.0, std::fabs(f))) { status = INLA_THETA_OK; break; }
  }
  std::copy(th.begin(), th.end(), theta_star);
  if (f_star) *f_star = -f;
  if (grad)
    for (int i = 0; i < t; ++i) grad[i] = i < (int)g.size() ? -g[i] : 0.0;
  if (iters) *iters = it;
  if (evals) *evals = ev.evals;
  if (info) *info = status;
  return INLA_OK;
}

// Central-difference negative Hessian of log pi~(theta | y) with the evaluator's route.
int theta_hessian_run(Evaluator &ev, int32_t t, const double *theta, double step, double *neg_hess, double *log_post,
                      int32_t *info) {
  double f0 = 0.0;
  int rc = ev.eval(1, theta, &f0);
  if (rc) return rc;
  if (info) *info = INLA_THETA_OK;
  if (!std::isfinite(f0)) {
    if (info) *info = INLA_THETA_EVAL_FAILED;
    return INLA_OK;
  }
  if ((rc = ev.set_centre(0))) return rc;
  // stencil: theta +- h e_i (2t), theta + h (s_i e_i + s_j e_j) for i < j and
  // the four sign pairs (2t(t-1)); with the centre 1 + 2t^2 evaluations
  std::vector<double> pts;
  auto add = [&](int i, double si, int j, double sj) {
    for (int k = 0; k < t; ++k) pts.push_back(theta[k]);
    double *p = &pts[pts.size() - t];
    p[i] += si * step;
    if (j >= 0) p[j] += sj * step;
  };
  for (int i = 0; i < t; ++i) { add(i, 1, -1, 0); add(i, -1, -1, 0); }
  for (int i = 0; i < t; ++i)
    for (int j = i + 1; j < t; ++j) {
      add(i, 1, j, 1); add(i, 1, j, -1); add(i, -1, j, 1); add(i, -1, j, -1);
    }
  const int P = (int)(pts.size() / t);
  std::vector<double> f(P);
  if ((rc = ev.eval(P, pts.data(), f.data()))) return rc;
  for (double v : f)
    if (!std::isfinite(v)) {
      if (info) *info = INLA_THETA_EVAL_FAILED;
      return INLA_OK;
    }
  const double h2 = step * step;
  for (int i = 0; i < t; ++i) neg_hess[(size_t)i * t + i] = (f[2 * i] - 2.0 * f0 + f[2 * i + 1]) / h2;
  int q = 2 * t;
  for (int i = 0; i < t; ++i)
    for (int j = i + 1; j < t; ++j) {
      const double v = (f[q] - f[q + 1] - f[q + 2] + f[q + 3]) / (4.0 * h2);
      neg_hess[(size_t)i * t + j] = neg_hess[(size_t)j * t + i] = v;
      q += 4;
    }
  if (log_post) *log_post = -f0;
  return INLA_OK;
}

}  // namespace

extern "C" {

int inla_theta_mode(inla_handle *h, const inla_model *model, int32_t t, const double *theta0,
                    const inla_theta_opts *opts, inla_log_prior_fn log_prior, void *user, double *theta_star,
                    double *f_star, double *grad, int32_t *iters, int32_t *evals, int32_t *info) {
  if (!h) return -1;
  if (!model) return -2;
  if (t != n_prior_params(model->prior) + 1) return -3;
  if (!theta0) return -4;
  if (!theta_star) return -8;
  for (int i = 0; i < t; ++i)
    if (!std::isfinite(theta0[i])) return -4;
  Evaluator ev{h, model, t, model->n, opts ? opts->eval : inla_opts{}, log_prior, user};
  ev.eo.start = 0;
  return theta_mode_run(ev, t, theta0, opts, theta_star, f_star, grad, iters, evals, info);
}

static bool pinv_model_ok(const inla_model *m) { return m->prior == INLA_PRIOR_PINV && m->k == 0 && m->n >= 1; }

int inla_theta_mode_pinv(inla_handle *h, const inla_model *model, const inla_pinv_prior *prior, int32_t t,
                         const double *theta0, const inla_theta_opts *opts, inla_log_prior_fn log_prior, void *user,
                         double *theta_star, double *f_star, double *grad, int32_t *iters, int32_t *evals,
                         int32_t *info) {
  if (!h) return -1;
  if (!model || !pinv_model_ok(model)) return -2;
  if (t < 1) return -4;
  if (inla::pinv_prior_check(prior, model->n, t)) return -3;
  if (!theta0) return -5;
  if (!theta_star) return -9;
  for (int i = 0; i < t; ++i)
    if (!std::isfinite(theta0[i])) return -5;
  Evaluator ev{h, model, t, model->n, opts ? opts->eval : inla_opts{}, log_prior, user};
  ev.eo.start = 0;
  ev.pp = prior;
  return theta_mode_run(ev, t, theta0, opts, theta_star, f_star, grad, iters, evals, info);
}

int inla_theta_hessian(inla_handle *h, const inla_model *model, int32_t t, const double *theta, double step,
                       const inla_opts *opts, inla_log_prior_fn log_prior, void *user, double *neg_hess,
                       double *log_post, int32_t *info) {
  if (!h) return -1;
  if (!model) return -2;
  if (t != n_prior_params(model->prior) + 1) return -3;
  if (!theta) return -4;
  if (!(step > 0)) step = 5e-3;
  if (!neg_hess) return -9;
  Evaluator ev{h, model, t, model->n, opts ? *opts : inla_opts{}, log_prior, user};
  ev.eo.start = 0;
  return theta_hessian_run(ev, t, theta, step, neg_hess, log_post, info);
}

int inla_theta_hessian_pinv(inla_handle *h, const inla_model *model, const inla_pinv_prior *prior, int32_t t,
                            const double *theta, double step, const inla_opts *opts, inla_log_prior_fn log_prior,
                            void *user, double *neg_hess, double *log_post, int32_t *info) {
  if (!h) return -1;
  if (!model || !pinv_model_ok(model)) return -2;
  if (t < 1) return -4;
  if (inla::pinv_prior_check(prior, model->n, t)) return -3;
  if (!theta) return -5;
  if (!(step > 0)) step = 5e-3;
  if (!neg_hess) return -10;
  Evaluator ev{h, model, t, model->n, opts ? *opts : inla_opts{}, log_prior, user};
  ev.eo.start = 0;
  ev.pp = prior;
  return theta_hessian_run(ev, t, theta, step, neg_hess, log_post, info);
}

int inla_ccd_design(int32_t t, double f0, int32_t *n_points, double *z, double *delta) {
  if (t < 1 || t > INLA_CCD_MAX_T) return -1;
  if (!(f0 > 1.0)) return -2;
  if (!n_points) return -3;
  // factorial part: full 2^t for t <= 4, the half fraction with the last factor
  // the product of the others (defining relation I = 12...t, resolution t) for
  // t >= 5; none for t = 1, whose corners would be the axial points
  const int nf = t == 1 ? 0 : (t <= 4 ? 1 << t : 1 << (t - 1));
  const int np = 1 + 2 * t + nf;
  const bool query = !z && !delta;
  if (!query && (!z || !delta)) return -4;
  if (!query && *n_points < np) {
    *n_points = np;
    return -3;
  }
  *n_points = np;
  if (query) return INLA_OK;
  const double r = f0 * std::sqrt((double)t);
  std::fill(z, z + (size_t)np * t, 0.0);
  int k = 1;
  for (int i = 0; i < t; ++i)
    for (int s = 0; s < 2; ++s, ++k) z[(size_t)k * t + i] = s ? -r : r;
  const int free_bits = t <= 4 ? t : t - 1;
  for (int m = 0; m < nf; ++m, ++k) {
    double prod = 1.0;
    for (int i = 0; i < free_bits; ++i) {
      const double sgn = (m >> i) & 1 ? -1.0 : 1.0;
      z[(size_t)k * t + i] = f0 * sgn;
      prod *= sgn;
    }
    if (free_bits < t) z[(size_t)k * t + t - 1] = f0 * prod;
  }
  // weights that integrate a standard Gaussian's mass, mean and covariance
  // exactly: a point on the sphere |z| = r gets exp(r^2 / 2) / (f0^2 (np - 1)),
  // the centre 1 - 1 / f0^2 (relative to the density's value at each point)
  delta[0] = 1.0 - 1.0 / (f0 * f0);
  for (int j = 1; j < np; ++j) delta[j] = std::exp(0.5 * r * r) / (f0 * f0 * (np - 1));
  return INLA_OK;
}

int inla_ccd_points(int32_t t, const double *theta_star, const double *neg_hess, double f0, int32_t *n_points,
                    double *theta_k, double *delta) {
  if (t < 1 || t > INLA_CCD_MAX_T) return -1;
  if (!theta_star) return -2;
  if (!neg_hess) return -3;
  if (!n_points || !theta_k || !delta) return -6;
  std::vector<double> H(neg_hess, neg_hess + (size_t)t * t), w, V;
  for (int i = 0; i < t; ++i)
    for (int j = 0; j < t; ++j)
      if (!std::isfinite(H[(size_t)i * t + j])) return -3;
  for (int i = 0; i < t; ++i)   // symmetrise
    for (int j = i + 1; j < t; ++j)
      H[(size_t)i * t + j] = H[(size_t)j * t + i] = 0.5 * (H[(size_t)i * t + j] + H[(size_t)j * t + i]);
  sym_eigen(t, H, w, V);
  for (double v : w)
    if (!(v > 0.0)) return INLA_THETA_NOT_PD;
  int np = *n_points;
  std::vector<double> z((size_t)std::max(np, 1) * t);
  int rc = inla_ccd_design(t, f0, &np, z.data(), delta);
  *n_points = np;
  if (rc) return rc == -2 ? -4 : -5;
  // theta(z) = theta* + V Lambda^{1/2} z with Sigma = neg_hess^{-1} = V diag(1 / w) V^T
  for (int k = 0; k < np; ++k)
    for (int i = 0; i < t; ++i) {
      double v = theta_star[i];
      for (int j = 0; j < t; ++j) v += V[(size_t)i * t + j] * z[(size_t)k * t + j] / std::sqrt(w[j]);
      theta_k[(size_t)k * t + i] = v;
    }
  return INLA_OK;
}

int inla_ccd_weights(int32_t n_points, const double *delta, const double *log_post, double *weights) {
  if (n_points < 1) return -1;
  if (!delta) return -2;
  if (!log_post) return -3;
  if (!weights) return -4;
  double m = -std::numeric_limits<double>::infinity();
  for (int k = 0; k < n_points; ++k) m = std::max(m, log_post[k]);
  if (!std::isfinite(m)) return -3;
  double s = 0.0;
  for (int k = 0; k < n_points; ++k) {
    weights[k] = std::isfinite(log_post[k]) ? delta[k] * std::exp(log_post[k] - m) : 0.0;
    s += weights[k];
  }
  for (int k = 0; k < n_points; ++k) weights[k] /= s;
  return INLA_OK;
}

}  // extern "C"
