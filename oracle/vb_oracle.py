"""Plain reference of the variational-Bayes correction of the posterior mean
(TEST INFRASTRUCTURE ONLY: imported by ``tests/`` alone).

Appendix "Variational Bayes approximation strategy", algorithm "Correction of
Posterior Mean using Variational Bayes": with x | y, theta ~ N(mu + lambda, Q*^{-1})
and Q*, hence the marginal variances s_i^2 of the Laplace approximation, held
fixed, lambda minimises the second-order expansion of
    E[-log pi(y | eta)] + KLD(N(mu + lambda, Q*^{-1}) || N(0, Q_prior^{-1})),
eta_i ~ N(eta_i(mu), s_i^2).  Its minimiser solves
    (Q_prior + diag I'') lambda = -(I' + Q_prior mu),
I' = E[-d log pi / d eta], I'' = E[-d^2 log pi / d eta^2] at eta(mu), and
mu <- mu + lambda is repeated until the step is below the tolerance.  With the
constraints C x = e the correction is kriged so that C mu stays e.  Written in
the equivalent form of a Newton step, mu_new solves
    (Q_prior + diag I'') mu_new = I'' mu - I'   (then kriged).

The expectations are taken in closed form here (no quadrature): for the
Poisson likelihood E[E e^eta] = E e^(eta(mu) + s^2 / 2) (the log-normal mean),
for the Gaussian likelihood they equal the derivatives at eta(mu).  The library
uses Gauss-Hermite quadrature as the paper does.

Readings: the paper's c = (I'(0) A)^T + Q mu* with "solve Q^c lambda = c" has the
sign of the minimiser reversed (lambda = -(Q^c)^{-1} c minimises c^T lambda +
lambda^T Q^c lambda / 2), and its KLD omits the factor 1/2 on the quadratic
term; the minimiser above uses the standard Gaussian KLD.  A = I.
"""
from __future__ import annotations

import math

import numpy as np

from . import inla_oracle as O

VB_TOL = 1e-11
VB_MAX_ITER = 50


def expected_terms(model, theta, eta, var):
    """(-I', I''): E[d log pi(y|eta')/d eta'] and E[-d^2 log pi/d eta'^2] for
    eta' ~ N(eta, var), in closed form."""
    y = np.asarray(model["y"], dtype=np.float64)
    if model["lik"] == "gaussian":
        s2 = math.exp(O.lik_param(model, theta))
        return (y - eta) / s2, np.full_like(eta, 1.0 / s2)
    E = model.get("E")
    E = np.ones_like(eta) if E is None else np.asarray(E, dtype=np.float64)
    m = E * np.exp(eta + 0.5 * np.asarray(var, dtype=np.float64))
    return y - m, m


def vb_mean(model, theta, x_mode, var, tol=VB_TOL, max_iter=VB_MAX_ITER):
    """Corrected posterior mean.  Returns (mu, iterations, info)."""
    if O.design(model) is not None:
        raise ValueError("the correction is written for A = I")
    Qp = O.prior_precision(model, theta)
    C, e = O.constraint_of(model)
    mu = np.array(x_mode, dtype=np.float64)
    for it in range(1, max_iter + 1):
        eta = O.linear_predictor(model, theta, mu)
        g, W = expected_terms(model, theta, eta, var)
        L, info = O.cholesky(O.assemble(model, Qp, W, mu))
        if info:
            return mu, it, info
        new = O.chol_solve(L, O.rhs(model, g, W, mu))
        if C is not None:
            new, _, _, LS = O.kriging(L, new, C, e)
            if LS is None:
                return mu, it, O.INFO_CONSTRAINT_RANK
        step = float(np.max(np.abs(new - mu)))
        scale = max(1.0, float(np.max(np.abs(new))))
        mu = new
        if step <= tol * scale:
            return mu, it, O.INFO_OK
    return mu, max_iter, O.INFO_NEWTON_MAXIT


def vb_objective(model, theta, mu, var):
    """The quantity the correction minimises, up to terms free of mu:
    sum_i E[-log pi(y_i | eta_i)] + mu^T Q_prior mu / 2, eta_i ~ N(eta_i(mu), s_i^2),
    in closed form (Poisson: E e^eta = e^(eta + s^2/2); Gaussian: the squared
    residual plus the variance)."""
    Qp = O.prior_precision(model, theta)
    y = np.asarray(model["y"], dtype=np.float64)
    eta = O.linear_predictor(model, theta, mu)
    var = np.asarray(var, dtype=np.float64)
    if model["lik"] == "gaussian":
        s2 = math.exp(O.lik_param(model, theta))
        nll = np.sum(((y - eta) ** 2 + var) / (2.0 * s2))
    else:
        E = model.get("E")
        E = np.ones_like(eta) if E is None else np.asarray(E, dtype=np.float64)
        nll = np.sum(E * np.exp(eta + 0.5 * var) - y * (np.log(E) + eta))
    return float(nll + 0.5 * mu @ Qp @ mu)
