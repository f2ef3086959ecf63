"""Pins of the Stage-1 reference (BFGS mode, finite-difference Hessian, CCD).

The Gaussian exponential-covariance model has a closed-form marginal
likelihood L(theta) = log N(y; 0, Sigma(rho)/tau + sigma^2 I), whose gradient and
Hessian are written out analytically here (standard derivatives of a Gaussian
log-density in the covariance parameters).  They pin the reference's BFGS
result (a stationary point of the exact function, and the optimum another
optimiser finds on the closed form) and its finite-difference Hessian.  The CCD
design is pinned by its point counts (45 at t = 6 in the paper), its geometry,
the orthogonality of its factorial part and by exact Gaussian moments.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import theta_oracle as T
from paper_2311_08050_amd import synth

PRIOR_MEAN = np.array([0.0, math.log(0.2), math.log(0.25)])


def log_prior(th):
    return -0.5 * float(np.sum((np.asarray(th) - PRIOR_MEAN) ** 2))


def gaussian_parts(model, th):
    """K(theta), its first and second derivatives in (log tau, log rho, log sigma^2)."""
    tau, rho, s2 = np.exp(th)
    p = model["coords"]
    d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
    S = np.exp(-d / rho)
    D = d / rho
    n = len(p)
    K = S / tau + s2 * np.eye(n)
    dK = [-S / tau, S * D / tau, s2 * np.eye(n)]
    ddK = [[S / tau, -S * D / tau, 0 * S], [None, S * (D * D - D) / tau, 0 * S], [None, None, s2 * np.eye(n)]]
    for i in range(3):
        for j in range(i):
            ddK[i][j] = ddK[j][i]
    return K, dK, ddK


def closed_form(model, th):
    K, _, _ = gaussian_parts(model, th)
    y = model["y"]
    sign, ld = np.linalg.slogdet(K)
    return -0.5 * (len(y) * math.log(2 * math.pi) + ld + y @ np.linalg.solve(K, y)) + log_prior(th)


def closed_grad_hess(model, th):
    K, dK, ddK = gaussian_parts(model, th)
    Ki = np.linalg.inv(K)
    a = Ki @ model["y"]
    g = np.array([0.5 * a @ dK[i] @ a - 0.5 * np.trace(Ki @ dK[i]) for i in range(3)])
    H = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            H[i, j] = (0.5 * a @ ddK[i][j] @ a - a @ dK[i] @ Ki @ dK[j] @ a - 0.5 * np.trace(Ki @ ddK[i][j])
                       + 0.5 * np.trace(Ki @ dK[i] @ Ki @ dK[j]))
    g -= np.asarray(th) - PRIOR_MEAN
    H -= np.eye(3)
    return g, H


@pytest.fixture(scope="module")
def gauss_mode():
    model = synth.expcov_gaussian(30, seed=7)
    res = T.theta_mode(model, PRIOR_MEAN + np.array([0.5, -0.3, 0.4]), log_prior=log_prior)
    return model, res


def test_bfgs_mode_is_a_stationary_point_of_the_closed_form(gauss_mode):
    model, res = gauss_mode
    assert res["info"] == T.OK, res
    g, H = closed_grad_hess(model, res["theta"])
    # the central-difference gradient is within gtol = 1e-3 of zero at the stop
    assert np.max(np.abs(g)) <= 3e-3, g
    assert np.all(np.linalg.eigvalsh(-H) > 0)
    assert abs(res["log_post"] - closed_form(model, res["theta"])) <= 1e-9 * abs(res["log_post"])


def test_bfgs_mode_matches_another_optimiser_on_the_closed_form(gauss_mode):
    model, res = gauss_mode
    opt = minimize(lambda th: -closed_form(model, th), PRIOR_MEAN, jac=lambda th: -closed_grad_hess(model, th)[0],
                   method="BFGS", options={"gtol": 1e-10})
    # the gap is bounded by the gradient tolerance over the smallest curvature
    _, H = closed_grad_hess(model, opt.x)
    bound = 3e-3 / np.min(np.linalg.eigvalsh(-H))
    assert np.max(np.abs(res["theta"] - opt.x)) <= bound, (res["theta"], opt.x, bound)


def test_finite_difference_hessian_matches_the_analytic_one(gauss_mode):
    model, res = gauss_mode
    Hfd, lp = T.neg_hessian(model, res["theta"], log_prior=log_prior)
    _, H = closed_grad_hess(model, res["theta"])
    assert np.max(np.abs(Hfd + H)) <= 1e-3 * np.max(np.abs(H)), (Hfd, -H)
    assert abs(lp - closed_form(model, res["theta"])) <= 1e-9 * abs(lp)


@pytest.mark.parametrize("t,count", [(1, 3), (2, 9), (3, 15), (4, 25), (5, 27), (6, 45)])
def test_ccd_counts_and_geometry(t, count):
    z, delta = T.ccd_design(t, f0=1.1)
    assert len(z) == count == len(delta)
    r = np.linalg.norm(z, axis=1)
    assert r[0] == 0 and np.allclose(r[1:], 1.1 * math.sqrt(t))
    assert len({tuple(np.round(v, 12)) for v in z}) == count   # distinct points


@pytest.mark.parametrize("t", [2, 3, 4, 5, 6])
def test_ccd_factorial_part_has_resolution_v(t):
    """Main effects and two-factor interactions of the factorial part are
    mutually orthogonal and orthogonal to the mean."""
    z, _ = T.ccd_design(t, f0=1.1)
    F = z[1 + 2 * t:] / 1.1
    cols = [np.ones(len(F))] + [F[:, i] for i in range(t)] + [F[:, i] * F[:, j] for i in range(t) for j in range(i + 1, t)]
    X = np.stack(cols, axis=1)
    assert np.allclose(X.T @ X, len(F) * np.eye(X.shape[1]))


@pytest.mark.parametrize("t", [1, 2, 4, 6])
def test_ccd_weights_exact_for_a_standard_gaussian(t):
    z, delta = T.ccd_design(t, f0=1.1)
    w = T.ccd_weights(delta, -0.5 * (z * z).sum(1))
    assert abs(w.sum() - 1) <= 1e-14
    assert np.max(np.abs(w @ z)) <= 1e-12
    assert np.max(np.abs((w[:, None] * z).T @ z - np.eye(t))) <= 1e-12


def test_ccd_points_reproduce_a_gaussian_posterior():
    rng = np.random.default_rng(3)
    t = 4
    A = rng.normal(size=(t, t))
    H = A @ A.T + t * np.eye(t)
    mu = rng.normal(size=t)
    th, delta = T.ccd_points(mu, H, f0=1.3)
    lp = np.array([-0.5 * (v - mu) @ H @ (v - mu) for v in th])
    w = T.ccd_weights(delta, lp)
    mean = w @ th
    cov = (w[:, None] * (th - mean)).T @ (th - mean)
    assert np.max(np.abs(mean - mu)) <= 1e-12
    assert np.max(np.abs(cov - np.linalg.inv(H))) <= 1e-12
