"""An independent route to the Laplace objective, mode and marginal variances
of a constrained Poisson latent Gaussian model, used to pin the kriging oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and the script that stores
its full-size values under ``tests/golden/``), never by the product path.  It
shares no code with ``inla_oracle``.

The kriging oracle conditions on C x = e through the Schur complements of
Eq. (41) with the constraint terms (log|Q_p|, log|C Q_p^{-1} C^T|,
e^T (C Q_p^{-1} C^T)^{-1} e, log|Q*|, log|C Q*^{-1} C^T|).  Here the
constrained field is written in coordinates of the constraint surface,

    x = x_p + N z,   C x_p = e,   N an orthonormal basis of null(C),

where the conditioned prior is an ordinary Gaussian in z with precision
P = N^T Q_p N and centre z_c = -P^{-1} N^T Q_p x_p.  The textbook Laplace
approximation of the marginal likelihood in z is

    log p(y | z*) - 1/2 (z* - z_c)^T P (z* - z_c) + 1/2 log|P| - 1/2 log|P + N^T A^T W A N|,

with z* the mode, found by scipy's trust-region Newton optimiser.  Since
det(N^T Q N) = det(Q) det(C Q^{-1} C^T) / det(C C^T) and
(x - mu_c)^T Q (x - mu_c) = x^T Q x - e^T (C Q^{-1} C^T)^{-1} e on {C x = e}, it
equals the kriging form term by term, so a dropped or mis-signed term of the
oracle's objective, a transposed design matrix or a wrong Poisson weight makes
the two disagree.  The posterior covariance of the Gaussian approximation on the
surface is N H^{-1} N^T (H the Hessian in z), which pins the oracle's kriging-
corrected marginal variances.  The prior precision, the likelihood and every
determinant are written here from their definitions.
"""
import math

import numpy as np
from scipy.linalg import null_space
from scipy.optimize import minimize


def kron_prior(model, theta):
    """tau (R_t kron Sigma_s(rho)^{-1} + delta I): R_t the first-order random
    walk structure, Sigma_s(rho)_ij = exp(-|p_i - p_j| / rho), index t n_s + s."""
    n_s, n_t = model["n_s"], model["n_t"]
    tau, rho, delta = math.exp(theta[0]), math.exp(theta[1]), math.exp(theta[2])
    p = np.asarray(model["coords"], dtype=np.float64)
    d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(axis=2))
    Sinv = np.linalg.inv(np.exp(-d / rho))
    R = 2.0 * np.eye(n_t) - np.eye(n_t, k=1) - np.eye(n_t, k=-1)
    R[0, 0] = R[-1, -1] = 1.0
    return tau * (np.kron(R, Sinv) + delta * np.eye(n_s * n_t))


def nullspace_laplace(Q, A, y, E, offset, C, e):
    """Mode, Laplace objective, largest gradient entry at the mode and marginal
    variances in constraint-surface coordinates (Poisson likelihood)."""
    n = Q.shape[0]
    if C is None:
        N, xp = np.eye(n), np.zeros(n)
    else:
        N = null_space(C)
        xp = np.linalg.lstsq(C, e, rcond=None)[0]
    P = N.T @ Q @ N
    zc = -np.linalg.solve(P, N.T @ (Q @ xp))
    AN = N if A is None else A @ N
    eta0 = offset + (xp if A is None else A @ xp)
    lgy = sum(math.lgamma(v + 1.0) for v in y)

    def parts(z):
        eta = eta0 + AN @ z
        mu = E * np.exp(eta)
        dz = z - zc
        return float(np.sum(y * (np.log(E) + eta) - mu) - lgy), mu, dz

    def f(z):
        ll, _, dz = parts(z)
        return -(ll - 0.5 * dz @ P @ dz)

    def grad(z):
        _, mu, dz = parts(z)
        return -(AN.T @ (y - mu) - P @ dz)

    def hess(z):
        _, mu, _ = parts(z)
        return P + AN.T @ (mu[:, None] * AN)

    res = minimize(f, zc, jac=grad, hess=hess, method="trust-exact", options={"gtol": 1e-10, "maxiter": 200})
    z = res.x
    # one more Newton step from the optimiser's answer (quadratic convergence
    # puts the iterate at the rounding level of the gradient)
    z = z - np.linalg.solve(hess(z), grad(z))
    ll, mu, dz = parts(z)
    H = hess(z)
    sp, ldP = np.linalg.slogdet(P)
    sh, ldH = np.linalg.slogdet(H)
    assert sp > 0 and sh > 0
    gmax = float(np.max(np.abs(grad(z))))
    obj = ll - 0.5 * dz @ P @ dz + 0.5 * ldP - 0.5 * ldH
    # posterior covariance of the Gaussian approximation on the surface: N H^{-1} N^T
    var = np.einsum("ij,ji->i", N, np.linalg.solve(H, N.T))
    return xp + N @ z, obj, gmax, var
