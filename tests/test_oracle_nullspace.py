"""Pin of the oracle's Laplace objective for Poisson likelihoods at sizes the
exact-rational twin cannot reach (n up to 240), through a route that shares
none of the oracle's algorithm.

The oracle conditions on C x = e by kriging (Eq. (41) with the constraint terms:
log|Q_p|, log|C Q_p^{-1} C^T|, e^T (C Q_p^{-1} C^T)^{-1} e, log|Q*| and
log|C Q*^{-1} C^T|).  Here the constrained field is instead written in
coordinates of the constraint surface,

    x = x_p + N z,   C x_p = e,   N an orthonormal basis of null(C),

where the conditioned prior is an ordinary Gaussian in z with precision
P = N^T Q_p N and centre z_c = -P^{-1} N^T Q_p x_p.  The textbook Laplace
approximation of the marginal likelihood in z is

    log p(y | z*) - 1/2 (z* - z_c)^T P (z* - z_c) + 1/2 log|P| - 1/2 log|P + N^T A^T W A N|,

with z* the mode, found here by scipy's trust-region Newton optimiser.  By
det(N^T Q N) = det(Q) det(C Q^{-1} C^T) / det(C C^T) and
(x - mu_c)^T Q (x - mu_c) = x^T Q x - e^T (C Q^{-1} C^T)^{-1} e on {C x = e},
this equals the kriging form term by term, so a dropped or mis-signed term of the
oracle's objective (the e-term, either Schur log-determinant), a transposed
design matrix or a wrong Poisson weight makes the two disagree.  The posterior
covariance of the Gaussian approximation on the surface is N H^{-1} N^T (H the
Hessian in z), which pins the oracle's kriging-corrected marginal variances.
The prior precision, the likelihood and every determinant are written here from
their definitions, not taken from the oracle.
"""
import math

import numpy as np
import pytest
from scipy.linalg import null_space
from scipy.optimize import minimize

from oracle import inla_oracle as O
from paper_2311_08050_amd import synth


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
    """Mode and Laplace objective in constraint-surface coordinates (Poisson)."""
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
    sp, ldP = np.linalg.slogdet(P)
    sh, ldH = np.linalg.slogdet(hess(z))
    assert sp > 0 and sh > 0
    gmax = float(np.max(np.abs(grad(z))))
    obj = ll - 0.5 * dz @ P @ dz + 0.5 * ldP - 0.5 * ldH
    # posterior covariance of the Gaussian approximation on the surface: N H^{-1} N^T
    var = np.einsum("ij,ji->i", N, np.linalg.solve(hess(z), N.T))
    return xp + N @ z, obj, gmax, var


def _kron_case(n_s, n_t, seed, e_scale, constrained=True):
    m = synth.kron_poisson(n_s, n_t, seed=seed, constrained=constrained)
    if constrained and e_scale:
        m["e"] = np.random.default_rng(seed + 1).normal(0.0, e_scale, size=m["C"].shape[0])
    th = synth.kron_theta0(n_t) + np.array([0.25, -0.2, 0.4, 0.1])
    return m, th, kron_prior(m, th), None, float(th[3])


def _crossed_case(seed):
    m = synth.crossed_effects(15, 10, 300, seed=seed, lik="poisson", sum_to_zero=True)
    m["e"] = np.array([0.7])
    th = np.array([0.15])                     # beta0; the dense prior has no parameters
    return m, th, np.eye(m["n"]), m["A"], 0.15


@pytest.mark.parametrize("case", ["kron_e0", "kron_e_nonzero", "kron_unconstrained", "crossed_A_e_nonzero"])
def test_laplace_objective_equals_nullspace_route(case):
    if case == "kron_e0":
        m, th, Q, A, off = _kron_case(20, 8, seed=41, e_scale=0.0)
    elif case == "kron_e_nonzero":
        m, th, Q, A, off = _kron_case(24, 10, seed=43, e_scale=0.5)
    elif case == "kron_unconstrained":
        m, th, Q, A, off = _kron_case(16, 6, seed=45, e_scale=0.0, constrained=False)
    else:
        m, th, Q, A, off = _crossed_case(seed=47)
    y = np.asarray(m["y"], dtype=np.float64)
    nobs = y.shape[0]
    E = np.ones(nobs) if m.get("E") is None else np.asarray(m["E"], dtype=np.float64)
    x_ns, obj_ns, gmax, var_ns = nullspace_laplace(Q, A, y, E, off, m.get("C"), m.get("e"))
    assert gmax <= 1e-9 * max(1.0, float(np.max(np.abs(y))))
    r = O.laplace_eval(m, th)
    assert r["info"] == O.INFO_OK
    assert np.max(np.abs(r["x"] - x_ns)) <= 1e-8 * max(1.0, float(np.max(np.abs(x_ns))))
    assert abs(r["objective"] - obj_ns) <= 1e-9 * abs(obj_ns)
    if m.get("C") is not None:
        assert np.max(np.abs(m["C"] @ x_ns - m["e"])) <= 1e-10 * max(1.0, float(np.max(np.abs(x_ns))))
    # marginal variances: the oracle's kriging-corrected diagonal equals the
    # diagonal of the surface covariance N H^{-1} N^T at the mode
    v = O.marginal_var(m, th, r["x"])
    assert np.max(np.abs(v - var_ns)) <= 1e-9 * float(np.max(var_ns))


@pytest.mark.slow
def test_laplace_objective_equals_nullspace_route_at_n3000():
    """The same pin at the n = 3000 configuration's shape (100 regions x 30
    times, k = 129 sum-to-zero rows): objective, mode and marginal variances of
    the oracle against the constraint-surface route (z of dimension 2871)."""
    m = synth.kron_poisson(100, 30, seed=2)
    th = synth.kron_theta0(30) + np.array([0.1, -0.1, 0.2, 0.05])
    Q = kron_prior(m, th)
    y, E = np.asarray(m["y"], dtype=np.float64), np.asarray(m["E"], dtype=np.float64)
    x_ns, obj_ns, gmax, var_ns = nullspace_laplace(Q, None, y, E, float(th[3]), m["C"], m["e"])
    assert gmax <= 1e-9 * max(1.0, float(np.max(np.abs(y))))
    r = O.laplace_eval(m, th)
    assert r["info"] == O.INFO_OK
    assert np.max(np.abs(r["x"] - x_ns)) <= 1e-8 * max(1.0, float(np.max(np.abs(x_ns))))
    assert abs(r["objective"] - obj_ns) <= 1e-9 * abs(obj_ns)
    assert np.max(np.abs(m["C"] @ x_ns - m["e"])) <= 1e-10 * max(1.0, float(np.max(np.abs(x_ns))))
    v = O.marginal_var(m, th, r["x"])
    assert np.max(np.abs(v - var_ns)) <= 1e-9 * float(np.max(var_ns))
