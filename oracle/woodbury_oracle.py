"""Plain reference of the Moore-Penrose route for intrinsic priors
(TEST INFRASTRUCTURE ONLY: imported by ``tests/`` alone).

Section "Bypassing constraints complexity in disease mapping models using dense
matrices": when Q_prior is rank deficient (an intrinsic GMRF such as a random
walk or a Besag model, or their Kronecker interaction), the latent field is
identified by working with the Moore-Penrose inverse Q_prior^+ instead of
conditioning on constraints C x = 0.  The null space N of Q_prior plays the role
of the constraints (N x = 0), and the rank of Q_prior plus the number of
constraints equals n.  The posterior covariance comes from the Woodbury variant
of Eq. (woodeqn):

    Sigma* = Q^+ - Q^+ (I + Q_l Q^+)^{-1} Q_l Q^+,   Q_l = A^T diag(W) A.

This module writes the route out step by step:
  * the pseudo-inverse by a symmetric eigen-decomposition (one per evaluation,
    as the section on the optimisation's cost states), eigenvalues at or below
    RANK_RTOL * max|lambda| treated as zero;
  * Newton for the mode in covariance form: b = A^T (g + W A x) as in the
    algorithm "Gaussian Approximation", x_new = Sigma*(x) b;
  * the Laplace objective as the Gaussian approximation on range(Q_prior), with
    pseudo-determinants:
        l = 1/2 log pdet(Q_prior) + 1/2 log pdet(Sigma*) - 1/2 x*^T Q_prior x*
            + sum_i log pi(y_i | eta*_i).
    The paper gives the covariance only; this objective is the textbook Laplace
    approximation of a Gaussian that lives on range(Q_prior) and equals the
    kriging objective with constraints that span null(Q_prior).

Model dict (as in ``inla_oracle``) with prior kind
    'rw1_besag': Q_prior = tau * (R_t kron R_s), R_t the first-order random walk
                 structure on n_t steps, R_s = D - Adj the Besag structure of the
                 region graph ``edges`` (pairs (i, j), i != j) on n_s regions,
                 latent index t*n_s + s;
    'intrinsic': Q_prior = tau * R with R = model['R'] given;
    'type4':     the simulation study's model (section "Simulation study"),
                 latent [mu, beta_t, alpha_time (n_t), alpha_space (n_s), zeta]
                 with Q_prior = blockdiag(c, c, tau_t R2_t, tau_s R_s,
                 tau_st R2_t kron R_s), c = model['fixed_precision'], R2_t the
                 second-order random walk structure, R_s the Besag structure,
                 and the design matrix model['A'];
theta = (log tau, lik) or, for 'type4', (log tau_t, log tau_s, log tau_st, lik);
lik = log sigma^2 (Gaussian) or beta0 (Poisson).
"""
from __future__ import annotations

import math

import numpy as np

from . import inla_oracle as O

RANK_RTOL = 1e-9
NEWTON_TOL = 1e-11
NEWTON_MAX_ITER = 50


# --------------------------------------------------------------------------- #
# Priors                                                                       #
# --------------------------------------------------------------------------- #
def besag_structure(n_s, edges):
    """R_s = D - Adj of the undirected region graph (each edge counted once)."""
    R = np.zeros((n_s, n_s))
    for i, j in edges:
        i, j = int(i), int(j)
        if i == j:
            continue
        R[i, j] -= 1.0
        R[j, i] -= 1.0
        R[i, i] += 1.0
        R[j, j] += 1.0
    return R


def rw2_structure(n_t):
    """Second-order random walk structure D^T D, D the (n_t - 2) x n_t matrix of
    second differences (rank n_t - 2; constants and linear trends are free)."""
    D = np.zeros((max(n_t - 2, 0), n_t))
    for i in range(n_t - 2):
        D[i, i], D[i, i + 1], D[i, i + 2] = 1.0, -2.0, 1.0
    return D.T @ D


def n_prior_params(model):
    return 3 if model["prior"] == "type4" else 1


def structure(model):
    """The unscaled structure matrix R (Q_prior = tau R)."""
    if model["prior"] == "rw1_besag":
        return np.kron(O.rw1_structure(model["n_t"]), besag_structure(model["n_s"], model["edges"]))
    if model["prior"] == "intrinsic":
        return np.array(model["R"], dtype=np.float64)
    raise ValueError(model["prior"])


def prior_precision(model, theta):
    if model["prior"] != "type4":
        return math.exp(float(theta[0])) * structure(model)
    n_s, n_t = model["n_s"], model["n_t"]
    R2 = rw2_structure(n_t)
    Rs = besag_structure(n_s, model["edges"])
    blocks = [np.array([[model["fixed_precision"]]]), np.array([[model["fixed_precision"]]]),
              math.exp(float(theta[0])) * R2, math.exp(float(theta[1])) * Rs,
              math.exp(float(theta[2])) * np.kron(R2, Rs)]
    n = sum(b.shape[0] for b in blocks)
    Q = np.zeros((n, n))
    o = 0
    for b in blocks:
        k = b.shape[0]
        Q[o:o + k, o:o + k] = b
        o += k
    return Q


def lik_view(model):
    """The model as the likelihood helpers of ``inla_oracle`` see it: one prior
    parameter in front of the likelihood parameter, A from the model."""
    v = dict(model)
    v["prior"] = "dense"
    return v


def theta_lik(model, theta):
    """(lik,) -- the theta the likelihood helpers take for a 'dense' view."""
    return np.asarray(theta, dtype=np.float64)[n_prior_params(model):]


# --------------------------------------------------------------------------- #
# Pseudo-inverse and the Woodbury covariance                                   #
# --------------------------------------------------------------------------- #
def pseudo_inverse(Q, rtol=RANK_RTOL):
    """Q^+ = V diag(1/lambda) V^T over the eigenvalues with |lambda| > rtol *
    max|lambda| (eigen-decomposition Q = V diag(lambda) V^T).  Returns
    (Q^+, rank, eigenvalues)."""
    lam, V = np.linalg.eigh(np.asarray(Q, dtype=np.float64))
    cut = rtol * float(np.max(np.abs(lam))) if lam.size else 0.0
    keep = np.abs(lam) > cut
    f = np.zeros_like(lam)
    f[keep] = 1.0 / lam[keep]
    return (V * f) @ V.T, int(np.count_nonzero(keep)), lam


def woodbury_cov(Qpinv, Ql):
    """Eq. (woodeqn): Sigma* = Q^+ - Q^+ (I + Q_l Q^+)^{-1} Q_l Q^+."""
    n = Qpinv.shape[0]
    return Qpinv - Qpinv @ np.linalg.solve(np.eye(n) + Ql @ Qpinv, Ql @ Qpinv)


def pseudo_logdet(M, rank):
    """log of the product of the `rank` largest-magnitude eigenvalues."""
    lam = np.linalg.eigvalsh(np.asarray(M, dtype=np.float64))
    top = np.sort(np.abs(lam))[::-1][:rank]
    return float(np.sum(np.log(top)))


# --------------------------------------------------------------------------- #
# Newton in covariance form and the objective                                  #
# --------------------------------------------------------------------------- #
def _lik(model, theta, x):
    view, th = lik_view(model), theta_lik(model, theta)
    eta = O.linear_predictor(view, th, x)
    g, W, ll = O.lik_terms(view, th, eta)
    return view, th, g, W, ll


def q_like(model, W):
    A = O.design(model)
    return np.diag(W) if A is None else A.T @ (W[:, None] * A)


# The covariance form loses accuracy in proportion to the condition of
# I + Q_l Q^+ (weak priors on fixed effects make Q^+ large), so its iterates
# settle on a rounding floor that can lie above NEWTON_TOL.  A step below
# FLOOR_TOL relative that is no longer at most half the previous one ends the
# iteration there.
FLOOR_TOL = 1e-7


def newton_mode(model, theta, Qpinv, x0=None, tol=NEWTON_TOL, max_iter=NEWTON_MAX_ITER):
    """x_new = Sigma*(x) b(x) until ||x_new - x||_inf <= tol * max(1, ||x_new||_inf),
    or until the step stops contracting below FLOOR_TOL relative.
    Returns (x, iters, info)."""
    n = model["n"]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    prev = math.inf
    for it in range(1, max_iter + 1):
        view, th, g, W, _ = _lik(model, theta, x)
        b = O.rhs(view, g, W, x)
        x_new = woodbury_cov(Qpinv, q_like(model, W)) @ b
        if not np.all(np.isfinite(x_new)):
            return x, it, O.INFO_NONFINITE
        step = float(np.max(np.abs(x_new - x)))
        scale = max(1.0, float(np.max(np.abs(x_new))))
        x = x_new
        if model["lik"] == "gaussian" or step <= tol * scale:
            return x, it, O.INFO_OK
        if step <= FLOOR_TOL * scale and step > 0.5 * prev:
            return x, it, O.INFO_OK
        prev = step
    return x, max_iter, O.INFO_NEWTON_MAXIT


def laplace_eval(model, theta, x0=None, rtol=RANK_RTOL, Qpinv=None):
    """log pi~(y | theta) by the Moore-Penrose route.  Returns a dict with the
    terms, the mode, the rank of Q_prior and the status."""
    theta = np.asarray(theta, dtype=np.float64)
    Qp = prior_precision(model, theta)
    if Qpinv is None:
        Qpinv, rank, lam = pseudo_inverse(Qp, rtol)
    else:
        lam = np.linalg.eigvalsh(Qp)
        rank = int(np.count_nonzero(np.abs(lam) > rtol * np.max(np.abs(lam))))
    x, iters, info = newton_mode(model, theta, Qpinv, x0=x0)
    out = {"x": x, "iters": iters, "info": info, "rank": rank}
    if info not in (O.INFO_OK, O.INFO_NEWTON_MAXIT):
        return out
    _, _, _, W, ll = _lik(model, theta, x)
    Sigma = woodbury_cov(Qpinv, q_like(model, W))
    keep = np.abs(lam) > rtol * np.max(np.abs(lam))
    ld_p = float(np.sum(np.log(np.abs(lam[keep]))))
    ld_sigma = pseudo_logdet(Sigma, rank)
    xqx = float(x @ Qp @ x)
    out.update(logdet_qprior=ld_p, logdet_sigma=ld_sigma, xqx=xqx, loglik=ll,
               objective=0.5 * ld_p + 0.5 * ld_sigma - 0.5 * xqx + ll, Sigma=Sigma)
    return out


def null_basis(Q, rtol=RANK_RTOL):
    """Orthonormal basis of the numerical null space of a symmetric Q."""
    lam, V = np.linalg.eigh(np.asarray(Q, dtype=np.float64))
    return V[:, np.abs(lam) <= rtol * float(np.max(np.abs(lam)))]
