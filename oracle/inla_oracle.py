"""Plain FP64 CPU oracle of the per-theta Laplace evaluation of dense INLA.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product path.

Every step follows the paper (arXiv 2311.08050, "INLA+ - Approximate Bayesian
inference for non-sparse models using HPC") in its order and notation, in
float64, with no blocking, fusion or reordering.  LAPACK routines reached through
scipy (``dpotrf`` Cholesky, triangular solves) serve as library primitives for
single steps, exactly like a matmul would.

Model (the latent Gaussian model of the Introduction):
    y_i | x, theta ~ f(eta_i, theta),   eta = offset + A x
    x | theta      ~ N(0, Q_prior(theta)^{-1}),   optionally conditioned on C x = e.

A model is a plain ``dict`` (the keys are listed in ``paper_2311_08050_amd.synth``):
``n``, ``lik`` ('gaussian' | 'poisson'), ``prior`` ('dense' | 'expcov' | 'kron'),
``y``, ``E`` (Poisson exposure phi; None means 1), ``A`` (dense m x n, None
means the identity), ``C`` (k x n, None means no constraint), ``e`` (k),
``coords`` (points for the exponential covariance), ``n_s``, ``n_t`` and, for
the dense prior kind, ``Qprior``.

Theta layout: prior parameters first, then the likelihood parameter.
    expcov: (log tau, log rho, lik)        Q_prior = tau * Sigma(rho)^{-1}
    kron:   (log tau, log rho, log delta, lik)
            Q_prior = tau * (R_t kron Sigma_s(rho)^{-1} + delta I), index t*n_s + s
    dense:  (lik,)                         Q_prior supplied by the caller
    lik = log sigma^2 (Gaussian, eta = x) or beta0 (Poisson, eta = beta0 + x).

Readings of the paper where it is silent or garbled (all listed in the design
notes as well):
  * Newton stopping rule: infinity norm, ||x_new - x||_inf <= tol*max(1, ||x_new||_inf),
    tol = 1e-11, at most 50 iterations, no damping.  A Gaussian likelihood has a
    curvature that does not depend on x, so one step is exact and is the only one.
  * Q_l is the *negative* second derivative of log pi(y | eta).
  * The constrained Laplace objective adds the Gaussian conditioning terms
    1/2 log|C Q_p^{-1} C^T| + 1/2 e^T (C Q_p^{-1} C^T)^{-1} e - 1/2 log|C Q*^{-1} C^T|
    (the last is the constrained Gaussian approximation's normaliser).
  * log|Q*| is taken from a fresh factorisation at the returned mode.
  * The marginal variance is the diagonal of the constrained posterior covariance,
    not 1/Q*_ii.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack

NEWTON_TOL = 1e-11
NEWTON_MAX_ITER = 50

# per-theta status codes (shared meaning with the C header, but not its code)
INFO_OK = 0
INFO_NEWTON_MAXIT = -1
INFO_CONSTRAINT_RANK = -2
INFO_NONFINITE = -3


class NotPositiveDefinite(Exception):
    def __init__(self, info):
        super().__init__(f"leading minor {info} is not positive definite")
        self.info = info


# --------------------------------------------------------------------------- #
# Priors (section "Application ... Model": Q_* = tau_* R_*; the configurations  #
# add an exponential covariance in space).                                      #
# --------------------------------------------------------------------------- #
def expcov(coords, rho):
    """Sigma_ij = exp(-||p_i - p_j|| / rho) for points p (rows of ``coords``)."""
    p = np.asarray(coords, dtype=np.float64)
    d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
    return np.exp(-d / rho)


def rw1_structure(n_t):
    """Unscaled first-order random-walk structure R_t (rank n_t - 1): tridiagonal,
    diagonal (1, 2, ..., 2, 1), off-diagonal -1."""
    R = np.zeros((n_t, n_t))
    for i in range(n_t - 1):
        R[i, i] += 1.0
        R[i + 1, i + 1] += 1.0
        R[i, i + 1] -= 1.0
        R[i + 1, i] -= 1.0
    return R


def n_prior_params(prior):
    return {"dense": 0, "expcov": 2, "kron": 3}[prior]


def spd_inverse(M):
    """M^{-1} for SPD M through its Cholesky factor: M^{-1} = L^{-T} L^{-1}."""
    L, info = cholesky(M)
    if info:
        raise NotPositiveDefinite(info)
    Linv = sla.solve_triangular(L, np.eye(M.shape[0]), lower=True)
    return Linv.T @ Linv


def prior_precision(model, theta):
    """Q_prior(theta) as a dense symmetric matrix."""
    kind = model["prior"]
    if kind == "dense":
        return np.array(model["Qprior"], dtype=np.float64)
    tau = math.exp(theta[0])
    rho = math.exp(theta[1])
    if kind == "expcov":
        return tau * spd_inverse(expcov(model["coords"], rho))
    if kind == "kron":
        delta = math.exp(theta[2])
        Sinv = spd_inverse(expcov(model["coords"], rho))
        R = rw1_structure(model["n_t"])
        n = model["n"]
        # np.kron(R, Sinv)[t1*n_s+s1, t2*n_s+s2] = R[t1,t2] * Sinv[s1,s2]
        return tau * (np.kron(R, Sinv) + delta * np.eye(n))
    raise ValueError(kind)


# --------------------------------------------------------------------------- #
# Dense linear algebra steps                                                    #
# --------------------------------------------------------------------------- #
def cholesky(Q):
    """Q = L L^T (lower).  Returns (L, info); info = j > 0 means the leading
    minor of order j is not positive definite (LAPACK convention)."""
    c, info = lapack.dpotrf(np.array(Q, dtype=np.float64, order="F"), lower=1, clean=1)
    return np.tril(c), int(info)


def logdet_from_chol(L):
    """log|Q| = 2 sum_i log L_ii."""
    return 2.0 * float(np.sum(np.log(np.diag(L))))


def logdet(Q):
    """(log|Q|, L, info) for a symmetric positive definite Q."""
    L, info = cholesky(Q)
    if info:
        return float("nan"), L, info
    return logdet_from_chol(L), L, 0


def chol_solve(L, B):
    """Q^{-1} B with Q = L L^T: forward then backward substitution."""
    Y = sla.solve_triangular(L, B, lower=True)
    return sla.solve_triangular(L.T, Y, lower=False)


# --------------------------------------------------------------------------- #
# Likelihood (sections "Bypassing constraints ..." and "Model": Poisson with    #
# exposure phi; the configurations add a Gaussian likelihood).                  #
# --------------------------------------------------------------------------- #
def lik_param(model, theta):
    """The likelihood parameter: the entry right after the prior parameters."""
    return float(theta[n_prior_params(model["prior"])])


def offset_of(model, theta):
    return lik_param(model, theta) if model["lik"] == "poisson" else 0.0


def lik_terms(model, theta, eta):
    """(g, W, loglik): g = d log pi(y|eta)/d eta, W = -d^2 log pi(y|eta)/d eta^2
    (the Q_l of the Gaussian approximation), loglik = sum_i log pi(y_i|eta_i)."""
    y = np.asarray(model["y"], dtype=np.float64)
    if model["lik"] == "gaussian":
        s2 = math.exp(lik_param(model, theta))
        r = y - eta
        g = r / s2
        W = np.full_like(eta, 1.0 / s2)
        ll = float(np.sum(-0.5 * math.log(2.0 * math.pi * s2) - r * r / (2.0 * s2)))
        return g, W, ll
    if model["lik"] == "poisson":
        E = model.get("E")
        E = np.ones_like(eta) if E is None else np.asarray(E, dtype=np.float64)
        mu = E * np.exp(eta)
        g = y - mu
        W = mu
        lgy = np.array([math.lgamma(v + 1.0) for v in y])
        ll = float(np.sum(y * (np.log(E) + eta) - mu - lgy))
        return g, W, ll
    raise ValueError(model["lik"])


def design(model):
    A = model.get("A")
    return None if A is None else np.asarray(A, dtype=np.float64)


def linear_predictor(model, theta, x):
    A = design(model)
    return offset_of(model, theta) + (x if A is None else A @ x)


def assemble(model, Qp, W, x):
    """Q* = Q_prior + A^T W A and b = A^T g + A^T W A x  (the algorithm
    'Gaussian Approximation'; with A = I: Q* = Q_prior + diag(W))."""
    A = design(model)
    if A is None:
        return Qp + np.diag(W)
    return Qp + A.T @ (W[:, None] * A)


def rhs(model, g, W, x):
    A = design(model)
    if A is None:
        return g + W * x
    return A.T @ (g + W * (A @ x))


# --------------------------------------------------------------------------- #
# Kriging correction (sections "Identifiability constraints" and the appendix   #
# on an IGMRF under linear constraints)                                         #
# --------------------------------------------------------------------------- #
# A constraint system S = C Q^{-1} C^T whose Cholesky factor has a squared pivot
# below this fraction of the largest one is treated as rank deficient (the paper
# does not discuss rank detection; exact dependence shows up as such a pivot).
RANK_RTOL = 1e-13


def constraint_cholesky(S):
    """Cholesky factor of S, or None if S is not (numerically) positive definite."""
    LS, info = cholesky(S)
    if info:
        return None
    d = np.diag(LS) ** 2
    if d.size and d.min() < RANK_RTOL * d.max():
        return None
    return LS


def kriging(L, x_u, C, e):
    """Condition the Gaussian N(x_u, Q^{-1}) (Q = L L^T) on C x = e:
        V = Q^{-1} C^T,  S = C V,  lambda = S^{-1}(C x_u - e),  x = x_u - V lambda.
    Returns (x, V, S, L_S); L_S is the Cholesky factor of S (None if S is not
    positive definite, i.e. C lacks full row rank)."""
    V = chol_solve(L, C.T)
    S = C @ V
    LS = constraint_cholesky(S)
    if LS is None:
        return x_u, V, S, None
    lam = chol_solve(LS, C @ x_u - e)
    return x_u - V @ lam, V, S, LS


def constraint_of(model):
    C = model.get("C")
    if C is None or np.asarray(C).size == 0:
        return None, None
    C = np.asarray(C, dtype=np.float64)
    e = model.get("e")
    e = np.zeros(C.shape[0]) if e is None else np.asarray(e, dtype=np.float64)
    return C, e


# --------------------------------------------------------------------------- #
# Gaussian approximation: Newton iteration for the mode                         #
# --------------------------------------------------------------------------- #
def newton_mode(model, theta, x0=None, tol=NEWTON_TOL, max_iter=NEWTON_MAX_ITER, Qp=None):
    """Algorithm 'Gaussian Approximation' (appendix 'Gaussian approximation
    strategy'), each iterate corrected by kriging onto C x = e.

    Returns (x, iters, info)."""
    n = model["n"]
    if Qp is None:
        Qp = prior_precision(model, theta)
    C, e = constraint_of(model)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if not (np.all(np.isfinite(x)) and np.all(np.isfinite(theta))):
        return x, 0, INFO_NONFINITE
    for it in range(1, max_iter + 1):
        eta = linear_predictor(model, theta, x)
        g, W, _ = lik_terms(model, theta, eta)
        Q = assemble(model, Qp, W, x)
        b = rhs(model, g, W, x)
        L, info = cholesky(Q)
        if info:
            return x, it, info
        x_u = chol_solve(L, b)
        if C is not None:
            x_new, _, _, LS = kriging(L, x_u, C, e)
            if LS is None:
                return x, it, INFO_CONSTRAINT_RANK
        else:
            x_new = x_u
        if not np.all(np.isfinite(x_new)):
            return x, it, INFO_NONFINITE
        step = float(np.max(np.abs(x_new - x))) if n else 0.0
        scale = max(1.0, float(np.max(np.abs(x_new))) if n else 0.0)
        x = x_new
        if model["lik"] == "gaussian" or step <= tol * scale:
            return x, it, INFO_OK
    return x, max_iter, INFO_NEWTON_MAXIT


# --------------------------------------------------------------------------- #
# Laplace approximation of pi(theta | y)  (Eq. (41), mode-approx)               #
# --------------------------------------------------------------------------- #
def laplace_eval(model, theta, x0=None, tol=NEWTON_TOL, max_iter=NEWTON_MAX_ITER):
    """log pi~(y | theta) (log pi(theta) excluded), evaluated at the mode x*:

        l = 1/2 log|Q_p| + 1/2 log|S_p| + 1/2 e^T S_p^{-1} e - 1/2 x*^T Q_p x*
            + sum_i log pi(y_i | eta*_i) - 1/2 log|Q*| - 1/2 log|S|

    with S_p = C Q_p^{-1} C^T, S = C Q*^{-1} C^T (constraint terms only if C).
    Returns a dict with every term, the mode and the status."""
    theta = np.asarray(theta, dtype=np.float64)
    out = {"info": INFO_OK}
    Qp = prior_precision(model, theta)
    C, e = constraint_of(model)
    ld_p, Lp, info = logdet(Qp)
    if info:
        out["info"] = info
        return out
    out["logdet_qprior"] = ld_p
    ld_sp = 0.0
    ese = 0.0
    if C is not None:
        Vp = chol_solve(Lp, C.T)
        Sp = C @ Vp
        LSp = constraint_cholesky(Sp)
        if LSp is None:
            out["info"] = INFO_CONSTRAINT_RANK
            return out
        ld_sp = logdet_from_chol(LSp)
        ese = float(e @ chol_solve(LSp, e))
    out["logdet_sprior"] = ld_sp
    out["ese"] = ese

    x, iters, info = newton_mode(model, theta, x0=x0, tol=tol, max_iter=max_iter, Qp=Qp)
    out["x"] = x
    out["iters"] = iters
    if info > 0 or info in (INFO_CONSTRAINT_RANK, INFO_NONFINITE):
        out["info"] = info
        return out
    out["info"] = info  # INFO_OK or INFO_NEWTON_MAXIT (objective still reported)

    # refactor at the mode
    eta = linear_predictor(model, theta, x)
    _, W, ll = lik_terms(model, theta, eta)
    Qs = assemble(model, Qp, W, x)
    ld_s, Ls, info = logdet(Qs)
    if info:
        out["info"] = info
        return out
    ld_S = 0.0
    if C is not None:
        V = chol_solve(Ls, C.T)
        LS = constraint_cholesky(C @ V)
        if LS is None:
            out["info"] = INFO_CONSTRAINT_RANK
            return out
        ld_S = logdet_from_chol(LS)
    xqx = float(x @ (Qp @ x))
    out.update(
        logdet_qstar=ld_s,
        logdet_s=ld_S,
        xqx=xqx,
        loglik=ll,
        objective=0.5 * ld_p + 0.5 * ld_sp + 0.5 * ese - 0.5 * xqx + ll - 0.5 * ld_s - 0.5 * ld_S,
    )
    return out


# --------------------------------------------------------------------------- #
# Marginal variances  (Eq. (VBA): x | theta ~ N(x*, Q*^{-1}); constrained      #
# covariance of the appendix on an IGMRF under linear constraints)             #
# --------------------------------------------------------------------------- #
def constrained_covariance(Qs, C=None):
    """Sigma_c = Q*^{-1} - V S^{-1} V^T with V = Q*^{-1} C^T, S = C V."""
    L, info = cholesky(Qs)
    if info:
        raise NotPositiveDefinite(info)
    Sigma = chol_solve(L, np.eye(Qs.shape[0]))
    if C is None:
        return Sigma
    C = np.asarray(C, dtype=np.float64)
    V = Sigma @ C.T
    S = C @ V
    return Sigma - V @ np.linalg.solve(S, V.T)


def marginal_var(model, theta, x_mode):
    """sigma_i^2 = sum_j (L^{-1})_{ji}^2 - sum_ab V_ia (S^{-1})_ab V_ib at the mode."""
    theta = np.asarray(theta, dtype=np.float64)
    Qp = prior_precision(model, theta)
    eta = linear_predictor(model, theta, np.asarray(x_mode, dtype=np.float64))
    _, W, _ = lik_terms(model, theta, eta)
    Qs = assemble(model, Qp, W, x_mode)
    L, info = cholesky(Qs)
    if info:
        raise NotPositiveDefinite(info)
    Z = sla.solve_triangular(L, np.eye(Qs.shape[0]), lower=True)
    var = np.sum(Z * Z, axis=0)
    C, _ = constraint_of(model)
    if C is not None:
        V = chol_solve(L, C.T)
        S = C @ V
        LS, info = cholesky(S)
        if info:
            raise NotPositiveDefinite(info)
        U = sla.solve_triangular(LS, V.T, lower=True)  # L_S^{-1} V^T
        var = var - np.sum(U * U, axis=0)
    return var
