"""Plain reference of Stage 1 around the Laplace evaluation (TEST INFRASTRUCTURE
ONLY: imported by ``tests/`` alone, never by the product path).

Follows the paper's section "Stage 1" and the appendix "Marginal posteriors of
the hyperparameters": theta* = argmin -log pi~(theta | y) by BFGS with
central-difference gradients, the negative Hessian at theta* by finite
differences, the z-parameterisation theta(z) = theta* + V Lambda^{1/2} z with
Sigma = (negative Hessian)^{-1} = V Lambda V^T, and central composite design
points for the exploration of Stage 2 (45 points at t = 6, section
"Hyperparameter exploration").  log pi~(y | theta) comes from
``inla_oracle.laplace_eval``; numpy's ``eigh`` is the eigen-decomposition.

Readings where the paper is silent (the same on the library side):
  * gradient step h = 1e-3, Hessian step 5e-3 (central differences; the
    paper allows forward or central);
  * BFGS: inverse-Hessian update, identity start scaled by s^T y / y^T y at the
    first update, steepest-descent restart on a non-descent direction, step
    scaled to a largest component of at most 1, backtracking over the step
    lengths 1, 1/2, ..., 1/2^11 with the Armijo constant 1e-4; stop when
    ||gradient||_inf <= 1e-3 or the decrease is <= 1e-12 max(1, |f|);
  * CCD: factorial part 2^t for t <= 4, for t >= 5 the half fraction whose last
    coordinate is the product of the others (1 + 2t + 2^(t-1) points, 45 at
    t = 6); all non-centre points on the sphere of radius f0 sqrt(t); design
    weights exact for the mass, mean and covariance of a standard Gaussian.
"""
from __future__ import annotations

import math

import numpy as np

from . import inla_oracle as O

OK, MAXIT, LINESEARCH, EVAL_FAILED = 0, 1, 2, 3


def neg_log_post(model, theta, log_prior=None, laplace=None):
    """f(theta) = -(log pi~(y | theta) + log pi(theta)); +inf if the evaluation
    fails.  `laplace(model, theta)` evaluates log pi~(y | theta) (default: the
    kriging route of ``inla_oracle``; the Moore-Penrose route passes its own)."""
    r = (laplace or O.laplace_eval)(model, np.asarray(theta, dtype=np.float64))
    lp = 0.0 if log_prior is None else float(log_prior(np.asarray(theta)))
    if r["info"] != 0 or not np.isfinite(r["objective"]) or not np.isfinite(lp):
        return math.inf
    return -(r["objective"] + lp)


def central_gradient(f, theta, h):
    t = len(theta)
    g = np.zeros(t)
    for i in range(t):
        e = np.zeros(t)
        e[i] = h
        g[i] = (f(theta + e) - f(theta - e)) / (2.0 * h)
    return g


def theta_mode(model, theta0, log_prior=None, h=1e-3, gtol=1e-3, ftol=1e-12, max_iter=100, max_step=1.0,
               laplace=None):
    """BFGS minimisation of -log pi~(theta | y).  Returns a dict with theta,
    log_post (= log pi~ at theta), grad (of log pi~), iters, info."""
    f = lambda th: neg_log_post(model, th, log_prior, laplace)   # noqa: E731
    th = np.asarray(theta0, dtype=np.float64).copy()
    t = len(th)
    fx = f(th)
    if not np.isfinite(fx):
        return {"theta": th, "log_post": -fx, "grad": np.zeros(t), "iters": 0, "info": EVAL_FAILED}
    g = central_gradient(f, th, h)
    if not np.all(np.isfinite(g)):
        return {"theta": th, "log_post": -fx, "grad": -g, "iters": 0, "info": EVAL_FAILED}
    Hi = np.eye(t)
    scaled = False
    status, it = MAXIT, 0
    while it < max_iter:
        if np.max(np.abs(g)) <= gtol:
            status = OK
            break
        it += 1
        p = -Hi @ g
        if not (g @ p < 0):
            Hi = np.eye(t)
            p = -g
            scaled = False
        pinf = np.max(np.abs(p))
        if pinf > max_step:
            p = p * (max_step / pinf)
        gp = g @ p
        # backtracking: the largest of 1, 1/2, ..., 1/2^11 meeting Armijo
        alpha = None
        for j in range(12):
            a = 0.5 ** j
            fa = f(th + a * p)
            if fa <= fx + 1e-4 * a * gp:
                alpha = a
                break
        if alpha is None:
            status = LINESEARCH
            break
        thn = th + alpha * p
        gn = central_gradient(f, thn, h)
        if not np.all(np.isfinite(gn)):
            status = EVAL_FAILED
            break
        s, y = thn - th, gn - g
        sy = s @ y
        if sy > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            if not scaled:
                Hi = np.eye(t) * (sy / (y @ y))
                scaled = True
            rho = 1.0 / sy
            I = np.eye(t)
            Hi = (I - rho * np.outer(s, y)) @ Hi @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
        df = fx - fa
        th, fx, g = thn, fa, gn
        if df <= ftol * max(1.0, abs(fx)):
            status = OK
            break
    return {"theta": th, "log_post": -fx, "grad": -g, "iters": it, "info": status}


def neg_hessian(model, theta, log_prior=None, h=5e-3, laplace=None):
    """-d^2 log pi~(theta | y) by central differences (diagonal three-point,
    off-diagonal four-point stencil)."""
    f = lambda th: neg_log_post(model, th, log_prior, laplace)   # noqa: E731
    th = np.asarray(theta, dtype=np.float64)
    t = len(th)
    f0 = f(th)
    H = np.zeros((t, t))
    E = np.eye(t) * h
    for i in range(t):
        H[i, i] = (f(th + E[i]) - 2.0 * f0 + f(th - E[i])) / (h * h)
        for j in range(i + 1, t):
            v = (f(th + E[i] + E[j]) - f(th + E[i] - E[j]) - f(th - E[i] + E[j]) + f(th - E[i] - E[j])) / (4 * h * h)
            H[i, j] = H[j, i] = v
    return H, -f0


def ccd_design(t, f0=1.1):
    """(z [n x t], delta [n]): centre, axial points +-f0 sqrt(t) e_i, factorial points f0 (+-1, ...)."""
    r = f0 * math.sqrt(t)
    pts = [np.zeros(t)]
    for i in range(t):
        for sgn in (1.0, -1.0):
            z = np.zeros(t)
            z[i] = sgn * r
            pts.append(z)
    if t >= 2:
        free = t if t <= 4 else t - 1
        for m in range(2 ** free):
            s = np.array([-1.0 if (m >> i) & 1 else 1.0 for i in range(free)])
            if free < t:
                s = np.append(s, np.prod(s))
            pts.append(f0 * s)
    z = np.array(pts)
    n = len(z)
    delta = np.full(n, math.exp(0.5 * r * r) / (f0 * f0 * (n - 1)))
    delta[0] = 1.0 - 1.0 / (f0 * f0)
    return z, delta


def ccd_points(theta_star, neg_hess, f0=1.1):
    """theta_k = theta* + V Lambda^{1/2} z_k, Sigma = neg_hess^{-1} = V Lambda V^T."""
    H = 0.5 * (np.asarray(neg_hess) + np.asarray(neg_hess).T)
    w, V = np.linalg.eigh(H)
    if np.any(w <= 0):
        raise ValueError("negative Hessian is not positive definite")
    z, delta = ccd_design(len(theta_star), f0)
    return np.asarray(theta_star)[None, :] + (z / np.sqrt(w)[None, :]) @ V.T, delta


def ccd_weights(delta, log_post):
    lp = np.asarray(log_post, dtype=np.float64)
    m = np.max(lp[np.isfinite(lp)])
    w = np.where(np.isfinite(lp), np.asarray(delta) * np.exp(lp - m), 0.0)
    return w / w.sum()
