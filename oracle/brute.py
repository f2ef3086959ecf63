"""Exact-rational brute-force twin of the oracle for tiny problems (n <= 8).

TEST INFRASTRUCTURE ONLY (see the package docstring).  It shares no code with
``inla_oracle``: every linear-algebra step here is Gaussian elimination over
``fractions.Fraction`` (exact), the constrained Newton step solves the KKT system
[[Q, C^T], [C, 0]] [x; lambda] = [b; e] instead of kriging, and determinants come
from exact elimination instead of a Cholesky factor.  The only rounding is in the
float64 inputs, in exp/log/lgamma and in the final conversions to float.
"""
from __future__ import annotations

import math
from fractions import Fraction


def F(v):
    return Fraction(float(v))


def mat(A):
    return [[F(v) for v in row] for row in A]


def eye(n):
    return [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]


def matmul(A, B):
    return [[sum((A[i][k] * B[k][j] for k in range(len(B))), Fraction(0))
             for j in range(len(B[0]))] for i in range(len(A))]


def transpose(A):
    return [list(r) for r in zip(*A)]


def det(A):
    """Exact determinant by Gaussian elimination with row swaps."""
    M = [row[:] for row in A]
    n = len(M)
    d = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            M[c], M[p] = M[p], M[c]
            d = -d
        d *= M[c][c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            if f:
                for j in range(c, n):
                    M[r][j] -= f * M[c][j]
    return d


def solve(A, B):
    """Exact A^{-1} B by Gauss-Jordan elimination (B is a list of rows)."""
    n = len(A)
    M = [A[i][:] + B[i][:] for i in range(n)]
    w = len(M[0])
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            raise ZeroDivisionError("singular")
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [M[r][j] - f * M[c][j] for j in range(w)]
    return [row[n:] for row in M]


def inverse(A):
    return solve(A, eye(len(A)))


def log_of(q):
    """log of a positive Fraction without overflow."""
    q = Fraction(q)
    if q <= 0:
        raise ValueError("log of non-positive value")
    return math.log(q.numerator) - math.log(q.denominator)


# ----------------------------- model pieces ---------------------------------- #
def prior_exact(model, theta):
    """Q_prior from its definition: tau * Sigma^{-1} (expcov) or
    tau * (R_t kron Sigma_s^{-1} + delta I) (kron), Sigma inverted exactly."""
    kind = model["prior"]
    if kind == "dense":
        return mat(model["Qprior"])
    tau = F(math.exp(theta[0]))
    rho = math.exp(theta[1])
    pts = [tuple(map(float, p)) for p in model["coords"]]
    m = len(pts)
    Sig = [[F(math.exp(-math.hypot(pts[i][0] - pts[j][0], pts[i][1] - pts[j][1]) / rho))
            for j in range(m)] for i in range(m)]
    Sinv = inverse(Sig)
    if kind == "expcov":
        return [[tau * v for v in row] for row in Sinv]
    delta = F(math.exp(theta[2]))
    n_t = model["n_t"]
    n_s = m
    # RW1: (x_{t+1} - x_t)^2 summed over t, written as a precision entry by entry
    R = [[Fraction(0)] * n_t for _ in range(n_t)]
    for t in range(n_t - 1):
        for a, b, s in ((t, t, 1), (t + 1, t + 1, 1), (t, t + 1, -1), (t + 1, t, -1)):
            R[a][b] += s
    n = n_t * n_s
    Q = [[Fraction(0)] * n for _ in range(n)]
    for t1 in range(n_t):
        for s1 in range(n_s):
            for t2 in range(n_t):
                for s2 in range(n_s):
                    Q[t1 * n_s + s1][t2 * n_s + s2] = tau * R[t1][t2] * Sinv[s1][s2]
    for i in range(n):
        Q[i][i] += tau * delta
    return Q


def _lik_param(model, theta):
    """Theta holds the prior parameters first, then the likelihood parameter."""
    return float(theta[{"dense": 0, "expcov": 2, "kron": 3}[model["prior"]]])


def lik_exact(model, theta, eta):
    """(g, W, loglik) at float eta; g and W returned as Fractions."""
    y = [float(v) for v in model["y"]]
    if model["lik"] == "gaussian":
        s2 = math.exp(_lik_param(model, theta))
        g = [F((yi - ei) / s2) for yi, ei in zip(y, eta)]
        W = [F(1.0 / s2)] * len(y)
        ll = sum(-0.5 * math.log(2 * math.pi * s2) - (yi - ei) ** 2 / (2 * s2) for yi, ei in zip(y, eta))
        return g, W, ll
    E = model.get("E")
    E = [1.0] * len(y) if E is None else [float(v) for v in E]
    mu = [Ei * math.exp(ei) for Ei, ei in zip(E, eta)]
    g = [F(yi - mi) for yi, mi in zip(y, mu)]
    W = [F(mi) for mi in mu]
    ll = sum(yi * (math.log(Ei) + ei) - mi - math.lgamma(yi + 1) for yi, Ei, ei, mi in zip(y, E, eta, mu))
    return g, W, ll


def _offset(model, theta):
    return _lik_param(model, theta) if model["lik"] == "poisson" else 0.0


def _A(model, n):
    A = model.get("A")
    return eye(n) if A is None else mat(A)


def _C(model):
    C = model.get("C")
    if C is None or len(C) == 0:
        return None, None
    e = model.get("e")
    e = [0.0] * len(C) if e is None else e
    return mat(C), [F(v) for v in e]


def newton_kkt(model, theta, x0=None, tol=1e-11, max_iter=50):
    """The Newton iteration with every step solved exactly as a KKT system."""
    n = model["n"]
    Qp = prior_exact(model, theta)
    A = _A(model, n)
    At = transpose(A)
    C, e = _C(model)
    off = _offset(model, theta)
    x = [0.0] * n if x0 is None else [float(v) for v in x0]
    for it in range(1, max_iter + 1):
        Ax = matmul(A, [[F(v)] for v in x])
        eta = [off + float(r[0]) for r in Ax]
        g, W, _ = lik_exact(model, theta, eta)
        AtWA = matmul(At, [[W[i] * A[i][j] for j in range(n)] for i in range(len(A))])
        Q = [[Qp[i][j] + AtWA[i][j] for j in range(n)] for i in range(n)]
        inner = [[g[i] + W[i] * Ax[i][0]] for i in range(len(A))]
        b = matmul(At, inner)
        if C is None:
            sol = solve(Q, b)
        else:
            k = len(C)
            K = [Q[i][:] + [C[a][i] for a in range(k)] for i in range(n)]
            K += [C[a][:] + [Fraction(0)] * k for a in range(k)]
            sol = solve(K, b + [[v] for v in e])[:n]
        x_new = [float(r[0]) for r in sol]
        step = max(abs(a - b_) for a, b_ in zip(x_new, x))
        scale = max(1.0, max(abs(v) for v in x_new))
        x = x_new
        if model["lik"] == "gaussian" or step <= tol * scale:
            return x, it
    return x, max_iter


def laplace_exact(model, theta, x):
    """The Laplace objective at a given mode x, every determinant, inverse and
    quadratic form exact: log pi(x | theta, Cx=e) + log pi(y | x) - log pi~_G."""
    n = model["n"]
    Qp = prior_exact(model, theta)
    A = _A(model, n)
    At = transpose(A)
    C, e = _C(model)
    off = _offset(model, theta)
    xf = [[F(v)] for v in x]
    Ax = matmul(A, xf)
    eta = [off + float(r[0]) for r in Ax]
    _, W, ll = lik_exact(model, theta, eta)
    AtWA = matmul(At, [[W[i] * A[i][j] for j in range(n)] for i in range(len(A))])
    Qs = [[Qp[i][j] + AtWA[i][j] for j in range(n)] for i in range(n)]
    xqx = matmul(transpose(xf), matmul(Qp, xf))[0][0]
    val = 0.5 * log_of(det(Qp)) - 0.5 * float(xqx) + ll - 0.5 * log_of(det(Qs))
    terms = {"logdet_qprior": log_of(det(Qp)), "logdet_qstar": log_of(det(Qs)),
             "xqx": float(xqx), "loglik": ll}
    if C is not None:
        Ct = transpose(C)
        Sp = matmul(C, solve(Qp, Ct))
        S = matmul(C, solve(Qs, Ct))
        ese = matmul([e], solve(Sp, [[v] for v in e]))[0][0]
        val += 0.5 * log_of(det(Sp)) + 0.5 * float(ese) - 0.5 * log_of(det(S))
        terms.update(logdet_sprior=log_of(det(Sp)), logdet_s=log_of(det(S)), ese=float(ese))
    terms["objective"] = val
    return terms


def marginal_var_exact(model, theta, x):
    """diag of Q*^{-1} - Q*^{-1} C^T (C Q*^{-1} C^T)^{-1} C Q*^{-1}, exact."""
    n = model["n"]
    Qp = prior_exact(model, theta)
    A = _A(model, n)
    At = transpose(A)
    C, _ = _C(model)
    off = _offset(model, theta)
    Ax = matmul(A, [[F(v)] for v in x])
    eta = [off + float(r[0]) for r in Ax]
    _, W, _ = lik_exact(model, theta, eta)
    AtWA = matmul(At, [[W[i] * A[i][j] for j in range(n)] for i in range(len(A))])
    Qs = [[Qp[i][j] + AtWA[i][j] for j in range(n)] for i in range(n)]
    Sig = inverse(Qs)
    if C is not None:
        V = matmul(Sig, transpose(C))
        S = matmul(C, V)
        corr = matmul(V, solve(S, transpose(V)))
        Sig = [[Sig[i][j] - corr[i][j] for j in range(n)] for i in range(n)]
    return [float(Sig[i][i]) for i in range(n)]
