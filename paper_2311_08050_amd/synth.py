"""Seeded synthetic latent-Gaussian-model inputs.

This module is shared by the tests, the benchmark and the CPU oracle's callers.
It draws inputs only: points, exposures, constraint rows, a smooth "true" field,
counts and hyperparameter batches.  It holds none of the method's arithmetic (no
covariance or precision is built here), so the oracle and the HIP library stay
independent of each other.

The shapes follow the paper's space x time Poisson interaction models (section
"Application to disease mapping ...", Type IV interaction, sum-to-zero
constraints per region and per time) and the exponential-covariance Gaussian
model; the paper's own data sets (prostate-cancer mortality in Spain, the
Penicillin crossed design) are not available and these draws stand in for them.

Model dict keys (consumed by the oracle and by the C-ABI binding alike):
    n, lik ('gaussian'|'poisson'), prior ('dense'|'expcov'|'kron'),
    y (n,), E (n,) or None, A None (identity) or (m, n), C (k, n) or None,
    e (k,) or None, coords (n_s, 2), n_s, n_t, Qprior (n, n) for 'dense'.
"""
from __future__ import annotations

import math

import numpy as np


def points(rng, n_s):
    """n_s points uniform in the unit square."""
    return rng.uniform(0.0, 1.0, size=(n_s, 2))


def smooth_field(rng, coords, n_t, n_waves=6, amp=0.35):
    """A smooth space-time field x(s, t) = sum_m a_m sin(2 pi u_m . p_s + w_m t/n_t + phi_m),
    laid out with index t*n_s + s.  It is not drawn from the prior."""
    n_s = coords.shape[0]
    t = np.arange(n_t)[:, None]
    x = np.zeros((n_t, n_s))
    for _ in range(n_waves):
        u = rng.normal(0.0, 2.0, size=2)
        w = rng.uniform(0.5, 6.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        a = amp * rng.uniform(0.3, 1.0)
        x += a * np.sin(2.0 * math.pi * (coords @ u)[None, :] + w * 2.0 * math.pi * t / n_t + ph)
    return x


def double_centre(x):
    """Remove per-region and per-time means of an (n_t, n_s) array so that every
    sum-to-zero row holds exactly: x - rowmean - colmean + grandmean."""
    return x - x.mean(axis=1, keepdims=True) - x.mean(axis=0, keepdims=True) + x.mean()


def sum_to_zero_rows(n_s, n_t):
    """Per-region rows (sum over time for each region) and per-time rows (sum
    over regions for each time), with the last per-time row dropped: the full set
    has rank n_s + n_t - 1, so the kept k = n_s + n_t - 1 rows have full row rank
    and span the same space."""
    n = n_s * n_t
    C = np.zeros((n_s + n_t - 1, n))
    idx = np.arange(n).reshape(n_t, n_s)  # index t*n_s + s
    for s in range(n_s):
        C[s, idx[:, s]] = 1.0
    for t in range(n_t - 1):
        C[n_s + t, idx[t, :]] = 1.0
    return C


def kron_theta0(n_t):
    """(log tau0, log 0.2, log 0.01, 0) with tau0 = (n_t^2 - 1)/(6 n_t 0.25), which
    sets the average prior marginal variance of a first-order random walk of
    length n_t to about 0.25 (trace of its pseudo-inverse is (n_t^2 - 1)/6)."""
    tau0 = (n_t * n_t - 1.0) / (6.0 * n_t * 0.25)
    return np.array([math.log(tau0), math.log(0.2), math.log(0.01), 0.0])


def kron_poisson(n_s, n_t, seed, beta0=0.0, constrained=True):
    """Poisson space x time interaction model, n = n_s * n_t latent (index t*n_s+s),
    exposures E ~ U(5, 50), y ~ Poisson(E exp(beta0 + x_true))."""
    rng = np.random.default_rng(seed)
    coords = points(rng, n_s)
    x = double_centre(smooth_field(rng, coords, n_t)).reshape(-1)
    n = n_s * n_t
    E = rng.uniform(5.0, 50.0, size=n)
    y = rng.poisson(E * np.exp(beta0 + x)).astype(np.float64)
    C = sum_to_zero_rows(n_s, n_t) if constrained else None
    return {
        "n": n, "lik": "poisson", "prior": "kron", "y": y, "E": E, "A": None,
        "C": C, "e": None if C is None else np.zeros(C.shape[0]),
        "coords": coords, "n_s": n_s, "n_t": n_t, "x_true": x,
    }


def expcov_gaussian(n, seed, sigma2=0.25, constrained=False):
    """Gaussian model y = x + eps on n uniform points, eps ~ N(0, sigma2).  With
    ``constrained`` a single sum-to-zero row is imposed (e = 0)."""
    rng = np.random.default_rng(seed)
    coords = points(rng, n)
    x = smooth_field(rng, coords, 1)[0]
    x = x - x.mean()
    y = x + rng.normal(0.0, math.sqrt(sigma2), size=n)
    C = np.ones((1, n)) if constrained else None
    return {
        "n": n, "lik": "gaussian", "prior": "expcov", "y": y, "E": None, "A": None,
        "C": C, "e": None if C is None else np.zeros(1),
        "coords": coords, "n_s": n, "n_t": 1, "x_true": x,
    }


def random_spd(n, seed, shift=0.5):
    """A dense symmetric positive-definite test matrix G G^T / m + shift I."""
    rng = np.random.default_rng(seed)
    m = n + 8
    G = rng.normal(size=(n, m))
    return G @ G.T / m + shift * np.eye(n)


def dense_poisson(n, k, seed):
    """Poisson model with a caller-supplied dense prior precision and k random
    full-rank constraint rows with a non-zero right-hand side."""
    rng = np.random.default_rng(seed)
    Q = random_spd(n, seed + 1000, shift=1.0)
    x = rng.normal(0.0, 0.3, size=n)
    E = rng.uniform(5.0, 50.0, size=n)
    y = rng.poisson(E * np.exp(x)).astype(np.float64)
    C = rng.integers(0, 2, size=(k, n)).astype(np.float64) if k else None
    if k:
        C[np.arange(k), np.arange(k)] = 1.0
    e = rng.normal(0.0, 0.2, size=k) if k else None
    return {
        "n": n, "lik": "poisson", "prior": "dense", "y": y, "E": E, "A": None,
        "C": C, "e": e, "coords": None, "n_s": n, "n_t": 1, "Qprior": Q,
    }


def crossed_effects(n_a, n_b, n_obs, seed, lik="gaussian", sigma2=1.0, sum_to_zero=False):
    """Crossed random effects (the LGM example of the paper's Introduction):
    eta_k = alpha_{i_k} + gamma_{j_k} with i_k, j_k drawn with replacement from
    n_a and n_b levels, alpha, gamma ~ N(0, 1) (dense prior precision I), A the
    n_obs x (n_a + n_b) design matrix with two ones per row.  Gaussian:
    y = eta + eps, eps ~ N(0, sigma2); Poisson: y ~ Poisson(E e^{beta0 + eta})
    with beta0 = 0 and E ~ U(5, 50).  With sum_to_zero the gamma levels sum to 0."""
    rng = np.random.default_rng(seed)
    n = n_a + n_b
    i = rng.integers(0, n_a, size=n_obs)
    j = rng.integers(0, n_b, size=n_obs)
    A = np.zeros((n_obs, n))
    A[np.arange(n_obs), i] = 1.0
    A[np.arange(n_obs), n_a + j] = 1.0
    x = rng.normal(0.0, 1.0 if lik == "gaussian" else 0.3, size=n)
    C = e = None
    if sum_to_zero:
        C = np.zeros((1, n))
        C[0, n_a:] = 1.0
        e = np.zeros(1)
        x[n_a:] -= x[n_a:].mean()
    E = None
    if lik == "gaussian":
        y = A @ x + rng.normal(0.0, math.sqrt(sigma2), size=n_obs)
    else:
        E = rng.uniform(5.0, 50.0, size=n_obs)
        y = rng.poisson(E * np.exp(A @ x)).astype(np.float64)
    return {
        "n": n, "lik": lik, "prior": "dense", "y": y, "E": E, "A": A,
        "C": C, "e": e, "coords": None, "n_s": n, "n_t": 1, "Qprior": np.eye(n), "x_true": x,
    }


def region_graph(coords):
    """Neighbouring-region pairs of points: the edges of their Delaunay
    triangulation (a connected planar graph, like the adjacency of a map)."""
    from scipy.spatial import Delaunay
    tri = Delaunay(np.asarray(coords, dtype=np.float64))
    e = set()
    for a, b, c in tri.simplices:
        for i, j in ((a, b), (b, c), (a, c)):
            e.add((min(int(i), int(j)), max(int(i), int(j))))
    return np.array(sorted(e), dtype=np.int64)


def rw1_besag(n_s, n_t, seed, lik="poisson", beta0=0.0, sigma2=0.25):
    """Space x time interaction with an intrinsic prior (Type IV: first-order
    random walk in time kron a Besag model on a random region graph), latent
    index t*n_s + s, no explicit constraints (the prior's null space identifies
    the field).  Poisson: E ~ U(5, 50), y ~ Poisson(E exp(beta0 + x_true));
    Gaussian: y = x_true + eps, eps ~ N(0, sigma2).  x_true is a smooth field
    with region and time means removed."""
    rng = np.random.default_rng(seed)
    coords = points(rng, n_s)
    edges = region_graph(coords)
    x = double_centre(smooth_field(rng, coords, n_t)).reshape(-1)
    n = n_s * n_t
    E = None
    if lik == "poisson":
        E = rng.uniform(5.0, 50.0, size=n)
        y = rng.poisson(E * np.exp(beta0 + x)).astype(np.float64)
    else:
        y = x + rng.normal(0.0, math.sqrt(sigma2), size=n)
    return {
        "n": n, "lik": lik, "prior": "rw1_besag", "y": y, "E": E, "A": None, "C": None, "e": None,
        "coords": coords, "edges": edges, "n_s": n_s, "n_t": n_t, "x_true": x,
    }


def rw1_besag_theta0(n_t, lik="poisson"):
    """(log tau0, lik0): tau0 = (n_t^2 - 1) / (6 n_t 0.25) as for the Kronecker
    prior; lik0 = beta0 = 0 (Poisson) or log 0.25 (Gaussian)."""
    tau0 = (n_t * n_t - 1.0) / (6.0 * n_t * 0.25)
    return np.array([math.log(tau0), 0.0 if lik == "poisson" else math.log(0.25)])


def random_besag_graph(n_s, rng, p=0.3):
    """Neighbour pairs of a random region graph in the manner of the paper's
    appendix on simulating a random Besag graph: every region draws n_s binary
    features with probability p, two regions are neighbours when they share a
    feature, and draws repeat until the graph is connected."""
    while True:
        F = rng.random((n_s, n_s)) < p
        share = (F.astype(np.int64) @ F.T.astype(np.int64)) > 0
        np.fill_diagonal(share, False)
        seen = np.zeros(n_s, dtype=bool)
        stack = [0]
        seen[0] = True
        while stack:
            i = stack.pop()
            for j in np.nonzero(share[i] & ~seen)[0]:
                seen[j] = True
                stack.append(int(j))
        if seen.all():
            i, j = np.nonzero(np.triu(share, 1))
            return np.stack([i, j], axis=1).astype(np.int64)


def type4(n_s, n_t, seed, graph="random", p=0.3):
    """The simulation study's space-time model (section "Simulation study"):
        eta_{st} = mu + beta_t t_c + alpha_time_t + alpha_space_s + zeta_{ts},
    Poisson counts y ~ Poisson(E exp(eta)), E ~ U(5, 50), t_c = (t - (n_t-1)/2) / n_t.
    Latent layout (s = n_t n_s + n_s + n_t + 2 effects): [mu, beta_t,
    alpha_time (n_t), alpha_space (n_s), zeta (index t*n_s + s)]; observation
    index t*n_s + s; A is the dense (n_t n_s) x s design matrix.  Priors (built
    by the consumers): low-precision Gaussian on mu and beta_t, RW2 in time,
    Besag in space on ``edges`` (graph "random": the appendix's random graph;
    "delaunay": the triangulation of random points), and the Type IV interaction
    RW2 kron Besag.  The true effects are smooth draws with the sum-to-zero
    and linear-trend parts removed."""
    rng = np.random.default_rng(seed)
    edges = random_besag_graph(n_s, rng, p) if graph == "random" else region_graph(points(rng, n_s))
    m = n_s * n_t
    n = m + n_s + n_t + 2
    t = np.repeat(np.arange(n_t), n_s)
    sidx = np.tile(np.arange(n_s), n_t)
    tc = (t - (n_t - 1) / 2.0) / n_t
    A = np.zeros((m, n))
    rows = np.arange(m)
    A[rows, 0] = 1.0
    A[rows, 1] = tc
    A[rows, 2 + t] = 1.0
    A[rows, 2 + n_t + sidx] = 1.0
    A[rows, 2 + n_t + n_s + rows] = 1.0
    tt = np.arange(n_t) / max(1, n_t - 1)
    a_time = 0.2 * np.sin(2.0 * math.pi * tt + rng.uniform(0, 2 * math.pi))
    a_time -= np.polyval(np.polyfit(tt, a_time, 1), tt) if n_t > 2 else a_time.mean()
    a_space = rng.normal(0.0, 0.2, size=n_s)
    a_space -= a_space.mean()
    zeta = rng.normal(0.0, 0.1, size=(n_t, n_s))
    zeta = double_centre(zeta).reshape(-1)
    x = np.concatenate([[0.1, 0.3], a_time, a_space, zeta])
    E = rng.uniform(5.0, 50.0, size=m)
    y = rng.poisson(E * np.exp(A @ x)).astype(np.float64)
    return {
        "n": n, "m": m, "lik": "poisson", "prior": "type4", "y": y, "E": E, "A": A, "C": None, "e": None,
        "edges": edges, "n_s": n_s, "n_t": n_t, "x_true": x, "fixed_precision": 1e-3,
    }


def type4_theta0():
    """(log tau_time, log tau_space, log tau_interaction, beta0 = 0)."""
    return np.array([math.log(10.0), math.log(2.0), math.log(5.0), 0.0])


def fd_batch(theta0, h, dims):
    """theta0 followed by theta0 +/- h e_j for each j in ``dims`` (the points of a
    central finite-difference gradient)."""
    th = [np.array(theta0, dtype=np.float64)]
    for j in dims:
        for s in (+1.0, -1.0):
            t = np.array(theta0, dtype=np.float64)
            t[j] += s * h
            th.append(t)
    return np.stack(th)


def normal_batch(theta0, B, sd, seed):
    """B draws of theta ~ N(theta0, sd^2 I)."""
    rng = np.random.default_rng(seed)
    return np.asarray(theta0)[None, :] + sd * rng.normal(size=(B, len(theta0)))


# ----------------------------- named workloads -------------------------------- #
def expcov400():
    """n = 400 Gaussian model, theta0 = (0, log 0.2, log 0.25); batch of 5 =
    theta0 and theta0 +/- 0.01 on log tau and log rho, then the two points
    +/- 0.01 on log sigma^2."""
    model = expcov_gaussian(400, seed=1)
    theta0 = np.array([0.0, math.log(0.2), math.log(0.25)])
    batch = fd_batch(theta0, 0.01, [0, 1, 2])
    return model, batch


def kron3000():
    """n = 100 regions x 30 times Poisson model, k = 129, 9 theta points."""
    model = kron_poisson(100, 30, seed=2)
    return model, fd_batch(kron_theta0(30), 0.01, [0, 1, 2, 3])


UNEVEN_SHAPES = [(32, 32), (64, 32), (100, 30), (128, 32), (192, 32)]


def uneven_batch(B=64, seed=3):
    """B theta points with n drawn from {1024, 2048, 3000, 4096, 6144}; one data
    set per distinct n (seed 30 + i); theta_b ~ N(theta0(n_b), 0.5^2 I)."""
    rng = np.random.default_rng(seed)
    which = rng.integers(0, len(UNEVEN_SHAPES), size=B)
    models = [kron_poisson(ns, nt, seed=30 + i) for i, (ns, nt) in enumerate(UNEVEN_SHAPES)]
    thetas = np.stack([kron_theta0(UNEVEN_SHAPES[w][1]) + 0.5 * rng.normal(size=4) for w in which])
    return [models[w] for w in which], thetas


def headline(B=64, seed=81, n_s=128, n_t=64):
    """n = 128 regions x 64 times = 8192 Poisson model, k = 191, B theta ~ N(theta0, 0.5^2 I)."""
    model = kron_poisson(n_s, n_t, seed=seed)
    return model, normal_batch(kron_theta0(n_t), B, 0.5, seed + 1)
