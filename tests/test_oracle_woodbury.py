"""Pins of the Moore-Penrose (Woodbury) reference against facts the paper and
the mathematics fix, independent of its own code:

* the worked example of the appendix on an IGMRF under linear constraints: the
  printed pseudo-inverse Q_e^+ and the printed corrected covariance Sigma*;
* the Penrose conditions and the identity Q^+ = (Q + N N^T)^{-1} - N N^T for an
  orthonormal basis N of the known null space of R_t kron R_s (constant in time
  per region, constant over regions per time);
* equality with the kriging route (a different algorithm in ``inla_oracle``) on
  the proper prior Q + N N^T conditioned on sum-to-zero constraints that span
  null(Q): same mode, same objective;
* the Gaussian likelihood's exact marginal likelihood log N(y; 0, Q^+ + s^2 I);
* the mode lies in range(Q) and satisfies the projected stationarity condition.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import inla_oracle as O
from oracle import woodbury_oracle as WB
from paper_2311_08050_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "appc_example.json")) as f:
        return json.load(f)


def known_null_basis(n_s, n_t):
    """Orthonormal basis of null(R_t kron R_s) for a connected region graph:
    1_t kron e_s (s = 1..n_s) and e_t kron 1_s (t = 1..n_t), orthonormalised."""
    cols = [np.kron(np.ones(n_t), np.eye(n_s)[:, s]) for s in range(n_s)]
    cols += [np.kron(np.eye(n_t)[:, t], np.ones(n_s)) for t in range(n_t)]
    Qr, Rr = np.linalg.qr(np.stack(cols, axis=1))
    keep = np.abs(np.diag(Rr)) > 1e-10
    return Qr[:, keep]


# ------------------------------------------------------------------ worked example
def test_appc_pseudo_inverse_printed():
    g = _golden()
    P, rank, lam = WB.pseudo_inverse(np.array(g["Q_e"], float))
    assert rank == 3
    # the printed entries are exact multiples of 1/8
    assert np.max(np.abs(P - np.array(g["Q_e_pinv"]))) < 1e-12


def test_appc_woodbury_covariance_printed():
    g = _golden()
    A = np.array(g["A"], float)
    P, _, _ = WB.pseudo_inverse(np.array(g["Q_e"], float))
    S = WB.woodbury_cov(P, A.T @ np.diag(g["Q_l_diag"]) @ A)
    assert np.max(np.abs(S - np.array(g["Sigma_star"]))) <= 5e-4
    # the correction keeps the null space: Sigma* 1 = 0
    assert np.max(np.abs(S @ np.ones(4))) < 1e-12


# ------------------------------------------------------------------ pseudo-inverse
@pytest.mark.parametrize("shape", [(5, 3), (13, 7)])
def test_pseudo_inverse_identities(shape):
    n_s, n_t = shape
    m = synth.rw1_besag(n_s, n_t, seed=11)
    Q = WB.prior_precision(m, np.array([0.4, 0.0]))
    P, rank, _ = WB.pseudo_inverse(Q)
    N = known_null_basis(n_s, n_t)
    assert rank == m["n"] - N.shape[1] == m["n"] - (n_s + n_t - 1)
    ref = np.linalg.inv(Q + N @ N.T) - N @ N.T
    sc = np.max(np.abs(ref))
    assert np.max(np.abs(P - ref)) <= 1e-12 * sc
    assert np.max(np.abs(Q @ P @ Q - Q)) <= 1e-12 * np.max(np.abs(Q))
    assert np.max(np.abs(P @ Q @ P - P)) <= 1e-12 * sc
    assert np.max(np.abs(P - P.T)) <= 1e-13 * sc


def test_besag_structure_definition():
    R = WB.besag_structure(4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)])
    assert np.array_equal(np.diag(R), [3, 2, 3, 2])
    assert R[0, 1] == -1 and R[1, 3] == 0 and R[0, 2] == -1
    assert np.allclose(R @ np.ones(4), 0)


# ------------------------------------------------------------------ against kriging
@pytest.mark.parametrize("lik", ["poisson", "gaussian"])
def test_equals_kriging_route(lik):
    """The pseudo-inverse route on Q equals the kriging route on Q + N N^T with
    C the per-region and per-time sum-to-zero rows (which span null(Q))."""
    n_s, n_t = 13, 7
    m = synth.rw1_besag(n_s, n_t, seed=5, lik=lik)
    th = synth.rw1_besag_theta0(n_t, lik) + np.array([0.2, 0.1])
    r = WB.laplace_eval(m, th)
    assert r["info"] == O.INFO_OK and r["rank"] == m["n"] - (n_s + n_t - 1)
    Q = WB.prior_precision(m, th)
    N = known_null_basis(n_s, n_t)
    C = synth.sum_to_zero_rows(n_s, n_t)
    km = {"n": m["n"], "lik": lik, "prior": "dense", "y": m["y"], "E": m["E"], "A": None,
          "C": C, "e": np.zeros(C.shape[0]), "Qprior": Q + N @ N.T}
    k = O.laplace_eval(km, th[1:])
    assert k["info"] == O.INFO_OK
    assert np.max(np.abs(r["x"] - k["x"])) <= 1e-9 * max(1.0, np.max(np.abs(k["x"])))
    assert abs(r["objective"] - k["objective"]) <= 1e-9 * abs(k["objective"])
    if lik == "poisson":
        assert 3 <= r["iters"] <= 8 and abs(r["iters"] - k["iters"]) <= 1
    # the posterior covariances agree as well
    _, W, _ = O.lik_terms(km, th[1:], O.linear_predictor(km, th[1:], k["x"]))
    Sk = O.constrained_covariance(O.assemble(km, km["Qprior"], W, k["x"]), C)
    assert np.max(np.abs(r["Sigma"] - Sk)) <= 1e-10 * np.max(np.abs(Sk))


def test_gaussian_marginal_likelihood_closed_form():
    """y = x + eps with x ~ N(0, Q^+) (degenerate): the Laplace objective is the
    exact log N(y; 0, Q^+ + sigma^2 I)."""
    m = synth.rw1_besag(9, 6, seed=3, lik="gaussian")
    th = np.array([0.7, math.log(0.3)])
    r = WB.laplace_eval(m, th)
    P, _, _ = WB.pseudo_inverse(WB.prior_precision(m, th))
    K = P + 0.3 * np.eye(m["n"])
    sign, ld = np.linalg.slogdet(K)
    y = m["y"]
    exact = -0.5 * (m["n"] * math.log(2 * math.pi) + ld + y @ np.linalg.solve(K, y))
    assert sign > 0
    assert abs(r["objective"] - exact) <= 1e-10 * abs(exact)
    assert r["iters"] == 1
    # the mode is the posterior mean Q^+ (Q^+ + s^2 I)^{-1} y
    assert np.max(np.abs(r["x"] - P @ np.linalg.solve(K, y))) <= 1e-10


def test_mode_invariants_poisson():
    n_s, n_t = 24, 10
    m = synth.rw1_besag(n_s, n_t, seed=8)
    th = synth.rw1_besag_theta0(n_t) + np.array([-0.3, 0.05])
    r = WB.laplace_eval(m, th)
    x = r["x"]
    N = known_null_basis(n_s, n_t)
    assert np.max(np.abs(N.T @ x)) <= 1e-12 * max(1.0, np.max(np.abs(x)))
    view = WB.lik_view(m)
    g, _, _ = O.lik_terms(view, th[1:], O.linear_predictor(view, th[1:], x))
    Q = WB.prior_precision(m, th)
    res = Q @ x - g
    res -= N @ (N.T @ res)          # stationarity on range(Q)
    assert np.max(np.abs(res)) <= 1e-8 * np.max(np.abs(g))
    # start independence
    r2 = WB.laplace_eval(m, th, x0=0.5 * x + 0.01)
    assert np.max(np.abs(r2["x"] - x)) <= 1e-10 * max(1.0, np.max(np.abs(x)))


# ------------------------------------------------------------------ Type IV model
def type4_null_basis(m):
    """Orthonormal basis of null(Q_prior) of the Type IV model, written from the
    structure of its blocks: alpha_time in span{1, t}, alpha_space constant,
    zeta in span{1_t kron e_s, t kron e_s, e_t kron 1_s}; mu and beta_t have
    proper priors."""
    n_s, n_t, n = m["n_s"], m["n_t"], m["n"]
    o_t, o_s, o_z = 2, 2 + n_t, 2 + n_t + n_s
    tt = np.arange(n_t, dtype=float)
    cols = []
    for v in (np.ones(n_t), tt):
        c = np.zeros(n); c[o_t:o_t + n_t] = v; cols.append(c)
    c = np.zeros(n); c[o_s:o_s + n_s] = 1.0; cols.append(c)
    for s in range(n_s):
        for v in (np.ones(n_t), tt):
            c = np.zeros(n); c[o_z:] = np.kron(v, np.eye(n_s)[s]); cols.append(c)
    for t in range(n_t):
        c = np.zeros(n); c[o_z:] = np.kron(np.eye(n_t)[t], np.ones(n_s)); cols.append(c)
    Qr, Rr = np.linalg.qr(np.stack(cols, axis=1))
    return Qr[:, np.abs(np.diag(Rr)) > 1e-10]


def test_type4_sizes_of_table3():
    """Effects size s = n_t n_s + n_s + n_t + 2 and constraint count k = the
    null-space dimension of Q_prior, as printed (first two rows; the third by
    the same formulas)."""
    with open(os.path.join(GOLDEN, "table3_sizes.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        m = synth.type4(r["n_s"], r["n_t"], seed=1)
        assert m["n"] == r["s"] and m["A"].shape == (r["n_s"] * r["n_t"], r["s"])
        assert r["k"] == r["n_t"] + 2 * r["n_s"] + 1
        if r["s"] <= 2500:
            Q = WB.prior_precision(m, synth.type4_theta0())
            _, rank, _ = WB.pseudo_inverse(Q)
            assert m["n"] - rank == r["k"]
            assert type4_null_basis(m).shape[1] == r["k"]


@pytest.mark.parametrize("graph", ["delaunay", "random"])
def test_type4_equals_kriging_route(graph):
    """Woodbury on the intrinsic Type IV prior with its design matrix equals
    kriging on Q + N N^T with the n_t + 2 n_s + 1 constraints N^T x = 0."""
    m = synth.type4(12, 5, seed=4, graph=graph)
    th = synth.type4_theta0() + np.array([0.2, -0.1, 0.3, 0.0])
    r = WB.laplace_eval(m, th)
    N = type4_null_basis(m)
    Q = WB.prior_precision(m, th)
    assert N.shape[1] == 5 + 2 * 12 + 1 and r["rank"] == m["n"] - N.shape[1]
    assert np.max(np.abs(Q @ N)) <= 1e-12 * np.max(np.abs(Q))
    km = {"n": m["n"], "lik": "poisson", "prior": "dense", "y": m["y"], "E": m["E"], "A": m["A"],
          "C": N.T, "e": np.zeros(N.shape[1]), "Qprior": Q + N @ N.T}
    k = O.laplace_eval(km, th[3:])
    assert r["info"] == k["info"] == O.INFO_OK
    assert np.max(np.abs(r["x"] - k["x"])) <= 1e-9 * max(1.0, np.max(np.abs(k["x"])))
    assert abs(r["objective"] - k["objective"]) <= 1e-9 * abs(k["objective"])
