"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
independent of the oracle's own code: the paper's worked example, exact rational
brute force on tiny inputs, the closed-form Gaussian posterior and marginal
likelihood, the Kronecker eigenvalue form of log|Q_prior|, the null space of the
first-order random walk, and invariants of the constrained mode."""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats as st

from oracle import brute
from oracle import inla_oracle as O
from paper_2311_08050_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ worked example
def _appc():
    with open(os.path.join(GOLDEN, "appc_example.json")) as f:
        g = json.load(f)
    A = np.array(g["A"], float)
    model = {"n": 4, "A": A}
    Qp = np.array(g["Q_e"], float) + g["epsilon"] * np.eye(4)
    Qs = O.assemble(model, Qp, np.array(g["Q_l_diag"]), np.zeros(4))
    return g, Qs


def test_appc_uncorrected_covariance():
    g, Qs = _appc()
    S = O.constrained_covariance(Qs, None)
    assert np.max(np.abs(S - np.array(g["Sigma_un"]))) <= 5e-4


def test_appc_kriging_corrected_covariance():
    g, Qs = _appc()
    S = O.constrained_covariance(Qs, np.array(g["C"], float))
    printed = np.array(g["Sigma_star"])
    assert np.max(np.abs(S - printed)) <= 5e-4
    assert np.allclose(np.diag(S), [0.274, 0.198, 0.198, 0.274], atol=5e-4)
    # the constrained covariance annihilates the constraint: Sigma_c C^T = 0
    assert np.max(np.abs(S @ np.array(g["C"], float).T)) < 1e-12


def test_appc_kriging_equals_woodbury():
    """Eq. (woodeqn) with the Moore-Penrose inverse of Q_e gives the same
    covariance as kriging, up to the epsilon regularisation."""
    g, Qs = _appc()
    A = np.array(g["A"], float)
    Qlike = A.T @ np.diag(g["Q_l_diag"]) @ A
    P = np.linalg.pinv(np.array(g["Q_e"], float))
    assert np.max(np.abs(P - np.array(g["Q_e_pinv"]))) < 1e-12
    wood = P - P @ np.linalg.solve(np.eye(4) + Qlike @ P, Qlike @ P)
    krig = O.constrained_covariance(Qs, np.array(g["C"], float))
    assert np.max(np.abs(wood - krig)) < 3e-5
    assert np.max(np.abs(wood - np.array(g["Sigma_star"]))) <= 5e-4


# ------------------------------------------------------------------ definitions
def test_expcov_worked_value():
    S = O.expcov(np.array([[0.0, 0.0], [0.3, 0.4]]), 0.2)
    assert S[0, 0] == 1.0 and S[1, 1] == 1.0
    assert abs(S[0, 1] - 0.0820849986238988) < 1e-15   # exp(-0.5/0.2)


def test_rw1_null_space_and_kron_order():
    """R_t 1 = 0, so a field constant in time is in the null space of
    R_t kron Sigma_s^{-1}: Q_prior x = tau*delta*x exactly when the index is t*n_s+s."""
    model = synth.kron_poisson(5, 4, seed=7)
    R = O.rw1_structure(4)
    assert np.allclose(R @ np.ones(4), 0.0)
    assert np.linalg.matrix_rank(R) == 3
    theta = np.array([0.3, math.log(0.3), math.log(0.05), 0.0])
    Qp = O.prior_precision(model, theta)
    f = np.random.default_rng(0).normal(size=5)
    x = np.tile(f, 4)                      # x[t*n_s+s] = f[s]
    tau, delta = math.exp(0.3), 0.05
    assert np.allclose(Qp @ x, tau * delta * x, rtol=1e-10, atol=1e-10)
    x_wrong = np.repeat(f, 4)              # the other ordering is not in the null space
    assert not np.allclose(Qp @ x_wrong, tau * delta * x_wrong, rtol=1e-3)


def test_kron_logdet_closed_form():
    """log|tau (R kron S^{-1} + delta I)| = sum_ij log(tau (lambda_i / mu_j + delta))."""
    model = synth.kron_poisson(12, 9, seed=3)
    theta = np.array([1.1, math.log(0.25), math.log(0.02), 0.0])
    Qp = O.prior_precision(model, theta)
    ld, _, info = O.logdet(Qp)
    assert info == 0
    lam = np.linalg.eigvalsh(O.rw1_structure(9))
    mu = np.linalg.eigvalsh(O.expcov(model["coords"], 0.25))
    closed = np.sum(np.log(math.exp(1.1) * (lam[:, None] / mu[None, :] + 0.02)))
    assert abs(ld - closed) <= 1e-12 * abs(closed)


def test_poisson_loglik_against_scipy():
    rng = np.random.default_rng(5)
    E = rng.uniform(5, 50, 30)
    eta = rng.normal(0, 0.4, 30)
    y = rng.poisson(E * np.exp(eta)).astype(float)
    model = {"lik": "poisson", "y": y, "E": E}
    _, W, ll = O.lik_terms(model, np.array([0.0]), eta)
    ref = st.poisson.logpmf(y, E * np.exp(eta)).sum()
    assert abs(ll - ref) <= 1e-11 * abs(ref)
    assert np.allclose(W, E * np.exp(eta))


# ------------------------------------------------------------------ brute force
def test_logdet_against_exact_determinant():
    for seed in range(3):
        Q = synth.random_spd(6, seed)
        ld, _, info = O.logdet(Q)
        exact = brute.log_of(brute.det(brute.mat(Q)))
        assert info == 0 and abs(ld - exact) <= 1e-13 * max(1.0, abs(exact))


def test_cholesky_reports_first_failing_minor():
    Q = synth.random_spd(6, 0)
    Q[3, 3] = -5.0
    _, _, info = O.logdet(Q)
    assert info == 4


def _tiny_models():
    dense = synth.dense_poisson(6, 2, seed=11)
    kron = synth.kron_poisson(3, 2, seed=12)
    kron["e"] = np.array([0.1, -0.2, 0.05, 0.0])
    expc = synth.expcov_gaussian(5, seed=13, constrained=True)
    expc["e"] = np.array([0.3])
    return [
        (dense, np.array([0.2])),
        (kron, np.array([0.4, math.log(0.3), math.log(0.05), 0.1])),
        (expc, np.array([0.1, math.log(0.2), math.log(0.3)])),
    ]


@pytest.mark.parametrize("case", range(3))
def test_laplace_against_exact_kkt_twin(case):
    model, theta = _tiny_models()[case]
    ours = O.laplace_eval(model, theta)
    assert ours["info"] == 0
    x_b, it_b = brute.newton_kkt(model, theta)
    assert np.max(np.abs(ours["x"] - np.array(x_b))) <= 1e-10 * max(1.0, np.max(np.abs(x_b)))
    ref = brute.laplace_exact(model, theta, x_b)
    for key in ("logdet_qprior", "logdet_qstar", "xqx", "loglik", "objective"):
        assert abs(ours[key] - ref[key]) <= 1e-9 * max(1.0, abs(ref[key])), key
    for key in ("logdet_sprior", "logdet_s", "ese"):
        assert abs(ours[key] - ref[key]) <= 1e-9 * max(1.0, abs(ref[key])), key
    C = np.asarray(model["C"])
    assert np.max(np.abs(C @ ours["x"] - model["e"])) < 1e-12


@pytest.mark.parametrize("case", range(3))
def test_marginal_var_against_exact_inverse(case):
    model, theta = _tiny_models()[case]
    ours = O.laplace_eval(model, theta)
    v = O.marginal_var(model, theta, ours["x"])
    ref = brute.marginal_var_exact(model, theta, ours["x"])
    assert np.max(np.abs(v - np.array(ref))) <= 1e-11 * max(1.0, max(abs(r) for r in ref))


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("constraint", [None, "zero", "nonzero"])
def test_gaussian_closed_form(constraint):
    """Gaussian likelihood: the Laplace approximation is exact, so the objective
    is log N(y; mu_c, Sigma_c + sigma^2 I) and the mode is the posterior mean, in
    the covariance form that never forms Q_prior:
        Sigma = Sigma(rho)/tau, S = C Sigma C^T, mu_c = Sigma C^T S^{-1} e,
        Sigma_c = Sigma - Sigma C^T S^{-1} C Sigma,
        x* = mu_c + Sigma_c (Sigma_c + sigma^2 I)^{-1} (y - mu_c)."""
    model = synth.expcov_gaussian(60, seed=21, constrained=constraint is not None)
    if constraint == "nonzero":
        model["e"] = np.array([1.7])
    theta = np.array([0.4, math.log(0.15), math.log(0.3)])
    tau, rho, s2 = math.exp(0.4), 0.15, 0.3
    out = O.laplace_eval(model, theta)
    Sig = O.expcov(model["coords"], rho) / tau
    mu = np.zeros(60)
    if constraint is not None:
        C = model["C"]
        S = C @ Sig @ C.T
        mu = Sig @ C.T @ np.linalg.solve(S, model["e"])
        Sig = Sig - Sig @ C.T @ np.linalg.solve(S, C @ Sig)
    K = Sig + s2 * np.eye(60)
    ref = st.multivariate_normal(mean=mu, cov=K).logpdf(model["y"])
    assert abs(out["objective"] - ref) <= 1e-9 * abs(ref)
    xstar = mu + Sig @ np.linalg.solve(K, model["y"] - mu)
    assert np.max(np.abs(out["x"] - xstar)) <= 1e-9 * np.max(np.abs(xstar))
    assert out["iters"] == 1


# ------------------------------------------------------------------ invariants
def test_poisson_mode_invariants():
    """Stationarity on {C x = e}: Q_p x* - A^T g(x*) = C^T lambda for some lambda
    (least-squares residual ~ 0), C x* = e, and independence from the start."""
    model = synth.kron_poisson(16, 8, seed=31)
    theta = synth.kron_theta0(8) + np.array([0.2, -0.1, 0.3, 0.05])
    out = O.laplace_eval(model, theta)
    assert out["info"] == 0 and 2 <= out["iters"] <= 12
    x = out["x"]
    Qp = O.prior_precision(model, theta)
    g, _, _ = O.lik_terms(model, theta, O.linear_predictor(model, theta, x))
    r = Qp @ x - g
    C = model["C"]
    lam, *_ = np.linalg.lstsq(C.T, r, rcond=None)
    assert np.max(np.abs(r - C.T @ lam)) <= 1e-9 * max(1.0, np.max(np.abs(r)))
    assert np.max(np.abs(C @ x)) <= 1e-10
    warm = O.laplace_eval(model, theta, x0=model["x_true"])
    assert np.max(np.abs(warm["x"] - x)) <= 1e-10 * max(1.0, np.max(np.abs(x)))
    assert abs(warm["objective"] - out["objective"]) <= 1e-10 * abs(out["objective"])


def test_constraint_rows_full_rank_and_satisfied_by_truth():
    for ns, nt in [(100, 30), (12, 5)]:
        C = synth.sum_to_zero_rows(ns, nt)
        assert C.shape == (ns + nt - 1, ns * nt)
        if ns * nt <= 3000:
            assert np.linalg.matrix_rank(C) == ns + nt - 1
    m = synth.kron_poisson(12, 5, seed=1)
    assert np.max(np.abs(m["C"] @ m["x_true"])) < 1e-12


def test_rank_deficient_constraints_flagged():
    model = synth.kron_poisson(4, 3, seed=2)
    model["C"] = np.vstack([model["C"], model["C"][:1]])   # a dependent row
    model["e"] = np.zeros(model["C"].shape[0])
    out = O.laplace_eval(model, synth.kron_theta0(3))
    assert out["info"] == O.INFO_CONSTRAINT_RANK


def test_theta_layout_padded_rows():
    """Theta rows may be padded: the likelihood parameter is the entry right
    after the prior parameters, whatever the row length."""
    m = synth.dense_poisson(12, 2, seed=3)
    a = O.laplace_eval(m, np.array([0.1]))
    b = O.laplace_eval(m, np.array([0.1, 0.0, 0.0, 0.0]))
    assert a["objective"] == b["objective"]
    g = synth.expcov_gaussian(10, seed=3)
    th = np.array([0.2, math.log(0.3), math.log(0.4)])
    assert O.laplace_eval(g, th)["objective"] == O.laplace_eval(g, np.append(th, 7.0))["objective"]


@pytest.mark.parametrize("sum_to_zero", [False, True])
def test_crossed_effects_gaussian_closed_form(sum_to_zero):
    """The Introduction's crossed random effects with a Gaussian likelihood:
    the mode is the posterior mean (A^T A / s2 + Q_prior)^{-1} A^T y / s2 (kriged
    onto C x = 0) and the objective equals the marginal likelihood
    log N(y; 0, A Sigma_c A^T + s2 I), Sigma_c the (constrained) prior covariance."""
    m = synth.crossed_effects(7, 5, 30, seed=12, sum_to_zero=sum_to_zero)
    s2 = 0.7
    th = np.array([math.log(s2)])
    r = O.laplace_eval(m, th)
    A, y = m["A"], m["y"]
    Sigma = np.linalg.inv(m["Qprior"])
    if sum_to_zero:
        C = m["C"]
        Sigma = Sigma - Sigma @ C.T @ np.linalg.solve(C @ Sigma @ C.T, C @ Sigma)
    K = A @ Sigma @ A.T + s2 * np.eye(len(y))
    mean = Sigma @ A.T @ np.linalg.solve(K, y)
    sign, ld = np.linalg.slogdet(K)
    ml = -0.5 * (len(y) * math.log(2 * math.pi) + ld + y @ np.linalg.solve(K, y))
    assert r["info"] == 0
    assert np.max(np.abs(r["x"] - mean)) <= 1e-12 * max(1.0, np.max(np.abs(mean)))
    assert abs(r["objective"] - ml) <= 1e-10 * abs(ml)
