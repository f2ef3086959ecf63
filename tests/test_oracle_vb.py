"""Pins of the variational-Bayes mean-correction reference (``oracle/vb_oracle.py``).

The corrected mean minimises sum_i E[-log pi(y_i | eta_i)] + mu^T Q_prior mu / 2 on
{C mu = e} with the Laplace variances held fixed (the expansion the algorithm
iterates is Newton's method on that function).  A general-purpose optimiser on
that objective, written in closed form over a null-space parameterisation of
the constraints, pins the reference; two special cases reduce it to the
Laplace mode: a Gaussian likelihood (the correction is zero) and zero variances.
"""
import numpy as np
import pytest
from scipy.linalg import null_space
from scipy.optimize import minimize

from oracle import inla_oracle as O
from oracle import vb_oracle as V
from paper_2311_08050_amd import synth


def laplace(model, th):
    x, it, info = O.newton_mode(model, th)
    assert info == 0
    return x, O.marginal_var(model, th, x)


def test_gaussian_correction_is_zero():
    m = synth.expcov_gaussian(25, seed=3, constrained=True)
    th = np.array([0.1, np.log(0.3), np.log(0.3)])
    x, var = laplace(m, th)
    mu, it, info = V.vb_mean(m, th, x, var)
    assert info == 0 and it == 1
    assert np.max(np.abs(mu - x)) <= 1e-12


def test_zero_variances_give_the_laplace_mode():
    m = synth.kron_poisson(5, 4, seed=8)
    th = synth.kron_theta0(4) + np.array([0.2, 0.0, 0.3, 0.1])
    x, _ = laplace(m, th)
    mu, it, info = V.vb_mean(m, th, x, np.zeros(m["n"]))
    assert info == 0 and np.max(np.abs(mu - x)) <= 1e-11


@pytest.mark.parametrize("shape", [(5, 4), (6, 3)])
def test_poisson_correction_minimises_the_expected_objective(shape):
    m = synth.kron_poisson(*shape, seed=9)
    th = synth.kron_theta0(shape[1]) + np.array([-0.2, 0.1, 0.2, 0.05])
    x, var = laplace(m, th)
    mu, it, info = V.vb_mean(m, th, x, var)
    assert info == 0 and it <= 10
    C, e = O.constraint_of(m)
    assert np.max(np.abs(C @ mu - e)) <= 1e-11
    N = null_space(C)
    x0 = np.linalg.lstsq(C, e, rcond=None)[0]
    res = minimize(lambda z: V.vb_objective(m, th, x0 + N @ z, var), N.T @ (x - x0), method="BFGS",
                   options={"gtol": 1e-9, "maxiter": 10000})
    ref = x0 + N @ res.x
    assert np.max(np.abs(mu - ref)) <= 1e-5, np.max(np.abs(mu - ref))
    assert V.vb_objective(m, th, mu, var) <= V.vb_objective(m, th, ref, var) + 1e-9
    # the correction moves the mean (the variances are not negligible here)
    assert np.max(np.abs(mu - x)) > 1e-4


# ----------------------------------------------------------------------------
# The closed-form expectations themselves, against numerical integration of
# their definitions: E[f(eta')] = int f(eta + s t) phi(t) dt, eta' ~ N(eta, s^2).
# A wrong variance factor in the log-normal mean (s^2 for s^2 / 2, or none) moves
# every Poisson value by at least e^(0.005) - 1 = 5e-3 relative at these variances.
# ----------------------------------------------------------------------------
def _gauss_expect(f, eta, s2):
    """E[f(eta')] for eta' ~ N(eta, s2), by adaptive quadrature over the standard
    normal density (the integrand is written as one exponential where it grows)."""
    from scipy.integrate import quad
    s = np.sqrt(s2)
    val, err = quad(lambda t: f(eta + s * t, t), -60.0, 60.0, epsabs=0.0, epsrel=1e-13, limit=400, points=[s])
    return val


_POIS = {"lik": "poisson", "y": np.array([3.0, 0.0, 12.0, 7.0, 41.0]),
         "E": np.array([5.0, 40.0, 17.3, 1.0, 8.5])}
_ETA = np.array([-1.2, 0.3, -0.05, 1.7, 1.5])
_VAR = np.array([0.01, 0.4, 1.3, 2.5, 0.07])


def test_poisson_expected_terms_equal_quadrature():
    """-I' = E[y - E e^eta'] and I'' = E[E e^eta'] (appendix "Variational Bayes
    approximation strategy": expectations of the first and second derivative of
    log pi(y | eta) under the Gaussian marginal) to 1e-12 relative."""
    g, W = V.expected_terms(_POIS, None, _ETA, _VAR)
    for i in range(_ETA.size):
        E, y = _POIS["E"][i], _POIS["y"][i]
        # E e^(eta + s t) phi(t) as one exponential
        m = _gauss_expect(lambda e, t: E * np.exp(e - 0.5 * t * t) / np.sqrt(2 * np.pi), _ETA[i], _VAR[i])
        assert abs(W[i] - m) <= 1e-12 * m, (i, W[i], m)
        gi = _gauss_expect(lambda e, t: (y - E * np.exp(e)) * np.exp(-0.5 * t * t) / np.sqrt(2 * np.pi),
                           _ETA[i], _VAR[i])
        assert abs(g[i] - gi) <= 1e-12 * max(1.0, abs(gi)), (i, g[i], gi)


def test_gaussian_expected_terms_equal_quadrature():
    m = {"lik": "gaussian", "y": np.array([0.4, -1.3, 2.2])}
    th = np.array([np.log(0.3)])          # dense prior: theta = (log sigma^2,)
    m["prior"] = "dense"
    eta, var = np.array([0.1, -0.7, 1.0]), np.array([0.2, 0.05, 1.1])
    g, W = V.expected_terms(m, th, eta, var)
    for i in range(3):
        gi = _gauss_expect(lambda e, t: (m["y"][i] - e) / 0.3 * np.exp(-0.5 * t * t) / np.sqrt(2 * np.pi),
                           eta[i], var[i])
        assert abs(g[i] - gi) <= 1e-12 * max(1.0, abs(gi))
        assert abs(W[i] - 1.0 / 0.3) <= 1e-15 / 0.3


@pytest.mark.parametrize("lik", ["poisson", "gaussian"])
def test_vb_objective_equals_quadrature(lik):
    """The expected negative log-likelihood of vb_objective (normalising
    constant lgamma(y + 1) and the Gaussian log(2 pi s^2) left out, as there)
    against quadrature of its definition, observation by observation; with a zero
    prior precision the quadratic term vanishes."""
    n = _ETA.size
    if lik == "poisson":
        m = dict(_POIS, prior="dense", n=n, Qprior=np.zeros((n, n)))
        th = np.array([0.0])                 # beta0 = 0: eta = x
    else:
        m = {"lik": "gaussian", "prior": "dense", "n": n, "y": _POIS["y"] / 10.0, "Qprior": np.zeros((n, n))}
        th = np.array([np.log(0.7)])
    total = 0.0
    for i in range(n):
        y = m["y"][i]
        if lik == "poisson":
            E = m["E"][i]
            f = lambda e, t: (E * np.exp(e - 0.5 * t * t) - y * (np.log(E) + e) * np.exp(-0.5 * t * t)) / np.sqrt(2 * np.pi)  # noqa: E731,E501
        else:
            f = lambda e, t: (y - e) ** 2 / (2 * 0.7) * np.exp(-0.5 * t * t) / np.sqrt(2 * np.pi)  # noqa: E731
        total += _gauss_expect(f, _ETA[i], _VAR[i])
    got = V.vb_objective(m, th, _ETA.copy(), _VAR)
    assert abs(got - total) <= 1e-12 * abs(total), (got, total)
