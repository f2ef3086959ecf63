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
