"""Pin of the oracle's Laplace objective for Poisson likelihoods at sizes the
exact-rational twin cannot reach, through the constraint-surface route of
``oracle/nullspace_route.py``, which shares none of the oracle's algorithm
(the reasoning is in that module's docstring): n = 96 ... 240 here, the n = 3000
configuration's shape as a slow test, and the stored full-size values (n = 8192
and 16384, ``tests/golden/kron*_theta0*.json``, written once by
``tests/golden/make_full_size.py``)."""
import json
import os

import numpy as np
import pytest

from oracle import inla_oracle as O
from oracle.nullspace_route import kron_prior, nullspace_laplace
from paper_2311_08050_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


@pytest.mark.parametrize("n", [8192, 16384])
def test_stored_oracle_values_equal_nullspace_route_at_full_size(n):
    """The stored oracle values of the full-size cases (the headline's theta 0,
    n = 8192, k = 191; the precision configuration at theta0, n = 16384,
    k = 255: objective, mode and marginal variances at every 8th index) against
    the same cases by the constraint-surface route (z of dimension 8001 and
    16129), both written by ``tests/golden/make_full_size.py`` from ``oracle/``
    only.  This pins the full-size parity tests' expected values by a route that
    shares none of the oracle's algorithm."""
    with open(os.path.join(GOLDEN, f"kron{n}_theta0.json")) as f:
        ref = json.load(f)
    with open(os.path.join(GOLDEN, f"kron{n}_theta0_nullspace.json")) as f:
        ns = json.load(f)
    assert ref["n"] == ns["n"] == n and ref["k"] == ns["k"] and ref["theta"] == ns["theta"]
    assert ref["index"] == ns["index"]
    assert ns["gradient_absmax"] <= 1e-8 and ns["constraint_residual"] <= 1e-10 * max(1.0, ns["x_absmax"])
    assert abs(ref["objective"] - ns["objective"]) <= 1e-9 * abs(ns["objective"])
    x_ref, x_ns = np.array(ref["x"]), np.array(ns["x"])
    assert np.max(np.abs(x_ref - x_ns)) <= 1e-8 * max(1.0, ns["x_absmax"])
    v_ref, v_ns = np.array(ref["var"]), np.array(ns["var"])
    assert np.max(np.abs(v_ref - v_ns)) <= 1e-9 * ns["var_max"]
