"""The host-only CCD entry points of the library (inla_ccd_design,
inla_ccd_points, inla_ccd_weights: no handle, no device) against the oracle's
central composite design and against the property that defines the rule: with a
Gaussian log-posterior -1/2 (theta - theta*)^T H (theta - theta*), the weighted
points reproduce the mean theta* and the covariance H^{-1} exactly (section
"Hyperparameter exploration")."""
import ctypes as C
import math
import os

import numpy as np
import pytest

from oracle import theta_oracle as T

PD = C.POINTER(C.c_double)
NOT_PD = -2000


@pytest.fixture(scope="module")
def lib():
    from paper_2311_08050_amd import binding, build
    if not os.path.exists(binding.LIBPATH):
        build.build()
    L = C.CDLL(binding.LIBPATH)
    L.inla_ccd_design.argtypes = [C.c_int32, C.c_double, C.POINTER(C.c_int32), PD, PD]
    L.inla_ccd_points.argtypes = [C.c_int32, PD, PD, C.c_double, C.POINTER(C.c_int32), PD, PD]
    L.inla_ccd_weights.argtypes = [C.c_int32, PD, PD, PD]
    return L


def design(lib, t, f0):
    n = C.c_int32(0)
    assert lib.inla_ccd_design(t, f0, C.byref(n), None, None) == 0
    z, d = np.zeros((n.value, t)), np.zeros(n.value)
    assert lib.inla_ccd_design(t, f0, C.byref(n), z.ctypes.data_as(PD), d.ctypes.data_as(PD)) == 0
    return z, d


def points(lib, th, H, f0):
    t = len(th)
    n = C.c_int32(0)
    assert lib.inla_ccd_design(t, f0, C.byref(n), None, None) == 0
    P, d = np.zeros((n.value, t)), np.zeros(n.value)
    rc = lib.inla_ccd_points(t, np.ascontiguousarray(th).ctypes.data_as(PD), np.ascontiguousarray(H).ctypes.data_as(PD),
                             f0, C.byref(n), P.ctypes.data_as(PD), d.ctypes.data_as(PD))
    return rc, P, d


def weights(lib, d, lp):
    w = np.zeros(len(d))
    assert lib.inla_ccd_weights(len(d), np.ascontiguousarray(d).ctypes.data_as(PD),
                                np.ascontiguousarray(lp, dtype=np.float64).ctypes.data_as(PD), w.ctypes.data_as(PD)) == 0
    return w


def sorted_rows(a):
    a = np.round(np.asarray(a), 12)
    return a[np.lexsort(a.T[::-1])]


def spd(t, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(t, t))
    return X @ X.T + 0.5 * np.eye(t)


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6])
def test_design_equals_the_oracle_and_the_stated_counts(lib, t):
    f0 = 1.1
    z, d = design(lib, t, f0)
    zr, dr = T.ccd_design(t, f0)
    count = {1: 3, 2: 9, 3: 15, 4: 25, 5: 27, 6: 45}[t]
    assert len(z) == len(zr) == count
    both = np.column_stack([z, d])
    ref = np.column_stack([zr, dr])
    assert np.max(np.abs(sorted_rows(both) - sorted_rows(ref))) <= 1e-12
    assert np.allclose(np.linalg.norm(z[1:], axis=1), f0 * math.sqrt(t))


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6])
def test_weights_reproduce_gaussian_mean_and_covariance(lib, t):
    th = np.linspace(-0.7, 0.9, t)
    H = spd(t, seed=10 + t)
    rc, P, d = points(lib, th, H, 1.1)
    assert rc == 0
    D = P - th[None, :]
    lp = -0.5 * np.einsum("ki,ij,kj->k", D, H, D)
    w = weights(lib, d, lp)
    assert abs(w.sum() - 1.0) <= 1e-14
    assert np.max(np.abs(w @ P - th)) <= 1e-12
    cov = (w[:, None] * D).T @ D
    assert np.max(np.abs(cov - np.linalg.inv(H))) <= 1e-12 * np.max(np.abs(np.linalg.inv(H)))
    if t <= 4:   # sign-symmetric designs: the point sets equal the oracle's
        Pr, dr = T.ccd_points(th, H, 1.1)
        assert np.max(np.abs(sorted_rows(np.column_stack([P, d])) - sorted_rows(np.column_stack([Pr, dr])))) <= 1e-10
        lpr = -0.5 * np.einsum("ki,ij,kj->k", Pr - th, H, Pr - th)
        assert np.max(np.abs(np.sort(w) - np.sort(T.ccd_weights(dr, lpr)))) <= 1e-12


def test_nonfinite_log_posterior_gets_zero_weight(lib):
    d = np.array([0.5, 1.0, 1.0, 2.0])
    lp = np.array([0.0, -np.inf, np.nan, -1.0])
    w = weights(lib, d, lp)
    ref = T.ccd_weights(d, lp)
    assert w[1] == 0.0 and w[2] == 0.0
    assert np.max(np.abs(w - ref)) <= 1e-15


def test_status_codes(lib):
    n = C.c_int32(3)
    z, d = np.zeros((3, 2)), np.zeros(3)
    assert lib.inla_ccd_design(2, 1.1, C.byref(n), z.ctypes.data_as(PD), d.ctypes.data_as(PD)) == -3
    assert n.value == 9    # the needed count comes back
    H = np.array([[1.0, 0.0], [0.0, -1.0]])
    rc, _, _ = points(lib, np.zeros(2), H, 1.1)
    assert rc == NOT_PD
