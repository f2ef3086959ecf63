"""GPU parity of the variational-Bayes mean correction (inla_vb_mean) against the
CPU reference on the same seeded models.  The library takes the expectations by
Gauss-Hermite quadrature (20 points), the reference in closed form, so the
comparison also bounds the quadrature error: 1e-9 relative on the corrected
mean.  At n = 3000 the corrected mean is checked by its stationarity."""
import sys

import numpy as np
import pytest

from oracle import inla_oracle as O
from oracle import vb_oracle as V
from paper_2311_08050_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-vb] {msg}", flush=True)
    sys.stdout.flush()


def dev_models(models):
    from paper_2311_08050_amd.binding import DeviceModel
    return [DeviceModel(m) for m in models]


@pytest.mark.parametrize("shape", [(13, 7), (40, 9)])
def test_vb_mean_matches_reference(lib, shape):
    m = synth.kron_poisson(*shape, seed=31)
    th0 = synth.kron_theta0(shape[1])
    thetas = np.stack([th0, th0 + np.array([0.3, -0.2, 0.4, 0.1])])
    dms = dev_models([m, m])
    say(f"vb {shape}: Laplace modes, marginal variances, correction")
    _, xs = lib.constrained_mode(dms, thetas)
    var, vinfo = lib.marginal_var(dms, thetas, xs)
    assert np.all(vinfo == 0)
    mus, its, info = lib.vb_mean(dms, thetas, var, xs)
    assert np.all(info == 0), info
    for b in range(2):
        x, _, _ = O.newton_mode(m, thetas[b])
        vr = O.marginal_var(m, thetas[b], x)
        ref, it_ref, _ = V.vb_mean(m, thetas[b], x, vr)
        mu = mus[b].cpu().numpy()
        err = np.max(np.abs(mu - ref)) / max(1.0, np.max(np.abs(ref)))
        say(f"  theta {b}: {its[b]} iterations (reference {it_ref}), error {err:.2e}, "
            f"shift from the mode {np.max(np.abs(ref - x)):.3e}")
        assert err <= 1e-9 and abs(int(its[b]) - it_ref) <= 1


def test_vb_gaussian_is_the_mode(lib):
    m = synth.expcov_gaussian(130, seed=4, constrained=True)
    th = np.array([[0.2, np.log(0.3), np.log(0.4)]])
    dms = dev_models([m])
    _, xs = lib.constrained_mode(dms, th)
    var, _ = lib.marginal_var(dms, th, xs)
    mus, its, info = lib.vb_mean(dms, th, var, xs)
    assert info[0] == 0 and its[0] == 1
    assert np.max(np.abs(mus[0].cpu().numpy() - xs[0].cpu().numpy())) <= 1e-12


def test_vb_at_n3000_is_stationary(lib):
    """The corrected mean satisfies the stationarity of the expected objective:
    E[-d log pi / d eta] + Q_prior mu lies in the span of C^T, and C mu = e."""
    m, thetas = synth.kron3000()
    thetas = thetas[:3]
    dms = dev_models([m]) * 3
    _, xs = lib.constrained_mode(dms, thetas)
    var, _ = lib.marginal_var(dms, thetas, xs)
    mus, its, info = lib.vb_mean(dms, thetas, var, xs)
    assert np.all(info == 0)
    C, e = O.constraint_of(m)
    for b in range(3):
        mu, v = mus[b].cpu().numpy(), var[b].cpu().numpy()
        g, _ = V.expected_terms(m, thetas[b], O.linear_predictor(m, thetas[b], mu), v)
        r = O.prior_precision(m, thetas[b]) @ mu - g
        lam = np.linalg.lstsq(C.T, r, rcond=None)[0]
        say(f"n=3000 theta {b}: {its[b]} iterations, stationarity residual "
            f"{np.max(np.abs(r - C.T @ lam)) / np.max(np.abs(r)):.2e}")
        assert np.max(np.abs(r - C.T @ lam)) <= 1e-8 * np.max(np.abs(r))
        assert np.max(np.abs(C @ mu - e)) <= 1e-10


@pytest.mark.timeout(600)
def test_vb_at_n8192_against_stored_oracle_values(lib):
    """The headline model at theta 0 of its batch (n = 8192, k = 191): the
    corrected mean from the library's FP64 mode and marginal variances against
    the oracle's, from the oracle's mode and variances (stored by
    tests/golden/make_full_size.py), at every 8th index, to 1e-9 relative."""
    import json
    import os

    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kron8192_theta0_vb.json")) as f:
        g = json.load(f)
    model, thetas = synth.headline(B=64)
    th = thetas[:1]
    assert np.array_equal(th[0], np.array(g["theta"]))
    dms = dev_models([model])
    say("n=8192: mode, marginal variances, correction")
    _, xs = lib.constrained_mode(dms, th)
    var, vinfo = lib.marginal_var(dms, th, xs)
    assert vinfo[0] == 0
    mus, its, info = lib.vb_mean(dms, th, var, xs)
    assert info[0] == 0, info
    idx = np.array(g["index"])
    mu = mus[0].cpu().numpy()
    err = np.max(np.abs(mu[idx] - np.array(g["mu"]))) / max(1.0, g["mu_absmax"])
    say(f"n=8192: {its[0]} iterations (oracle {g['iters']}), error {err:.2e}, "
        f"shift from the mode {g['shift_from_mode_absmax']:.3e}")
    assert err <= 1e-9 and abs(int(its[0]) - g["iters"]) <= 1
