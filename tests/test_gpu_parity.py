"""GPU parity: every C-ABI call against the FP64 CPU oracle on the same seeded
inputs, element by element at small sizes (several tiles plus a ragged tail),
and by properties plus sampled oracle evaluations at the full headline size.

Tolerance: 1e-9 relative for log-determinants, objective and mode (FP64 path).
"""
import math
import sys

import numpy as np
import pytest

from oracle import inla_oracle as O
from paper_2311_08050_amd import synth

pytestmark = pytest.mark.gpu
RTOL = 1e-9


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


def dev_models(models):
    from paper_2311_08050_amd.binding import DeviceModel
    return [DeviceModel(m) for m in models]


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def check_eval(res, x_gpu, ref, what):
    assert res["info"] == ref["info"] == 0, (what, res["info"], ref["info"])
    # the iteration count is unique except when a step lands at the tolerance,
    # where either side may take one more (equally converged) step
    assert abs(res["iters"] - ref["iters"]) <= 1, (what, res["iters"], ref["iters"])
    for key in ("objective", "logdet_qprior", "logdet_sprior", "ese", "logdet_qstar", "logdet_s", "xqx", "loglik"):
        assert rel(res[key], ref[key]) <= RTOL, (what, key, res[key], ref[key])
    xr = ref["x"]
    err = np.max(np.abs(x_gpu - xr)) / max(1.0, np.max(np.abs(xr)))
    assert err <= RTOL, (what, "mode", err)


def run_and_compare(lib, models, thetas, what):
    say(f"{what}: B={len(models)} n={[m['n'] for m in models]}")
    res, xs = lib.laplace_eval(dev_models(models), thetas)
    for b, (m, th) in enumerate(zip(models, thetas)):
        ref = O.laplace_eval(m, th)
        check_eval(res[b], xs[b].cpu().numpy(), ref, f"{what}[{b}]")
    return res


# ---------------------------------------------------------------- log-det
def test_logdet_batch_against_oracle(lib):
    import torch
    sizes = [1, 5, 64, 65, 127, 128, 129, 300, 513, 1000]
    say(f"logdet sizes {sizes}")
    mats = [synth.random_spd(n, seed=100 + n) for n in sizes]
    dev = [torch.tensor(M).cuda() for M in mats]
    ld, info = lib.logdet(dev)
    for n, M, d, l, i in zip(sizes, mats, dev, ld, info):
        ref, Lref, iref = O.logdet(M)
        assert i == iref == 0
        assert rel(l, ref) <= 1e-11, (n, l, ref)
        L = np.tril(d.cpu().numpy().T)   # column-major lower triangle
        assert np.max(np.abs(L - Lref)) <= 1e-12 * np.max(np.abs(Lref)), n


def test_logdet_reports_failing_minor_and_empty(lib):
    import torch
    M = synth.random_spd(200, seed=7)
    M[70, 70] = -3.0
    _, _, iref = O.logdet(M)
    say("logdet non-PD n=200 and n=0")
    ld, info = lib.logdet([torch.tensor(M).cuda(), torch.zeros((0, 0), dtype=torch.float64).cuda()])
    assert info[0] == iref == 71 and math.isnan(ld[0])
    assert info[1] == 0 and ld[1] == 0.0


# ---------------------------------------------------------------- laplace_eval
def test_laplace_expcov400_configuration(lib):
    model, batch = synth.expcov400()
    run_and_compare(lib, [model] * len(batch), batch, "expcov400")


def test_laplace_kron_ragged_with_nonzero_rhs(lib):
    m = synth.kron_poisson(13, 7, seed=5)          # n = 91, k = 19
    m["e"] = np.linspace(-0.3, 0.2, m["C"].shape[0])
    th = synth.kron_theta0(7)
    thetas = np.stack([th, th + np.array([0.3, -0.2, 0.4, 0.1]), th + np.array([-0.4, 0.3, -0.5, -0.2])])
    run_and_compare(lib, [m] * 3, thetas, "kron 13x7")


def test_laplace_dense_prior(lib):
    m = synth.dense_poisson(150, 3, seed=2)
    run_and_compare(lib, [m, m], np.array([[0.1], [-0.2]]), "dense 150")


def test_laplace_unconstrained_poisson(lib):
    m = synth.kron_poisson(20, 10, seed=6, constrained=False)
    run_and_compare(lib, [m], synth.kron_theta0(10)[None, :], "kron 20x10 unconstrained")


def test_laplace_uneven_batch_one_call(lib):
    ms = [synth.kron_poisson(13, 7, seed=5), synth.kron_poisson(40, 9, seed=8), synth.dense_poisson(150, 3, seed=2),
          synth.kron_poisson(100, 3, seed=9), synth.expcov_gaussian(130, seed=4, constrained=True)]
    ths = [synth.kron_theta0(7), synth.kron_theta0(9) + 0.2, np.array([0.1, 0, 0, 0]),
           synth.kron_theta0(3) - 0.3, np.array([0.2, math.log(0.3), math.log(0.4), 0.0])]
    run_and_compare(lib, ms, np.stack(ths), "uneven batch")


def test_laplace_kron3000_configuration(lib):
    model, batch = synth.kron3000()
    run_and_compare(lib, [model] * 3, batch[:3], "kron3000 (first 3 of 9)")


# ---------------------------------------------------------------- mode / var
def test_constrained_mode_and_warm_start(lib):
    import torch
    m = synth.kron_poisson(40, 9, seed=8)
    th = synth.kron_theta0(9) + 0.1
    ref = O.laplace_eval(m, th)
    say("constrained_mode zero start")
    dm = dev_models([m])
    res, xs = lib.constrained_mode(dm, th[None, :])
    assert res[0]["info"] == 0 and abs(res[0]["iters"] - ref["iters"]) <= 1
    assert np.max(np.abs(xs[0].cpu().numpy() - ref["x"])) <= RTOL * max(1.0, np.max(np.abs(ref["x"])))
    say("laplace_eval warm start from the mode")
    x0 = [torch.tensor(ref["x"]).cuda()]
    res2, xs2 = lib.laplace_eval(dm, th[None, :], x=x0, start=1)
    assert res2[0]["info"] == 0 and res2[0]["iters"] <= 2
    assert np.max(np.abs(xs2[0].cpu().numpy() - ref["x"])) <= 1e-10 * max(1.0, np.max(np.abs(ref["x"])))
    assert rel(res2[0]["objective"], ref["objective"]) <= RTOL


@pytest.mark.parametrize("case", ["kron", "dense", "expcov"])
def test_marginal_var_against_oracle(lib, case):
    import torch
    if case == "kron":
        m, th = synth.kron_poisson(13, 7, seed=5), synth.kron_theta0(7) + 0.2
    elif case == "dense":
        m, th = synth.dense_poisson(150, 3, seed=2), np.array([0.1])
    else:
        m, th = synth.expcov_gaussian(100, seed=3), np.array([0.0, math.log(0.2), math.log(0.25)])
    ref_mode = O.laplace_eval(m, th)["x"]
    ref = O.marginal_var(m, th, ref_mode)
    say(f"marginal_var {case} n={m['n']}")
    var, info = lib.marginal_var(dev_models([m]), th[None, :], [torch.tensor(ref_mode).cuda()])
    assert info[0] == 0
    v = var[0].cpu().numpy()
    assert np.max(np.abs(v - ref) / np.abs(ref)) <= RTOL, case


# ---------------------------------------------------------------- failures
def test_status_codes(lib):
    from paper_2311_08050_amd import binding
    m = synth.kron_poisson(13, 7, seed=5)
    th = synth.kron_theta0(7)
    say("status: non-finite theta, max_iter=1")
    bad = np.stack([th, th])
    bad[1, 0] = np.nan
    res, _ = lib.laplace_eval(dev_models([m, m]), bad)
    assert res[0]["info"] == 0 and res[1]["info"] == binding.INFO_NONFINITE
    res, _ = lib.laplace_eval(dev_models([m]), th[None, :], max_iter=1)
    assert res[0]["info"] == binding.INFO_NEWTON_MAXIT and res[0]["iters"] == 1
    say("status: dependent constraint row")
    m2 = dict(m)
    m2["C"] = np.vstack([m["C"], m["C"][:1]])
    m2["e"] = np.zeros(m2["C"].shape[0])
    res, _ = lib.laplace_eval(dev_models([m2]), th[None, :])
    assert res[0]["info"] == binding.INFO_CONSTRAINT_RANK
    assert O.laplace_eval(m2, th)["info"] == O.INFO_CONSTRAINT_RANK
    say("status: empty batch")
    assert lib.laplace_eval([], np.zeros((0, 4)))[0] == []


# ---------------------------------------------------------------- full size
@pytest.mark.timeout(600)
def test_headline_size_properties_and_sampled_oracle(lib):
    """n = 8192 (128 regions x 64 times), k = 191, in the configuration the
    benchmark times: log|Q_prior| against its Kronecker eigenvalue form, C x* = e,
    and theta 0 against the oracle's stored values (every term of the objective,
    the mode at every 8th element)."""
    model, thetas = synth.headline(B=2)
    say("headline n=8192 B=2")
    res, xs = lib.laplace_eval(dev_models([model] * 2), thetas)
    lam = np.linalg.eigvalsh(O.rw1_structure(model["n_t"]))
    for b in range(2):
        r = res[b]
        assert r["info"] == 0 and 2 <= r["iters"] <= 12
        th = thetas[b]
        tau, rho, delta = math.exp(th[0]), math.exp(th[1]), math.exp(th[2])
        mu = np.linalg.eigvalsh(O.expcov(model["coords"], rho))
        closed = np.sum(np.log(tau * (lam[:, None] / mu[None, :] + delta)))
        assert rel(r["logdet_qprior"], closed) <= 1e-10
        x = xs[b].cpu().numpy()
        assert np.max(np.abs(model["C"] @ x)) <= 1e-10
    say("headline: theta 0 against the oracle's stored values")
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kron8192_theta0.json")) as f:
        g = json.load(f)
    assert np.array_equal(np.array(g["theta"]), thetas[0])
    r = res[0]
    assert r["info"] == 0 and abs(r["iters"] - g["iters"]) <= 1
    for key in ("objective", "logdet_qprior", "logdet_sprior", "ese", "logdet_qstar", "logdet_s", "xqx", "loglik"):
        assert rel(r[key], g[key]) <= RTOL, (key, r[key], g[key])
    idx = np.array(g["index"])
    assert np.max(np.abs(xs[0].cpu().numpy()[idx] - np.array(g["x"]))) / max(1.0, g["x_absmax"]) <= RTOL
