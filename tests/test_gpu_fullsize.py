"""Marginal variances (diag(Q*^{-1}) with the kriging correction, Eq. (VBA) and
the appendix on an IGMRF under linear constraints) against the FP64 oracle on
the paths that only sizes beyond one 512-wide panel reach: trailing updates
over the n identity border rows that turn into L^{-1}, with their zero-tile
skip, at both trailing tile sizes, with and without constraints; the n = 3000
configuration; and the headline model (n = 8192, k = 191) at theta 0 of its
batch against stored oracle values (``tests/golden/make_full_size.py``).

Bound: 1e-9 relative, element by element (the FP64 bar)."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import inla_oracle as O
from paper_2311_08050_amd import synth

pytestmark = pytest.mark.gpu
RTOL = 1e-9
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(f"[gpu-fullsize] {msg}", flush=True)
    sys.stdout.flush()


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("constrained", [True, False])
def test_marginal_var_three_panels(lib, tile, constrained):
    """n = 1110 (37 regions x 30 times; padded order 1152 = three 512-wide
    panels), k = 66 sum-to-zero rows or none, two theta, the trailing tile forced
    to `tile` for the factorisation of the variance pass."""
    from paper_2311_08050_amd.binding import DeviceModel
    m = synth.kron_poisson(37, 30, seed=17, constrained=constrained)
    th0 = synth.kron_theta0(30)
    thetas = np.stack([th0, th0 + np.array([0.3, -0.2, 0.4, 0.1])])
    refs = []
    for th in thetas:
        r = O.laplace_eval(m, th)
        assert r["info"] == 0
        refs.append((r["x"], O.marginal_var(m, th, r["x"])))
    lib.tune_set("fp64", m["n"], 2, nb=512, tm=tile)
    try:
        say(f"marginal_var n={m['n']} k={0 if m.get('C') is None else m['C'].shape[0]} tile {tile}")
        var, info = lib.marginal_var([DeviceModel(m)] * 2, thetas, [dev(x) for x, _ in refs])
    finally:
        lib.tune_set("fp64", m["n"], 2)   # back to the tuned / default configuration
    assert np.all(info == 0), info
    for b in range(2):
        v, ref = var[b].cpu().numpy(), refs[b][1]
        err = np.max(np.abs(v - ref) / np.abs(ref))
        say(f"  theta {b}: max relative error {err:.2e}")
        assert err <= RTOL, (b, err)


def test_marginal_var_n3000_configuration(lib):
    """The n = 3000 configuration (100 regions x 30 times, k = 129): theta0 and
    two points of its finite-difference batch, at the modes the GPU finds."""
    from paper_2311_08050_amd.binding import DeviceModel
    m, thetas = synth.kron3000()
    thetas = thetas[[0, 1, 6]]
    dm = DeviceModel(m)
    say("n=3000: modes (FP64) and marginal variances of 3 theta")
    res, xs = lib.laplace_eval([dm] * 3, thetas)
    assert all(r["info"] == 0 for r in res)
    var, info = lib.marginal_var([dm] * 3, thetas, xs)
    assert np.all(info == 0)
    for b in range(3):
        x = xs[b].cpu().numpy()
        ref = O.marginal_var(m, thetas[b], x)
        err = np.max(np.abs(var[b].cpu().numpy() - ref) / np.abs(ref))
        say(f"  theta {b}: max relative error {err:.2e}")
        assert err <= RTOL, (b, err)


@pytest.mark.timeout(300)
def test_headline_theta0_against_stored_oracle(lib):
    """n = 8192 (128 x 64), k = 191, theta 0 of the headline batch: every term of
    the objective, the mode (every 8th element) and the marginal variances
    (every 8th element) against the oracle's stored values, in the FP64 path."""
    from paper_2311_08050_amd.binding import DeviceModel
    g = golden("kron8192_theta0.json")
    model, thetas = synth.headline(B=64)
    assert np.array_equal(thetas[0], np.array(g["theta"])) and model["n"] == g["n"]
    dm = DeviceModel(model)
    say("headline theta 0: FP64 evaluation")
    res, xs = lib.laplace_eval([dm], thetas[:1])
    r = res[0]
    assert r["info"] == 0 and abs(r["iters"] - g["iters"]) <= 1
    for key in ("objective", "logdet_qprior", "logdet_sprior", "ese", "logdet_qstar", "logdet_s", "xqx", "loglik"):
        assert abs(r[key] - g[key]) <= RTOL * max(1.0, abs(g[key])), (key, r[key], g[key])
    idx = np.array(g["index"])
    x = xs[0].cpu().numpy()
    assert np.max(np.abs(x[idx] - np.array(g["x"]))) <= RTOL * max(1.0, g["x_absmax"])
    say("headline theta 0: marginal variances")
    var, info = lib.marginal_var([dm], thetas[:1], xs)
    assert info[0] == 0
    v = var[0].cpu().numpy()[idx]
    err = np.max(np.abs(v - np.array(g["var"])) / np.array(g["var"]))
    say(f"  max relative error of the sampled variances {err:.2e}")
    assert err <= RTOL
