"""GPU parity for models with a general design matrix A (eta = offset + A x,
Q* = Q_prior + A^T W A): the crossed random effects of the paper's Introduction,
whose A^T A makes the posterior precision dense.  Element by element against
the FP64 oracle (which applies A densely), 1e-9 relative, including a batch that
mixes A = I and general-A models in one call."""
import math
import sys

import numpy as np
import pytest

from oracle import inla_oracle as O
from paper_2311_08050_amd import synth

pytestmark = pytest.mark.gpu
RTOL = 1e-9


def say(msg):
    print(f"[gpu-design] {msg}", flush=True)
    sys.stdout.flush()


def dev_models(models):
    from paper_2311_08050_amd.binding import DeviceModel
    return [DeviceModel(m) for m in models]


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def check(res, x, ref, what):
    assert res["info"] == ref["info"] == 0, (what, res["info"])
    assert abs(res["iters"] - ref["iters"]) <= 1, (what, res["iters"], ref["iters"])
    for key in ("objective", "logdet_qprior", "logdet_sprior", "logdet_qstar", "logdet_s", "xqx", "loglik"):
        assert rel(res[key], ref[key]) <= RTOL, (what, key, res[key], ref[key])
    err = np.max(np.abs(x - ref["x"])) / max(1.0, np.max(np.abs(ref["x"])))
    assert err <= RTOL, (what, "mode", err)


@pytest.mark.parametrize("lik,stz", [("gaussian", False), ("gaussian", True), ("poisson", False), ("poisson", True)])
def test_crossed_effects_against_oracle(lib, lik, stz):
    m = synth.crossed_effects(30, 20, 300, seed=41, lik=lik, sum_to_zero=stz)
    th = np.array([[math.log(0.6)], [math.log(1.4)]]) if lik == "gaussian" else np.array([[0.0], [0.2]])
    say(f"crossed effects {lik} (sum to zero: {stz}): n={m['n']}, m={len(m['y'])}")
    dms = dev_models([m, m])
    res, xs = lib.laplace_eval(dms, th)
    for b in range(2):
        check(res[b], xs[b].cpu().numpy(), O.laplace_eval(m, th[b]), f"{lik}[{b}]")
    var, info = lib.marginal_var(dms, th, xs)
    for b in range(2):
        ref = O.marginal_var(m, th[b], O.laplace_eval(m, th[b])["x"])
        assert info[b] == 0
        assert np.max(np.abs(var[b].cpu().numpy() - ref)) <= RTOL * np.max(np.abs(ref))


def test_mixed_batch_of_identity_and_general_designs(lib):
    ms = [synth.crossed_effects(40, 25, 500, seed=42, lik="poisson", sum_to_zero=True), synth.kron_poisson(13, 7, seed=5),
          synth.crossed_effects(10, 90, 300, seed=43, lik="poisson")]
    th = [np.array([0.1, 0, 0, 0]), synth.kron_theta0(7), np.array([-0.1, 0, 0, 0])]
    say("mixed batch: crossed effects, space-time (A = I), crossed effects")
    res, xs = lib.laplace_eval(dev_models(ms), np.stack(th))
    for b, (m, t) in enumerate(zip(ms, th)):
        check(res[b], xs[b].cpu().numpy(), O.laplace_eval(m, t), f"mixed[{b}]")


def test_general_design_rejects_low_precision_and_vb(lib):
    from paper_2311_08050_amd.binding import LibraryError
    m = synth.crossed_effects(10, 10, 50, seed=44, lik="poisson")
    dms = dev_models([m])
    with pytest.raises(LibraryError, match="-1002"):
        lib.laplace_eval(dms, np.array([[0.0]]), prec="fp32")
    _, xs = lib.constrained_mode(dms, np.array([[0.0]]))
    var, _ = lib.marginal_var(dms, np.array([[0.0]]), xs)
    with pytest.raises(LibraryError, match="-1002"):
        lib.vb_mean(dms, np.array([[0.0]]), var, xs)


def test_crossed_effects_at_n2048(lib):
    """1024 x 1024 levels, 8192 Poisson observations: a dense 2048 x 2048 Q*."""
    import time
    m = synth.crossed_effects(1024, 1024, 8192, seed=45, lik="poisson", sum_to_zero=True)
    th = np.array([[0.0], [0.1], [-0.1], [0.05]])
    dms = dev_models([m])
    dms = dms * 4
    lib.laplace_eval(dms[:1], th[:1])
    t0 = time.perf_counter()
    res, xs = lib.laplace_eval(dms, th)
    dt = time.perf_counter() - t0
    say(f"crossed effects n=2048 (m=8192): {4 / dt:.1f} theta-evals/s, iterations {[r['iters'] for r in res]}")
    ref = O.laplace_eval(m, th[0])
    check(res[0], xs[0].cpu().numpy(), ref, "n2048")
