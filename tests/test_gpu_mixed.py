"""Mixed precision (FP32 storage and FP32 MFMA for the Newton and final-pass
factorisations, FP64 prior pass, FP64 log-det sums, FP64 kriging system and
FP64 iterative refinement of every constrained Newton solve) against the FP64
oracle.

Bounds: the mode is refined to FP64 accuracy, so it must meet the FP64 bar
(1e-9 relative).  Log-determinants come from the FP32 factor: each pivot
carries a relative error of order kappa(Q*) u_32 (u_32 = 6e-8, kappa(Q*) <= ~1e2
here), so log|Q*| is within n * kappa * u_32 absolute; the tests state 2e-6
relative for log|Q*| and the objective, and 1e-5 relative for log|S|.
"""
import sys

import numpy as np
import pytest

from oracle import inla_oracle as O
from paper_2311_08050_amd import synth

pytestmark = pytest.mark.gpu
MODE_RTOL = 1e-9
LOGDET_RTOL = 2e-6
LOGDET_S_RTOL = 1e-5


def say(msg):
    print(f"[gpu-mixed] {msg}", flush=True)
    sys.stdout.flush()


def dev_models(models):
    from paper_2311_08050_amd.binding import DeviceModel
    return [DeviceModel(m) for m in models]


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def check_mixed(res, x, ref, what):
    assert res["info"] == 0 and ref["info"] == 0, (what, res["info"])
    assert res["fallback"] == 0, what
    assert res["ir_steps"] >= 1, what   # the converged step is always refined
    assert abs(res["iters"] - ref["iters"]) <= 1, (what, res["iters"], ref["iters"])
    err = np.max(np.abs(x - ref["x"])) / max(1.0, np.max(np.abs(ref["x"])))
    assert err <= MODE_RTOL, (what, "mode", err)
    # the prior pass is FP64
    for key in ("logdet_qprior", "logdet_sprior", "ese"):
        assert rel(res[key], ref[key]) <= 1e-9, (what, key)
    assert rel(res["logdet_qstar"], ref["logdet_qstar"]) <= LOGDET_RTOL, (what, res["logdet_qstar"], ref["logdet_qstar"])
    assert rel(res["logdet_s"], ref["logdet_s"]) <= LOGDET_S_RTOL, (what, res["logdet_s"], ref["logdet_s"])
    assert rel(res["objective"], ref["objective"]) <= LOGDET_RTOL, (what, res["objective"], ref["objective"])


@pytest.mark.parametrize("shape", [(13, 7), (40, 9), (100, 30)])
def test_fp32_laplace_against_oracle(lib, shape):
    m = synth.kron_poisson(*shape, seed=11)
    th0 = synth.kron_theta0(shape[1])
    thetas = np.stack([th0, th0 + np.array([0.3, -0.2, 0.4, 0.1])])
    say(f"fp32 kron {shape}")
    res, xs = lib.laplace_eval(dev_models([m, m]), thetas, prec="fp32")
    for b in range(2):
        check_mixed(res[b], xs[b].cpu().numpy(), O.laplace_eval(m, thetas[b]), f"{shape}[{b}]")


def test_fp32_dense_prior_nonzero_rhs_and_gaussian(lib):
    ms = [synth.dense_poisson(150, 3, seed=2), synth.expcov_gaussian(130, seed=4, constrained=True)]
    ths = np.array([[0.1, 0, 0, 0], [0.2, np.log(0.3), np.log(0.4), 0.0]])
    say("fp32 dense + gaussian")
    res, xs = lib.laplace_eval(dev_models(ms), ths, prec="fp32")
    for b in range(2):
        check_mixed(res[b], xs[b].cpu().numpy(), O.laplace_eval(ms[b], ths[b]), f"mixed[{b}]")


def test_fp32_matches_fp64_path_on_the_same_gpu(lib):
    """All theta of a batch: modes agree with the FP64 GPU path to 1e-9."""
    m, thetas = synth.headline(B=4, n_s=32, n_t=16)
    dm = dev_models([m] * 4)
    say("fp32 vs fp64 on GPU, n=512")
    r64, x64 = lib.laplace_eval(dm, thetas)
    r32, x32 = lib.laplace_eval(dm, thetas, prec="fp32")
    for b in range(4):
        assert r32[b]["info"] == 0 and r32[b]["fallback"] == 0
        a, c = x32[b].cpu().numpy(), x64[b].cpu().numpy()
        assert np.max(np.abs(a - c)) <= MODE_RTOL * max(1.0, np.max(np.abs(c)))
        assert rel(r32[b]["objective"], r64[b]["objective"]) <= LOGDET_RTOL
