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


# ---------------------------------------------------------------- BF16 trailing
# Unrefined Newton steps factor with BF16 trailing operands; refined steps and
# the factor behind log|Q*| are FP32, so the FP32 bounds above still apply.  A
# BF16 step is a less exact Newton step, so the iteration count may exceed the
# oracle's by up to two.
BF16_LOGDET_RTOL = 1e-4   # log-det of a factorisation with BF16 trailing operands throughout


@pytest.mark.parametrize("shape", [(40, 9), (100, 30)])
def test_bf16_laplace_against_oracle(lib, shape):
    from paper_2311_08050_amd import binding
    m = synth.kron_poisson(*shape, seed=11)
    th0 = synth.kron_theta0(shape[1])
    thetas = np.stack([th0, th0 + np.array([0.3, -0.2, 0.4, 0.1])])
    say(f"bf16 kron {shape}")
    lib.profile(True)
    res, xs = lib.laplace_eval(dev_models([m, m]), thetas, prec="bf16")
    bf = lib.profile_get(binding.K_TRAIL, "bf16")
    lib.profile(False)
    # with n within one 512-wide panel there is no trailing update of Q* itself
    # (the correction-form steps still run); beyond it the BF16 kernel must run
    assert (bf["launches"] > 0) == (m["n"] > 512), bf
    for b in range(2):
        ref = O.laplace_eval(m, thetas[b])
        r, x = res[b], xs[b].cpu().numpy()
        assert r["info"] == 0 and r["fallback"] == 0 and r["ir_steps"] >= 1
        assert ref["iters"] - 1 <= r["iters"] <= ref["iters"] + 2, (r["iters"], ref["iters"])
        assert np.max(np.abs(x - ref["x"])) / max(1.0, np.max(np.abs(ref["x"]))) <= MODE_RTOL
        for key in ("logdet_qprior", "logdet_sprior", "ese"):
            assert rel(r[key], ref[key]) <= 1e-9, key
        assert rel(r["logdet_qstar"], ref["logdet_qstar"]) <= LOGDET_RTOL
        assert rel(r["logdet_s"], ref["logdet_s"]) <= LOGDET_S_RTOL
        assert rel(r["objective"], ref["objective"]) <= LOGDET_RTOL


def test_logdet_precisions_on_posterior_precision(lib):
    """log|Q*| of the posterior precision at the mode (n = 2048: several panels,
    trailing updates of every size) in FP64, FP32 and with BF16 trailing operands."""
    import torch
    m = synth.kron_poisson(64, 32, seed=12)
    th = synth.kron_theta0(32) + np.array([0.2, -0.1, 0.3, 0.0])
    ref = O.laplace_eval(m, th)
    Q = O.prior_precision(m, th) + np.diag(m["E"] * np.exp(th[3] + ref["x"]))
    ld_ref, _, info = O.logdet(Q)
    assert info == 0
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6), ("bf16", BF16_LOGDET_RTOL)):
        ld, inf = lib.logdet([torch.tensor(Q).cuda()], prec=prec)
        say(f"logdet {prec}: relative error {abs(ld[0] - ld_ref) / abs(ld_ref):.2e}")
        assert inf[0] == 0 and abs(ld[0] - ld_ref) <= tol * abs(ld_ref), (prec, ld[0], ld_ref)


def ill_conditioned_model(n=300, seed=11):
    """Poisson model with a dense prior whose eigenvalues run geometrically from
    1 down to 1e-10 (condition 1e10): positive definite in FP64 (u_64 cond ~
    1e-6), far beyond FP32 (u_32 cond ~ 6e2), so an FP32 Cholesky of Q* meets a
    non-positive pivot (LAPACK's spotrf fails at pivot 216 on it).  y = 0 and an
    exposure of 1e-17 keep W = E e^x ~ 1e-17, so Q* ~ Q_prior, and the mode of
    order 1e-7, where FP64 Newton converges in two steps (the oracle's too)."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.normal(size=(n, n)))
    Q = (U * np.logspace(0.0, -10.0, n)) @ U.T
    Q = 0.5 * (Q + Q.T)
    return {"n": n, "lik": "poisson", "prior": "dense", "y": np.zeros(n), "E": np.full(n, 1e-17), "A": None,
            "C": None, "e": None, "coords": None, "n_s": n, "n_t": 1, "Qprior": Q}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_low_precision_breakdown_is_redone_in_fp64(lib, prec):
    """A Q* that is positive definite in FP64 but whose low-precision factor
    breaks down is re-evaluated in FP64 (fallback bit 0, info 0) and matches the
    FP64 path; a well-conditioned theta of the same batch stays mixed.  From a
    warm start the same holds: the FP64 re-evaluation, not a zero-start retry in
    the failing precision."""
    import torch
    bad = ill_conditioned_model()
    good = synth.kron_poisson(13, 7, seed=5)
    th_bad, th_good = np.array([0.0, 0, 0, 0]), synth.kron_theta0(7)
    dms = dev_models([bad, good])
    ths = np.stack([th_bad, th_good])
    say(f"{prec} breakdown on an FP64-definite Q* (cond 1e10)")
    r64, x64 = lib.laplace_eval(dms, ths, prec="fp64")
    assert r64[0]["info"] == 0 and r64[1]["info"] == 0, (r64[0]["info"], r64[1]["info"])
    for start in (0, 1):
        xs = [torch.zeros(bad["n"], dtype=torch.float64, device="cuda"),
              torch.zeros(good["n"], dtype=torch.float64, device="cuda")]
        r, xs = lib.laplace_eval(dms, ths, x=xs, start=start, prec=prec)
        assert r[0]["info"] == 0 and r[0]["fallback"] & 1 and not r[0]["fallback"] & 2, (start, r[0])
        assert abs(r[0]["objective"] - r64[0]["objective"]) <= 1e-12 * max(1.0, abs(r64[0]["objective"]))
        assert torch.equal(xs[0], x64[0])
        assert r[1]["info"] == 0 and r[1]["fallback"] == 0
        assert rel(r[1]["objective"], r64[1]["objective"]) <= LOGDET_RTOL
    ref = O.laplace_eval(bad, th_bad)
    assert ref["info"] == 0
    assert np.max(np.abs(x64[0].cpu().numpy() - ref["x"])) <= MODE_RTOL * max(1.0, np.max(np.abs(ref["x"])))
