"""The learned warm start: the GPU network's forward pass, gradients and Adam
step against the FP64 reference (oracle/mlp_oracle.py, itself pinned by finite
differences), and what the trained network gains over the zero start on a held-out
batch: fewer Newton iterations with the same converged evaluation (1e-10)."""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2311_08050_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-mlp] {msg}", flush=True)
    sys.stdout.flush()


def params(I, H, O, seed):
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, (H, I)) * np.sqrt(6 / I), rng.normal(0, 0.1, H),
             rng.uniform(-1, 1, (H, H)) * np.sqrt(6 / H), rng.normal(0, 0.1, H),
             rng.uniform(-1, 1, (O, H)) * np.sqrt(3 / H), rng.normal(0, 0.1, O)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


@pytest.fixture(scope="module")
def net(lib):
    import torch
    from paper_2311_08050_amd.binding import Mlp
    I, H, O, B = 4, 256, 300, 64
    p = params(I, H, O, 1)
    m = Mlp(lib, I, H, O)
    assert m.num_params == p.size
    m.set_params(torch.tensor(p))
    rng = np.random.default_rng(2)
    u = rng.normal(size=(B, I)).astype(np.float32)
    t = rng.normal(size=(B, O))
    return m, p.astype(np.float64), u, t, (I, H, O)


def blockwise_err(a, b, I, H, O):
    out, off = [], 0
    for _, shp in M.sizes(I, H, O):
        c = int(np.prod(shp))
        out.append(np.max(np.abs(a[off:off + c] - b[off:off + c])) / max(1e-30, np.max(np.abs(b[off:off + c]))))
        off += c
    return max(out)


def test_forward_matches_reference(net):
    import torch
    m, p, u, _, (I, H, O) = net
    say("mlp forward")
    y = m.forward(torch.tensor(u)).cpu().numpy()
    ref, _ = M.forward(p, u.astype(np.float64), I, H, O)
    assert np.max(np.abs(y - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


def test_gradients_match_reference(net):
    import torch
    m, p, u, t, (I, H, O) = net
    say("mlp gradients")
    loss, g = m.grad(torch.tensor(u), torch.tensor(t))
    ref_loss, ref_g = M.grad(p, u.astype(np.float64), t, I, H, O)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert blockwise_err(g.cpu().numpy().astype(np.float64), ref_g, I, H, O) <= 1e-4


def test_adam_step_matches_reference(net):
    import torch
    m, p, u, t, (I, H, O) = net
    say("mlp adam step")
    m.set_params(torch.tensor(p.astype(np.float32)))
    U, T = torch.tensor(u).cuda(), torch.tensor(t).cuda()
    m.train_step(U, T, 1e-3)
    new = m.get_params().cpu().numpy().astype(np.float64)
    _, g = M.grad(p, u.astype(np.float64), t, I, H, O)
    ref, _, _ = M.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    # The first Adam step is -lr g / (|g| + eps): about -lr sign(g) where |g| is
    # well above the FP32 gradient error, and at most lr everywhere.
    move, ref_move = new - p, ref - p
    assert np.max(np.abs(move)) <= 1e-3 * (1 + 1e-5) + 1e-7
    big = np.abs(g) >= 1e-3 * np.max(np.abs(g))
    assert big.sum() > 0.5 * g.size
    assert np.max(np.abs(move[big] - ref_move[big])) <= 1e-3 * 1e-3 + 1e-7
    m.set_params(torch.tensor(p.astype(np.float32)))


def test_adam_sequence_matches_reference(net):
    """Six Adam steps in a row: moment accumulation and bias correction from
    step 2 on.  Each GPU step is compared with the FP64 reference's Adam update
    applied to the same parameters and the same gradient (the GPU's own, read
    with inla_mlp_grad, which runs the kernels the step runs), with moments
    accumulated in FP64 over the sequence; the bound is the FP32 rounding of
    the parameters plus 1e-5 of a step."""
    import torch
    m, p, u, t, (I, H, O) = net
    steps, lr = 6, 1e-3
    say("mlp adam, six steps")
    m.set_params(torch.tensor(p.astype(np.float32)))
    U, T = torch.tensor(u).cuda(), torch.tensor(t).cuda()
    cur = m.get_params().cpu().numpy().astype(np.float64)
    mom, vel = np.zeros_like(cur), np.zeros_like(cur)
    for s in range(1, steps + 1):
        _, g = m.grad(U, T)
        g = g.cpu().numpy().astype(np.float64)
        m.train_step(U, T, lr)
        new = m.get_params().cpu().numpy().astype(np.float64)
        ref, mom, vel = M.adam(cur, g, mom, vel, s, lr)
        err = np.max(np.abs(new - ref))
        tol = 2 * np.finfo(np.float32).eps * np.max(np.abs(cur)) + 1e-5 * lr
        assert err <= tol, (s, err, tol)
        if s == steps:
            say(f"step {s}: max |GPU - reference| {err:.2e} (bound {tol:.2e}), "
                f"max |move / lr| {np.max(np.abs(new - cur)) / lr:.3f}")
        cur = new
    m.set_params(torch.tensor(p.astype(np.float32)))


def test_trained_warm_start_saves_newton_iterations(lib):
    import torch
    from paper_2311_08050_amd import warmstart
    from paper_2311_08050_amd.binding import DeviceModel
    model = synth.kron_poisson(40, 16, seed=21)        # n = 640, k = 55
    dm = DeviceModel(model)
    th0 = synth.kron_theta0(16)
    scale = np.full(4, 0.5)
    train = synth.normal_batch(th0, 192, 0.5, seed=51)
    test = synth.normal_batch(th0, 32, 0.5, seed=52)
    say("mlp warm start: training")
    mlp, info = warmstart.train(lib, dm, train, th0, scale, hidden=128, epochs=150, lr=2e-3)
    assert info["loss_last"] < 0.05 * info["loss_first"], info
    say("mlp warm start: zero vs warm on held-out theta")
    r0, x0 = lib.laplace_eval([dm] * 32, test)
    xw = mlp.predict_modes(test, th0, scale)
    rw, xw = lib.laplace_eval([dm] * 32, test, x=xw, start=1)
    it0 = np.mean([r["iters"] for r in r0])
    itw = np.mean([r["iters"] for r in rw])
    say(f"mean Newton iterations: zero start {it0:.2f}, warm start {itw:.2f}")
    assert itw < it0 - 1.0
    for b in range(32):
        assert rw[b]["info"] == 0 and rw[b]["fallback"] == 0
        a, c = xw[b].cpu().numpy(), x0[b].cpu().numpy()
        assert np.max(np.abs(a - c)) <= 1e-10 * max(1.0, np.max(np.abs(c)))
        assert abs(rw[b]["objective"] - r0[b]["objective"]) <= 1e-10 * abs(r0[b]["objective"])


def test_failed_warm_start_falls_back_to_zero_start(lib):
    """A start vector full of NaN is rejected and the theta re-solved from zero."""
    import torch
    from paper_2311_08050_amd.binding import DeviceModel
    model = synth.kron_poisson(13, 7, seed=5)
    dm = DeviceModel(model)
    th = synth.kron_theta0(7)[None, :]
    say("warm start fallback")
    r0, x0 = lib.laplace_eval([dm], th)
    bad = [torch.full((model["n"],), float("nan"), dtype=torch.float64, device="cuda")]
    r1, x1 = lib.laplace_eval([dm], th, x=bad, start=1)
    assert r1[0]["info"] == 0 and r1[0]["fallback"] & 2
    assert abs(r1[0]["objective"] - r0[0]["objective"]) <= 1e-12 * abs(r0[0]["objective"])
