"""Pins of the FP64 warm-start network reference: the hand-written
backpropagation against central finite differences of the forward pass, and the
GELU derivative against finite differences of the erf form."""
import numpy as np

from oracle import mlp_oracle as M


def test_gelu_derivative_matches_finite_differences():
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(z))) < 1e-8
    assert abs(M.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15   # Phi(1)


def test_backprop_matches_central_differences():
    I, H, O, B = 4, 7, 5, 3
    rng = np.random.default_rng(0)
    P = sum(int(np.prod(s)) for _, s in M.sizes(I, H, O))
    p = rng.normal(0, 0.5, P)
    u = rng.normal(size=(B, I))
    t = rng.normal(size=(B, O))
    _, g = M.grad(p, u, t, I, H, O)
    h = 1e-6
    fd = np.empty(P)
    for i in range(P):
        e = np.zeros(P)
        e[i] = h
        fd[i] = (M.loss(p + e, u, t, I, H, O) - M.loss(p - e, u, t, I, H, O)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_adam_first_step_is_signed_lr():
    """With zero moments the bias-corrected first Adam step is -lr * sign(g)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = M.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 1e-3)
    assert np.allclose(p, -1e-3 * np.sign(g), rtol=1e-4)


def test_adam_sequence_matches_torch_adam():
    """Moment accumulation and bias correction over many steps: the reference's
    Adam against torch.optim.Adam (CPU, FP64) fed the same gradient sequence,
    with sign changes and magnitudes spread over six decades."""
    import torch
    rng = np.random.default_rng(7)
    P, steps, lr = 50, 12, 3e-3
    p0 = rng.normal(size=P)
    grads = rng.normal(size=(steps, P)) * 10.0 ** rng.uniform(-4, 2, size=(steps, P))
    tp = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(P), np.zeros(P)
    for s in range(steps):
        tp.grad = torch.tensor(grads[s], dtype=torch.float64)
        opt.step()
        p, m, v = M.adam(p, grads[s], m, v, s + 1, lr)
        ref = tp.detach().numpy()
        assert np.max(np.abs(p - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref))), s
        state = opt.state[tp]
        assert np.max(np.abs(m - state["exp_avg"].numpy())) <= 1e-15 * np.max(np.abs(m))
        assert np.max(np.abs(v - state["exp_avg_sq"].numpy())) <= 1e-15 * np.max(np.abs(v))
    # the steps differ from the signed-lr first step: the bias correction matters
    assert np.max(np.abs((p - p0) + lr * steps * np.sign(grads).mean(0))) > 1e-4
