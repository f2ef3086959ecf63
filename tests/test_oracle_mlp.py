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
