"""Training driver of the learned warm start (the network and its kernels live
in the C-ABI library; this module only sequences calls).

The training set is a batch of hyperparameter points solved by the method
itself (inla_constrained_mode writes the modes straight into the rows of one
FP64 device array, which are the regression targets).  Inputs are the
normalised points u = (theta - centre) / scale, prepared on the host.  Batches
are contiguous slices of the (already randomly drawn) training set.
"""
from __future__ import annotations

import time

import numpy as np


def solve_modes(lib, dmodel, thetas, prec="fp32", batch=64):
    """Modes of `dmodel` at each theta (rows of one (N x n) float64 device tensor)."""
    import torch

    N, n = len(thetas), dmodel.n
    X = torch.zeros((N, n), dtype=torch.float64, device="cuda")
    iters = []
    for s in range(0, N, batch):
        e = min(N, s + batch)
        res, _ = lib.constrained_mode([dmodel] * (e - s), thetas[s:e], x=[X[i] for i in range(s, e)], prec=prec)
        bad = [r["info"] for r in res if r["info"] != 0]
        if bad:
            raise RuntimeError(f"training targets: Newton failed with info {bad}")
        iters += [r["iters"] for r in res]
    return X, iters


def train(lib, dmodel, thetas, centre, scale, hidden=256, epochs=200, batch=64, lr=1e-3, seed=0, prec="fp32",
          lr_final=0.01, normalise=True):
    """Solve the training points, fit the network, return (mlp, info dict).

    Adam with a cosine learning-rate decay from `lr` to `lr_final * lr`; the
    training set is visited in a fresh random order every epoch (seeded).
    With `normalise` the network is fitted to the modes centred on their mean
    and divided by their standard deviation, and the two are folded into the
    last layer afterwards (W3 <- s W3, b3 <- s b3 + mean), so that it predicts
    modes directly."""
    import math

    import torch

    from .binding import Mlp

    t0 = time.perf_counter()
    X, iters = solve_modes(lib, dmodel, thetas, prec=prec)
    t_solve = time.perf_counter() - t0
    mean, sd = None, 1.0
    if normalise:
        mean = X.mean(0)
        sd = float((X - mean).std()) or 1.0
        X = (X - mean) / sd
    U = torch.tensor(((np.asarray(thetas) - centre) / scale).astype(np.float32), device="cuda")
    mlp = Mlp(lib, U.shape[1], hidden, dmodel.n, seed=seed)
    N = len(thetas)
    rng = np.random.default_rng(seed)
    per_epoch = max(1, N // batch)
    total, k = epochs * per_epoch, 0
    losses = []
    t1 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(N), device="cuda")
        Us, Xs = U.index_select(0, perm), X.index_select(0, perm)
        last = N - batch   # the epoch's last batch reports its loss; the others do not wait for the device
        for s in range(0, N - batch + 1, batch):
            step_lr = lr * (lr_final + (1.0 - lr_final) * 0.5 * (1.0 + math.cos(math.pi * k / total)))
            loss = mlp.train_step(Us[s:s + batch], Xs[s:s + batch], step_lr, want_loss=(s + batch > last))
            k += 1
        losses.append(loss)
    if normalise:
        # fold the target normalisation into the output layer (flat layout
        # W1, b1, W2, b2, W3 (O x H), b3 (O))
        I, H, O = mlp.dims
        p = mlp.get_params().double()
        o_w3 = H * I + H + H * H + H
        o_b3 = o_w3 + O * H
        p[o_w3:o_b3] *= sd
        p[o_b3:] = p[o_b3:] * sd + mean
        mlp.set_params(p.float())
    t_train = time.perf_counter() - t1
    # losses: the last batch's mean squared error (before its step) in the first and last epoch
    return mlp, {"solve_s": t_solve, "train_s": t_train, "loss_first": losses[0], "loss_last": losses[-1],
                 "zero_start_iters_mean": float(np.mean(iters)), "n_train": N, "epochs": epochs,
                 "target_scale": sd}
