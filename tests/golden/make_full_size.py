"""Write the stored oracle values of the full-size parity tests.

The FP64 oracle needs minutes per evaluation at n = 8192 and n = 16384 on a
host CPU, too long to rerun inside a GPU test.  This script evaluates it once,
on the seeded synthetic models that the tests rebuild with ``synth``, and writes
what the tests compare against:

  kron8192_theta0.json   the headline model (128 regions x 64 times, k = 191)
                         at theta 0 of its 64-point batch (seed 81);
  kron16384_theta0.json  the precision configuration (128 regions x 128 times,
                         k = 255, seed 4) at theta0.

Each file holds every scalar term of the Laplace objective (Eq. (41) with the
constraint terms), the Newton iteration count, the mode and the kriging-
corrected marginal variances at sampled indices (every STRIDE-th index plus the
last one), and their maxima.

With ``ns8192`` or ``ns16384``, it writes instead the same case's objective,
mode and marginal variances by the constraint-surface route of
``oracle/nullspace_route.py`` (``*_nullspace.json``), which pins the stored
kriging-oracle values at full size.  With ``vb8192`` it writes the
variational-Bayes corrected mean of the headline case (``oracle/vb_oracle.py``
from the oracle's mode and marginal variances) at the same sampled indices
(``kron8192_theta0_vb.json``).  It calls only ``oracle/`` and the input
generator ``synth`` (which holds none of the method's arithmetic); nothing here
reads the GPU library.

    python tests/golden/make_full_size.py [8192|16384|ns8192|ns16384|vb8192 ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import inla_oracle as O  # noqa: E402
from oracle import nullspace_route as NS  # noqa: E402
from oracle import vb_oracle as V  # noqa: E402
from paper_2311_08050_amd import synth  # noqa: E402

STRIDE = 8
SCALARS = ("objective", "logdet_qprior", "logdet_sprior", "ese", "logdet_qstar", "logdet_s", "xqx", "loglik")


def case(n):
    """(file name, model, theta, description) of a full-size case."""
    if n == 8192:
        model, thetas = synth.headline(B=64)
        return "kron8192_theta0.json", model, thetas[0], "synth.headline(B=64): theta 0 of the batch"
    if n == 16384:
        return ("kron16384_theta0.json", synth.kron_poisson(128, 128, seed=4), synth.kron_theta0(128),
                "synth.kron_poisson(128, 128, seed=4) at synth.kron_theta0(128)")
    raise ValueError(n)


def sample_index(n):
    idx = list(range(0, n, STRIDE))
    if idx[-1] != n - 1:
        idx.append(n - 1)
    return idx


def write(n):
    fname, model, theta, what = case(n)
    t0 = time.perf_counter()
    ref = O.laplace_eval(model, theta)
    t1 = time.perf_counter()
    assert ref["info"] == O.INFO_OK, ref["info"]
    var = O.marginal_var(model, theta, ref["x"])
    t2 = time.perf_counter()
    idx = sample_index(model["n"])
    out = {
        "what": f"FP64 oracle (oracle/inla_oracle.py laplace_eval, marginal_var) on {what}",
        "n": int(model["n"]), "k": int(model["C"].shape[0]),
        "theta": [float(v) for v in theta],
        "iters": int(ref["iters"]),
        **{key: float(ref[key]) for key in SCALARS},
        "index": idx,
        "x": [float(ref["x"][i]) for i in idx],
        "x_absmax": float(np.max(np.abs(ref["x"]))),
        "var": [float(var[i]) for i in idx],
        "var_max": float(np.max(var)),
        "oracle_seconds": {"laplace_eval": t1 - t0, "marginal_var": t2 - t1},
    }
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"{fname}: n={model['n']} iters={ref['iters']} objective={ref['objective']!r} "
          f"({t1 - t0:.0f} s + {t2 - t1:.0f} s)", flush=True)


def write_nullspace(n):
    fname, model, theta, what = case(n)
    t0 = time.perf_counter()
    Q = NS.kron_prior(model, theta)
    y = np.asarray(model["y"], dtype=np.float64)
    E = np.asarray(model["E"], dtype=np.float64)
    x, obj, gmax, var = NS.nullspace_laplace(Q, None, y, E, float(theta[3]), model["C"], model["e"])
    t1 = time.perf_counter()
    idx = sample_index(model["n"])
    out = {
        "what": f"constraint-surface route (oracle/nullspace_route.py) on {what}",
        "n": int(model["n"]), "k": int(model["C"].shape[0]),
        "theta": [float(v) for v in theta],
        "objective": float(obj),
        "gradient_absmax": gmax,
        "constraint_residual": float(np.max(np.abs(model["C"] @ x - model["e"]))),
        "index": idx,
        "x": [float(x[i]) for i in idx],
        "x_absmax": float(np.max(np.abs(x))),
        "var": [float(var[i]) for i in idx],
        "var_max": float(np.max(var)),
        "seconds": t1 - t0,
    }
    name = fname.replace(".json", "_nullspace.json")
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"{name}: objective={obj!r} ({t1 - t0:.0f} s)", flush=True)


def write_vb(n):
    fname, model, theta, what = case(n)
    t0 = time.perf_counter()
    ref = O.laplace_eval(model, theta)
    assert ref["info"] == O.INFO_OK, ref["info"]
    var = O.marginal_var(model, theta, ref["x"])
    t1 = time.perf_counter()
    mu, iters, info = V.vb_mean(model, theta, ref["x"], var)
    t2 = time.perf_counter()
    assert info == O.INFO_OK, info
    idx = sample_index(model["n"])
    out = {
        "what": f"variational-Bayes corrected mean (oracle/vb_oracle.py vb_mean from the oracle's mode and marginal "
                f"variances) on {what}",
        "n": int(model["n"]), "k": int(model["C"].shape[0]),
        "theta": [float(v) for v in theta],
        "iters": int(iters),
        "index": idx,
        "mu": [float(mu[i]) for i in idx],
        "mu_absmax": float(np.max(np.abs(mu))),
        "shift_from_mode_absmax": float(np.max(np.abs(mu - ref["x"]))),
        "oracle_seconds": {"mode_and_variances": t1 - t0, "vb_mean": t2 - t1},
    }
    name = fname.replace(".json", "_vb.json")
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"{name}: {iters} iterations, shift from the mode {out['shift_from_mode_absmax']:.3e} "
          f"({t2 - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["8192", "16384"]:
        if arg.startswith("ns"):
            write_nullspace(int(arg[2:]))
        elif arg.startswith("vb"):
            write_vb(int(arg[2:]))
        else:
            write(int(arg))
