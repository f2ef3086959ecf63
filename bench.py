"""Benchmark: batched Laplace evaluations of pi(theta | y) per second on one MI355X.

Workload: the n = 8192 Poisson space x time interaction model (128 regions x 64
times, Q_prior = tau (R_t kron Sigma_s(rho)^{-1} + delta I), k = 191 independent
sum-to-zero constraints), a batch of 64 theta ~ N(theta0, 0.5^2 I).  One step =
one inla_laplace_eval over the batch (prior build, FP64 prior pass, Newton
iterations with kriging, final pass at the mode, objective; the prior pass runs
beside the Newton iterations on a second stream of the handle unless
--no-overlap).  Inputs are synthetic (seeded) and resident in HBM before the
timed region.

Variants (each timed separately, same batch):
  fp64        FP64 everywhere, Newton from x = 0
  fp32        FP32-storage FP32-MFMA factorisations of Q* with FP64 refinement,
              Newton from x = 0
  bf16        as fp32, but the unrefined Newton steps factor with BF16 trailing
              operands (FP32 accumulation)
  fp32+mlp,   as fp32 / bf16, Newton started from the learned warm start (the
  bf16+mlp    network's prediction runs inside the timed step; its one-time
              training on modes of separately drawn theta is reported, not timed)
The headline `value` is the last variant in --variants.

Prints one JSON line.  The roofline object describes the dominant trailing-update
MFMA kernel of the headline variant, timed with HIP events on the library's
stream over the timed region.  cpu_baseline is the CPU
oracle timed on this host on a bounded sample (one theta of the batch).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "θ-evals/sec + TFLOP/s vs MFMA peak at n=8192, FP64 vs mixed+warm-start"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # dense MFMA peaks
TYPE_NAME = {"fp64": "double", "fp32": "float"}


def trail_kernel_name(precision, tile, aux=False):
    """Symbol of the trailing-update kernel of a precision at the tuned tile
    (`aux`: the kernel of a factorisation on the handle's aux stream, i.e. the
    concurrent prior pass)."""
    if precision == "bf16":
        return "trail_bf16_kernel<128,128>"
    name = "trail_update_aux_kernel" if aux else "trail_update_kernel"
    return f"{name}<{TYPE_NAME[precision]},{tile},{tile}>"
MLP_TRAIN = {"n_train": 2048, "epochs": 6400, "batch": 256, "hidden": 256, "lr": 4e-3, "lr_final": 0.01, "seed": 91}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def traffic_from_profile(kernel_source, summary_md, kernel_instance, alg_bytes_per_launch=None):
    """HBM bytes per launch of the trailing-update kernel from the committed
    counter summary (its `kernel_instance:`, `kernel_source_sha256:`,
    `traffic_bytes_per_launch:` and, if present, `traffic_alg_ratio:` lines),
    or None if the summary is missing, was taken on a different kernel source
    or on another instance (tile size) than the one this run timed.  With a
    ratio and this run's algorithmic bytes per launch the figure is their
    product (the counters may come from another launch mix of the same
    kernel), else the summary's bytes per launch."""
    import hashlib
    try:
        with open(summary_md) as f:
            lines = f.read().splitlines()
        with open(kernel_source, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    fields = {}
    for ln in lines:
        ln = ln.strip().lstrip("-* ").replace("`", "")
        if ":" in ln:
            key, val = ln.split(":", 1)
            fields[key.strip()] = val.strip()
    if fields.get("kernel_source_sha256") != digest or fields.get("kernel_instance") != kernel_instance:
        return None
    try:
        if alg_bytes_per_launch and "traffic_alg_ratio" in fields:
            return float(fields["traffic_alg_ratio"]) * float(alg_bytes_per_launch)
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def rocprof_window(csv_path, bench_json, precision=None):
    """Average a rocprofv3 per-dispatch CSV (kernel trace or counter collection)
    over the timed region: the last `launches` dispatches of the headline's
    roofline kernel (or of its trailing-update kernel of `precision`) named in
    the JSON line that the profiled bench run printed."""
    import csv

    with open(bench_json) as f:
        line = json.loads([ln for ln in f if ln.startswith("{")][-1])
    roof = line["roofline"]
    if precision:
        tk = line["variants"][line["config"]["variant"]]["trail_kernels"][precision]
        roof = {"kernel": tk["kernel"], "launches": tk["launches"], "avg_launch_ms": tk["avg_launch_ms"]}
    name = roof["kernel"].split(" ")[0].replace("inla::", "")
    nlast = int(roof["launches"])
    rows = []
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row["Kernel_Name"].replace(" ", "").split("(")[0].endswith(name):
                key = int(row.get("Dispatch_Id") or row["Correlation_Id"])
                if "Counter_Value" in row:
                    rows.append((key, float(row["Counter_Value"]), row["Counter_Name"]))
                else:
                    rows.append((key, (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-6, "duration_ms"))
    rows.sort()
    win = [v for _, v, _ in rows[-nlast:]]
    what = rows[0][2] if rows else "none"
    return {"kernel": name, "dispatches_in_csv": len(rows), "window": len(win), "quantity": what,
            "window_mean": sum(win) / len(win) if win else None,
            "all_mean": sum(v for _, v, _ in rows) / len(rows) if rows else None,
            "bench_avg_launch_ms": roof["avg_launch_ms"], "bench_launches": roof["launches"],
            "bench_alg_bytes_per_launch": roof.get("alg_bytes_per_launch")}


def run_variant(lib, binding, dms, thetas, xs, variant, steps, warmup, warm=None):
    import numpy as np
    import torch

    prec = variant.split("+")[0]

    def tname(p):   # the trailing kernel at the tile the handle uses for this batch
        # (a mixed variant's FP64 updates are its prior pass, on the aux stream
        # with overlap on; the fp64 variant's are mostly its Newton passes)
        aux = p == "fp64" and prec != "fp64" and lib.overlap
        return trail_kernel_name(p, lib.tune_get(p, dms[0].n, len(dms))[1], aux)

    def step():
        if warm is None:
            return lib.laplace_eval(dms, thetas, x=xs, prec=prec)
        mlp, centre, scale, max_iter = warm
        mlp.predict_modes(thetas, centre, scale, x=xs)
        return lib.laplace_eval(dms, thetas, x=xs, start=1, max_iter=max_iter, prec=prec)

    for w in range(warmup):
        res, _ = step()
        log(f"{variant}: warmup {w} done, iters {[r['iters'] for r in res][:8]}...")
    torch.cuda.synchronize()
    lib.profile(True)
    t0 = time.perf_counter()
    for s in range(steps):
        res, _ = step()
        log(f"{variant}: step {s} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # counters per precision: a mixed variant files its FP64 prior pass under fp64
    stats_by = {p: {binding.K_NAMES[c]: lib.profile_get(c, p) for c in binding.K_NAMES}
                for p in ("fp64", "fp32", "bf16")}
    lib.profile(False)
    # the dominant trailing-update kernel of the variant (a BF16 variant runs
    # both BF16 and FP32 trailing updates; the prior pass is FP64 in every variant)
    key = max(("fp32", "bf16") if prec != "fp64" else ("fp64",), key=lambda p: stats_by[p]["trail"]["time_ms"])
    stats = stats_by[key]
    infos = [r["info"] for r in res]
    assert all(i == 0 for i in infos), infos
    iters = np.array([r["iters"] for r in res])
    trail = stats["trail"]
    achieved = trail["flops"] / (trail["time_ms"] * 1e-3) / 1e12 if trail["time_ms"] > 0 else 0.0
    fact = ("trail", "panel", "potf2", "border")
    fact_ms = sum(stats[c]["time_ms"] for c in fact)
    fact_flops = sum(stats[c]["flops"] for c in fact)
    peak = PEAK_TFLOPS[key]
    return {
        "value": steps * len(dms) / dt,
        "ms_per_step": dt / steps * 1e3,
        "newton_iters": {"mean": float(iters.mean()), "max": int(iters.max()), "min": int(iters.min())},
        "ir_steps_mean": float(np.mean([r["ir_steps"] for r in res])),
        "fp64_fallbacks": int(sum(r["fallback"] & 1 for r in res)),
        "zero_start_fallbacks": int(sum((r["fallback"] >> 1) & 1 for r in res)),
        "roofline": {
            "bound": "mfma",
            "kernel": f"{tname(key)} ({key.upper()} MFMA trailing update of the blocked Cholesky)",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "precision": key,
            "launches": trail["launches"],
            "avg_launch_ms": trail["time_ms"] / max(1, trail["launches"]),
            "alg_flops_per_launch": trail["flops"] / max(1, trail["launches"]),
            "alg_bytes_per_launch": trail["bytes"] / max(1, trail["launches"]),
        },
        "trail_kernels": {
            p: {"kernel": tname(p), "launches": sb["trail"]["launches"],
                "avg_launch_ms": sb["trail"]["time_ms"] / sb["trail"]["launches"],
                "achieved_tflops": sb["trail"]["flops"] / (sb["trail"]["time_ms"] * 1e-3) / 1e12,
                "frac_of_peak": sb["trail"]["flops"] / (sb["trail"]["time_ms"] * 1e-3) / 1e12 / PEAK_TFLOPS[p]}
            for p, sb in stats_by.items() if sb["trail"]["launches"] and sb["trail"]["time_ms"] > 0},
        "factorization_tflops": fact_flops / (fact_ms * 1e-3) / 1e12 if fact_ms > 0 else 0.0,
        "kernel_time_ms": {p: {name: st["time_ms"] / steps for name, st in sb.items() if st["launches"]}
                           for p, sb in stats_by.items()},
        "alg_tflops_end_to_end": sum(st["flops"] for sb in stats_by.values() for st in sb.values()) / dt / 1e12,
    }


def time_unprofiled(lib, dms, thetas, xs, variant, steps, warmup, warm=None):
    """Whole steps of a variant with profiling off (no per-launch events), so
    that the whole-pass graphs, which profiling turns off, can run."""
    import torch
    prec = variant.split("+")[0]

    def step():
        if warm is None:
            return lib.laplace_eval(dms, thetas, x=xs, prec=prec)
        mlp, centre, scale, max_iter = warm
        mlp.predict_modes(thetas, centre, scale, x=xs)
        return lib.laplace_eval(dms, thetas, x=xs, start=1, max_iter=max_iter, prec=prec)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res, _ = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert all(r["info"] == 0 for r in res)
    return {"value": steps * len(dms) / dt, "ms_per_step": dt / steps * 1e3, "steps": steps}


def amortised_warm_start(results, train_info, counts=(512, 4096)):
    """What the learned warm start buys an INLA run once its one-time cost is
    charged to the evaluations it speeds up.  For each mixed precision p with a
    '+mlp' variant and a zero-start variant in this run: theta-evals/s over N
    evaluations, N / (setup + N / v_warm), with setup = the training targets'
    solves + the training itself, and with setup = the training alone (targets
    taken from modes the run computes anyway, e.g. its Stage-1 evaluations);
    and the break-even count setup / (1 / v_zero - 1 / v_warm).  N = 512 is
    about one run at t = 4 (Stage 1 took 457 evaluations at n = 3000, plus the
    Hessian and CCD points)."""
    out = {}
    for p in ("fp32", "bf16"):
        if f"{p}+mlp" not in results or p not in results:
            continue
        vz, vw = results[p]["value"], results[f"{p}+mlp"]["value"]
        row = {"zero_start": vz, "warm_start": vw}
        for label, setup in (("with_target_solves", train_info["solve_s"] + train_info["train_s"]),
                             ("targets_from_run", train_info["train_s"])):
            row[label] = {"setup_s": setup,
                          **{f"N{n}": n / (setup + n / vw) for n in counts},
                          "break_even_evals": setup / (1.0 / vz - 1.0 / vw) if vw > vz else None}
        out[p] = row
    out["unit"] = "θ-evals/s"
    return out


def run_extras(lib, binding, synth, dms, thetas, xs):
    """Separately timed figures (not part of `value`): marginal variances and the
    variational-Bayes mean correction of the headline batch (FP64, from the modes
    the last variant left in xs), Stage 1 plus the CCD exploration on the
    n = 3000 space-time configuration, and the Moore-Penrose route against
    kriging on an intrinsic n = 3000 model."""
    import numpy as np
    import torch

    out = {}
    B = len(dms)
    torch.cuda.synchronize()
    lib.marginal_var(dms[:1], thetas[:1], xs[:1])           # warm-up (workspace, graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    var, info = lib.marginal_var(dms, thetas, xs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert np.all(info == 0), info
    out["marginal_var"] = {"value": B / dt, "unit": "var-evals/s", "batch": B, "s": dt, "precision": "fp64"}
    log(f"marginal variances: {B / dt:.2f} var-evals/s")
    t0 = time.perf_counter()
    mus, its, vinfo = lib.vb_mean(dms, thetas, var, xs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert np.all(vinfo == 0), vinfo
    out["vb_mean"] = {"value": B / dt, "unit": "VB corrections/s", "batch": B, "s": dt,
                      "iterations_mean": float(np.mean(its)), "precision": "fp64"}
    log(f"VB mean correction: {B / dt:.2f} corrections/s, {np.mean(its):.2f} iterations")
    m3, _ = synth.kron3000()
    d3 = binding.DeviceModel(m3)
    th0 = synth.kron_theta0(30)
    prior = lambda th: -0.5 * float(np.sum((np.asarray(th) - th0) ** 2))   # noqa: E731
    t0 = time.perf_counter()
    g = lib.theta_mode(d3, th0 + np.array([0.2, 0.2, -0.2, 0.05]), log_prior=prior)
    t1 = time.perf_counter()
    H, _, hinfo = lib.theta_hessian(d3, g["theta"], log_prior=prior)
    pts, delta = lib.ccd_points(g["theta"], H)
    res, _ = lib.laplace_eval([d3] * len(pts), pts)
    lib.ccd_weights(delta, [q["objective"] + prior(p) for q, p in zip(res, pts)])
    t2 = time.perf_counter()
    out["stage1_n3000"] = {"workload": "Poisson space-time n=3000 (100 regions x 30 times), k=129, t=4, "
                                       "N(theta0, I) log prior", "mode_s": t1 - t0, "bfgs_iterations": g["iters"],
                           "evaluations": g["evals"], "theta_evals_per_s": g["evals"] / (t1 - t0),
                           "hessian_and_ccd_s": t2 - t1, "ccd_points": len(pts), "info": [g["info"], hinfo]}
    log(f"stage 1 at n=3000: {t1 - t0:.2f} s ({g['iters']} iterations), Hessian + CCD {t2 - t1:.2f} s")
    out["uneven_batch"] = run_uneven_batch(lib, binding, synth)
    out["n16384_precision"] = run_n16384(lib, binding, synth)
    out["moore_penrose_n3000"] = run_moore_penrose(lib, binding, synth)
    out["table3_type4"] = run_table3(lib, binding, synth)
    out["stage1_type4_moore_penrose"] = run_stage1_type4(lib, binding, synth)
    return out


def run_uneven_batch(lib, binding, synth, steps=3):
    """The batching configuration: 64 theta in one call, n drawn from {1024,
    2048, 3000, 4096, 6144} (Poisson space-time models, k = n_s + n_t - 1),
    theta_b ~ N(theta0(n_b), 0.5^2 I), FP64, zero start, autotuned panel width
    and tile for the batch's shape; `steps` timed calls after one untimed one."""
    import numpy as np
    import torch
    models, thetas = synth.uneven_batch(B=64, seed=3)
    seen, dms = {}, []
    for m in models:
        if id(m) not in seen:
            seen[id(m)] = binding.DeviceModel(m)
        dms.append(seen[id(m)])
    t0 = time.perf_counter()
    chosen, _ = lib.autotune([m["n"] for m in models], [m["C"].shape[0] + 1 for m in models], prec="fp64", reps=2)
    t_tune = time.perf_counter() - t0
    lib.laplace_eval(dms, thetas)
    torch.cuda.synchronize()
    g0 = lib.graph_stats()
    t0 = time.perf_counter()
    for _ in range(steps):
        res, _ = lib.laplace_eval(dms, thetas)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    g1 = lib.graph_stats()
    assert all(r["info"] == 0 for r in res), [r["info"] for r in res]
    ns = [m["n"] for m in models]
    out = {"workload": "64 theta in one call, n in {1024, 2048, 3000, 4096, 6144} (Poisson space-time, k = n_s + n_t "
                       "- 1), theta ~ N(theta0, 0.5^2 I), FP64, zero start",
           "value": 64 / dt, "unit": "θ-evals/s", "ms_per_call": dt * 1e3, "steps": steps,
           "n_counts": {str(v): ns.count(v) for v in sorted(set(ns))},
           "newton_iters_mean": float(np.mean([r["iters"] for r in res])),
           "autotune": {"nb": chosen[0], "tm": chosen[1], "lookahead": chosen[2], "tune_s": t_tune},
           "graph_replays_per_call": (g1["replays"] - g0["replays"]) / steps,
           "graphs_captured_in_timed_calls": g1["captured"] - g0["captured"], "precision": "fp64"}
    log(f"uneven batch: {64 / dt:.1f} theta-evals/s ({dt * 1e3:.0f} ms per call), tuned {chosen}")
    return out


def run_n16384(lib, binding, synth):
    """The precision configuration: n = 16384 (128 regions x 128 times, k =
    255), the 9-point finite-difference batch at theta0 (h = 0.01) in FP64, FP32
    and BF16 (one untimed and one timed call each, autotuned), and the errors
    of theta0's evaluation against the FP64 oracle's stored values
    (tests/golden/kron16384_theta0.json, written by a script that calls only
    the oracle): mode (every 8th element), log|Q*|, log|S| and the objective,
    relative and absolute."""
    import numpy as np
    import torch
    model = synth.kron_poisson(128, 128, seed=4)
    th0 = synth.kron_theta0(128)
    batch = synth.fd_batch(th0, 0.01, [0, 1, 2, 3])
    dm = binding.DeviceModel(model)
    with open(os.path.join(ROOT, "tests", "golden", "kron16384_theta0.json")) as f:
        g = json.load(f)
    idx = np.array(g["index"])
    k = model["C"].shape[0]
    out = {"workload": "Poisson space-time n=16384 (128 regions x 128 times), k=255, 9-point finite-difference "
                       "batch at theta0", "precisions": {}}
    for prec in ("fp64", "fp32", "bf16"):
        chosen, _ = lib.autotune([16384] * 9, [k + 1] * 9, prec=prec, reps=1)
        lib.laplace_eval([dm] * 9, batch, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, xs = lib.laplace_eval([dm] * 9, batch, prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert all(r["info"] == 0 for r in res), [r["info"] for r in res]
        r0, x0 = res[0], xs[0].cpu().numpy()
        errs = {"mode_max_rel": float(np.max(np.abs(x0[idx] - np.array(g["x"]))) / max(1.0, g["x_absmax"])),
                "objective_abs": abs(r0["objective"] - g["objective"])}
        for key in ("objective", "logdet_qstar", "logdet_s", "logdet_qprior"):
            errs[f"{key}_rel"] = abs(r0[key] - g[key]) / abs(g[key])
        out["precisions"][prec] = {
            "value": 9 / dt, "unit": "θ-evals/s", "s_per_call": dt,
            "newton_iters": [r["iters"] for r in res], "fp64_fallbacks": int(sum(r["fallback"] & 1 for r in res)),
            "autotune": {"nb": chosen[0], "tm": chosen[1], "lookahead": chosen[2]},
            "theta0_errors_vs_oracle": errs}
        log(f"n=16384 9-point batch {prec}: {9 / dt:.2f} theta-evals/s, iterations "
            f"{[r['iters'] for r in res]}, theta0 objective error {errs['objective_abs']:.1e} abs")
    return out


def intrinsic_inputs(model):
    """Caller-side inputs of the intrinsic RW1 x Besag model: its structure
    matrix R = R_t kron (D - Adj) and an orthonormal basis of its null space
    (time-constant per region, region-constant per time)."""
    import numpy as np
    n_s, n_t = model["n_s"], model["n_t"]
    Rt = np.diag(np.r_[1.0, 2.0 * np.ones(n_t - 2), 1.0]) - np.eye(n_t, k=1) - np.eye(n_t, k=-1)
    Rs = np.zeros((n_s, n_s))
    for i, j in model["edges"]:
        Rs[i, j] = Rs[j, i] = -1.0
    Rs -= np.diag(Rs.sum(axis=1))
    cols = np.hstack([np.kron(np.ones((n_t, 1)), np.eye(n_s)), np.kron(np.eye(n_t), np.ones((n_s, 1)))])
    Qr, Rr = np.linalg.qr(cols)
    return np.kron(Rt, Rs), Qr[:, np.abs(np.diag(Rr)) > 1e-10]


def type4_inputs(model, theta):
    """Caller-side inputs of the Type IV model: the structure blocks of its
    prior (RW2 in time, Besag in space and their Kronecker product), the full
    Q_prior(theta), and an orthonormal basis of its null space written from the
    blocks (time effect: constant and linear trend; space effect: constant;
    interaction: constant and linear in time per region, constant over regions
    per time)."""
    import math

    import numpy as np
    n_s, n_t, n = model["n_s"], model["n_t"], model["n"]
    D = np.zeros((n_t - 2, n_t))
    for i in range(n_t - 2):
        D[i, i:i + 3] = (1.0, -2.0, 1.0)
    R2 = D.T @ D
    Rs = np.zeros((n_s, n_s))
    Rs[model["edges"][:, 0], model["edges"][:, 1]] = -1.0
    Rs[model["edges"][:, 1], model["edges"][:, 0]] = -1.0
    Rs -= np.diag(Rs.sum(axis=1))
    Rk = np.kron(R2, Rs)
    c = model["fixed_precision"]
    tau = [math.exp(v) for v in theta[:3]]
    Q = np.zeros((n, n))
    Q[0, 0] = Q[1, 1] = c
    o = 2
    for blk, t in ((R2, tau[0]), (Rs, tau[1]), (Rk, tau[2])):
        k = blk.shape[0]
        Q[o:o + k, o:o + k] = t * blk
        o += k
    tt = np.arange(n_t, dtype=float)
    cols = []
    o_t, o_s, o_z = 2, 2 + n_t, 2 + n_t + n_s
    for v in (np.ones(n_t), tt):
        col = np.zeros(n); col[o_t:o_t + n_t] = v; cols.append(col)
    col = np.zeros(n); col[o_s:o_s + n_s] = 1.0; cols.append(col)
    for sr in range(n_s):
        for v in (np.ones(n_t), tt):
            col = np.zeros(n); col[o_z + sr:o_z + n_t * n_s:n_s] = v; cols.append(col)
    for t in range(n_t):
        col = np.zeros(n); col[o_z + t * n_s:o_z + (t + 1) * n_s] = 1.0; cols.append(col)
    Qr, Rr = np.linalg.qr(np.stack(cols, axis=1))
    return (R2, Rs, Rk), Q, Qr[:, np.abs(np.diag(Rr)) > 1e-10]


def run_table3(lib, binding, synth, B=8, sizes=((200, 5), (400, 5), (800, 5))):
    """The paper's comparison table of the simulation study (kriging against the
    Moore-Penrose route on the Type IV model with intercept, trend, RW2 time,
    random-graph Besag space and RW2 x Besag interaction), at its three sizes:
    B theta ~ N(theta0, 0.3^2 I) each.  Moore-Penrose: the pseudo-inverses of
    the three structure blocks from one batched GPU Jacobi call (timed apart),
    Q_prior(theta)^+ assembled block-diagonally with the 1/tau scalings, then
    inla_woodbury_eval with the design matrix.  Kriging: inla_laplace_eval on
    Q_prior + N N^T with the n_t + 2 n_s + 1 constraints N^T x = 0.  FP64."""
    import math

    import numpy as np
    import torch
    out = []
    for n_s, n_t in sizes:
        m = synth.type4(n_s, n_t, seed=90 + n_s)
        th0 = synth.type4_theta0()
        thetas = synth.normal_batch(th0, B, 0.3, seed=91 + n_s)
        thetas[:, 3] = 0.0
        blocks, _, N = type4_inputs(m, th0)
        mats = [torch.as_tensor(b).cuda() for b in blocks]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Pb, ranks, sweeps, pinfo = lib.pinv(mats)
        torch.cuda.synchronize()
        t_pinv = time.perf_counter() - t0
        n = m["n"]
        Ps = []
        for th in thetas:
            P = torch.zeros((n, n), dtype=torch.float64, device="cuda")
            P[0, 0] = P[1, 1] = 1.0 / m["fixed_precision"]
            o = 2
            for Pk, v in zip(Pb, th[:3]):
                k = Pk.shape[0]
                P[o:o + k, o:o + k] = Pk / math.exp(v)
                o += k
            Ps.append(P)
        dm = binding.DeviceModel(m)
        lib.woodbury_eval([dm], [0.0], Ps[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rw, xw = lib.woodbury_eval([dm] * B, thetas[:, 3], Ps)
        torch.cuda.synchronize()
        t_wood = time.perf_counter() - t0
        kms = []
        for th in thetas:
            _, Q, _ = type4_inputs(m, th)
            kms.append(binding.DeviceModel({"n": n, "lik": "poisson", "prior": "dense", "y": m["y"], "E": m["E"],
                                            "A": m["A"], "C": N.T, "e": np.zeros(N.shape[1]),
                                            "Qprior": Q + N @ N.T}))
        lib.laplace_eval(kms[:1], thetas[:1, 3:])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rk, xk = lib.laplace_eval(kms, thetas[:, 3:])
        torch.cuda.synchronize()
        t_krig = time.perf_counter() - t0
        d = max(abs(a["objective"] - b["objective"]) / abs(b["objective"]) for a, b in zip(rw, rk))
        dx = max(float((xa - xb).abs().max()) for xa, xb in zip(xw, xk))
        row = {"n_s": n_s, "n_t": n_t, "effects": n, "constraints": int(N.shape[1]), "observations": m["m"],
               "pinv_blocks": [int(b.shape[0]) for b in blocks], "pinv_s": t_pinv,
               "pinv_sweeps": [int(v) for v in sweeps], "pinv_info": [int(v) for v in pinfo],
               "woodbury_theta_evals_per_s": B / t_wood, "kriging_theta_evals_per_s": B / t_krig,
               "woodbury_iters_mean": float(np.mean([r["iters"] for r in rw])),
               "kriging_iters_mean": float(np.mean([r["iters"] for r in rk])),
               "max_rel_objective_diff": d, "max_abs_mode_diff": dx,
               "info": [r["info"] for r in rw] + [r["info"] for r in rk]}
        log(f"table 3 size s={n} k={N.shape[1]}: pinv of blocks {t_pinv:.2f} s; Woodbury {B / t_wood:.1f} vs "
            f"kriging {B / t_krig:.1f} theta-evals/s; objectives agree to {d:.1e}, modes to {dx:.1e}")
        out.append(row)
        del Ps, kms, dm
        torch.cuda.empty_cache()
    return {"workload": f"Type IV Poisson model of the simulation study, random Besag graph, batch {B} theta ~ "
                        "N(theta0, 0.3^2 I) per size", "rows": out, "precision": "fp64"}


def run_stage1_type4(lib, binding, synth, n_s=200, n_t=5):
    """Stage 1 and the CCD exploration on the Moore-Penrose route for the Type IV
    model at the simulation table's first size (s = 1207, k = 406 implicit
    constraints): block pseudo-inverses of the three structures (one batched
    call), BFGS mode and Hessian of log pi~(theta | y) over theta = (log tau_time,
    log tau_space, log tau_interaction) with a N(theta0, I) log prior, the CCD
    points, their Woodbury evaluations and weights.  FP64."""
    import numpy as np
    import torch
    m = synth.type4(n_s, n_t, seed=90 + n_s)
    th0 = synth.type4_theta0()[:3]
    blocks, _, _ = type4_inputs(m, np.r_[th0, 0.0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, _, sweeps, pinfo = lib.pinv([torch.as_tensor(b).cuda() for b in blocks])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    one = torch.ones((1, 1), dtype=torch.float64, device="cuda")
    c = m["fixed_precision"]
    prior = binding.PinvPrior([{"offset": 0, "P": one, "tau_index": -1, "fixed_scale": 1.0 / c},
                               {"offset": 1, "P": one, "tau_index": -1, "fixed_scale": 1.0 / c},
                               {"offset": 2, "P": P[0], "tau_index": 0},
                               {"offset": 2 + n_t, "P": P[1], "tau_index": 1},
                               {"offset": 2 + n_t + n_s, "P": P[2], "tau_index": 2}], lik_index=-1, lik_value=0.0)
    dm = binding.DeviceModel(m)
    lp = lambda th: -0.5 * float(np.sum((np.asarray(th) - th0) ** 2))   # noqa: E731
    g = lib.theta_mode_pinv(dm, prior, th0 + np.array([0.3, -0.3, 0.3]), log_prior=lp)
    t2 = time.perf_counter()
    H, lpost, hinfo = lib.theta_hessian_pinv(dm, prior, g["theta"], log_prior=lp)
    pts, delta = lib.ccd_points(g["theta"], H)
    Ps = lib.pinv_prior_assemble(prior, m["n"], pts)
    res, _ = lib.woodbury_eval([dm] * len(pts), np.zeros(len(pts)), Ps)
    w = lib.ccd_weights(delta, [q["objective"] + lp(p) for q, p in zip(res, pts)])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out = {"workload": f"Type IV Poisson model, s={m['n']} effects, k={n_t + 2 * n_s + 1} implicit constraints, "
                       "t=3, N(theta0, I) log prior, Moore-Penrose route",
           "pinv_blocks_s": t1 - t0, "pinv_sweeps": [int(v) for v in sweeps], "mode_s": t2 - t1,
           "bfgs_iterations": g["iters"], "evaluations": g["evals"], "theta_evals_per_s": g["evals"] / (t2 - t1),
           "hessian_and_ccd_s": t3 - t2, "ccd_points": len(pts), "weights_sum": float(np.sum(w)),
           "theta_star": [float(v) for v in g["theta"]], "info": [g["info"], hinfo] + [q["info"] for q in res]}
    log(f"stage 1 on the Moore-Penrose route (s={m['n']}): pinv {t1 - t0:.2f} s, mode {t2 - t1:.2f} s "
        f"({g['iters']} iterations, {g['evals']} evaluations), Hessian + {len(pts)} CCD points {t3 - t2:.2f} s")
    return out


def run_moore_penrose(lib, binding, synth, B=9):
    """The paper's comparison of its Moore-Penrose route with kriging, on one
    posterior: the intrinsic RW1 x Besag Poisson model at n = 3000 (100 regions
    x 30 times, null space of dimension 129), B theta.  Woodbury route:
    Q_prior(theta)^+ = R^+ / tau from one GPU pseudo-inverse of R (timed apart),
    then inla_woodbury_eval.  Kriging route: inla_laplace_eval on the proper
    prior tau R + N N^T with the 129 sum-to-zero constraints.  Both FP64; the two
    objectives agree to rounding."""
    import math

    import numpy as np
    import torch
    m = synth.rw1_besag(100, 30, seed=72)
    R, N = intrinsic_inputs(m)
    th0 = synth.rw1_besag_theta0(30)
    thetas = synth.normal_batch(th0, B, 0.3, seed=73)
    Rd = torch.as_tensor(R).cuda()
    lib.pinv([Rd])                     # warm-up (workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, rank, sweeps, info = lib.pinv([Rd])
    torch.cuda.synchronize()
    t_pinv = time.perf_counter() - t0
    Ps = [P[0] / math.exp(th[0]) for th in thetas]
    dm = binding.DeviceModel(m)
    lib.woodbury_eval([dm], [thetas[0][1]], Ps[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rw, _ = lib.woodbury_eval([dm] * B, thetas[:, 1], Ps)
    torch.cuda.synchronize()
    t_wood = time.perf_counter() - t0
    xw = [torch.zeros(m["n"], dtype=torch.float64, device="cuda") for _ in range(B)]
    lib.woodbury_eval([dm] * B, thetas[:, 1], Ps, x=xw)
    lib.woodbury_var([dm], [thetas[0][1]], Ps[:1], xw[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, vinfo = lib.woodbury_var([dm] * B, thetas[:, 1], Ps, xw)
    torch.cuda.synchronize()
    t_var = time.perf_counter() - t0
    C = synth.sum_to_zero_rows(100, 30)
    kms = [binding.DeviceModel({"n": m["n"], "lik": "poisson", "prior": "dense", "y": m["y"], "E": m["E"], "A": None,
                                "C": C, "e": np.zeros(C.shape[0]),
                                "Qprior": math.exp(th[0]) * R + N @ N.T}) for th in thetas]
    lib.laplace_eval(kms[:1], thetas[:1, 1:])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rk, _ = lib.laplace_eval(kms, thetas[:, 1:])
    torch.cuda.synchronize()
    t_krig = time.perf_counter() - t0
    d = max(abs(a["objective"] - b["objective"]) / abs(b["objective"]) for a, b in zip(rw, rk))
    res = {"workload": "Poisson RW1 x Besag (intrinsic) n=3000 (100 regions x 30 times), null space 129, "
                       f"batch {B} theta ~ N(theta0, 0.3^2 I)",
           "pinv_s": t_pinv, "pinv_sweeps": int(sweeps[0]), "pinv_rank": int(rank[0]), "pinv_info": int(info[0]),
           "woodbury_theta_evals_per_s": B / t_wood, "kriging_theta_evals_per_s": B / t_krig,
           "woodbury_var_evals_per_s": B / t_var, "woodbury_var_info": [int(v) for v in vinfo],
           "woodbury_iters_mean": float(np.mean([r["iters"] for r in rw])),
           "kriging_iters_mean": float(np.mean([r["iters"] for r in rk])),
           "max_rel_objective_diff": d, "info": [r["info"] for r in rw] + [r["info"] for r in rk],
           "precision": "fp64"}
    log(f"Moore-Penrose n=3000: pinv {t_pinv:.2f} s ({int(sweeps[0])} sweeps); Woodbury {B / t_wood:.1f} vs "
        f"kriging {B / t_krig:.1f} theta-evals/s; objectives agree to {d:.1e}; variances {B / t_var:.1f}/s")
    return res


def run_logdet_batch(binding, n=8192, B=64, seed=5):
    """Two batched FP32 factorisations of B seeded synthetic SPD matrices
    M M^T / n + 2 I of order n (nb 512, tile 128), the second one profiled: its
    trailing-update launches, their algorithmic bytes and average duration, in
    the form that --rocprof-window reads."""
    import torch

    lib = binding.Library()
    gen = torch.Generator(device="cuda").manual_seed(seed)
    mats = []
    for _ in range(B):
        m = torch.randn(n, n, device="cuda", dtype=torch.float64, generator=gen)
        q = m @ m.T / n
        q.diagonal().add_(2.0)
        mats.append(q)
        del m
    lib.tune_set("fp32", n, B, 512, 128, 0)
    work = [q.clone() for q in mats]
    lib.logdet(work, prec="fp32")
    for w, q in zip(work, mats):
        w.copy_(q)
    torch.cuda.synchronize()
    lib.profile(True)
    _, info = lib.logdet(work, prec="fp32")
    torch.cuda.synchronize()
    st = lib.profile_get(binding.K_TRAIL, "fp32")
    lib.profile(False)
    assert all(i == 0 for i in info), info
    return {"logdet_batch": {"n": n, "batch": B, "precision": "fp32", "nb": 512, "tile": 128},
            "roofline": {"kernel": trail_kernel_name("fp32", 128) + " (full-batch FP32 factorisation)",
                         "launches": st["launches"], "avg_launch_ms": st["time_ms"] / st["launches"],
                         "alg_bytes_per_launch": st["bytes"] / st["launches"]}}


def main():
    import faulthandler
    faulthandler.enable()   # a crash in native code prints the Python stack that led to it
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--ns", type=int, default=128)
    ap.add_argument("--nt", type=int, default=64)
    ap.add_argument("--variants", default="fp64,fp32,bf16,bf16+mlp,fp32+mlp")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="factor with the default panel width and tile instead of tuning them first")
    ap.add_argument("--no-graphs", action="store_true", help="launch every kernel directly (no hipGraph replays)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run each evaluation's FP64 prior pass in order instead of beside the Newton iteration "
                         "(inla_set_overlap; on by default here: +3.7%% at the headline)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the separately timed marginal-variance, VB-correction and Stage-1 figures")
    ap.add_argument("--timed-only", action="store_true",
                    help="skip the headline's second timings (prior pass in order, unprofiled), so that the "
                         "variants' timed regions are the last dispatches of a profiled run")
    ap.add_argument("--rocprof-window", metavar="CSV",
                    help="only summarise a rocprofv3 per-dispatch CSV over the timed region of --bench-json")
    ap.add_argument("--bench-json", metavar="FILE", help="the JSON line printed by the profiled bench run")
    ap.add_argument("--window-precision", choices=("fp64", "fp32", "bf16"),
                    help="window the trailing-update kernel of this precision instead of the roofline kernel")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (HBM counter calibration)")
    ap.add_argument("--logdet-batch", action="store_true",
                    help="only factor one full batch twice (64 synthetic SPD matrices of order 8192, FP32, nb 512, "
                         "tile 128, through inla_logdet) and print the second factorisation's trailing launches "
                         "(for counter runs of the kernel on a full batch)")
    ap.add_argument("--moore-penrose-only", action="store_true",
                    help="only run the Moore-Penrose vs kriging comparison at n = 3000 (for profiling)")
    args = ap.parse_args()
    if args.rocprof_window:
        print(json.dumps(rocprof_window(args.rocprof_window, args.bench_json, args.window_precision)))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2311_08050_amd import binding, synth

    torch.cuda.set_device(0)
    if args.moore_penrose_only:
        lib = binding.Library()
        print(json.dumps({"moore_penrose_n3000": run_moore_penrose(lib, binding, synth),
                          "table3_type4": run_table3(lib, binding, synth),
                          "stage1_type4_moore_penrose": run_stage1_type4(lib, binding, synth)}), flush=True)
        return
    if args.logdet_batch:
        print(json.dumps(run_logdet_batch(binding)), flush=True)
        return
    if args.calibrate_copy:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy": {"bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                                             "copies": 3}}), flush=True)
        return
    model, thetas = synth.headline(B=args.batch, n_s=args.ns, n_t=args.nt)
    n, k = model["n"], model["C"].shape[0]
    log(f"workload n={n} k={k} batch={args.batch}")
    lib = binding.Library()
    dm = binding.DeviceModel(model)
    dms = [dm] * args.batch
    xs = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(args.batch)]
    variants = [v.strip() for v in args.variants.split(",") if v.strip()]
    if args.no_graphs:
        lib.set_graphs(False)
    lib.set_overlap(not args.no_overlap)
    tuning = {}
    if not args.no_autotune:
        # one-time setup, not timed: the tuner factors synthetic batches of the
        # Newton passes' shape (n latent columns, k + 1 border rows)
        for p in dict.fromkeys(v.split("+")[0] for v in variants):
            t0 = time.perf_counter()
            chosen, times = lib.autotune([n] * args.batch, [k + 1] * args.batch, prec=p, reps=2)
            tuning[p] = {"nb": chosen[0], "tm": chosen[1], "lookahead": chosen[2], "tune_s": time.perf_counter() - t0,
                         "candidate_ms": {f"nb{c[0]}_tm{c[1]}_la{c[2]}": round(v, 3) for c, v in times.items()}}
            log(f"autotune {p}: {chosen} {tuning[p]['candidate_ms']}")
    results, train_info, trained = {}, None, {}
    for v in variants:
        warm = None
        if v.endswith("+mlp"):
            from paper_2311_08050_amd import warmstart
            pv = v.split("+")[0]
            centre, scale = synth.kron_theta0(args.nt), np.full(4, 0.5)
            if "net" not in trained:
                # one network for every +mlp variant: its targets are modes solved
                # by the mixed-precision path (equal to the FP64 modes to 1e-9);
                # their zero-start iteration mean sets the warm start's cap
                train = synth.normal_batch(centre, MLP_TRAIN["n_train"], 0.5, seed=MLP_TRAIN["seed"])
                log(f"training the warm start on {len(train)} theta (fp32 solves)")
                trained["net"] = warmstart.train(lib, dm, train, centre, scale, hidden=MLP_TRAIN["hidden"],
                                                 epochs=MLP_TRAIN["epochs"], batch=MLP_TRAIN["batch"],
                                                 lr=MLP_TRAIN["lr"], prec="fp32", seed=MLP_TRAIN["seed"],
                                                 lr_final=MLP_TRAIN["lr_final"])
                log(f"warm start trained: {trained['net'][1]}")
            mlp, train_info = trained["net"]
            # a warm start that needs more iterations than the zero-start median is
            # re-solved from zero (counted in zero_start_fallbacks)
            warm = (mlp, centre, scale, int(np.ceil(train_info["zero_start_iters_mean"])))
        results[v] = run_variant(lib, binding, dms, thetas, xs, v, args.steps, args.warmup, warm)
    head = variants[-1]
    hv = results[head]
    in_order = None
    if not args.no_overlap and not args.timed_only:
        # the headline variant once more with the prior pass in order: the
        # trailing kernel's own rate, which the concurrent prior pass stretches
        lib.set_overlap(False)
        w = max(3, args.steps // 4)
        r = run_variant(lib, binding, dms, thetas, xs, head, w, 1, warm)
        lib.set_overlap(True)
        in_order = {"value": r["value"], "ms_per_step": r["ms_per_step"], "steps": w,
                    "newton_iters": r["newton_iters"], "kernel_time_ms": r["kernel_time_ms"],
                    "roofline": {k: r["roofline"][k] for k in ("achieved", "peak", "unit", "frac", "launches",
                                                               "avg_launch_ms")}}
    unprofiled = None
    if not args.no_graphs and not args.timed_only:
        # the headline variant without per-launch events, with and without the
        # whole-pass graphs (each Newton pass and refinement step one hipGraph)
        w = max(3, args.steps // 4)
        st0 = lib.pass_graph_stats()
        with_pg = time_unprofiled(lib, dms, thetas, xs, head, w, 2, warm)
        st1 = lib.pass_graph_stats()
        lib.set_pass_graphs(False)
        direct = time_unprofiled(lib, dms, thetas, xs, head, w, 1, warm)
        lib.set_pass_graphs(True)
        unprofiled = {"pass_graphs": dict(with_pg, captured=st1["captured"] - st0["captured"],
                                          replays=st1["replays"] - st0["replays"]),
                      "chain_graphs_only": direct}
        log(f"unprofiled headline: {unprofiled}")
    for v in variants:
        roof = results[v]["roofline"]
        pv = roof["precision"]
        summary = os.path.join(ROOT, "profiles", f"trail_update_{pv}_n8192_b64.md")
        roof["traffic"] = traffic_from_profile(
            os.path.join(ROOT, "paper_2311_08050_amd", "csrc", "k_factor.hip"), summary,
            roof["kernel"].split(" ")[0], roof["alg_bytes_per_launch"])
        if roof["traffic"] is not None:
            roof["traffic_basis"] = (f"HBM bytes per launch = this run's algorithmic bytes per launch x the ratio of "
                                     f"FETCH_SIZE + WRITE_SIZE (copy-calibrated) to algorithmic bytes in "
                                     f"profiles/{os.path.basename(summary)}")
    if in_order is not None:
        # the same kernel's rate in the in-order repeat of the headline (the
        # figure above is measured beside the concurrent prior pass, with which
        # it shares the MFMA units)
        hv["roofline"]["frac_prior_pass_in_order"] = in_order["roofline"]["frac"]
    out = {
        "metric": METRIC,
        "value": hv["value"],
        "unit": "θ-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hv["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f32+f64"}[head.split("+")[0]],
        "data": "synthetic",
        "config": {
            "workload": f"Poisson space-time interaction, n={n} ({args.ns} regions x {args.nt} times), "
                        f"k={k} sum-to-zero constraints, batch {args.batch} theta ~ N(theta0, 0.5^2 I), "
                        f"variant {head}",
            "n": n, "k": k, "batch": args.batch, "variant": head,
        },
        "roofline": hv["roofline"],
        "headline_prior_pass_in_order": in_order,
        "headline_unprofiled": unprofiled,
        "variants": results,
        "autotune": tuning or None,
        "graphs": not args.no_graphs,
        "overlap": not args.no_overlap,
    }
    if train_info is not None:
        out["warm_start_training"] = dict(train_info, **MLP_TRAIN)
        out["warm_start_amortised"] = amortised_warm_start(results, train_info)
    if "fp64" in results and head != "fp64":
        out["speedup_vs_fp64"] = hv["value"] / results["fp64"]["value"]
    if not args.no_extras:
        out["extras"] = run_extras(lib, binding, synth, dms, thetas, xs)
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info

        from oracle import inla_oracle as O

        log("cpu baseline: oracle on theta 0")
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        t0 = time.perf_counter()
        ref = O.laplace_eval(model, thetas[0])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": 1.0 / dt, "unit": "θ-evals/s", "cores": int(threads), "kind": "oracle",
            "sample": f"1 theta (theta 0 of the batch), full oracle Laplace evaluation at n={n}, {dt:.1f} s"}
        errs = {}
        for v in variants:
            if v.endswith("+mlp"):
                x0 = mlp.predict_modes(thetas[:1], centre, scale)
                r0, x0 = lib.laplace_eval([dm], thetas[:1], x=x0, start=1, prec=v.split("+")[0])
            else:
                r0, x0 = lib.laplace_eval([dm], thetas[:1], prec=v.split("+")[0])
            r0 = r0[0]
            errs[v] = {
                "objective_rel": abs(r0["objective"] - ref["objective"]) / abs(ref["objective"]),
                "objective_abs": abs(r0["objective"] - ref["objective"]),
                "logdet_qstar_rel": abs(r0["logdet_qstar"] - ref["logdet_qstar"]) / abs(ref["logdet_qstar"]),
                "logdet_s_rel": abs(r0["logdet_s"] - ref["logdet_s"]) / abs(ref["logdet_s"]),
                "mode_max_abs": float(np.max(np.abs(x0[0].cpu().numpy() - ref["x"]))),
                "iters": r0["iters"], "iters_oracle": ref["iters"],
            }
        out["errors_vs_oracle"] = errs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
