"""ctypes binding of ``libinla_dense.so`` (C-ABI in ``include/inla_dense.h``).

Argument marshalling only: device buffers are torch tensors on the current HIP
device, host outputs are numpy arrays, and every step of the computation runs in
the library's HIP kernels.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libinla_dense.so")

LIK = {"gaussian": 0, "poisson": 1}
PRIOR = {"dense": 0, "expcov": 1, "kron": 2, "pinv": 3, "rw1_besag": 3, "intrinsic": 3, "type4": 3}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
N_PRIOR_PARAMS = {"dense": 0, "expcov": 2, "kron": 3}

INFO_OK = 0
INFO_NEWTON_MAXIT = -1
INFO_CONSTRAINT_RANK = -2
INFO_NONFINITE = -3
ERR_TOO_LARGE = -1003
INFO_EIG_MAXIT = -4

K_TRAIL, K_PANEL, K_POTF2, K_ASSEMBLE, K_SOLVE, K_BORDER = 0, 1, 2, 3, 4, 5
K_NAMES = {K_TRAIL: "trail", K_PANEL: "panel", K_POTF2: "potf2", K_ASSEMBLE: "assemble", K_SOLVE: "solve",
           K_BORDER: "border"}

# Symbols declared by include/inla_dense.h
EXPORTS = [
    "inla_create", "inla_destroy", "inla_set_stream", "inla_logdet", "inla_logdet_noalloc", "inla_constrained_mode",
    "inla_laplace_eval", "inla_marginal_var", "inla_profile", "inla_profile_get", "inla_version",
    "inla_mlp_create", "inla_mlp_destroy", "inla_mlp_num_params", "inla_mlp_get_params", "inla_mlp_set_params",
    "inla_mlp_forward", "inla_mlp_grad", "inla_mlp_train_step", "inla_mlp_predict_modes",
    "inla_set_graphs", "inla_set_lookahead", "inla_set_overlap", "inla_graph_stats", "inla_set_pass_graphs",
    "inla_pass_graph_stats",
    "inla_vb_mean", "inla_theta_mode", "inla_theta_hessian", "inla_ccd_design", "inla_ccd_points", "inla_ccd_weights", "inla_autotune", "inla_tune_set", "inla_tune_get",
    "inla_pinv", "inla_woodbury_eval", "inla_woodbury_var",
    "inla_pinv_prior_assemble", "inla_theta_mode_pinv", "inla_theta_hessian_pinv",
]
# Autotuner candidates (nb, tm) without lookahead, in the order inla_autotune
# reports their times; the fastest is then timed with lookahead as well.
TUNE_CANDIDATES = {p: [(nb, tm) for nb in (128, 256, 512, 1024) for tm in (64, 128) if p != "bf16" or tm == 128]
                   for p in PREC}


def tune_default(prec, n_max):
    """The (nb, tm, lookahead) a batch of largest order n_max factorises with
    when the handle's table has no entry for it: BF16 batches of padded order
    4096 and above take 1024-wide panels."""
    if prec == "bf16" and -(-n_max // 128) * 128 >= 4096:
        return (1024, 128, 0)
    return {"fp64": (512, 64, 0), "fp32": (512, 128, 0), "bf16": (512, 128, 0)}[prec]


class Model(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("k", C.c_int32), ("lik", C.c_int32), ("prior", C.c_int32),
        ("n_s", C.c_int32), ("n_t", C.c_int32), ("ldq", C.c_int32), ("reserved", C.c_int32),
        ("y", C.c_void_p), ("E", C.c_void_p), ("C", C.c_void_p), ("e", C.c_void_p),
        ("coords", C.c_void_p), ("Qprior", C.c_void_p),
        ("m", C.c_int32), ("nnz", C.c_int32), ("A_rowptr", C.c_void_p), ("A_col", C.c_void_p), ("A_val", C.c_void_p),
    ]


class Opts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("start", C.c_int32), ("reserved", C.c_int32)]


class Result(C.Structure):
    _fields_ = [
        ("objective", C.c_double), ("logdet_qprior", C.c_double), ("logdet_sprior", C.c_double),
        ("ese", C.c_double), ("xqx", C.c_double), ("loglik", C.c_double), ("logdet_qstar", C.c_double),
        ("logdet_s", C.c_double), ("step", C.c_double), ("iters", C.c_int32), ("info", C.c_int32),
        ("ir_steps", C.c_int32), ("fallback", C.c_int32),
    ]

    def asdict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ThetaOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("reserved", C.c_int32), ("h", C.c_double), ("gtol", C.c_double),
                ("ftol", C.c_double), ("max_step", C.c_double), ("eval", Opts)]


class PinvPriorStruct(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("offset", C.POINTER(C.c_int32)), ("size", C.POINTER(C.c_int32)),
                ("P", C.POINTER(C.c_void_p)), ("ld", C.POINTER(C.c_int32)), ("tau_index", C.POINTER(C.c_int32)),
                ("fixed_scale", C.POINTER(C.c_double)), ("lik_index", C.c_int32), ("reserved", C.c_int32),
                ("lik_value", C.c_double)]


class PinvPrior:
    """A prior given through its diagonal blocks' pseudo-inverses (inla_pinv_prior):
    blocks is a list of dicts {"offset", "P" (square float64 device tensor R_k^+),
    "tau_index" (theta component of log tau_k, or -1), "fixed_scale" (1 / tau_k
    for tau_index -1)}; the likelihood parameter is theta[lik_index], or
    lik_value for lik_index -1.  Keeps its arrays alive."""

    def __init__(self, blocks, lik_index=-1, lik_value=0.0):
        k = len(blocks)
        self.tensors = [b["P"] for b in blocks]
        self._off = (C.c_int32 * k)(*[int(b["offset"]) for b in blocks])
        self._size = (C.c_int32 * k)(*[int(b["P"].shape[0]) for b in blocks])
        self._ptr = (C.c_void_p * k)(*[b["P"].data_ptr() for b in blocks])
        self._ld = (C.c_int32 * k)(*[int(b["P"].shape[0]) for b in blocks])
        self._tau = (C.c_int32 * k)(*[int(b.get("tau_index", -1)) for b in blocks])
        self._fix = (C.c_double * k)(*[float(b.get("fixed_scale", 0.0)) for b in blocks])
        self.struct = PinvPriorStruct(n_blocks=k, offset=self._off, size=self._size, P=self._ptr, ld=self._ld,
                                      tau_index=self._tau, fixed_scale=self._fix, lik_index=int(lik_index),
                                      reserved=0, lik_value=float(lik_value))


LOG_PRIOR_FN = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_int32, C.c_void_p)
THETA_STATUS = {0: "ok", 1: "max_iter", 2: "line_search", 3: "eval_failed"}


class KStats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("time_ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


def load_library(path: str = LIBPATH):
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    P = C.c_void_p
    i32, pi32 = C.c_int32, C.POINTER(C.c_int32)
    pd = C.POINTER(C.c_double)
    lib.inla_create.argtypes = [C.POINTER(P), P]
    lib.inla_destroy.argtypes = [P]
    lib.inla_set_stream.argtypes = [P, P]
    lib.inla_logdet.argtypes = [P, i32, pi32, C.POINTER(P), pi32, i32, pd, pi32]
    lib.inla_logdet_noalloc.argtypes = [P, i32, pi32, C.POINTER(P), pi32, i32, pd, pi32]
    for f in (lib.inla_constrained_mode, lib.inla_laplace_eval, lib.inla_woodbury_eval):
        f.argtypes = [P, i32, C.POINTER(Model), pd, i32, C.POINTER(P), C.POINTER(Opts), C.POINTER(Result)]
    lib.inla_pinv.argtypes = [P, i32, pi32, C.POINTER(P), pi32, C.POINTER(P), pi32, C.c_double, pi32, pi32, pi32]
    lib.inla_marginal_var.argtypes = [P, i32, C.POINTER(Model), pd, i32, C.POINTER(P), C.POINTER(P), pi32]
    lib.inla_woodbury_var.argtypes = [P, i32, C.POINTER(Model), pd, i32, C.POINTER(P), C.POINTER(P), pi32]
    lib.inla_profile.argtypes = [P, i32]
    lib.inla_profile_get.argtypes = [P, i32, i32, C.POINTER(KStats)]
    pf = C.c_void_p
    lib.inla_mlp_create.argtypes = [P, i32, i32, i32, C.c_uint64, C.POINTER(P)]
    lib.inla_mlp_destroy.argtypes = [P]
    lib.inla_mlp_num_params.argtypes = [P, C.POINTER(C.c_int64)]
    lib.inla_mlp_get_params.argtypes = [P, pf]
    lib.inla_mlp_set_params.argtypes = [P, pf]
    lib.inla_mlp_forward.argtypes = [P, i32, pf, pf]
    lib.inla_mlp_grad.argtypes = [P, i32, pf, pf, pf, pd]
    lib.inla_mlp_train_step.argtypes = [P, i32, pf, pf, C.c_float, pd]
    lib.inla_mlp_predict_modes.argtypes = [P, i32, pd, i32, pd, pd, C.POINTER(P)]
    lib.inla_set_graphs.argtypes = [P, i32]
    lib.inla_set_lookahead.argtypes = [P, i32]
    lib.inla_set_overlap.argtypes = [P, i32]
    lib.inla_graph_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.inla_set_pass_graphs.argtypes = [P, i32]
    lib.inla_pass_graph_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.inla_autotune.argtypes = [P, i32, pi32, pi32, i32, i32, pi32, pd, pi32]
    lib.inla_tune_set.argtypes = [P, i32, i32, i32, pi32]
    lib.inla_tune_get.argtypes = [P, i32, i32, i32, pi32]
    lib.inla_vb_mean.argtypes = [P, i32, C.POINTER(Model), pd, i32, C.POINTER(P), C.POINTER(P), i32, C.POINTER(Opts),
                                 pi32, pi32]
    lib.inla_theta_mode.argtypes = [P, C.POINTER(Model), i32, pd, C.POINTER(ThetaOpts), LOG_PRIOR_FN, P, pd, pd, pd,
                                    pi32, pi32, pi32]
    lib.inla_theta_hessian.argtypes = [P, C.POINTER(Model), i32, pd, C.c_double, C.POINTER(Opts), LOG_PRIOR_FN, P, pd,
                                       pd, pi32]
    pp = C.POINTER(PinvPriorStruct)
    lib.inla_pinv_prior_assemble.argtypes = [P, pp, i32, i32, pd, i32, C.POINTER(P)]
    lib.inla_theta_mode_pinv.argtypes = [P, C.POINTER(Model), pp, i32, pd, C.POINTER(ThetaOpts), LOG_PRIOR_FN, P, pd,
                                         pd, pd, pi32, pi32, pi32]
    lib.inla_theta_hessian_pinv.argtypes = [P, C.POINTER(Model), pp, i32, pd, C.c_double, C.POINTER(Opts),
                                            LOG_PRIOR_FN, P, pd, pd, pi32]
    lib.inla_ccd_design.argtypes = [i32, C.c_double, pi32, pd, pd]
    lib.inla_ccd_points.argtypes = [i32, pd, pd, C.c_double, pi32, pd, pd]
    lib.inla_ccd_weights.argtypes = [i32, pd, pd, pd]
    lib.inla_version.restype = C.c_char_p
    for name in EXPORTS:
        if name != "inla_version":
            getattr(lib, name).restype = C.c_int
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class DeviceModel:
    """A model dict (see ``synth``) with its arrays copied to the GPU."""

    def __init__(self, model: dict, device="cuda"):
        import torch

        def dev(a):
            if a is None:
                return None
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device)

        self.model = model
        self.n = int(model["n"])
        Cm = model.get("C")
        self.k = 0 if Cm is None else int(np.asarray(Cm).shape[0])
        self.y = dev(model["y"])
        self.E = dev(model.get("E"))
        self.C = dev(Cm) if self.k else None
        self.e = dev(model.get("e")) if self.k else None
        self.coords = dev(model.get("coords"))
        Q = model.get("Qprior")
        # column-major n x n: the transpose of a C-order array is its column-major view
        self.Q = dev(np.asarray(Q).T) if Q is not None else None
        # a general design matrix travels in CSR form (built from the dense array)
        A = model.get("A")
        self.m, self.nnz = 0, 0
        self.A_rowptr = self.A_col = self.A_val = None
        if A is not None:
            A = np.asarray(A, dtype=np.float64)
            rows, cols = np.nonzero(A)
            self.m, self.nnz = int(A.shape[0]), int(len(rows))
            rowptr = np.zeros(self.m + 1, dtype=np.int32)
            np.add.at(rowptr, rows + 1, 1)
            rowptr = np.cumsum(rowptr).astype(np.int32)
            self.A_rowptr = torch.as_tensor(rowptr).to(device)
            self.A_col = torch.as_tensor(cols.astype(np.int32)).to(device)
            self.A_val = dev(A[rows, cols])
        self.struct = Model(
            n=self.n, k=self.k, lik=LIK[model["lik"]], prior=PRIOR[model["prior"]],
            n_s=int(model.get("n_s") or self.n), n_t=int(model.get("n_t") or 1),
            ldq=self.n if Q is not None else 0, reserved=0,
            y=_ptr(self.y), E=_ptr(self.E), C=_ptr(self.C), e=_ptr(self.e),
            coords=_ptr(self.coords), Qprior=_ptr(self.Q),
            m=self.m, nnz=self.nnz, A_rowptr=_ptr(self.A_rowptr), A_col=_ptr(self.A_col), A_val=_ptr(self.A_val),
        )


class LibraryError(RuntimeError):
    pass


class Library:
    """One handle bound to torch's current stream on the current device."""

    def __init__(self, path: str = LIBPATH):
        import torch

        if not torch.cuda.is_available():
            raise LibraryError("no HIP device available")
        self.torch = torch
        self.lib = load_library(path)
        self.h = C.c_void_p()
        self.overlap = False   # concurrent prior pass (set_overlap)
        rc = self.lib.inla_create(C.byref(self.h), C.c_void_p(torch.cuda.current_stream().cuda_stream))
        self._check(rc, "inla_create")

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                self.lib.inla_destroy(self.h)
                self.h = C.c_void_p()
        except Exception:
            pass

    @staticmethod
    def _check(rc, what):
        if rc != 0:
            raise LibraryError(f"{what} returned {rc}")

    def set_stream(self, stream=None):
        """Rebind the handle to ``stream`` (a torch.cuda.Stream of the same
        device; None: torch's current stream).  The library first waits for the
        work it queued on the previous stream; ordering of the caller's own work
        across the two streams stays the caller's (``wait_stream``)."""
        s = self.torch.cuda.current_stream() if stream is None else stream
        self._check(self.lib.inla_set_stream(self.h, C.c_void_p(s.cuda_stream)), "inla_set_stream")

    # ------------------------------------------------------------- entry points
    def logdet(self, mats, prec="fp64"):
        """log|Q_b| for a list of square float64 device tensors (C-order symmetric
        matrices; C order is the column-major transpose, identical for symmetric
        input).  Overwrites their lower (column-major) triangle with L (the FP32
        factor converted to FP64 for prec "fp32" or "bf16")."""
        B = len(mats)
        n = (C.c_int32 * B)(*[int(m.shape[0]) for m in mats])
        ld = (C.c_int32 * B)(*[max(1, int(m.shape[0])) for m in mats])
        ptrs = (C.c_void_p * B)(*[m.data_ptr() for m in mats])
        out = (C.c_double * B)()
        info = (C.c_int32 * B)()
        rc = self.lib.inla_logdet(self.h, B, n, ptrs, ld, PREC[prec], out, info)
        self._check(rc, "inla_logdet")
        return np.array(out[:]), np.array(info[:], dtype=np.int32)

    def logdet_noalloc(self, mats, prec="fp64"):
        """As logdet, through inla_logdet_noalloc (scratch in the library's fixed
        device array, nothing allocated).  Returns (logdets, info, status code):
        the status is returned rather than raised, so that INLA_ERR_TOO_LARGE
        (-1003) can be seen."""
        B = len(mats)
        n = (C.c_int32 * B)(*[int(m.shape[0]) for m in mats])
        ld = (C.c_int32 * B)(*[max(1, int(m.shape[0])) for m in mats])
        ptrs = (C.c_void_p * B)(*[m.data_ptr() for m in mats])
        out = (C.c_double * B)()
        info = (C.c_int32 * B)()
        rc = self.lib.inla_logdet_noalloc(self.h, B, n, ptrs, ld, PREC[prec], out, info)
        return np.array(out[:]), np.array(info[:], dtype=np.int32), int(rc)

    def _common(self, dmodels, theta, x):
        B = len(dmodels)
        theta = np.ascontiguousarray(np.atleast_2d(np.asarray(theta, dtype=np.float64)))
        assert theta.shape[0] == B
        models = (Model * B)(*[m.struct for m in dmodels])
        if x is None:
            x = [self.torch.zeros(m.n, dtype=self.torch.float64, device="cuda") for m in dmodels]
        ptrs = (C.c_void_p * B)(*[t.data_ptr() for t in x])
        return B, theta, models, x, ptrs

    def _run(self, fn, dmodels, theta, x=None, start=0, max_iter=0, tol=0.0, prec="fp64"):
        B, theta, models, x, ptrs = self._common(dmodels, theta, x)
        opts = Opts(prec=PREC[prec], max_iter=max_iter, tol=tol, start=start, reserved=0)
        res = (Result * B)()
        rc = fn(self.h, B, models, theta.ctypes.data_as(C.POINTER(C.c_double)), theta.shape[1], ptrs,
                C.byref(opts), res)
        self._check(rc, fn.__name__)
        return [r.asdict() for r in res], x

    def laplace_eval(self, dmodels, theta, x=None, start=0, max_iter=0, tol=0.0, prec="fp64"):
        """(results, modes): per-theta dicts of inla_result fields and device modes."""
        return self._run(self.lib.inla_laplace_eval, dmodels, theta, x, start, max_iter, tol, prec)

    def constrained_mode(self, dmodels, theta, x=None, start=0, max_iter=0, tol=0.0, prec="fp64"):
        return self._run(self.lib.inla_constrained_mode, dmodels, theta, x, start, max_iter, tol, prec)

    def pinv(self, mats, rtol=0.0):
        """Moore-Penrose inverses of symmetric float64 device tensors (inla_pinv;
        C order equals column-major for symmetric input).  Returns (list of
        device tensors Q^+, ranks, Jacobi sweeps, info codes)."""
        B = len(mats)
        n = (C.c_int32 * B)(*[int(m.shape[0]) for m in mats])
        ld = (C.c_int32 * B)(*[int(m.shape[0]) for m in mats])
        out = [self.torch.empty_like(m) for m in mats]
        qp = (C.c_void_p * B)(*[m.data_ptr() for m in mats])
        pp = (C.c_void_p * B)(*[o.data_ptr() for o in out])
        rank, sweeps, info = (C.c_int32 * B)(), (C.c_int32 * B)(), (C.c_int32 * B)()
        rc = self.lib.inla_pinv(self.h, B, n, qp, ld, pp, ld, float(rtol), rank, sweeps, info)
        self._check(rc, "inla_pinv")
        return out, np.array(rank[:]), np.array(sweeps[:]), np.array(info[:], dtype=np.int32)

    def woodbury_eval(self, dmodels, lik_params, qpinv, x=None, start=0, max_iter=0, tol=0.0):
        """Laplace evaluation through the pseudo-inverse route (inla_woodbury_eval):
        dmodels are DeviceModels of intrinsic-prior models, lik_params the per-theta
        likelihood parameter (log sigma^2 or beta0), qpinv the device tensors
        Q_prior(theta_b)^+.  Returns (results, modes)."""
        B = len(dmodels)
        th = np.ascontiguousarray(np.asarray(lik_params, dtype=np.float64).reshape(B, 1))
        models = self._pinv_models(dmodels, qpinv)
        if x is None:
            x = [self.torch.zeros(m.n, dtype=self.torch.float64, device="cuda") for m in dmodels]
        ptrs = (C.c_void_p * B)(*[t.data_ptr() for t in x])
        opts = Opts(prec=0, max_iter=max_iter, tol=tol, start=start, reserved=0)
        res = (Result * B)()
        rc = self.lib.inla_woodbury_eval(self.h, B, models, th.ctypes.data_as(C.POINTER(C.c_double)), 1, ptrs,
                                         C.byref(opts), res)
        self._check(rc, "inla_woodbury_eval")
        return [r.asdict() for r in res], x

    def _pinv_models(self, dmodels, qpinv):
        structs = []
        for dm, P in zip(dmodels, qpinv):
            s = Model.from_buffer_copy(dm.struct)
            s.prior, s.k, s.C, s.e, s.Qprior, s.ldq = 3, 0, None, None, P.data_ptr(), int(P.shape[0])
            structs.append(s)
        return (Model * len(structs))(*structs)

    def woodbury_var(self, dmodels, lik_params, qpinv, x_modes):
        """diag(Sigma*) of the Woodbury covariance at the given device modes
        (inla_woodbury_var).  Returns (list of device tensors, info)."""
        B = len(dmodels)
        th = np.ascontiguousarray(np.asarray(lik_params, dtype=np.float64).reshape(B, 1))
        models = self._pinv_models(dmodels, qpinv)
        var = [self.torch.empty(m.n, dtype=self.torch.float64, device="cuda") for m in dmodels]
        xp = (C.c_void_p * B)(*[t.data_ptr() for t in x_modes])
        vp = (C.c_void_p * B)(*[t.data_ptr() for t in var])
        info = (C.c_int32 * B)()
        rc = self.lib.inla_woodbury_var(self.h, B, models, th.ctypes.data_as(C.POINTER(C.c_double)), 1, xp, vp, info)
        self._check(rc, "inla_woodbury_var")
        return var, np.array(info[:], dtype=np.int32)

    def marginal_var(self, dmodels, theta, x_modes):
        B, theta, models, x_modes, xptrs = self._common(dmodels, theta, x_modes)
        var = [self.torch.empty(m.n, dtype=self.torch.float64, device="cuda") for m in dmodels]
        vptrs = (C.c_void_p * B)(*[t.data_ptr() for t in var])
        info = (C.c_int32 * B)()
        rc = self.lib.inla_marginal_var(self.h, B, models, theta.ctypes.data_as(C.POINTER(C.c_double)),
                                        theta.shape[1], xptrs, vptrs, info)
        self._check(rc, "inla_marginal_var")
        return var, np.array(info[:], dtype=np.int32)

    # ------------------------------------------------------------- theta mode, Hessian, CCD
    @staticmethod
    def _prior(log_prior):
        if log_prior is None:
            return LOG_PRIOR_FN()
        return LOG_PRIOR_FN(lambda th, t, user: float(log_prior(np.ctypeslib.as_array(th, shape=(t,)).copy())))

    def theta_mode(self, dmodel, theta0, log_prior=None, max_iter=0, h=0.0, gtol=0.0, ftol=0.0, max_step=0.0,
                   prec="fp64"):
        """BFGS mode of log pi~(theta | y); returns a dict (theta, log_post, grad,
        iters, evals, info)."""
        th0 = np.ascontiguousarray(theta0, dtype=np.float64)
        t = len(th0)
        o = ThetaOpts(max_iter=max_iter, reserved=0, h=h, gtol=gtol, ftol=ftol, max_step=max_step,
                      eval=Opts(prec=PREC[prec], max_iter=0, tol=0.0, start=0, reserved=0))
        cb = self._prior(log_prior)
        out, grad = np.zeros(t), np.zeros(t)
        fs = C.c_double()
        it, ev, info = C.c_int32(), C.c_int32(), C.c_int32()
        pd = C.POINTER(C.c_double)
        rc = self.lib.inla_theta_mode(self.h, C.byref(dmodel.struct), t, th0.ctypes.data_as(pd), C.byref(o), cb, None,
                                      out.ctypes.data_as(pd), C.byref(fs), grad.ctypes.data_as(pd), C.byref(it),
                                      C.byref(ev), C.byref(info))
        self._check(rc, "inla_theta_mode")
        return {"theta": out, "log_post": fs.value, "grad": grad, "iters": it.value, "evals": ev.value,
                "info": info.value}

    def theta_hessian(self, dmodel, theta, step=0.0, log_prior=None, prec="fp64"):
        """(negative Hessian t x t, log pi~ at theta, info)."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        t = len(th)
        H = np.zeros((t, t))
        lp = C.c_double()
        info = C.c_int32()
        o = Opts(prec=PREC[prec], max_iter=0, tol=0.0, start=0, reserved=0)
        pd = C.POINTER(C.c_double)
        rc = self.lib.inla_theta_hessian(self.h, C.byref(dmodel.struct), t, th.ctypes.data_as(pd), step, C.byref(o),
                                         self._prior(log_prior), None, H.ctypes.data_as(pd), C.byref(lp),
                                         C.byref(info))
        self._check(rc, "inla_theta_hessian")
        return H, lp.value, info.value

    @staticmethod
    def _pinv_model_struct(dmodel):
        s = Model.from_buffer_copy(dmodel.struct)
        s.prior, s.k, s.C, s.e = 3, 0, None, None
        return s

    def pinv_prior_assemble(self, prior, n, thetas):
        """Q_prior(theta_b)^+ (n x n device tensors) for the rows of thetas."""
        th = np.ascontiguousarray(np.atleast_2d(np.asarray(thetas, dtype=np.float64)))
        B = th.shape[0]
        out = [self.torch.empty((n, n), dtype=self.torch.float64, device="cuda") for _ in range(B)]
        ptrs = (C.c_void_p * B)(*[o.data_ptr() for o in out])
        rc = self.lib.inla_pinv_prior_assemble(self.h, C.byref(prior.struct), n, B,
                                               th.ctypes.data_as(C.POINTER(C.c_double)), th.shape[1], ptrs)
        self._check(rc, "inla_pinv_prior_assemble")
        return out

    def theta_mode_pinv(self, dmodel, prior, theta0, log_prior=None, max_iter=0, h=0.0, gtol=0.0, ftol=0.0,
                        max_step=0.0):
        """inla_theta_mode on the Moore-Penrose route (inla_theta_mode_pinv)."""
        th0 = np.ascontiguousarray(theta0, dtype=np.float64)
        t = len(th0)
        o = ThetaOpts(max_iter=max_iter, reserved=0, h=h, gtol=gtol, ftol=ftol, max_step=max_step,
                      eval=Opts(prec=0, max_iter=0, tol=0.0, start=0, reserved=0))
        cb = self._prior(log_prior)
        out, grad = np.zeros(t), np.zeros(t)
        fs = C.c_double()
        it, ev, info = C.c_int32(), C.c_int32(), C.c_int32()
        pd = C.POINTER(C.c_double)
        ms = self._pinv_model_struct(dmodel)
        rc = self.lib.inla_theta_mode_pinv(self.h, C.byref(ms), C.byref(prior.struct), t, th0.ctypes.data_as(pd),
                                           C.byref(o), cb, None, out.ctypes.data_as(pd), C.byref(fs),
                                           grad.ctypes.data_as(pd), C.byref(it), C.byref(ev), C.byref(info))
        self._check(rc, "inla_theta_mode_pinv")
        return {"theta": out, "log_post": fs.value, "grad": grad, "iters": it.value, "evals": ev.value,
                "info": info.value}

    def theta_hessian_pinv(self, dmodel, prior, theta, step=0.0, log_prior=None):
        """(negative Hessian, log pi~ at theta, info) on the Moore-Penrose route."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        t = len(th)
        H = np.zeros((t, t))
        lp = C.c_double()
        info = C.c_int32()
        o = Opts(prec=0, max_iter=0, tol=0.0, start=0, reserved=0)
        pd = C.POINTER(C.c_double)
        ms = self._pinv_model_struct(dmodel)
        rc = self.lib.inla_theta_hessian_pinv(self.h, C.byref(ms), C.byref(prior.struct), t, th.ctypes.data_as(pd),
                                              step, C.byref(o), self._prior(log_prior), None, H.ctypes.data_as(pd),
                                              C.byref(lp), C.byref(info))
        self._check(rc, "inla_theta_hessian_pinv")
        return H, lp.value, info.value

    def ccd_points(self, theta_star, neg_hess, f0=1.1):
        """(theta_k [n x t], delta [n]) of the CCD exploration around theta*."""
        th = np.ascontiguousarray(theta_star, dtype=np.float64)
        t = len(th)
        H = np.ascontiguousarray(neg_hess, dtype=np.float64)
        n = C.c_int32(0)
        self._check(self.lib.inla_ccd_design(t, f0, C.byref(n), None, None), "inla_ccd_design")
        pts, delta = np.zeros((n.value, t)), np.zeros(n.value)
        pd = C.POINTER(C.c_double)
        rc = self.lib.inla_ccd_points(t, th.ctypes.data_as(pd), H.ctypes.data_as(pd), f0, C.byref(n),
                                      pts.ctypes.data_as(pd), delta.ctypes.data_as(pd))
        self._check(rc, "inla_ccd_points")
        return pts, delta

    def ccd_weights(self, delta, log_post):
        d = np.ascontiguousarray(delta, dtype=np.float64)
        lp = np.ascontiguousarray(log_post, dtype=np.float64)
        w = np.zeros(len(d))
        pd = C.POINTER(C.c_double)
        self._check(self.lib.inla_ccd_weights(len(d), d.ctypes.data_as(pd), lp.ctypes.data_as(pd),
                                              w.ctypes.data_as(pd)), "inla_ccd_weights")
        return w

    # ------------------------------------------------------------- graphs and tuning
    def set_graphs(self, on: bool):
        self._check(self.lib.inla_set_graphs(self.h, 1 if on else 0), "inla_set_graphs")

    def set_lookahead(self, on: bool):
        self._check(self.lib.inla_set_lookahead(self.h, 1 if on else 0), "inla_set_lookahead")

    def set_overlap(self, on: bool):
        """Run each evaluation's FP64 prior pass beside its Newton iteration on a
        stream of the handle (default off; results identical either way)."""
        self._check(self.lib.inla_set_overlap(self.h, 1 if on else 0), "inla_set_overlap")
        self.overlap = bool(on)

    def graph_stats(self):
        cap, rep = C.c_int64(), C.c_int64()
        self._check(self.lib.inla_graph_stats(self.h, C.byref(cap), C.byref(rep)), "inla_graph_stats")
        return {"captured": cap.value, "replays": rep.value}

    def set_pass_graphs(self, on: bool):
        """One hipGraph per Newton pass and per refinement step (default on)."""
        self._check(self.lib.inla_set_pass_graphs(self.h, 1 if on else 0), "inla_set_pass_graphs")

    def pass_graph_stats(self):
        cap, rep = C.c_int64(), C.c_int64()
        self._check(self.lib.inla_pass_graph_stats(self.h, C.byref(cap), C.byref(rep)), "inla_pass_graph_stats")
        return {"captured": cap.value, "replays": rep.value}

    def autotune(self, ns, kbs, prec="fp64", reps=2):
        """Tune the factorisation of a batch of orders ``ns`` with border heights
        ``kbs``; returns the chosen (nb, tm, lookahead) and each candidate's mean
        time in ms, keyed by (nb, tm, lookahead)."""
        B = len(ns)
        n = (C.c_int32 * B)(*[int(v) for v in ns])
        kb = (C.c_int32 * B)(*[int(v) for v in kbs])
        cfg, nc = (C.c_int32 * 3)(), C.c_int32()
        ms = (C.c_double * 9)()
        rc = self.lib.inla_autotune(self.h, B, n, kb, PREC[prec], reps, cfg, ms, C.byref(nc))
        self._check(rc, "inla_autotune")
        base = TUNE_CANDIDATES[prec]
        times = {(c[0], c[1], 0): ms[i] for i, c in enumerate(base)}
        if nc.value > len(base):
            fastest = min(times, key=times.get)
            times[(fastest[0], fastest[1], 1)] = ms[len(base)]
        return tuple(cfg[:]), times

    def tune_set(self, prec, n_max, B, nb=None, tm=128, look=0):
        """Set (nb, tm, lookahead) for such batches; nb=None erases the entry."""
        cfg = None if nb is None else (C.c_int32 * 3)(nb, tm, look)
        self._check(self.lib.inla_tune_set(self.h, PREC[prec], n_max, B, cfg), "inla_tune_set")

    def tune_get(self, prec, n_max, B):
        cfg = (C.c_int32 * 3)()
        self._check(self.lib.inla_tune_get(self.h, PREC[prec], n_max, B, cfg), "inla_tune_get")
        return tuple(cfg[:])

    def vb_mean(self, dmodels, theta, var, x_mode, n_gh=0, max_iter=0, tol=0.0):
        """Variational-Bayes corrected means (device tensors, new) from the Laplace
        modes and marginal variances; returns (means, iterations, info)."""
        B, theta, models, _, _ = self._common(dmodels, theta, None)
        xs = [t.clone() for t in x_mode]
        xp = (C.c_void_p * B)(*[t.data_ptr() for t in xs])
        vp = (C.c_void_p * B)(*[t.data_ptr() for t in var])
        it, info = (C.c_int32 * B)(), (C.c_int32 * B)()
        o = Opts(prec=0, max_iter=max_iter, tol=tol, start=0, reserved=0)
        rc = self.lib.inla_vb_mean(self.h, B, models, theta.ctypes.data_as(C.POINTER(C.c_double)), theta.shape[1],
                                   vp, xp, n_gh, C.byref(o), it, info)
        self._check(rc, "inla_vb_mean")
        return xs, np.array(it[:], dtype=np.int32), np.array(info[:], dtype=np.int32)

    # ------------------------------------------------------------- profiling
    def profile(self, on: bool):
        self._check(self.lib.inla_profile(self.h, 1 if on else 0), "inla_profile")

    def profile_get(self, kclass, prec="fp64"):
        s = KStats()
        self._check(self.lib.inla_profile_get(self.h, kclass, PREC[prec], C.byref(s)), "inla_profile_get")
        return {"launches": s.launches, "time_ms": s.time_ms, "flops": s.flops, "bytes": s.bytes}


class Mlp:
    """The warm-start network (I -> H -> H -> O, GELU, FP32) living on the GPU."""

    def __init__(self, library: "Library", n_in: int, n_hidden: int, n_out: int, seed: int = 0):
        self.L = library
        self.lib = library.lib
        self.dims = (n_in, n_hidden, n_out)
        self.m = C.c_void_p()
        Library._check(self.lib.inla_mlp_create(library.h, n_in, n_hidden, n_out, seed, C.byref(self.m)),
                       "inla_mlp_create")
        cnt = C.c_int64()
        Library._check(self.lib.inla_mlp_num_params(self.m, C.byref(cnt)), "inla_mlp_num_params")
        self.num_params = cnt.value

    def __del__(self):
        try:
            if self.m and self.m.value:
                self.lib.inla_mlp_destroy(self.m)
                self.m = C.c_void_p()
        except Exception:
            pass

    def get_params(self):
        t = self.L.torch.empty(self.num_params, dtype=self.L.torch.float32, device="cuda")
        Library._check(self.lib.inla_mlp_get_params(self.m, t.data_ptr()), "inla_mlp_get_params")
        return t

    def set_params(self, t):
        t = t.to(dtype=self.L.torch.float32, device="cuda").contiguous()
        Library._check(self.lib.inla_mlp_set_params(self.m, t.data_ptr()), "inla_mlp_set_params")

    def forward(self, x):
        x = x.to(dtype=self.L.torch.float32, device="cuda").contiguous()
        y = self.L.torch.empty((x.shape[0], self.dims[2]), dtype=self.L.torch.float32, device="cuda")
        Library._check(self.lib.inla_mlp_forward(self.m, x.shape[0], x.data_ptr(), y.data_ptr()), "inla_mlp_forward")
        return y

    def grad(self, x, target):
        x = x.to(dtype=self.L.torch.float32, device="cuda").contiguous()
        target = target.to(dtype=self.L.torch.float64, device="cuda").contiguous()
        g = self.L.torch.empty(self.num_params, dtype=self.L.torch.float32, device="cuda")
        loss = C.c_double()
        Library._check(self.lib.inla_mlp_grad(self.m, x.shape[0], x.data_ptr(), target.data_ptr(), g.data_ptr(),
                                              C.byref(loss)), "inla_mlp_grad")
        return loss.value, g

    def train_step(self, x, target, lr=1e-3, want_loss=True):
        """x: float32 (B x I) device tensor, target: float64 (B x O) device tensor.
        Returns the batch loss before the step, or None with want_loss=False
        (then the call does not wait for the device)."""
        loss = C.c_double()
        Library._check(self.lib.inla_mlp_train_step(self.m, x.shape[0], x.data_ptr(), target.data_ptr(), lr,
                                                    C.byref(loss) if want_loss else None), "inla_mlp_train_step")
        return loss.value if want_loss else None

    def predict_modes(self, theta, centre, scale, x=None):
        theta = np.ascontiguousarray(np.atleast_2d(np.asarray(theta, dtype=np.float64)))
        B = theta.shape[0]
        centre = np.ascontiguousarray(centre, dtype=np.float64)
        scale = np.ascontiguousarray(scale, dtype=np.float64)
        if x is None:
            x = [self.L.torch.empty(self.dims[2], dtype=self.L.torch.float64, device="cuda") for _ in range(B)]
        ptrs = (C.c_void_p * B)(*[t.data_ptr() for t in x])
        pd = C.POINTER(C.c_double)
        Library._check(self.lib.inla_mlp_predict_modes(self.m, B, theta.ctypes.data_as(pd), theta.shape[1],
                                                       centre.ctypes.data_as(pd), scale.ctypes.data_as(pd), ptrs),
                       "inla_mlp_predict_modes")
        return x
