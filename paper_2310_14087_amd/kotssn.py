"""Thin ctypes binding of libkotssn (include/kotssn.h).  Argument marshalling only: every step of the solver
runs in the library's HIP kernels.  Tensors are torch tensors on the GPU (float64, contiguous); the binding
passes their data pointers and the current torch stream.

The library is loaded from this package directory (built by ``python -m paper_2310_14087_amd.build``);
importing a function raises if it is missing.  There is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from pathlib import Path

import numpy as np

_LIBPATH = Path(__file__).resolve().parent / "libkotssn.so"

KOT_OK, KOT_NOT_CONVERGED = 0, 1
KOT_ERR_ARG, KOT_ERR_HIP, KOT_ERR_OOM, KOT_ERR_FACTOR, KOT_ERR_NUMERIC, KOT_ERR_EIG = -1, -2, -3, -4, -5, -6
KOT_FP64, KOT_FP32, KOT_MIXED_BF16, KOT_MIXED_BF16X3 = 0, 1, 2, 3
KOT_SAFEGUARD_EG, KOT_SAFEGUARD_NONE, KOT_SAFEGUARD_EG_ONLY = 0, 1, 2
KOT_PRECOND_NONE, KOT_PRECOND_JACOBI = 0, 1
KOT_SCHUR_CG, KOT_SCHUR_SQMR = 0, 1

STATUS_NAMES = {0: "KOT_OK", 1: "KOT_NOT_CONVERGED", -1: "KOT_ERR_ARG", -2: "KOT_ERR_HIP", -3: "KOT_ERR_OOM",
                -4: "KOT_ERR_FACTOR", -5: "KOT_ERR_NUMERIC", -6: "KOT_ERR_EIG"}

EXPORTED = ["kot_params_default", "kot_create", "kot_destroy", "kot_last_error", "kot_setup", "kot_solve",
            "kot_solve_core", "kot_eigh", "kot_residual", "kot_ssn_direction", "kot_schur_matvec", "kot_eg_step",
            "kot_cholesky",
            "kot_gemm", "kot_profile", "kot_mlp_params", "kot_features", "kot_mlp_forward", "kot_mlp_loss_grad",
            "kot_mlp_adam", "kot_warmstart", "kot_solve_batched", "kot_autotune", "kot_autotune_load",
            "kot_potentials", "kot_eigh_noalloc"]


class KotParams(C.Structure):
    _fields_ = [("sigma", C.c_double), ("lambda1", C.c_double), ("lambda2", C.c_double),
                ("eps_jitter", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int), ("cg_max_iter", C.c_int),
                ("tau", C.c_double), ("kappa", C.c_double), ("alpha1", C.c_double), ("alpha2", C.c_double),
                ("beta0", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("theta0", C.c_double),
                ("theta_min", C.c_double), ("theta_max", C.c_double), ("eg_step", C.c_double),
                ("precision", C.c_int), ("safeguard", C.c_int), ("null_step", C.c_int),
                ("eig_max_sweeps", C.c_int), ("warm_eig", C.c_int), ("lift_x0", C.c_int), ("ws_F", C.c_int),
                ("ws_H", C.c_int), ("ws_theta", C.c_void_p), ("overlap", C.c_int),
                ("lowp_min_rows", C.c_int), ("precond", C.c_int),
                ("schur_solver", C.c_int), ("eig_inner_sweeps", C.c_int), ("closed_start", C.c_int),
                ("kdiag_tol", C.c_double)]


class KotProblem(C.Structure):
    _fields_ = [("n_src", C.c_int), ("n_tgt", C.c_int), ("d", C.c_int), ("l", C.c_int),
                ("xs", C.c_void_p), ("ys", C.c_void_p), ("xf", C.c_void_p), ("yf", C.c_void_p)]


class KotResult(C.Structure):
    _fields_ = [("gamma", C.c_void_p), ("X", C.c_void_p), ("res_hist", C.c_void_p), ("res_v_hist", C.c_void_p),
                ("hist_cap", C.c_int), ("ot", C.c_double), ("residual", C.c_double), ("iters", C.c_int),
                ("cg_iters_total", C.c_int), ("eg_accepts", C.c_int), ("null_steps", C.c_int),
                ("eig_sweeps_total", C.c_int), ("alpha_last", C.c_int), ("warm_used", C.c_int),
                ("lowp_directions", C.c_int), ("time_ms", C.c_double), ("kdiag", C.c_int)]


_lib = None


def load(path: str | os.PathLike | None = None) -> C.CDLL:
    """Load libkotssn.so (raises OSError with a build hint if it is missing)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else _LIBPATH
    if not p.exists():
        raise OSError(f"{p} not found: build it with `python -m paper_2310_14087_amd.build`")
    # torch first: the library must bind to the HIP runtime that allocates the tensors it is handed (loaded
    # first, it would pull in the system's copy, whose context does not see torch's device memory)
    import torch  # noqa: F401
    lib = C.CDLL(str(p))
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    P = C.POINTER
    sig = {
        "kot_params_default": (None, [P(KotParams)]),
        "kot_create": (i, [P(vp), i, vp]),
        "kot_destroy": (i, [vp]),
        "kot_last_error": (C.c_char_p, [vp]),
        "kot_setup": (i, [vp, P(KotProblem), P(KotParams), vp, vp, vp, vp, P(d)]),
        "kot_solve": (i, [vp, P(KotProblem), P(KotParams), vp, P(KotResult)]),
        "kot_solve_core": (i, [vp, i, vp, vp, vp, d, vp, P(KotParams), vp, P(KotResult)]),
        "kot_eigh": (i, [vp, i, vp, vp, vp, P(KotParams)]),
        "kot_eigh_noalloc": (i, [i, vp, i, vp, vp, vp, P(KotParams)]),
        "kot_residual": (i, [vp, i, vp, vp, vp, vp, vp, P(KotParams), vp, vp, P(d)]),
        "kot_ssn_direction": (i, [vp, i, vp, vp, vp, vp, vp, d, P(KotParams), vp, vp, P(d)]),
        "kot_schur_matvec": (i, [vp, i, vp, vp, vp, vp, vp, d, P(KotParams), i, vp, vp, P(d)]),
        "kot_eg_step": (i, [vp, i, vp, vp, vp, vp, vp, d, P(KotParams), vp, vp]),
        "kot_cholesky": (i, [vp, i, vp, d, vp, vp]),
        "kot_gemm": (i, [vp, i, i, i, i, i, d, vp, i, vp, vp, i, d, vp, i, i, i]),
        "kot_profile": (i, [vp, i, vp, i]),
        "kot_mlp_params": (i, [i, i]),
        "kot_features": (i, [vp, i, vp, vp, vp, vp, d, P(KotParams), vp]),
        "kot_mlp_forward": (i, [vp, i, i, i, vp, vp, vp]),
        "kot_mlp_loss_grad": (i, [vp, i, i, i, vp, vp, vp, vp, P(d)]),
        "kot_mlp_adam": (i, [vp, i, vp, vp, vp, vp, i, C.c_float, C.c_float, C.c_float, C.c_float]),
        "kot_warmstart": (i, [vp, P(KotProblem), P(KotParams), i, i, vp, vp]),
        "kot_solve_batched": (i, [vp, i, P(KotProblem), P(KotParams), i, vp, P(KotResult), P(i), i]),
        "kot_autotune": (i, [vp, P(i), i, C.c_char_p, P(i)]),
        "kot_autotune_load": (i, [vp, C.c_char_p]),
        "kot_potentials": (i, [vp, P(KotProblem), P(KotParams), vp, i, vp, vp, vp, vp, vp]),
    }
    for name, (rt, args) in sig.items():
        f = getattr(lib, name)
        f.restype = rt
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


class KotError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def default_params(**kw) -> KotParams:
    p = KotParams()
    load().kot_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def eigh_noalloc(Z, prm: KotParams, P=None, w=None):
    """kot_eigh_noalloc on Z's device and torch's current stream there (no context; l <= 512).  P and w may be
    given (preallocated outputs) so that the call itself allocates nothing."""
    import torch
    l = Z.shape[0]
    P = torch.empty_like(Z) if P is None else P
    w = torch.empty(l, device=Z.device, dtype=torch.float64) if w is None else w
    lib = load()
    st = lib.kot_eigh_noalloc(Z.device.index or 0, torch.cuda.current_stream(Z.device).cuda_stream, l, _ptr(Z),
                              _ptr(P), _ptr(w), C.byref(prm))
    if st != KOT_OK:
        raise KotError(st, lib.kot_last_error(None).decode())
    return w, P


def _ptr(t, dtype=None) -> int | None:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    dtype = dtype or torch.float64
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    return t.data_ptr()


def _fptr(t) -> int | None:
    import torch
    return _ptr(t, torch.float32)


def mlp_params(F: int, H: int) -> int:
    return load().kot_mlp_params(F, H)


N_FEATURES = 12


@dataclass
class SolveResult:
    status: int
    ot: float
    residual: float
    iters: int
    cg_iters_total: int
    eg_accepts: int
    null_steps: int
    eig_sweeps_total: int
    alpha_last: int
    warm_used: int
    lowp_directions: int
    time_ms: float
    res_hist: np.ndarray
    res_v_hist: np.ndarray
    kdiag: int = 0


class Context:
    """Owns a kot_ctx on a device; uses torch's current stream on that device."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.device = device
        with torch.cuda.device(device):
            s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = C.c_void_p()
        st = self.lib.kot_create(C.byref(h), device, C.c_void_p(s.cuda_stream))
        if st != KOT_OK:
            raise KotError(st, "kot_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.kot_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, allow=(KOT_OK,)) -> int:
        if st not in allow:
            raise KotError(st, self.lib.kot_last_error(self.h).decode())
        return st

    # ---- entry points (same names as the C-ABI, without the prefix) ----
    def setup(self, xs, ys, xf, yf, prm: KotParams):
        import torch
        l, dd = xf.shape
        pb = KotProblem(xs.shape[0], ys.shape[0], dd, l, _ptr(xs), _ptr(ys), _ptr(xf), _ptr(yf))
        opts = dict(device=xs.device, dtype=torch.float64)
        Q = torch.empty((l, l), **opts)
        z = torch.empty(l, **opts)
        R = torch.empty((l, l), **opts)
        wsum = torch.empty(l, **opts)
        q2 = C.c_double()
        self._check(self.lib.kot_setup(self.h, C.byref(pb), C.byref(prm), _ptr(Q), _ptr(z), _ptr(R), _ptr(wsum),
                                       C.byref(q2)))
        return Q, z, R, wsum, q2.value

    def _result(self, l, device, want_X, hist_cap):
        import torch
        gamma = torch.empty(l, device=device, dtype=torch.float64)
        X = torch.empty((l, l), device=device, dtype=torch.float64) if want_X else None
        rh = np.zeros(hist_cap)
        rvh = np.zeros(hist_cap)
        res = KotResult()
        res.gamma = _ptr(gamma)
        res.X = _ptr(X) if X is not None else None
        res.res_hist = rh.ctypes.data
        res.res_v_hist = rvh.ctypes.data
        res.hist_cap = hist_cap
        return gamma, X, rh, rvh, res

    @staticmethod
    def _pack(st, res, rh, rvh) -> SolveResult:
        n = min(res.iters + 1, len(rh))
        return SolveResult(st, res.ot, res.residual, res.iters, res.cg_iters_total, res.eg_accepts, res.null_steps,
                           res.eig_sweeps_total, res.alpha_last, res.warm_used, res.lowp_directions, res.time_ms, rh[:n].copy(),
                           rvh[:n].copy(), kdiag=res.kdiag)

    def solve(self, xs, ys, xf, yf, prm: KotParams, gamma0=None, want_X=False, hist_cap=1024):
        l, dd = xf.shape
        pb = KotProblem(xs.shape[0], ys.shape[0], dd, l, _ptr(xs), _ptr(ys), _ptr(xf), _ptr(yf))
        gamma, X, rh, rvh, res = self._result(l, xs.device, want_X, hist_cap)
        st = self._check(self.lib.kot_solve(self.h, C.byref(pb), C.byref(prm), _ptr(gamma0), C.byref(res)),
                         (KOT_OK, KOT_NOT_CONVERGED))
        return gamma, X, self._pack(st, res, rh, rvh)

    def solve_batched(self, problems, prms, lanes=0, hist_cap=256):
        """problems: list of (xs, ys, xf, yf) device tensors; prms: one KotParams or a list of them."""
        nprob = len(problems)
        probs = (KotProblem * nprob)()
        for i, (xs, ys, xf, yf) in enumerate(problems):
            l, dd = xf.shape
            probs[i] = KotProblem(xs.shape[0], ys.shape[0], dd, l, _ptr(xs), _ptr(ys), _ptr(xf), _ptr(yf))
        plist = prms if isinstance(prms, (list, tuple)) else [prms]
        parr = (KotParams * len(plist))(*plist)
        outs = [self._result(xf.shape[0], xf.device, False, hist_cap) for (_, _, xf, _) in problems]
        res = (KotResult * nprob)(*[o[4] for o in outs])
        st = (C.c_int * nprob)()
        self._check(self.lib.kot_solve_batched(self.h, nprob, probs, parr, len(plist), None, res, st, int(lanes)),
                    (KOT_OK, KOT_NOT_CONVERGED))
        return [(outs[i][0], self._pack(st[i], res[i], outs[i][2], outs[i][3])) for i in range(nprob)]

    def autotune(self, sizes, path=None):
        arr = (C.c_int * len(sizes))(*sizes)
        out = (C.c_int * 33)()
        self._check(self.lib.kot_autotune(self.h, arr, len(sizes), path.encode() if path else None, out))
        return list(out)

    def autotune_load(self, path):
        self._check(self.lib.kot_autotune_load(self.h, str(path).encode()))

    def solve_core(self, Q, z, R, q2, wsum, prm: KotParams, gamma0=None, want_X=False, hist_cap=1024):
        l = Q.shape[0]
        gamma, X, rh, rvh, res = self._result(l, Q.device, want_X, hist_cap)
        st = self._check(self.lib.kot_solve_core(self.h, l, _ptr(Q), _ptr(z), _ptr(R), float(q2), _ptr(wsum),
                                                 C.byref(prm), _ptr(gamma0), C.byref(res)),
                         (KOT_OK, KOT_NOT_CONVERGED))
        return gamma, X, self._pack(st, res, rh, rvh)

    def eigh(self, Z, prm: KotParams):
        import torch
        l = Z.shape[0]
        P = torch.empty_like(Z)
        w = torch.empty(l, device=Z.device, dtype=torch.float64)
        self._check(self.lib.kot_eigh(self.h, l, _ptr(Z), _ptr(P), _ptr(w), C.byref(prm)))
        return w, P

    def residual(self, Q, z, R, gamma, X, prm: KotParams):
        import torch
        l = Q.shape[0]
        r1 = torch.empty(l, device=Q.device, dtype=torch.float64)
        r2 = torch.empty((l, l), device=Q.device, dtype=torch.float64)
        norms = (C.c_double * 3)()
        self._check(self.lib.kot_residual(self.h, l, _ptr(Q), _ptr(z), _ptr(R), _ptr(gamma), _ptr(X), C.byref(prm),
                                          _ptr(r1), _ptr(r2), norms))
        return r1, r2, (norms[0], norms[1], int(norms[2]))

    def ssn_direction(self, Q, z, R, gamma, X, mu, prm: KotParams):
        import torch
        l = Q.shape[0]
        dg = torch.empty(l, device=Q.device, dtype=torch.float64)
        dX = torch.empty((l, l), device=Q.device, dtype=torch.float64)
        info = (C.c_double * 4)()
        self._check(self.lib.kot_ssn_direction(self.h, l, _ptr(Q), _ptr(z), _ptr(R), _ptr(gamma), _ptr(X),
                                               float(mu), C.byref(prm), _ptr(dg), _ptr(dX), info))
        return dg, dX, dict(cg_iters=int(info[0]), cg_res=info[1], alpha=int(info[2]), res=info[3])

    def schur_matvec(self, Q, z, R, gamma, X, mu, v, prm: KotParams, reps=1):
        import torch
        l = Q.shape[0]
        y = torch.empty(l, device=Q.device, dtype=torch.float64)
        info = (C.c_double * 4)()
        self._check(self.lib.kot_schur_matvec(self.h, l, _ptr(Q), _ptr(z), _ptr(R), _ptr(gamma), _ptr(X), float(mu),
                                              C.byref(prm), int(reps), _ptr(v), _ptr(y), info))
        return y, dict(alpha=int(info[0]), m=int(info[1]), complement=bool(info[2]), ms=info[3])

    def eg_step(self, Q, z, R, gamma, X, eta, prm: KotParams):
        import torch
        l = Q.shape[0]
        go = torch.empty(l, device=Q.device, dtype=torch.float64)
        Xo = torch.empty((l, l), device=Q.device, dtype=torch.float64)
        self._check(self.lib.kot_eg_step(self.h, l, _ptr(Q), _ptr(z), _ptr(R), _ptr(gamma), _ptr(X), float(eta),
                                         C.byref(prm), _ptr(go), _ptr(Xo)))
        return go, Xo

    def cholesky(self, A, eps=0.0, inverse=False):
        """R with R^T R = A + eps I; with inverse, (R, R^-T)."""
        import torch
        R = torch.empty_like(A)
        Rit = torch.empty_like(A) if inverse else None
        self._check(self.lib.kot_cholesky(self.h, A.shape[0], _ptr(A), float(eps), _ptr(R),
                                          _ptr(Rit) if inverse else None))
        return (R, Rit) if inverse else R

    # ---- warm-start network ----
    def features(self, Q, z, R, wsum, q2, prm: KotParams):
        import torch
        l = Q.shape[0]
        X = torch.empty((l, N_FEATURES), device=Q.device, dtype=torch.float32)
        self._check(self.lib.kot_features(self.h, l, _ptr(Q), _ptr(z), _ptr(R), _ptr(wsum), float(q2), C.byref(prm),
                                          _fptr(X)))
        return X

    def mlp_forward(self, X, theta, H):
        import torch
        n, F = X.shape
        out = torch.empty(n, device=X.device, dtype=torch.float32)
        self._check(self.lib.kot_mlp_forward(self.h, n, F, H, _fptr(X), _fptr(theta), _fptr(out)))
        return out

    def mlp_loss_grad(self, X, y, theta, H, grad=None):
        import torch
        n, F = X.shape
        if grad is None:
            grad = torch.empty_like(theta)
        loss = C.c_double()
        self._check(self.lib.kot_mlp_loss_grad(self.h, n, F, H, _fptr(X), _fptr(y), _fptr(theta), _fptr(grad),
                                               C.byref(loss)))
        return loss.value, grad

    def mlp_adam(self, theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.kot_mlp_adam(self.h, theta.numel(), _fptr(theta), _fptr(grad), _fptr(m), _fptr(v), int(t),
                                          float(lr), float(beta1), float(beta2), float(eps)))

    def warmstart(self, xs, ys, xf, yf, prm: KotParams, theta, H):
        import torch
        l, dd = xf.shape
        pb = KotProblem(xs.shape[0], ys.shape[0], dd, l, _ptr(xs), _ptr(ys), _ptr(xf), _ptr(yf))
        g0 = torch.empty(l, device=xs.device, dtype=torch.float64)
        self._check(self.lib.kot_warmstart(self.h, C.byref(pb), C.byref(prm), N_FEATURES, H, _fptr(theta), _ptr(g0)))
        return g0

    def potentials(self, xs, ys, xf, yf, prm: KotParams, gamma, xq=None, yq=None, want_map=True):
        """(u(xq), v(yq), T(xq)) of a solved problem; entries for a missing query set are None."""
        import torch
        l, dd = xf.shape
        pb = KotProblem(xs.shape[0], ys.shape[0], dd, l, _ptr(xs), _ptr(ys), _ptr(xf), _ptr(yf))
        q = xq if xq is not None else yq
        m = 0 if q is None else q.shape[0]
        mk = lambda *shape: torch.empty(shape, device=xf.device, dtype=torch.float64)
        u = mk(m) if xq is not None else None
        v = mk(m) if yq is not None else None
        T = mk(m, dd) if (xq is not None and want_map) else None
        if xq is not None and yq is not None and xq.shape[0] != yq.shape[0]:
            raise ValueError("xq and yq must have the same number of rows")
        self._check(self.lib.kot_potentials(self.h, C.byref(pb), C.byref(prm), _ptr(gamma), m, _ptr(xq), _ptr(yq),
                                            _ptr(u), _ptr(v), _ptr(T)))
        return u, v, T

    PROFILE_CLASSES = ("gemm_f64", "eig_sweep", "gemv_f64", "gemm_f32", "gemm_bf16", "potential", "chain_f64")

    def profile_start(self):
        self._check(self.lib.kot_profile(self.h, 1, None, 0))

    def profile_stop(self) -> dict:
        n = len(self.PROFILE_CLASSES)
        buf = (C.c_double * (4 * n))()
        self._check(self.lib.kot_profile(self.h, 0, buf, n))
        return {c: dict(launches=int(buf[4 * i]), ms=buf[4 * i + 1], flops=buf[4 * i + 2], bytes=buf[4 * i + 3])
                for i, c in enumerate(self.PROFILE_CLASSES)}

    def gemm(self, A, B, transa=False, transb=False, s=None, alpha=1.0, beta=0.0, Cm=None, tri=0, sym=False):
        import torch
        m = A.shape[1] if transa else A.shape[0]
        k = A.shape[0] if transa else A.shape[1]
        n = B.shape[0] if transb else B.shape[1]
        if Cm is None:
            Cm = torch.zeros((m, n), device=A.device, dtype=torch.float64)
        self._check(self.lib.kot_gemm(self.h, int(transa), int(transb), m, n, k, float(alpha), _ptr(A), A.shape[1],
                                      _ptr(s), _ptr(B), B.shape[1], float(beta), _ptr(Cm), Cm.shape[1], int(tri),
                                      int(bool(sym))))
        return Cm
