"""Python binding of libpd, the MI355X (gfx950) polynomial-diagram library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libpd.so`` (built by ``paper_2605_20816_amd.build``).  Torch tensors
provide device memory and the current stream.  If the library is missing this
module raises on import of any entry point; there is no fallback path.

Paper: Bourne, Buze, Gallouet, Merigot, "Polynomial diagrams for microstructure
modelling" (arXiv 2605.20816).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpd.so")

PD_OK = 0
STATUS = {0: "PD_OK", 1: "PD_ERR_INVALID_ARG", 2: "PD_ERR_UNSUPPORTED", 3: "PD_ERR_OOM",
          4: "PD_ERR_HIP", 5: "PD_ERR_NONFINITE", 6: "PD_ERR_NOT_CONVERGED"}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
GAUGE = {"last": 0, "centered": 1, "none": 2}
INIT = {"given": 0, "zero": 1, "mlp": 2, "heuristic": 3}
FIT_STATUS = {0: "target", 1: "budget", 2: "gtol", 3: "linesearch", 4: "nonfinite"}
MAX_DEGREE = 8
DESC_DIM = 32
FRAME_DIM = 8
MLP_WIDTH = 256
# pd_objective_grad_noalloc: fixed scratch per device and maps per call
NOALLOC_SCRATCH_BYTES = 64 << 20
NOALLOC_MAX_MAPS = 4


class PdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("labels", ctypes.c_void_p), ("n_grains", ctypes.c_int32),
                ("degree", ctypes.c_int32), ("eps", ctypes.c_double)]


class _Points(ctypes.Structure):
    _fields_ = [("coords", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("n_points", ctypes.c_int64), ("dim", ctypes.c_int32),
                ("n_grains", ctypes.c_int32), ("degree", ctypes.c_int32), ("eps", ctypes.c_double)]


class _FitOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("gauge", ctypes.c_int), ("init", ctypes.c_int),
                ("history", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("target_acc", ctypes.c_double), ("gtol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("precondition", ctypes.c_int32), ("anneal_levels", ctypes.c_int32),
                ("anneal_factor", ctypes.c_double), ("anneal_iters", ctypes.c_int32),
                ("trace", ctypes.c_void_p), ("trace_cap", ctypes.c_int32),
                ("state", ctypes.c_void_p), ("resume", ctypes.c_int32)]


class _Mlp(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p * 9)]


class _FitReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("evals", ctypes.c_int32),
                ("phi", ctypes.c_double), ("acc", ctypes.c_double),
                ("seconds_total", ctypes.c_double), ("seconds_to_target", ctypes.c_double),
                ("seconds_iterating", ctypes.c_double), ("evals_iterating", ctypes.c_int32)]


class _NewtonOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("max_iter", ctypes.c_int32), ("cg_max", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32), ("target_acc", ctypes.c_double),
                ("gtol", ctypes.c_double)]


class _NewtonReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("evals", ctypes.c_int32),
                ("hvps", ctypes.c_int32), ("phi", ctypes.c_double), ("acc", ctypes.c_double),
                ("seconds_total", ctypes.c_double), ("seconds_to_target", ctypes.c_double)]


_lib = None

# Every symbol the C ABI declares, with its ctypes signature.
_SIGS = {
    "pd_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "pd_destroy": (None, [ctypes.c_void_p]),
    "pd_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "pd_num_features": (ctypes.c_int32, [ctypes.c_int32]),
    "pd_fit_state_size": (ctypes.c_int64, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "pd_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_validate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                   ctypes.c_void_p]),
    "pd_objective_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                         ctypes.c_void_p]),
    "pd_objective_grad_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem),
                                                 ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                                 ctypes.c_int, ctypes.c_void_p]),
    "pd_objective_grad_rows": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem),
                                              ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                              ctypes.c_int32, ctypes.c_void_p]),
    "pd_recover_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "pd_assign": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                 ctypes.c_void_p, ctypes.c_void_p]),
    "pd_fit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(_FitOpts),
                              ctypes.POINTER(_FitReport), ctypes.c_void_p]),
    "pd_profile_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "pd_probe_peak": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "pd_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "pd_hessian_diag": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                       ctypes.c_void_p]),
    "pd_hessian_vec": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                      ctypes.c_void_p]),
    "pd_fit_newton_cg": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(_NewtonOpts),
                                        ctypes.POINTER(_NewtonReport), ctypes.c_void_p]),
    "pd_points_num_features": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32]),
    "pd_points_objective_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Points), ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                                ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                                ctypes.c_void_p]),
    "pd_points_assign": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Points), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "pd_probe_math": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "pd_mlp_num_params": (ctypes.c_int64, [ctypes.c_int32]),
    "pd_descriptors": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "pd_heuristic": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "pd_warm_targets": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "pd_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "pd_mlp_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_mlp_adam": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_void_p]),
    "pd_warm_start": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                     ctypes.POINTER(_Mlp), ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_void_p]),
}

STAGES = ("tables", "center", "prep", "lse", "grad", "reduce")
# columns of a fit trace row (pd_fit_opts.trace)
TRACE_COLUMNS = ("iter", "evals", "phi", "grad_inf", "step", "acc")
TRACE_FIELDS = len(TRACE_COLUMNS)


def lib():
    """Load libpd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_20816_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def num_features(d: int) -> int:
    """Section 3.1: K_d = (d+1)(d+2)/2."""
    return int(lib().pd_num_features(int(d)))


def fit_state_size(n_grains: int, degree: int, history: int) -> int:
    """Doubles of one map's L-BFGS state buffer (pd_fit_state_size); 0 if invalid."""
    return int(lib().pd_fit_state_size(int(n_grains), int(degree), int(history)))


def mlp_num_params(k_out: int) -> int:
    """Parameter count of the warm-start network 32 -> 256 -> 256 -> k_out."""
    return int(lib().pd_mlp_num_params(int(k_out)))


class Mlp:
    """Warm-start networks by degree: params[d] is a float32 CUDA tensor of
    mlp_num_params(K_d) entries (or absent)."""

    def __init__(self, params=None):
        self.params = dict(params or {})

    def handle(self):
        m = _Mlp()
        for d, t in self.params.items():
            if t is None:
                continue
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise ValueError("network parameters must be a contiguous float32 CUDA tensor")
            if t.numel() != mlp_num_params(num_features(d)):
                raise ValueError(f"degree {d}: expected {mlp_num_params(num_features(d))} parameters")
            m.params[d] = t.data_ptr()
        self._keep = m
        return ctypes.pointer(m)


@dataclass
class Problem:
    """One grain map on the device: labels int32 (H*W,) values in [0, N)."""
    labels: torch.Tensor
    H: int
    W: int
    N: int
    d: int
    eps: float

    def c(self) -> _Problem:
        lab = self.labels
        if not (lab.is_cuda and lab.dtype == torch.int32 and lab.is_contiguous()):
            raise ValueError("labels must be a contiguous int32 CUDA tensor")
        if lab.numel() != self.H * self.W:
            raise ValueError("labels must have H*W entries")
        return _Problem(self.H, self.W, lab.data_ptr(), self.N, self.d, float(self.eps))


@dataclass
class Points:
    """An unstructured point set on the device: coords float64 (n, dim) in
    [-1, 1]^dim (dim 2 or 3), labels int32 (n,) values in [0, N)."""
    coords: torch.Tensor
    labels: torch.Tensor
    N: int
    d: int
    eps: float

    @property
    def dim(self) -> int:
        return int(self.coords.shape[1])

    @property
    def n(self) -> int:
        return int(self.coords.shape[0])

    def c(self) -> _Points:
        X, lab = self.coords, self.labels
        if not (X.is_cuda and X.dtype == torch.float64 and X.is_contiguous() and X.dim() == 2):
            raise ValueError("coords must be a contiguous float64 CUDA tensor (n, dim)")
        if not (lab.is_cuda and lab.dtype == torch.int32 and lab.is_contiguous()):
            raise ValueError("labels must be a contiguous int32 CUDA tensor")
        if lab.numel() != X.shape[0]:
            raise ValueError("one label per point")
        return _Points(X.data_ptr(), lab.data_ptr(), X.shape[0], X.shape[1], self.N, self.d,
                       float(self.eps))


def points_num_features(dim: int, degree: int) -> int:
    return int(lib().pd_points_num_features(dim, degree))


def _check_thetas(probs, thetas):
    if len(probs) != len(thetas):
        raise ValueError("one theta per map")
    for p, t in zip(probs, thetas):
        K = num_features(p.d)   # 0 for an invalid degree: the library reports it
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("theta must be a contiguous float64 CUDA tensor")
        if K and tuple(t.shape) != (p.N, K):
            raise ValueError(f"theta must have shape (N, K) = ({p.N}, {K})")


def _ptrs(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for k, t in enumerate(ts):
        arr[k] = None if t is None else t.data_ptr()
    return arr


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """A libpd context on one device (owns the library's workspace)."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        st = lib().pd_create(int(device), ctypes.byref(self._h))
        if st != PD_OK:
            raise PdError(st, "pd_create failed")
        self.device = device

    def close(self):
        if self._h:
            lib().pd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != PD_OK:
            raise PdError(st, lib().pd_last_error(self._h).decode())

    def features(self, H, W, d, prec="fp64", stream=None):
        """Design matrix eta_L(Omega) (K x n); 'bf16' returns (2, K, n) raw bf16 bits."""
        K = num_features(d)
        n = H * W
        dev = torch.device("cuda", self.device)
        if prec == "fp64":
            out = torch.empty((K, n), dtype=torch.float64, device=dev)
        elif prec == "fp32":
            out = torch.empty((K, n), dtype=torch.float32, device=dev)
        else:
            out = torch.empty((2, K, n), dtype=torch.int16, device=dev)
        self._check(lib().pd_features(self._h, H, W, d, PREC[prec], ctypes.c_void_p(out.data_ptr()),
                                      _stream(stream)))
        return out

    def validate(self, probs, stream=None):
        arr = (_Problem * len(probs))(*[p.c() for p in probs])
        self._check(lib().pd_validate(self._h, arr, len(probs), _stream(stream)))

    def objective_grad(self, probs, thetas, prec="fp64", grad=True, phi_out=None,
                       grad_out=None, stream=None):
        """Phi and grad Phi for each map.  Returns (phi (n,) float64, [grad N x K])."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        dev = thetas[0].device
        _check_thetas(probs, thetas)
        phi = phi_out if phi_out is not None else torch.empty(n, dtype=torch.float64, device=dev)
        if grad:
            grads = grad_out if grad_out is not None else [torch.empty_like(t) for t in thetas]
            gp = _ptrs(grads)
        else:
            grads, gp = None, None
        self._check(lib().pd_objective_grad(self._h, arr, n, _ptrs(thetas),
                                            ctypes.c_void_p(phi.data_ptr()), gp, PREC[prec],
                                            _stream(stream)))
        return phi, grads

    def objective_grad_noalloc(self, probs, thetas, phi_out, grad_out, prec="fp64",
                               stream=None):
        """pd_objective_grad_noalloc: the caller passes every output (phi_out (n,)
        float64, grad_out a list of N x K float64 tensors or None); the library
        allocates nothing."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        _check_thetas(probs, thetas)
        gp = _ptrs(grad_out) if grad_out is not None else None
        self._check(lib().pd_objective_grad_noalloc(
            self._h, arr, n, _ptrs(thetas), ctypes.c_void_p(phi_out.data_ptr()), gp, PREC[prec],
            _stream(stream)))
        return phi_out, grad_out

    def objective_grad_rows(self, probs, thetas, rows, prec="fp64", onehot_precomputed=False,
                            grad=True, stream=None):
        """Phi and grad Phi summed over the row band [r0, r1) of each map (rows: one
        (r0, r1) pair per map), both scaled by 1/n of the whole map.  With
        onehot_precomputed, the evaluation takes the form pd_fit uses."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        dev = thetas[0].device
        _check_thetas(probs, thetas)
        if len(rows) != n:
            raise ValueError("one (r0, r1) pair per map")
        rr = (ctypes.c_int32 * (2 * n))(*[int(v) for pair in rows for v in pair])
        phi = torch.empty(n, dtype=torch.float64, device=dev)
        grads = [torch.empty_like(t) for t in thetas] if grad else None
        self._check(lib().pd_objective_grad_rows(
            self._h, arr, n, rr, _ptrs(thetas), ctypes.c_void_p(phi.data_ptr()),
            _ptrs(grads) if grad else None, PREC[prec],
            1 if onehot_precomputed else 0, _stream(stream)))
        return phi, grads

    def hessian_diag(self, probs, thetas, prec="fp64", stream=None):
        """Diagonal of the Hessian of -Phi (N x K float64 per map)."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        _check_thetas(probs, thetas)
        out = [torch.empty_like(t) for t in thetas]
        self._check(lib().pd_hessian_diag(self._h, arr, n, _ptrs(thetas), _ptrs(out), PREC[prec],
                                          _stream(stream)))
        return out

    def hessian_vec(self, probs, thetas, vs, prec="fp64", stream=None):
        """H v for the Hessian H of -Phi at each theta (N x K float64 per map)."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        _check_thetas(probs, thetas)
        _check_thetas(probs, vs)
        out = [torch.empty_like(t) for t in thetas]
        self._check(lib().pd_hessian_vec(self._h, arr, n, _ptrs(thetas), _ptrs(vs), _ptrs(out),
                                         PREC[prec], _stream(stream)))
        return out

    def fit_newton_cg(self, probs, thetas, prec="fp64", max_iter=100, cg_max=20, max_halvings=30,
                      target_acc=0.99, gtol=0.0, stream=None):
        """Newton-CG ascent of Phi for every map; thetas are updated in place (and
        moved into the gauge theta_N = 0).  Returns a list of report dicts."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        _check_thetas(probs, thetas)
        opts = _NewtonOpts(PREC[prec], max_iter, cg_max, max_halvings, target_acc, gtol)
        reps = (_NewtonReport * n)()
        self._check(lib().pd_fit_newton_cg(self._h, arr, n, _ptrs(thetas), ctypes.byref(opts), reps,
                                           _stream(stream)))
        return [dict(status=FIT_STATUS.get(r.status, r.status), iters=r.iters, evals=r.evals,
                     hvps=r.hvps, phi=r.phi, acc=r.acc, seconds_total=r.seconds_total,
                     seconds_to_target=r.seconds_to_target) for r in reps]

    def recover_params(self, theta, degree, margin=1e-3, stream=None):
        """Physical parameters of a degree-1/2 fit: (params N x 6 float64 with
        columns y1, y2, w, A11, A12, A22; the shift lambda as a 1-element tensor)."""
        if not (theta.dtype == torch.float64 and theta.is_cuda and theta.is_contiguous()):
            raise ValueError("theta must be a contiguous float64 CUDA tensor")
        N = theta.shape[0]
        out = torch.empty((N, 6), dtype=torch.float64, device=theta.device)
        lam = torch.empty(1, dtype=torch.float64, device=theta.device)
        self._check(lib().pd_recover_params(self._h, N, degree, ctypes.c_void_p(theta.data_ptr()),
                                            float(margin), ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(lam.data_ptr()), _stream(stream)))
        return out, lam

    def assign(self, probs, thetas, labels_out=True, stream=None):
        """F_theta per map and #correct.  Returns ([labels int32 (n,)] or None, counts int64)."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        dev = thetas[0].device
        _check_thetas(probs, thetas)
        cnt = torch.empty(n, dtype=torch.int64, device=dev)
        outs = None
        lp = None
        if labels_out:
            outs = [torch.empty(p.H * p.W, dtype=torch.int32, device=dev) for p in probs]
            lp = _ptrs(outs)
        self._check(lib().pd_assign(self._h, arr, n, _ptrs(thetas), lp,
                                    ctypes.c_void_p(cnt.data_ptr()), _stream(stream)))
        return outs, cnt

    def probe_math(self, fn, x, stream=None):
        """The kernels' exp2/log2 on a float64 CUDA tensor x: fn 'exp2_f64' (x <= 0),
        'exp2_f32', 'log2_f64' or 'log2_f32'.  Returns a float64 tensor."""
        code = {"exp2_f64": 0, "exp2_f32": 1, "log2_f64": 2, "log2_f32": 3}[fn]
        if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
            raise ValueError("x must be a contiguous float64 CUDA tensor")
        out = torch.empty_like(x)
        self._check(lib().pd_probe_math(self._h, code, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), x.numel(), _stream(stream)))
        return out

    # ------------------------------------------------------------ point sets
    def points_objective_grad(self, sets, thetas, prec="fp64", grad=True, stream=None):
        """Phi and grad Phi of each point set.  Returns (phi float64 (n,), [grads] or None)."""
        n = len(sets)
        arr = (_Points * n)(*[q.c() for q in sets])
        if len(thetas) != n:
            raise ValueError("one theta per point set")
        for q, t in zip(sets, thetas):
            K = points_num_features(q.dim, q.d)
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("theta must be a contiguous float64 CUDA tensor")
            if K and tuple(t.shape) != (q.N, K):
                raise ValueError(f"theta must have shape (N, K) = ({q.N}, {K})")
        dev = thetas[0].device
        phi = torch.empty(n, dtype=torch.float64, device=dev)
        grads = [torch.empty_like(t) for t in thetas] if grad else None
        self._check(lib().pd_points_objective_grad(self._h, arr, n, _ptrs(thetas),
                                                   ctypes.c_void_p(phi.data_ptr()),
                                                   _ptrs(grads) if grad else None, PREC[prec],
                                                   _stream(stream)))
        return phi, grads

    def points_assign(self, sets, thetas, stream=None):
        """F_theta of each point set and #correct: ([labels int32 (n,)], counts int64)."""
        n = len(sets)
        arr = (_Points * n)(*[q.c() for q in sets])
        dev = thetas[0].device
        cnt = torch.empty(n, dtype=torch.int64, device=dev)
        outs = [torch.empty(q.n, dtype=torch.int32, device=dev) for q in sets]
        self._check(lib().pd_points_assign(self._h, arr, n, _ptrs(thetas), _ptrs(outs),
                                           ctypes.c_void_p(cnt.data_ptr()), _stream(stream)))
        return outs, cnt

    def profile_eval(self, probs, thetas, prec="fp64", reps=10, stream=None):
        """Average milliseconds per launch of each evaluation stage (dict)."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        _check_thetas(probs, thetas)
        ms = (ctypes.c_double * len(STAGES))()
        self._check(lib().pd_profile_eval(self._h, arr, n, _ptrs(thetas), PREC[prec], int(reps),
                                          ms, _stream(stream)))
        return dict(zip(STAGES, list(ms)))

    PEAK_KINDS = ("fp32_fma", "exp2", "fp32_fma4_exp2", "fp64_fma", "mfma_bf16")

    def probe_peak(self, kind, stream=None):
        """Measured rate of one unit (pd_probe_peak): flop/s for the FMA and
        matrix-core kinds, exponentials/s for "exp2" and "fp32_fma4_exp2"."""
        rate = ctypes.c_double(0.0)
        self._check(lib().pd_probe_peak(self._h, self.PEAK_KINDS.index(kind), ctypes.byref(rate),
                                        _stream(stream)))
        return float(rate.value)

    def autotune(self, probs, thetas, prec="fp64", stream=None):
        """Time the candidate work decompositions on this batch; returns the chosen
        waves-per-map, which later plans with the same key use."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        _check_thetas(probs, thetas)
        best = ctypes.c_int32(0)
        self._check(lib().pd_autotune(self._h, arr, n, _ptrs(thetas), PREC[prec], ctypes.byref(best),
                                      _stream(stream)))
        return int(best.value)

    def fit(self, probs, thetas, prec="fp64", gauge="last", init="given", history=10,
            max_iter=2000, target_acc=0.99, gtol=0.0, check_every=1, mlp=None, precondition=0,
            anneal=None, trace=None, state=None, resume=False, stream=None):
        """Device L-BFGS fit of every map; thetas are updated in place.
        anneal: None, or (levels, factor, iters per level) for the schedule of eps.
        trace: None, or one float64 CUDA tensor (cap, TRACE_FIELDS) per map (or
        None): the ring of per-iteration metrics (TRACE_COLUMNS).
        state: None, or one float64 CUDA tensor of fit_state_size(N, d, history)
        entries per map: receives the L-BFGS state; with resume=True the fit
        continues from it (init="given", theta the iterate it was written with).
        Returns a list of report dicts."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        h = None if mlp is None else mlp.handle()
        al, af, ai = anneal if anneal is not None else (0, 0.0, 0)
        tr, cap = None, 0
        if trace is not None:
            if len(trace) != n:
                raise ValueError("one trace buffer (or None) per map")
            caps = {int(t.shape[0]) for t in trace if t is not None}
            for t in trace:
                if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                                          and t.dim() == 2 and t.shape[1] == TRACE_FIELDS):
                    raise ValueError("trace buffers must be contiguous float64 CUDA (cap, 6) tensors")
            if len(caps) != 1:
                raise ValueError("trace buffers must share one capacity")
            tr, cap = _ptrs(trace), caps.pop()
        st = None
        if state is not None:
            if len(state) != n:
                raise ValueError("one state buffer (or None) per map")
            for p, t in zip(probs, state):
                if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                                          and t.numel() == fit_state_size(p.N, p.d, history)):
                    raise ValueError("state buffers must be contiguous float64 CUDA tensors of "
                                     "fit_state_size(N, d, history) entries")
            st = _ptrs(state)
        opts = _FitOpts(PREC[prec], GAUGE[gauge], INIT[init], history, max_iter, target_acc, gtol,
                        check_every, None if h is None else ctypes.cast(h, ctypes.c_void_p),
                        int(precondition), int(al), float(af), int(ai),
                        None if tr is None else ctypes.cast(tr, ctypes.c_void_p), int(cap),
                        None if st is None else ctypes.cast(st, ctypes.c_void_p), int(bool(resume)))
        reps = (_FitReport * n)()
        self._check(lib().pd_fit(self._h, arr, n, _ptrs(thetas), ctypes.byref(opts), reps,
                                 _stream(stream)))
        return [dict(status=FIT_STATUS.get(r.status, r.status), iters=r.iters, evals=r.evals,
                     phi=r.phi, acc=r.acc, seconds_total=r.seconds_total,
                     seconds_to_target=r.seconds_to_target,
                     seconds_iterating=r.seconds_iterating,
                     evals_iterating=r.evals_iterating) for r in reps]

    # ------------------------------------------------------------ warm start
    def descriptors(self, probs, frames=False, stream=None):
        """Per-grain descriptors (N x 32 float32) and, if asked, frames (N x 8 float64)."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        dev = torch.device("cuda", self.device)
        desc = [torch.empty((p.N, DESC_DIM), dtype=torch.float32, device=dev) for p in probs]
        fr = [torch.empty((p.N, FRAME_DIM), dtype=torch.float64, device=dev) for p in probs] if frames else None
        self._check(lib().pd_descriptors(self._h, arr, n, _ptrs(desc), _ptrs(fr) if fr else None,
                                         _stream(stream)))
        return (desc, fr) if frames else desc

    def heuristic(self, probs, stream=None):
        """Moment seed theta' (N x K float64) of each map (Section 5.6.2)."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        dev = torch.device("cuda", self.device)
        out = [torch.empty((p.N, num_features(p.d)), dtype=torch.float64, device=dev) for p in probs]
        self._check(lib().pd_heuristic(self._h, arr, n, _ptrs(out), _stream(stream)))
        return out

    def warm_targets(self, probs, thetas, stream=None):
        """Local-frame training targets (N x K float32) and the scales lambda (n,)."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        _check_thetas(probs, thetas)
        dev = torch.device("cuda", self.device)
        tg = [torch.empty((p.N, num_features(p.d)), dtype=torch.float32, device=dev) for p in probs]
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        self._check(lib().pd_warm_targets(self._h, arr, n, _ptrs(thetas), _ptrs(tg),
                                          ctypes.c_void_p(lam.data_ptr()), _stream(stream)))
        return tg, lam

    def mlp_forward(self, params, x, k_out, prec="fp32", stream=None):
        """Network outputs (B x k_out float32) for descriptors x (B x 32 float32)."""
        y = torch.empty((x.shape[0], k_out), dtype=torch.float32, device=x.device)
        self._check(lib().pd_mlp_forward(self._h, int(k_out), ctypes.c_void_p(params.data_ptr()),
                                         ctypes.c_void_p(x.data_ptr()), int(x.shape[0]),
                                         PREC[prec], ctypes.c_void_p(y.data_ptr()), _stream(stream)))
        return y

    def mlp_backward(self, params, x, target, loss_out=None, grad_out=None, stream=None):
        """(loss (1,) float64, gradient like params) of mean((y - target)^2)."""
        k_out = int(target.shape[1])
        loss = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float64, device=x.device)
        grad = grad_out if grad_out is not None else torch.empty_like(params)
        self._check(lib().pd_mlp_backward(self._h, k_out, ctypes.c_void_p(params.data_ptr()),
                                          ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(target.data_ptr()), int(x.shape[0]),
                                          ctypes.c_void_p(loss.data_ptr()),
                                          ctypes.c_void_p(grad.data_ptr()), _stream(stream)))
        return loss, grad

    def mlp_adam(self, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        """One in-place Adam step on params (moments m, v updated)."""
        self._check(lib().pd_mlp_adam(self._h, int(params.numel()), ctypes.c_void_p(params.data_ptr()),
                                      ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                                      ctypes.c_void_p(v.data_ptr()), int(step), float(lr),
                                      float(beta1), float(beta2), float(eps), _stream(stream)))

    def warm_start(self, probs, mlp=None, prec="fp32", stream=None):
        """Warm-start theta (N x K float64) per map and the chosen scales s*."""
        n = len(probs)
        arr = (_Problem * n)(*[p.c() for p in probs])
        dev = torch.device("cuda", self.device)
        out = [torch.empty((p.N, num_features(p.d)), dtype=torch.float64, device=dev) for p in probs]
        sc = (ctypes.c_double * n)()
        self._check(lib().pd_warm_start(self._h, arr, n, None if mlp is None else mlp.handle(),
                                        _ptrs(out), PREC[prec], sc, _stream(stream)))
        return out, list(sc)
