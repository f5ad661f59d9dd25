"""FP64 CPU oracle for Legendre polynomial diagrams.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU library (``paper_2605_20816_amd``) and neither imports the other.

The arithmetic of the per-pixel objective, gradient and arg-min lives in the
plain C file ``pd_oracle.c`` (built into ``liborc.so`` next to it); this module
marshals numpy arrays into it and adds the few pieces that are clearer in numpy
(the dense Hessian of tiny problems, gauge projections, the L-BFGS iteration, the
warm-start network).

Paper: Bourne, Buze, Gallouet, Merigot, "Polynomial diagrams for microstructure
modelling" (arXiv 2605.20816).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile pd_oracle.c with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    L = ctypes.CDLL(_LIB)
    c_int, c_dbl, c_i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
    L.orc_num_features.argtypes = [c_int]
    L.orc_num_features.restype = c_int
    L.orc_multi_index.argtypes = [c_int, _i32p, _i32p]
    L.orc_coord.argtypes = [c_int, c_int]
    L.orc_coord.restype = c_dbl
    L.orc_legendre.argtypes = [c_dbl, c_int, _f64p]
    L.orc_features.argtypes = [c_int, c_int, c_int, _f64p]
    L.orc_points_num_features.argtypes = [c_int, c_int]
    L.orc_points_num_features.restype = c_int
    L.orc_points_features.argtypes = [c_i64, c_int, c_int, _f64p, _f64p]
    L.orc_points_assign.argtypes = [c_i64, c_int, c_int, c_int, _f64p, _f64p, ctypes.c_void_p,
                                    _i32p, ctypes.POINTER(c_i64)]
    L.orc_points_assign.restype = c_i64
    L.orc_assign.argtypes = [c_int, c_int, c_int, c_int, _f64p, ctypes.c_void_p,
                             _i32p, ctypes.POINTER(c_i64)]
    L.orc_assign.restype = c_i64
    L.orc_objective_grad.argtypes = [c_int, c_int, c_int, c_int, c_dbl, _f64p, _i32p,
                                     ctypes.c_void_p]
    L.orc_objective_grad.restype = c_dbl
    L.orc_assign_rows.argtypes = [c_int, c_int, c_int, c_int, _f64p, ctypes.c_void_p,
                                  c_int, c_int, _i32p, ctypes.POINTER(c_i64)]
    L.orc_assign_rows.restype = c_i64
    L.orc_objective_grad_rows.argtypes = [c_int, c_int, c_int, c_int, c_dbl, _f64p, _i32p,
                                          c_int, c_int, ctypes.c_void_p]
    L.orc_objective_grad_rows.restype = c_dbl
    L.orc_num_threads.restype = c_int
    _lib = L
    return L


def num_threads() -> int:
    return int(_load().orc_num_threads())


def num_features(d: int) -> int:
    """Section 3.1: K_d = (d+1)(d+2)/2."""
    return int(_load().orc_num_features(int(d)))


def multi_index(d: int):
    """Section 3.1: exponent pairs (a, b) in the fixed graded order."""
    K = num_features(d)
    a = np.zeros(K, np.int32)
    b = np.zeros(K, np.int32)
    _load().orc_multi_index(int(d), a, b)
    return a, b


def coord(idx: int, length: int) -> float:
    """Section 2.1: pixel-centre coordinate of index idx on an axis of given length."""
    return float(_load().orc_coord(int(idx), int(length)))


def legendre(t: float, d: int) -> np.ndarray:
    """Section 3.3: P_0..P_d at t by the three-term recurrence."""
    P = np.zeros(max(d + 1, 2), np.float64)
    _load().orc_legendre(float(t), int(d), P)
    return P[: d + 1]


def features(H: int, W: int, d: int) -> np.ndarray:
    """Section 3.3: design matrix eta_L(Omega), shape (K, H*W), row-major pixels."""
    K = num_features(d)
    out = np.zeros((K, H * W), np.float64)
    _load().orc_features(int(H), int(W), int(d), out)
    return out


def _theta(theta, d):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.ndim != 2 or th.shape[1] != num_features(d):
        raise ValueError(f"theta must be N x K_d, got {th.shape}")
    return th


def assign(theta, H: int, W: int, d: int, labels=None):
    """Section 2.1: F_theta with smallest-index ties; -1 where a score is NaN.

    Returns (F as int32[H*W], n_correct against labels (0 if None), n_nan).
    """
    th = _theta(theta, d)
    N = th.shape[0]
    out = np.zeros(H * W, np.int32)
    nc = ctypes.c_int64(0)
    lab = None
    if labels is not None:
        lab = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    nn = _load().orc_assign(int(H), int(W), int(N), int(d), th.reshape(-1),
                            lab.ctypes.data if lab is not None else None, out,
                            ctypes.byref(nc))
    return out, int(nc.value), int(nn)


def assign_rows(theta, H: int, W: int, d: int, r0: int, r1: int, labels=None):
    """Section 2.1 over the pixel rows [r0, r1) only: returns (F of those rows as
    int32[(r1 - r0) * W], n_correct over them, n_nan)."""
    th = _theta(theta, d)
    N = th.shape[0]
    out = np.full(H * W, -2, np.int32)
    nc = ctypes.c_int64(0)
    lab = None
    if labels is not None:
        lab = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    nn = _load().orc_assign_rows(int(H), int(W), int(N), int(d), th.reshape(-1),
                                 lab.ctypes.data if lab is not None else None, int(r0), int(r1),
                                 out, ctypes.byref(nc))
    return out[r0 * W:r1 * W].copy(), int(nc.value), int(nn)


def objective_grad(theta, labels, H: int, W: int, d: int, eps: float, grad: bool = True):
    """eq:Phi and eq:grad: returns (Phi, grad N x K or None); L = n * Phi."""
    th = _theta(theta, d)
    N = th.shape[0]
    lab = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    if lab.size != H * W:
        raise ValueError("labels must have H*W entries")
    if lab.min() < 0 or lab.max() >= N:
        raise ValueError("labels must lie in [0, N)")
    g = np.zeros_like(th) if grad else None
    phi = _load().orc_objective_grad(int(H), int(W), int(N), int(d), float(eps),
                                     th.reshape(-1), lab,
                                     g.ctypes.data if g is not None else None)
    return float(phi), g


def objective_rows(theta, labels, H, W, d, eps, r0, r1, grad=True):
    """eq:Phi and eq:grad summed over the pixel rows [r0, r1) only, unscaled:
    (sum of log p_G(x), sum of (delta_G - p) psi as N x K).  Over a partition of
    the rows these sum to n Phi and -(eps n) grad Phi."""
    th = _theta(theta, d)
    lab = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    g = np.zeros_like(th) if grad else None
    v = _load().orc_objective_grad_rows(int(H), int(W), int(th.shape[0]), int(d), float(eps),
                                        th.reshape(-1), lab, int(r0), int(r1),
                                        g.ctypes.data if g is not None else None)
    return float(v), g


def softmax_probs(theta, H, W, d, eps):
    """p^eps_i(x) of eq p-e for every pixel (dense N x n; tiny problems only)."""
    th = _theta(theta, d)
    X = features(H, W, d)
    s = -(th @ X) / eps
    s = s - s.max(axis=0, keepdims=True)
    e = np.exp(s)
    return e / e.sum(axis=0, keepdims=True)


def hessian(theta, labels, H, W, d, eps):
    """eq:hess of Proposition 4.4 as a dense (N K) x (N K) matrix (tiny problems)."""
    th = _theta(theta, d)
    N, K = th.shape
    X = features(H, W, d)
    P = softmax_probs(th, H, W, d, eps)
    n = H * W
    Hm = np.zeros((N, K, N, K))
    for i in range(N):
        for k in range(N):
            w = P[i] * ((1.0 if i == k else 0.0) - P[k])
            Hm[i, :, k, :] = (X * w) @ X.T
    return -Hm.reshape(N * K, N * K) / (eps * eps * n)


def hessian_diag(theta, labels, H, W, d, eps):
    """Diagonal of the Hessian of -Phi (eq. hess): D_ik = (1/(eps^2 n))
    sum_x p_i(x) (1 - p_i(x)) psi_k(x)^2, N x K (dense probabilities: small maps)."""
    th = _theta(theta, d)
    X = features(H, W, d)
    P = softmax_probs(th, H, W, d, eps)
    return ((P * (1.0 - P)) @ (X * X).T) / (eps * eps * H * W)


def gauge_project(v, mode: str):
    """Remark 4.3: 'last' zeroes the reference grain N-1; 'centered' removes the
    common-shift component; 'none' leaves v unchanged."""
    v = np.array(v, dtype=np.float64, copy=True)
    if mode == "last":
        v[-1, :] = 0.0
    elif mode == "centered":
        v -= v.mean(axis=0, keepdims=True)
    elif mode != "none":
        raise ValueError(mode)
    return v


from .lbfgs import annealed_fit, lbfgs_fit, newton_cg_fit, newton_fit  # noqa: E402,F401
from .recover import recover_params, to_monomial  # noqa: E402,F401
from . import points  # noqa: E402,F401
