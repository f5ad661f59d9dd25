"""FP64 oracle for polynomial diagrams on unstructured point sets in 2-D and 3-D.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper defines the diagram and the objective for any finite set of points in
a domain of R^D (Section 2.1 takes Omega as a set of pixel centres and notes that
nothing restricts it to two dimensions or to a grid; Section 3.3 builds the
Legendre basis as tensor products).  For points x_1..x_n in [-1, 1]^D with labels
G, parameters theta (N x K) and eps > 0:

  psi_alpha(x) = prod_j P_{alpha_j}(x_j),  |alpha| <= d  (Section 3.3, in D dims)
  h_i(x) = theta_i . psi(x),  s_i(x) = -h_i(x) / eps
  Phi = (1/n) sum_x [ s_{G(x)}(x) - log sum_j exp s_j(x) ]        (eq. log-res)
  grad_i Phi = (1/(eps n)) sum_x (p_i(x) - [G(x) = i]) psi(x)     (eq. grad)
  F(x) = the smallest i minimising h_i(x)                         (Section 2.1)

Multi-indices in the degree-graded order: for total degree k = 0..d, in 2-D
(a, b) = (k - b, b) for b = 0..k (the grid's order); in 3-D (a, b, c) =
(k - b - c, b, c) for c = 0..k, then b = 0..k - c.
"""
from __future__ import annotations

import numpy as np


def multi_index(D: int, d: int) -> np.ndarray:
    """Exponent tuples (K x D) in the degree-graded order above."""
    if D not in (2, 3):
        raise ValueError("dimension 2 or 3")
    out = []
    for k in range(d + 1):
        if D == 2:
            for b in range(k + 1):
                out.append((k - b, b))
        else:
            for c in range(k + 1):
                for b in range(k - c + 1):
                    out.append((k - b - c, b, c))
    return np.array(out, dtype=np.int64)


def num_features(D: int, d: int) -> int:
    return len(multi_index(D, d))


def legendre_all(t: np.ndarray, d: int) -> np.ndarray:
    """P_0..P_d at every entry of t ((d+1) x len(t)) by Bonnet's recurrence
    (m + 1) P_{m+1} = (2m + 1) t P_m - m P_{m-1}."""
    t = np.asarray(t, np.float64)
    P = np.zeros((d + 1,) + t.shape)
    P[0] = 1.0
    if d >= 1:
        P[1] = t
    for m in range(1, d):
        P[m + 1] = ((2 * m + 1) * t * P[m] - m * P[m - 1]) / (m + 1)
    return P


def features(X: np.ndarray, d: int) -> np.ndarray:
    """psi(x) of every point (K x n), from the C oracle's 1-D recurrence (the grid
    oracle's, so pixel centres give the grid's design matrix bit for bit):
    psi = (P_a(x1) P_b(x2)) P_c(x3)."""
    from . import _load
    X = np.ascontiguousarray(X, np.float64)
    n, D = X.shape
    if D not in (2, 3):
        raise ValueError("dimension 2 or 3")
    out = np.zeros((num_features(D, d), n))
    _load().orc_points_features(int(n), int(D), int(d), X, out)
    return out


def features_numpy(X: np.ndarray, d: int) -> np.ndarray:
    """The same products from legendre_all (Bonnet's recurrence without a fused
    multiply-add): equal to features() to rounding."""
    X = np.asarray(X, np.float64)
    n, D = X.shape
    mi = multi_index(D, d)
    tabs = [legendre_all(X[:, j], d) for j in range(D)]
    out = np.ones((len(mi), n))
    for k, alpha in enumerate(mi):
        for j in range(D):
            out[k] *= tabs[j][alpha[j]]
    return out


def objective_grad(theta, X, labels, d: int, eps: float, grad: bool = True):
    """Phi and grad Phi (N x K) of eq. log-res / eq. grad over the point set."""
    th = np.asarray(theta, np.float64)
    Psi = features(X, d)
    n = Psi.shape[1]
    lab = np.asarray(labels, np.int64)
    s = -(th @ Psi) / eps                       # N x n
    m = s.max(axis=0)
    lse = m + np.log(np.exp(s - m).sum(axis=0))
    phi = float(np.mean(s[lab, np.arange(n)] - lse))
    if not grad:
        return phi, None
    P = np.exp(s - lse)
    P[lab, np.arange(n)] -= 1.0
    return phi, (P @ Psi.T) / (eps * n)


def assign(theta, X, d: int, labels=None):
    """F (smallest index on ties; scores theta_i0 then one FMA per feature, in
    index order) and the number of points with F = G."""
    import ctypes
    from . import _load
    X = np.ascontiguousarray(X, np.float64)
    n, D = X.shape
    th = np.ascontiguousarray(theta, np.float64)
    F = np.zeros(n, np.int32)
    nc = ctypes.c_int64(0)
    lab = np.ascontiguousarray(labels, np.int32) if labels is not None else None
    _load().orc_points_assign(int(n), int(D), int(th.shape[0]), int(d), th, X,
                              lab.ctypes.data if lab is not None else None, F,
                              ctypes.byref(nc))
    return F, int(nc.value)
