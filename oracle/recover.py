"""Recovery of physical diagram parameters from fitted coefficients.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 5.6.3: a degree-1 fit is a power diagram and a degree-2 fit an
anisotropic power diagram.  The coefficients are converted to the monomial basis
and read with eq. pd-lr-to-phys / apd-lr-to-phys (Section 2.3.1):
  h(x) = x.A x + c_lin . x + c_0,   A = [[c_xx, c_xy/2], [c_xy/2, c_yy]],
  y = -(1/2) A^{-1} c_lin,   w = y.A y - c_0.
The conversion is defined only up to the gauge of Lemma 4.2; adding lambda (x1^2 +
x2^2) to every score (A_i -> A_i + lambda I) changes no cell, and choosing
lambda > -min_i lambda_min(A_i) makes every anisotropy positive definite.  Here
lambda = max(0, margin - min_i lambda_min(A_i)), so that every A_i + lambda I has
smallest eigenvalue >= margin.  At degree 1 the common |x|^2 is the dropped gauge
term itself: A_i = I, y = -c_lin / 2, w = |y|^2 - c_0, lambda = 0.
"""
from __future__ import annotations

import numpy as np


def to_monomial(theta, d):
    """Coefficients of the Legendre-basis scores in the monomials
    (1, x1, x2, x1^2, x1 x2, x2^2) (degree 2; the first three at degree 1), from
    P_2(t) = (3 t^2 - 1) / 2 (Section 3.3)."""
    th = np.asarray(theta, np.float64)
    if d == 1:
        return th.copy()
    if d != 2:
        raise ValueError("physical parameters exist for degree 1 and 2 only")
    c = np.empty_like(th)
    c[:, 0] = th[:, 0] - 0.5 * th[:, 3] - 0.5 * th[:, 5]
    c[:, 1] = th[:, 1]
    c[:, 2] = th[:, 2]
    c[:, 3] = 1.5 * th[:, 3]
    c[:, 4] = th[:, 4]
    c[:, 5] = 1.5 * th[:, 5]
    return c


def recover_params(theta, d, margin=1e-3):
    """Returns (y (N, 2), w (N,), A (N, 2, 2), lam) for a degree-1 or degree-2 fit."""
    c = to_monomial(theta, d)
    N = c.shape[0]
    if d == 1:
        y = -0.5 * c[:, 1:3]
        w = (y * y).sum(1) - c[:, 0]
        A = np.broadcast_to(np.eye(2), (N, 2, 2)).copy()
        return y, w, A, 0.0
    A = np.empty((N, 2, 2))
    A[:, 0, 0] = c[:, 3]
    A[:, 0, 1] = A[:, 1, 0] = 0.5 * c[:, 4]
    A[:, 1, 1] = c[:, 5]
    lmin = np.linalg.eigvalsh(A)[:, 0]
    lam = max(0.0, margin - float(lmin.min()))
    A = A + lam * np.eye(2)
    y = -0.5 * np.linalg.solve(A, c[:, 1:3][:, :, None])[:, :, 0]
    w = np.einsum("ni,nij,nj->n", y, A, y) - c[:, 0]
    return y, w, A, lam
