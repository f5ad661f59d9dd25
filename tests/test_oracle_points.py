"""Pins of the point-set oracle (oracle/points.py): unstructured 2-D and 3-D
point sets (Section 2.1's Omega need not be a grid nor two-dimensional; Section
3.3's tensor-product Legendre basis in D dimensions)."""
import math

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import synth


def test_feature_counts_are_the_simplex_numbers(orc):
    for d in range(0, 9):
        assert orc.points.num_features(2, d) == (d + 1) * (d + 2) // 2 == orc.num_features(d)
        assert orc.points.num_features(3, d) == (d + 1) * (d + 2) * (d + 3) // 6


def test_legendre_closed_forms_and_orthogonality(orc):
    t = np.linspace(-1, 1, 17)
    P = orc.points.legendre_all(t, 5)
    assert np.allclose(P[2], (3 * t**2 - 1) / 2, atol=1e-15)
    assert np.allclose(P[3], (5 * t**3 - 3 * t) / 2, atol=1e-15)
    assert np.allclose(P[5], (63 * t**5 - 70 * t**3 + 15 * t) / 8, atol=1e-14)
    x, w = npleg.leggauss(12)
    Q = orc.points.legendre_all(x, 6)
    G = (Q * w) @ Q.T
    assert np.allclose(G, np.diag(2.0 / (2 * np.arange(7) + 1)), atol=1e-14)
    # the C oracle's features (fused recurrence) and numpy's agree to rounding
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, size=(500, 3))
    A, B = orc.points.features(X, 6), orc.points.features_numpy(X, 6)
    assert np.max(np.abs(A - B)) <= 1e-14


def test_pixel_centres_reproduce_the_grid_oracle(orc):
    """2-D points at the pixel centres, in row-major order, are the grid of
    Section 2.1: the same features, Phi, gradient and assignment."""
    gm = synth.config_c1()
    H, W, d, eps = gm.H, gm.W, 1, 1e-2
    c = np.array([orc.coord(j, W) for j in range(W)])
    r = np.array([orc.coord(i, H) for i in range(H)])
    X = np.stack([np.tile(c, H), np.repeat(r, W)], axis=1)
    assert np.array_equal(orc.points.features(X, 3), orc.features(H, W, 3))
    rng = np.random.default_rng(3)
    th = rng.normal(size=(gm.N, 3))
    p1, g1 = orc.points.objective_grad(th, X, gm.labels, d, eps)
    p2, g2 = orc.objective_grad(th, gm.labels, H, W, d, eps)
    assert abs(p1 - p2) <= 1e-13 * abs(p2)
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g2))
    F1, n1 = orc.points.assign(th, X, d, gm.labels)
    F2, n2, _ = orc.assign(th, H, W, d, gm.labels)
    assert np.array_equal(F1, F2) and n1 == n2


def test_third_coordinate_at_one_reduces_to_two_dimensions(orc):
    """With x3 = 1 every P_c(x3) = 1: a 3-D theta that is zero off c = 0 gives the
    2-D Phi, and the gradient entry of (a, b, c) is the 2-D entry of (a, b)."""
    rng = np.random.default_rng(4)
    n, N, d, eps = 300, 5, 3, 0.05
    X2 = rng.uniform(-1, 1, size=(n, 2))
    X3 = np.concatenate([X2, np.ones((n, 1))], axis=1)
    lab = rng.integers(0, N, size=n).astype(np.int32)
    mi2 = [tuple(a) for a in orc.points.multi_index(2, d)]
    mi3 = [tuple(a) for a in orc.points.multi_index(3, d)]
    th2 = rng.normal(size=(N, len(mi2))) * 0.2
    th3 = np.zeros((N, len(mi3)))
    for k, a in enumerate(mi3):
        if a[2] == 0:
            th3[:, k] = th2[:, mi2.index(a[:2])]
    p2, g2 = orc.points.objective_grad(th2, X2, lab, d, eps)
    p3, g3 = orc.points.objective_grad(th3, X3, lab, d, eps)
    assert abs(p3 - p2) <= 1e-14 * abs(p2)
    for k, a in enumerate(mi3):
        if a[0] + a[1] + a[2] <= d:
            j = mi2.index((a[0], a[1])) if a[0] + a[1] <= d else None
            assert np.allclose(g3[:, k], g2[:, j], rtol=0, atol=1e-14 * np.max(np.abs(g2)))


def test_3d_gradient_by_finite_differences_and_gauge(orc):
    rng = np.random.default_rng(5)
    n, N, d, eps = 200, 4, 2, 0.1
    X = rng.uniform(-1, 1, size=(n, 3))
    lab = rng.integers(0, N, size=n).astype(np.int32)
    K = orc.points.num_features(3, d)
    th = rng.normal(size=(N, K)) * 0.1
    phi, g = orc.points.objective_grad(th, X, lab, d, eps)
    # sum_i grad_i = 0: a common shift of every grain changes nothing (Lemma 4.2)
    assert np.max(np.abs(g.sum(axis=0))) <= 1e-13 * np.max(np.abs(g))
    h = 1e-6
    for (i, k) in [(0, 0), (1, 3), (3, K - 1), (2, 5)]:
        e = np.zeros_like(th)
        e[i, k] = h
        fd = (orc.points.objective_grad(th + e, X, lab, d, eps, grad=False)[0]
              - orc.points.objective_grad(th - e, X, lab, d, eps, grad=False)[0]) / (2 * h)
        assert abs(fd - g[i, k]) <= 1e-6 * max(1.0, abs(g[i, k]))


def test_two_grains_are_the_binary_logistic(orc):
    """N = 2: log p_G = -log(1 + exp(s_other - s_G)), written out per point."""
    rng = np.random.default_rng(6)
    n, d, eps = 50, 2, 0.2
    X = rng.uniform(-1, 1, size=(n, 3))
    lab = rng.integers(0, 2, size=n).astype(np.int32)
    K = orc.points.num_features(3, d)
    th = rng.normal(size=(2, K))
    Psi = orc.points.features(X, d)
    s = -(th @ Psi) / eps
    ref = 0.0
    for j in range(n):
        g = lab[j]
        ref += -math.log1p(math.exp(s[1 - g, j] - s[g, j])) if s[1 - g, j] < s[g, j] else \
            (s[g, j] - s[1 - g, j]) - math.log1p(math.exp(s[g, j] - s[1 - g, j]))
    phi, _ = orc.points.objective_grad(th, X, lab, d, eps)
    assert abs(phi - ref / n) <= 1e-13 * abs(ref / n)


def test_3d_assignment_by_exact_scores(orc):
    """Brute force with exact rationals on a tiny set: integer theta and points on
    a dyadic grid make every score exact in FP64 and in Fractions."""
    from fractions import Fraction as Fr
    rng = np.random.default_rng(7)
    d, N = 2, 6
    X = rng.integers(-4, 5, size=(40, 3)) / 4.0
    th = rng.integers(-3, 4, size=(N, orc.points.num_features(3, d))).astype(np.float64)
    F, _ = orc.points.assign(th, X, d)
    mi = orc.points.multi_index(3, d)

    def P(m, t):
        t = Fr(t)
        return [Fr(1), t, (3 * t * t - 1) / 2][m]

    for j, x in enumerate(X):
        sc = [sum(Fr(th[i, k]) * P(a[0], x[0]) * P(a[1], x[1]) * P(a[2], x[2])
                  for k, a in enumerate(mi)) for i in range(N)]
        best = min(range(N), key=lambda i: (sc[i], i))
        assert F[j] == best
