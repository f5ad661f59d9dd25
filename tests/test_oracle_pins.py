"""Pins of the FP64 oracle to what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself: a table
the paper prints, closed forms, exact rational / 40-digit arithmetic, the
invariances and bounds of Section 4, independent library routines, or
finite differences of its own objective.
"""
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- features ---

def test_table1_compression_ratio(orc):
    """Section 5.6.1, Table 1: K_d N / (3|Omega|) for both EBSD maps, d = 1..8."""
    rows = [l.split() for l in open(os.path.join(GOLD, "table1_compression.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for name, N, n, *pcts in rows:
        for d, pct in enumerate(pcts, start=1):
            val = 100.0 * orc.num_features(d) * int(N) / (3 * int(n))
            assert f"{val:.2f}" == pct, (name, d, val, pct)


def test_multi_index_order(orc):
    """Section 3.1: A_d = {|alpha| <= d}, K_d = (d+1)(d+2)/2, graded order;
    d = 1 lists (1, x, y) and d = 2 adds P2(x), xy, P2(y)."""
    a, b = orc.multi_index(1)
    assert list(zip(a, b)) == [(0, 0), (1, 0), (0, 1)]
    a, b = orc.multi_index(2)
    assert list(zip(a, b)) == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    for d in range(1, 9):
        a, b = orc.multi_index(d)
        pairs = set(zip(a.tolist(), b.tolist()))
        assert len(pairs) == orc.num_features(d) == (d + 1) * (d + 2) // 2
        assert pairs == {(i, j) for i in range(d + 1) for j in range(d + 1) if i + j <= d}
        k = a + b
        assert np.all(np.diff(k) >= 0)


def test_grid_matches_section_2_1(orc):
    """Pixel centres (-1,-1) + (k - 1/2)/M, k in [2M], exactly (correct rounding)."""
    for M in (1, 2, 3, 32, 50, 128):
        for k in range(1, 2 * M + 1):
            exact = Fraction(-1) + Fraction(2 * k - 1, 2 * M)
            assert orc.coord(k - 1, 2 * M) == float(exact)
    for L in (5, 7, 129, 768):
        xs = [orc.coord(i, L) for i in range(L)]
        assert all(xs[i] == -xs[L - 1 - i] for i in range(L))  # exact antisymmetry
        assert abs(xs[1] - xs[0] - 2.0 / L) < 1e-15


_CLOSED = {
    2: lambda t: (3 * t**2 - 1) / 2,
    3: lambda t: (5 * t**3 - 3 * t) / 2,
    4: lambda t: (35 * t**4 - 30 * t**2 + 3) / 8,
    5: lambda t: (63 * t**5 - 70 * t**3 + 15 * t) / 8,
    6: lambda t: (231 * t**6 - 315 * t**4 + 105 * t**2 - 5) / 16,
    7: lambda t: (429 * t**7 - 693 * t**5 + 315 * t**3 - 35 * t) / 16,
    8: lambda t: (6435 * t**8 - 12012 * t**6 + 6930 * t**4 - 1260 * t**2 + 35) / 128,
}


def test_legendre_closed_forms_parity_endpoints(orc):
    """Section 3.3: textbook closed forms of P_2..P_8 (exact rationals), parity
    P_m(-t) = (-1)^m P_m(t) and P_m(1) = 1."""
    rng = np.random.default_rng(0)
    ts = np.concatenate([rng.uniform(-1, 1, 200), [-1.0, 0.0, 1.0, 0.5]])
    for t in ts:
        P = orc.legendre(float(t), 8)
        Pm = orc.legendre(float(-t), 8)
        for m, f in _CLOSED.items():
            exact = float(f(Fraction(float(t))))
            assert abs(P[m] - exact) <= m * 2.3e-16, (t, m)  # a few ulp of |P_m| <= 1
            assert Pm[m] == (-1) ** m * P[m]
    assert np.all(orc.legendre(1.0, 8) == 1.0)


def test_legendre_orthogonality_gauss(orc):
    """Section 3.3: int P_m P_n = 2 delta_mn / (2n+1), by 20-point Gauss-Legendre
    quadrature (numpy's nodes, exact for degree <= 39)."""
    x, w = np.polynomial.legendre.leggauss(20)
    V = np.array([orc.legendre(float(t), 8) for t in x])
    G = (V * w[:, None]).T @ V
    ref = np.diag([2.0 / (2 * n + 1) for n in range(9)])
    assert np.max(np.abs(G - ref)) < 1e-14


def test_design_matrix_products_and_rank(orc):
    """psi_alpha = P_a(x1) P_b(x2); psi_0 = 1; the design matrix spans R^K
    (assumption of Proposition 4.5) on a 12 x 10 grid for d <= 4."""
    H, W = 10, 12
    for d in (1, 2, 4):
        X = orc.features(H, W, d)
        a, b = orc.multi_index(d)
        assert X.shape == (orc.num_features(d), H * W)
        assert np.all(X[0] == 1.0)
        r, c = 7, 3
        Px = orc.legendre(orc.coord(c, W), d)
        Py = orc.legendre(orc.coord(r, H), d)
        for k in range(X.shape[0]):
            assert X[k, r * W + c] == Px[a[k]] * Py[b[k]]
        assert np.linalg.matrix_rank(X) == X.shape[0]


# ---------------------------------------------------------------- assignment --

def _exact_scores(theta, H, W, d, orc):
    """Exact rational scores theta_i . psi(x) with exact Legendre values."""
    a, b = orc.multi_index(d)

    def leg(t, dd):
        P = [Fraction(1), t]
        for m in range(1, dd):
            P.append(((2 * m + 1) * t * P[m] - m * P[m - 1]) / (m + 1))
        return P[: dd + 1]

    out = []
    th = [[Fraction(float(v)) for v in row] for row in theta]
    for r in range(H):
        Py = leg(Fraction(2 * r + 1 - H, H), d)
        for c in range(W):
            Px = leg(Fraction(2 * c + 1 - W, W), d)
            psi = [Px[a[k]] * Py[b[k]] for k in range(len(a))]
            out.append([sum(t * p for t, p in zip(row, psi)) for row in th])
    return out


def test_assign_brute_force_exact(orc):
    """Section 2.1 arg-min with smallest-index ties against exact rational scores
    wherever the exact best-vs-second gap exceeds FP64 rounding."""
    rng = np.random.default_rng(1)
    H, W, N, d = 6, 7, 5, 3
    a, b = orc.multi_index(d)
    theta = synth.random_theta(N, d, rng, multi_index=(a, b))
    F, _, nn = orc.assign(theta, H, W, d)
    assert nn == 0
    ex = _exact_scores(theta, H, W, d, orc)
    checked = 0
    for j, sc in enumerate(ex):
        order = sorted(range(N), key=lambda i: (sc[i], i))
        gap = float(sc[order[1]] - sc[order[0]])
        if gap > 1e-12:
            assert F[j] == order[0]
            checked += 1
    assert checked > 0.9 * H * W


def test_assign_ties_and_scaling(orc):
    """Fully ambiguous theta = 0 assigns every pixel to grain 0 (tie-break,
    Section 2.1); F_{2^k theta} = F_theta bit for bit (Lemma 4.1: positive scaling
    leaves F unchanged, and power-of-two scaling is exact); exact duplicate grains
    resolve to the smaller index."""
    H, W, d = 16, 20, 2
    F, _, _ = orc.assign(np.zeros((4, 6)), H, W, d)
    assert np.all(F == 0)
    rng = np.random.default_rng(2)
    a, b = orc.multi_index(d)
    th = synth.random_theta(7, d, rng, multi_index=(a, b))
    F0, _, _ = orc.assign(th, H, W, d)
    for k in (-7, -1, 3, 30):
        assert np.array_equal(orc.assign(th * 2.0**k, H, W, d)[0], F0)
    th2 = np.vstack([th, th[2:3]])      # grain 7 duplicates grain 2
    F2, _, _ = orc.assign(th2, H, W, d)
    assert np.array_equal(F2, F0) and not np.any(F2 == 7)


def test_assign_nan_flag(orc):
    th = np.zeros((3, 3))
    th[1, 0] = np.nan
    F, _, nn = orc.assign(th, 4, 4, 1)
    assert nn == 16 and np.all(F == -1)


def test_assign_two_site_bisector(orc):
    """Two-site power diagram with w = 0: x goes to site 0 iff it is closer,
    i.e. the sign of (y1 - y0).(x - (y0 + y1)/2) (Section 2.3.1, Voronoi case)."""
    y0, y1 = np.array([-0.31, 0.2]), np.array([0.45, -0.17])
    th = np.array([[y0 @ y0, -2 * y0[0], -2 * y0[1]],
                   [y1 @ y1, -2 * y1[0], -2 * y1[1]]])   # Legendre order (1, x, y)
    H, W = 24, 30
    F, _, _ = orc.assign(th, H, W, 1)
    xs = (2.0 * np.arange(W) + 1 - W) / W
    ys = (2.0 * np.arange(H) + 1 - H) / H
    X1, X2 = np.meshgrid(xs, ys)
    side = (y1[0] - y0[0]) * (X1 - (y0[0] + y1[0]) / 2) + (y1[1] - y0[1]) * (X2 - (y0[1] + y1[1]) / 2)
    ok = np.abs(side.reshape(-1)) > 1e-12
    assert np.array_equal(F[ok], (side.reshape(-1)[ok] > 0).astype(np.int32))


def test_power_and_anisotropic_maps_reconstruct(orc):
    """Section 2.3.1: a PD is the d = 1 diagram with theta = (|y|^2 - w, -2y_1, -2y_2)
    in the order (1, x, y); an APD is the d = 2 diagram with, after x^2 = (2 P_2 + 1)/3,
    theta = (y.Ay - w + (A11 + A22)/3, -2(Ay)_1, -2(Ay)_2, 2A11/3, 2A12, 2A22/3).
    Both reproduce the generator's physical labelling."""
    rng = np.random.default_rng(7)
    gm = synth.power_diagram(48, 40, 12, rng, wmax=0.05)
    y, w = gm.sites, gm.weights
    th = np.stack([(y ** 2).sum(1) - w, -2 * y[:, 0], -2 * y[:, 1]], 1)
    F, nc, _ = orc.assign(th, gm.H, gm.W, 1, gm.labels)
    assert nc >= gm.H * gm.W - 2
    gm = synth.anisotropic_power_diagram(50, 64, 15, rng)
    y, w, A = gm.sites, gm.weights, gm.aniso
    Ay = np.einsum("nij,nj->ni", A, y)
    th = np.stack([(y * Ay).sum(1) - w + (A[:, 0, 0] + A[:, 1, 1]) / 3, -2 * Ay[:, 0], -2 * Ay[:, 1],
                   2 * A[:, 0, 0] / 3, 2 * A[:, 0, 1], 2 * A[:, 1, 1] / 3], 1)
    F, nc, _ = orc.assign(th, gm.H, gm.W, 2, gm.labels)
    assert nc >= gm.H * gm.W - 2


# ---------------------------------------------------------------- objective ---

def _mp_phi_grad(theta, labels, H, W, d, eps, orc, dps=40, rows=None):
    """40-digit Phi and gradient from exact rational scores (eq:Phi, eq:grad).
    With rows = (r0, r1): the unscaled sums over those pixel rows only,
    (sum of log p_G, sum of (delta - p) psi)."""
    mpmath.mp.dps = dps
    N, K = theta.shape
    a, b = orc.multi_index(d)
    sc = _exact_scores(theta, H, W, d, orc)
    e = mpmath.mpf(Fraction(eps).numerator) / Fraction(eps).denominator
    n = H * W
    total = mpmath.mpf(0)
    grad = [[mpmath.mpf(0)] * K for _ in range(N)]

    def leg(t, dd):
        P = [Fraction(1), t]
        for m in range(1, dd):
            P.append(((2 * m + 1) * t * P[m] - m * P[m - 1]) / (m + 1))
        return P[: dd + 1]

    for j, f in enumerate(sc):
        r, c = divmod(j, W)
        if rows is not None and not rows[0] <= r < rows[1]:
            continue
        Px, Py = leg(Fraction(2 * c + 1 - W, W), d), leg(Fraction(2 * r + 1 - H, H), d)
        psi = [Px[a[k]] * Py[b[k]] for k in range(K)]
        s = [-(mpmath.mpf(fi.numerator) / fi.denominator) / e for fi in f]
        mx = max(s)
        S = mpmath.fsum(mpmath.exp(si - mx) for si in s)
        lse = mx + mpmath.log(S)
        g = int(labels[j])
        total += s[g] - lse
        for i in range(N):
            wgt = (1 if i == g else 0) - mpmath.exp(s[i] - lse)
            for k in range(K):
                grad[i][k] += wgt * (mpmath.mpf(psi[k].numerator) / psi[k].denominator)
    if rows is not None:
        return float(total), np.array([[float(v) for v in row] for row in grad])
    phi = total / n
    G = np.array([[float(-v / (e * n)) for v in row] for row in grad])
    return float(phi), G


def test_objective_gradient_40_digit(orc):
    """eq:Phi and eq:grad against 40-digit arithmetic on exact rational features."""
    rng = np.random.default_rng(3)
    for (H, W, N, d, eps, scale) in ((4, 5, 3, 2, 0.1, 1.0), (3, 6, 4, 3, 0.05, 0.3), (5, 4, 2, 1, 1.0, 2.0)):
        a, b = orc.multi_index(d)
        th = synth.random_theta(N, d, rng, scale=scale, multi_index=(a, b))
        lab = synth.random_labels(H, W, N, rng)
        phi, g = orc.objective_grad(th, lab, H, W, d, eps)
        phi_x, g_x = _mp_phi_grad(th, lab, H, W, d, eps, orc)
        assert abs(phi - phi_x) <= 1e-14 * max(1.0, abs(phi_x))
        assert np.max(np.abs(g - g_x)) <= 1e-13 * np.max(np.abs(g_x))


def test_row_bands_40_digit_and_partition(orc):
    """eq:Phi and eq:grad restricted to pixel rows (the share of one device when a
    map is split by rows): each band against 40-digit arithmetic over the same
    rows, and the bands of a partition sum to n Phi and -(eps n) grad Phi."""
    rng = np.random.default_rng(31)
    H, W, N, d, eps = 7, 5, 4, 2, 0.07
    a, b = orc.multi_index(d)
    th = synth.random_theta(N, d, rng, scale=0.5, multi_index=(a, b))
    lab = synth.random_labels(H, W, N, rng)
    cuts = [0, 2, 3, 7]
    tot, gtot = 0.0, np.zeros_like(th)
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        v, g = orc.objective_rows(th, lab, H, W, d, eps, r0, r1)
        vx, gx = _mp_phi_grad(th, lab, H, W, d, eps, orc, rows=(r0, r1))
        assert abs(v - vx) <= 1e-14 * max(1.0, abs(vx))
        assert np.max(np.abs(g - gx)) <= 1e-13 * np.max(np.abs(gx))
        tot += v
        gtot += g
    phi, gf = orc.objective_grad(th, lab, H, W, d, eps)
    n = H * W
    assert abs(tot - n * phi) <= 1e-13 * abs(n * phi)
    assert np.max(np.abs(gtot + eps * n * gf)) <= 1e-13 * np.max(np.abs(gtot))
    v, g = orc.objective_rows(th, lab, H, W, d, eps, 3, 3)
    assert v == 0.0 and not g.any()


def test_assign_rows_is_the_band_of_the_full_assignment(orc):
    """Section 2.1 over a band of rows: exactly the full map's labels there, and
    the band counts of a partition add up to the full count."""
    rng = np.random.default_rng(32)
    H, W, N, d = 9, 11, 6, 3
    th = synth.random_theta(N, d, rng, multi_index=orc.multi_index(d))
    lab = synth.random_labels(H, W, N, rng)
    F, nc, _ = orc.assign(th, H, W, d, lab)
    ex = _exact_scores(th, H, W, d, orc)
    tot = 0
    for r0, r1 in ((0, 4), (4, 5), (5, 9)):
        Fb, ncb, nn = orc.assign_rows(th, H, W, d, r0, r1, lab)
        assert nn == 0 and np.array_equal(Fb, F[r0 * W:r1 * W])
        for j in range(r0 * W, r1 * W):
            sc = ex[j]
            best = min(range(N), key=lambda i: (sc[i], i))
            gap = min(float(sc[i] - sc[best]) for i in range(N) if i != best)
            if gap > 1e-12:
                assert Fb[j - r0 * W] == best
        tot += ncb
    assert tot == nc


def test_phi_at_zero_and_gradient_closed_form(orc):
    """Fully ambiguous start (Section 2.1, Section 5.2): Phi(0) = -log N and
    grad_i Phi(0) = -(m_i - (1/N) sum_x psi(x)) / (eps n), m_i = sum_{x in G_i} psi(x)."""
    gm = synth.config_c1()
    H, W, d, eps = gm.H, gm.W, 2, 0.03
    K = orc.num_features(d)
    phi, g = orc.objective_grad(np.zeros((gm.N, K)), gm.labels, H, W, d, eps)
    assert abs(phi - (-math.log(gm.N))) <= 2e-16 * math.log(gm.N)
    X = orc.features(H, W, d)
    n = H * W
    for i in range(gm.N):
        m_i = X[:, gm.labels == i].sum(1)
        ref = -(m_i - X.sum(1) / gm.N) / (eps * n)
        assert np.allclose(g[i], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_two_grain_is_binary_logistic(orc):
    """N = 2: log p_G = -softplus((h_G - h_other)/eps), the textbook binary
    logistic likelihood (numpy's logaddexp as the independent routine)."""
    rng = np.random.default_rng(4)
    H, W, d, eps = 9, 11, 3, 0.2
    a, b = orc.multi_index(d)
    th = synth.random_theta(2, d, rng, multi_index=(a, b))
    lab = synth.random_labels(H, W, 2, rng)
    X = orc.features(H, W, d)
    h = th @ X
    z = (h[lab, np.arange(H * W)] - h[1 - lab, np.arange(H * W)]) / eps
    ref = -np.mean(np.logaddexp(0.0, z))
    phi, _ = orc.objective_grad(th, lab, H, W, d, eps)
    assert abs(phi - ref) <= 1e-14 * abs(ref)


def test_eps_scaling_gauge_and_bounds(orc):
    """Lemma 4.1 (bit for bit at eps = 2^-k), Lemma 4.2, eq:Phi (Phi <= 0),
    Proposition 4.7 (0 <= -eps Phi - E_0 <= eps log N), Lemma 4.9
    (Phi <= -log2 Err)."""
    rng = np.random.default_rng(5)
    H, W, N, d = 20, 18, 6, 2
    a, b = orc.multi_index(d)
    th = synth.random_theta(N, d, rng, scale=0.5, multi_index=(a, b))
    lab = synth.random_labels(H, W, N, rng)
    for k in (1, 4, 7):
        eps = 2.0 ** -k
        p1, g1 = orc.objective_grad(th, lab, H, W, d, eps)
        p2, g2 = orc.objective_grad(th / eps, lab, H, W, d, 1.0)
        assert p1 == p2
        assert np.array_equal(g1, g2 * (1.0 / eps)) or np.allclose(g1, g2 / eps, rtol=1e-15)
    c = rng.normal(size=th.shape[1])
    for eps in (1.0, 0.1, 0.01):
        p1, g1 = orc.objective_grad(th, lab, H, W, d, eps)
        p2, g2 = orc.objective_grad(th + c, lab, H, W, d, eps)
        assert abs(p1 - p2) <= 1e-12 * abs(p1)
        assert np.max(np.abs(g1 - g2)) <= 1e-10 * np.max(np.abs(g1))
        assert p1 <= 0.0
        X = orc.features(H, W, d)
        h = th @ X
        E0 = np.mean(h[lab, np.arange(H * W)] - h.min(0))
        gap = -eps * p1 - E0
        assert -1e-12 <= gap <= eps * math.log(N) + 1e-12
        _, ncorr, _ = orc.assign(th, H, W, d, lab)
        err = 1.0 - ncorr / (H * W)
        assert p1 <= -math.log(2.0) * err + 1e-15


def test_gradient_sums_to_zero_and_finite_differences(orc):
    """Proposition 4.4: sum_i grad_i Phi = 0 (gauge direction), and eq:grad matches
    central differences of Phi."""
    rng = np.random.default_rng(6)
    H, W, N, d, eps = 12, 13, 5, 3, 0.2
    a, b = orc.multi_index(d)
    th = synth.random_theta(N, d, rng, scale=0.3, multi_index=(a, b))
    lab = synth.random_labels(H, W, N, rng)
    phi, g = orc.objective_grad(th, lab, H, W, d, eps)
    assert np.max(np.abs(g.sum(0))) <= 1e-13 * np.max(np.abs(g))
    h = 1e-5
    for (i, k) in [(0, 0), (1, 3), (4, 9), (2, 5), (3, 1)]:
        tp, tm = th.copy(), th.copy()
        tp[i, k] += h
        tm[i, k] -= h
        fd = (orc.objective_grad(tp, lab, H, W, d, eps, grad=False)[0]
              - orc.objective_grad(tm, lab, H, W, d, eps, grad=False)[0]) / (2 * h)
        assert abs(fd - g[i, k]) <= 1e-6 * np.max(np.abs(g)), (i, k, fd, g[i, k])


def test_hessian_variance_form_and_gradient_differences(orc):
    """eq:hess and Proposition 4.5: v.Hv = -(1/(eps^2 n)) sum_x Var_{P_x}(v_i . eta(x)),
    zero along the gauge direction, and H v matches differences of the gradient."""
    rng = np.random.default_rng(8)
    H, W, N, d, eps = 7, 8, 4, 2, 0.3
    a, b = orc.multi_index(d)
    K = orc.num_features(d)
    th = synth.random_theta(N, d, rng, multi_index=(a, b))
    lab = synth.random_labels(H, W, N, rng)
    Hm = orc.hessian(th, lab, H, W, d, eps)
    X = orc.features(H, W, d)
    P = orc.softmax_probs(th, H, W, d, eps)
    for _ in range(3):
        v = rng.normal(size=(N, K))
        u = v @ X                                       # N x n: v_i . eta(x)
        var = (P * u * u).sum(0) - (P * u).sum(0) ** 2
        q = -var.sum() / (eps * eps * H * W)
        assert abs(v.reshape(-1) @ Hm @ v.reshape(-1) - q) <= 1e-12 * abs(q)
        assert q <= 0.0
        hstep = 1e-5
        gp = orc.objective_grad(th + hstep * v, lab, H, W, d, eps)[1]
        gm_ = orc.objective_grad(th - hstep * v, lab, H, W, d, eps)[1]
        fd = ((gp - gm_) / (2 * hstep)).reshape(-1)
        assert np.max(np.abs(fd - Hm @ v.reshape(-1))) <= 1e-6 * np.max(np.abs(fd))
    c = np.tile(rng.normal(size=K), N)
    assert np.max(np.abs(Hm @ c)) <= 1e-10 * np.max(np.abs(Hm))


# ---------------------------------------------------------------- fits --------

def _fit(orc, gm, d, eps, **kw):
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    acc = lambda th: orc.assign(th, gm.H, gm.W, d, gm.labels)[1] / (gm.H * gm.W)
    return orc.lbfgs_fit(obj, np.zeros((gm.N, orc.num_features(d))), accuracy=acc, **kw)


def test_fit_power_diagram_reaches_target(orc):
    """Section 5.4: from theta = 0 the d = 1 fit of a power-diagram map reaches
    >= 99% accuracy; the accepted iterates increase Phi."""
    gm = synth.config_c1()
    r = _fit(orc, gm, 1, 1e-2, target_acc=0.99, max_iter=500)
    assert r["status"] == "target" and r["acc"] >= 0.99
    phis = [rec["phi"] for rec in r["records"]]
    assert all(b >= a for a, b in zip(phis, phis[1:]))
    assert r["theta"][-1].tolist() == [0.0, 0.0, 0.0]     # gauge theta_N = 0 held


def test_separable_certificate_and_scaling_to_zero(orc):
    """Proposition 4.8 and Corollary 4.10 on a map generated by a known theta*:
    Phi(t theta*) increases to 0 in t, and once Phi > -log2/n the reconstruction is exact."""
    rng = np.random.default_rng(9)
    H, W, N, d = 16, 16, 4, 1
    gm = synth.power_diagram(H, W, N, rng, wmax=0.05)
    y, w = gm.sites, gm.weights
    th = np.stack([(y ** 2).sum(1) - w, -2 * y[:, 0], -2 * y[:, 1]], 1)
    F, nc, _ = orc.assign(th, H, W, d, gm.labels)
    assert nc == H * W
    phis = [orc.objective_grad(t * th, gm.labels, H, W, d, 1.0, grad=False)[0]
            for t in (1, 10, 100, 1000, 10000)]
    assert all(b > a for a, b in zip(phis, phis[1:])) and phis[-1] > -1e-3
    n = H * W
    for t in (1, 10, 100, 1000, 10000, 1e5):
        phi = orc.objective_grad(t * th, gm.labels, H, W, d, 1.0, grad=False)[0]
        if phi > -math.log(2) / n:
            assert orc.assign(t * th, H, W, d, gm.labels)[1] == n


def test_nonseparable_fit_matches_newton(orc):
    """Proposition 4.11: with random labels no exact reconstruction exists, the
    gauge-fixed maximiser is unique; L-BFGS and a dense Newton solve with eq:hess
    agree on it."""
    rng = np.random.default_rng(10)
    H, W, N, d, eps = 8, 9, 3, 2, 0.5
    lab = synth.random_labels(H, W, N, rng)
    K = orc.num_features(d)
    obj = lambda th: orc.objective_grad(th, lab, H, W, d, eps)
    hes = lambda th: orc.hessian(th, lab, H, W, d, eps)
    xn = orc.newton_fit(np.zeros((N, K)), obj, hes)
    r = orc.lbfgs_fit(obj, np.zeros((N, K)), accuracy=None, max_iter=500, gtol=1e-12)
    assert np.max(np.abs(r["theta"] - xn)) <= 1e-6 * np.max(np.abs(xn))
    assert np.max(np.abs(obj(xn)[1][:-1])) <= 1e-10


def test_nested_degree_monotone(orc):
    """Section 5.6.1: the optimum of Phi does not decrease with d (a degree-d fit,
    zero-padded, is admissible at degree d+1)."""
    rng = np.random.default_rng(11)
    H, W, N, eps = 10, 10, 3, 0.5
    lab = synth.random_labels(H, W, N, rng)
    prev_phi, prev_th = None, None
    for d in (1, 2, 3):
        K = orc.num_features(d)
        a, b = orc.multi_index(d)
        th0 = np.zeros((N, K))
        if prev_th is not None:
            pa, pb = orc.multi_index(d - 1)
            for k, (aa, bb) in enumerate(zip(pa, pb)):
                th0[:, [kk for kk in range(K) if a[kk] == aa and b[kk] == bb][0]] = prev_th[:, k]
            assert abs(orc.objective_grad(th0, lab, H, W, d, eps, grad=False)[0] - prev_phi) < 1e-12
        obj = lambda th, d=d: orc.objective_grad(th, lab, H, W, d, eps)
        r = orc.lbfgs_fit(obj, th0, accuracy=None, max_iter=300, gtol=1e-11)
        if prev_phi is not None:
            assert r["phi"] >= prev_phi - 1e-12
        prev_phi, prev_th = r["phi"], r["theta"]


# ---------------------------------------------------------------- generators --

def test_generators_deterministic_and_compact():
    a = synth.config_c2()
    b = synth.config_c2()
    assert np.array_equal(a.labels, b.labels)
    assert a.labels.min() == 0 and a.labels.max() == a.N - 1
    assert len(np.unique(a.labels)) == a.N
    assert a.meta["noise_pixels"] == round(0.01 * a.meta["boundary_pixels"])
    shapes = synth.config_c4_shapes()
    assert len(shapes) == 64
    assert all(128 <= H <= 768 and 128 <= W <= 768 and 20 <= N <= 500 and d in (2, 3, 4)
               for H, W, N, d in shapes)


def test_polynomial_generator_reconstructs(orc):
    """A random degree-3 polynomial diagram is recovered by the oracle's arg-min
    at its own coefficients (Section 3.3 basis, graded order)."""
    rng = np.random.default_rng(12)
    gm = synth.polynomial_diagram(40, 48, 20, 3, rng)
    th = synth.coef_to_theta(gm.coef, orc.multi_index(3))
    _, nc, _ = orc.assign(th, gm.H, gm.W, 3, gm.labels)
    assert nc >= gm.H * gm.W - 3


def test_oracle_fit_start_keeps_phi_under_gauge_shift(orc):
    """Lemma 4.2: the oracle fit moves a given start into the gauge theta_{N-1} = 0
    by a common shift, so its starting Phi equals Phi of the given theta."""
    gm = synth.config_c1()
    rng = np.random.default_rng(8)
    th0 = rng.normal(size=(gm.N, 3)) * 0.05
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, 1, 1e-2)
    r = orc.lbfgs_fit(obj, th0, max_iter=0)
    assert np.array_equal(r["theta"], th0 - th0[-1])
    assert abs(r["phi"] - obj(th0)[0]) <= 1e-12 * abs(obj(th0)[0])


def test_hessian_diag_is_the_diagonal_of_eq_hess(orc):
    """The preconditioner's diagonal equals minus the diagonal of the dense
    Hessian of eq. hess (itself pinned by finite differences above)."""
    rng = np.random.default_rng(12)
    H, W, N, d, eps = 7, 9, 4, 2, 0.3
    lab = synth.random_labels(H, W, N, rng)
    th = synth.random_theta(N, d, rng, scale=0.5, multi_index=orc.multi_index(d))
    D = orc.hessian_diag(th, lab, H, W, d, eps)
    Hm = orc.hessian(th, lab, H, W, d, eps)
    assert np.allclose(D.reshape(-1), -np.diag(Hm), rtol=1e-13, atol=1e-15)


def test_preconditioned_fit_reaches_target_in_fewer_iterations(orc):
    """Diagonal-preconditioned L-BFGS on a degree-3 polynomial diagram: the same
    target accuracy in fewer iterations than the plain L-BFGS, and the gauge row
    stays zero."""
    gm = synth.polynomial_diagram(64, 64, 16, 3, np.random.default_rng(3))
    d, eps = 3, 1e-3
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    acc = lambda th: orc.assign(th, gm.H, gm.W, d, gm.labels)[1] / gm.labels.size
    pre = lambda th: orc.hessian_diag(th, gm.labels, gm.H, gm.W, d, eps)
    K = orc.num_features(d)
    r0 = orc.lbfgs_fit(obj, np.zeros((gm.N, K)), accuracy=acc, target_acc=0.99)
    r1 = orc.lbfgs_fit(obj, np.zeros((gm.N, K)), accuracy=acc, target_acc=0.99, precondition=pre)
    assert r0["status"] == r1["status"] == "target"
    assert r1["iters"] < r0["iters"]
    assert np.all(r1["theta"][-1] == 0)


# ------------------------------------------------ eps annealing (f2) --------

def test_preconditioned_fit_is_eps_covariant(orc):
    """Lemma 4.1 (Phi_eps(theta) = Phi_1(theta / eps)) carried through the fit: the
    diagonal-preconditioned L-BFGS (unit first step, D scaling as 1/eps^2) from
    theta0 at eps takes the iterates eps * u_k of the same fit at eps = 1 from
    theta0 / eps, so rescaling the start and changing eps are the same thing
    (the end of Section 5.6.4)."""
    gm = synth.polynomial_diagram(24, 20, 6, 2, np.random.default_rng(31))
    d, eps = 2, 1e-2
    K = orc.num_features(d)
    th0 = synth.random_theta(gm.N, d, np.random.default_rng(32), scale=0.02,
                             multi_index=orc.multi_index(d))
    th0 = th0 - th0[-1]
    traj = {}
    for e, start in ((eps, th0), (1.0, th0 / eps)):
        xs = []
        obj = lambda th, e=e: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, e)
        pre = lambda th, e=e: orc.hessian_diag(th, gm.labels, gm.H, gm.W, d, e)
        orc.lbfgs_fit(obj, start, max_iter=8, precondition=pre, diag_every=3,
                      callback=lambda it, x, phi, acc: xs.append(x.copy()))
        traj[e] = xs
    assert len(traj[eps]) == len(traj[1.0]) == 8
    for a, b in zip(traj[eps], traj[1.0]):
        assert np.max(np.abs(a - eps * b)) <= 1e-9 * np.max(np.abs(a))
    assert K == 6


def test_annealed_fit_without_levels_is_the_plain_fit(orc):
    gm = synth.config_c1()
    d, eps = 1, 1e-2
    obj_e = lambda th, e: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, e)
    acc = lambda th: orc.assign(th, gm.H, gm.W, d, gm.labels)[1] / gm.labels.size
    z = np.zeros((gm.N, 3))
    r0 = orc.lbfgs_fit(lambda th: obj_e(th, eps), z, accuracy=acc, max_iter=40)
    r1 = orc.annealed_fit(obj_e, z, eps, stages=0, factor=4.0, stage_iters=10, accuracy=acc,
                          max_iter=40)
    assert r0["iters"] == r1["iters"] and r0["evals"] == r1["evals"]
    assert np.array_equal(r0["theta"], r1["theta"]) and r0["phi"] == r1["phi"]


def test_annealed_fit_levels_and_err_aligned_stop(orc):
    """eps_k = eps * factor**(S - k); each level starts from the last one's theta,
    where the accuracy is unchanged (F_theta does not depend on eps); the fit ends
    at the first iterate, at any level, whose accuracy reaches the target; phi is
    reported at the target eps."""
    gm = synth.polynomial_diagram(48, 48, 10, 2, np.random.default_rng(33))
    d, eps = 2, 1e-3
    obj_e = lambda th, e: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, e)
    acc = lambda th: orc.assign(th, gm.H, gm.W, d, gm.labels)[1] / gm.labels.size
    seen = []
    r = orc.annealed_fit(obj_e, np.zeros((gm.N, 6)), eps, stages=2, factor=8.0, stage_iters=15,
                         accuracy=acc, target_acc=0.99, max_iter=2000,
                         callback=lambda it, x, phi, a: seen.append((x.copy(), a)))
    lv = r["levels"]
    assert [v["eps"] for v in lv] == [eps * 64.0, eps * 8.0, eps][:len(lv)]
    assert r["status"] == "target" and r["acc"] >= 0.99
    assert all(v["status"] != "target" for v in lv[:-1]) and lv[-1]["status"] == "target"
    assert all(v["iters"] <= 15 for v in lv[:-1])
    assert r["iters"] == sum(v["iters"] for v in lv)
    # the first iterate to reach the target is the last one
    accs = [a for _, a in seen]
    assert accs[-1] >= 0.99 and all(a < 0.99 for a in accs[:-1])
    # phi at the target eps
    assert r["phi"] == orc.objective_grad(r["theta"], gm.labels, gm.H, gm.W, d, eps,
                                          grad=False)[0]


# ------------------------------------------ physical parameters (f1) --------

def _forward_pd(y, w):
    """Section 2.3.1: theta = (|y|^2 - w, -2 y1, -2 y2) in the order (1, x, y)."""
    return np.stack([(y ** 2).sum(1) - w, -2 * y[:, 0], -2 * y[:, 1]], 1)


def _forward_apd_legendre(y, w, A):
    """eq. h-APD in monomials, then x^2 = (2 P_2(x) + 1) / 3 (Section 3.3)."""
    Ay = np.einsum("nij,nj->ni", A, y)
    return np.stack([(y * Ay).sum(1) - w + (A[:, 0, 0] + A[:, 1, 1]) / 3, -2 * Ay[:, 0],
                     -2 * Ay[:, 1], 2 * A[:, 0, 0] / 3, 2 * A[:, 0, 1], 2 * A[:, 1, 1] / 3], 1)


def test_recover_power_diagram_round_trip(orc):
    rng = np.random.default_rng(60)
    y = rng.uniform(-1, 1, (20, 2))
    w = rng.uniform(0, 0.05, 20)
    y2, w2, A2, lam = orc.recover_params(_forward_pd(y, w), 1)
    assert lam == 0.0 and np.allclose(A2, np.eye(2))
    assert np.max(np.abs(y2 - y)) <= 1e-15 and np.max(np.abs(w2 - w)) <= 1e-14


def test_recover_anisotropic_round_trip(orc):
    """The generator's own (y, w, A) come back from its Legendre coefficients
    (every A_i has lambda_min >= 0.5 > margin, so no shift)."""
    gm = synth.anisotropic_power_diagram(32, 32, 25, np.random.default_rng(61))
    th = _forward_apd_legendre(gm.sites, gm.weights, gm.aniso)
    y2, w2, A2, lam = orc.recover_params(th, 2, margin=0.1)
    assert lam == 0.0
    assert np.max(np.abs(A2 - gm.aniso)) <= 1e-14
    assert np.max(np.abs(y2 - gm.sites)) <= 1e-12
    assert np.max(np.abs(w2 - gm.weights)) <= 1e-12


def test_recover_gauge_shift_keeps_the_diagram(orc):
    """Section 5.6.3: in the fit's gauge theta_N = 0 the last anisotropy is 0 (not
    positive definite); the common shift A_i + lambda I makes every smallest
    eigenvalue >= margin, the smallest exactly margin, and the recovered
    parameters generate scores that differ from the given ones by one common
    function (Lemma 4.2), so the diagram is the same."""
    gm = synth.anisotropic_power_diagram(40, 36, 18, np.random.default_rng(62))
    th = _forward_apd_legendre(gm.sites, gm.weights, gm.aniso)
    th = th - th[-1]  # the gauge theta_N = 0
    margin = 0.05
    y2, w2, A2, lam = orc.recover_params(th, 2, margin=margin)
    lmin = np.linalg.eigvalsh(A2)[:, 0]
    assert lam > 0 and np.all(lmin >= margin - 1e-12) and abs(lmin.min() - margin) <= 1e-12
    back = _forward_apd_legendre(y2, w2, A2)
    diff = back - th
    assert np.max(np.abs(diff - diff[0])) <= 1e-11 * np.max(np.abs(th))
    F0 = orc.assign(th, gm.H, gm.W, 2)[0]
    F1 = orc.assign(back, gm.H, gm.W, 2)[0]
    assert np.mean(F0 == F1) >= 1 - 2 / F0.size
    assert np.array_equal(F0, gm.labels) or np.mean(F0 == gm.labels) >= 0.995


def test_recover_rejects_higher_degree(orc):
    with pytest.raises(ValueError):
        orc.recover_params(np.zeros((3, 10)), 3)


# -------------------------------------------------- Newton-CG (f4) ----------

def _hvp_dense(orc, lab, H, W, d, eps):
    """H v with H the Hessian of -Phi from the dense eq. hess (itself pinned above
    by finite differences and the variance form)."""
    def hv(th, v):
        N, K = th.shape
        return (-orc.hessian(th, lab, H, W, d, eps) @ v.reshape(-1)).reshape(N, K)
    return hv


def test_newton_cg_reaches_the_newton_maximiser(orc):
    """Proposition 4.11: random labels leave no exact reconstruction and a unique
    gauge-fixed maximiser; the inexact Newton iteration with Hessian-vector
    products reaches the point the dense damped Newton solve finds."""
    rng = np.random.default_rng(12)
    H, W, N, d, eps = 7, 9, 4, 2, 0.3
    lab = synth.random_labels(H, W, N, rng)
    K = orc.num_features(d)
    obj = lambda th: orc.objective_grad(th, lab, H, W, d, eps)
    ref = orc.newton_fit(np.zeros((N, K)), obj, lambda th: orc.hessian(th, lab, H, W, d, eps))
    r = orc.newton_cg_fit(obj, _hvp_dense(orc, lab, H, W, d, eps), np.zeros((N, K)),
                          max_iter=60, cg_max=40, gtol=1e-11)
    assert r["status"] == "gtol"
    assert np.max(np.abs(r["theta"] - ref)) <= 1e-8 * np.max(np.abs(ref))
    phis = [rec["phi"] for rec in r["records"]]
    assert all(b >= a for a, b in zip(phis, phis[1:]))


def test_newton_cg_reaches_target_on_a_power_diagram(orc):
    gm = synth.config_c1()
    d, eps = 1, 1e-2
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    acc = lambda th: orc.assign(th, gm.H, gm.W, d, gm.labels)[1] / gm.labels.size
    # H v for the 64x64 map from the variance form of eq. hess (no dense matrix)
    X = orc.features(gm.H, gm.W, d)

    def hv(th, v):
        P = orc.softmax_probs(th, gm.H, gm.W, d, eps)
        u = v @ X
        ub = (P * u).sum(0)
        return ((P * (u - ub)) @ X.T) / (eps * eps * gm.labels.size)

    # the variance-form product equals the dense Hessian on a random direction
    rng = np.random.default_rng(5)
    th = rng.normal(size=(gm.N, 3)) * 0.05
    v = rng.normal(size=(gm.N, 3))
    dense = _hvp_dense(orc, gm.labels, gm.H, gm.W, d, eps)(th, v)
    assert np.max(np.abs(hv(th, v) - dense)) <= 1e-10 * np.max(np.abs(dense))
    r = orc.newton_cg_fit(obj, hv, np.zeros((gm.N, 3)), accuracy=acc, max_iter=200, cg_max=20)
    assert r["status"] == "target" and r["acc"] >= 0.99
    assert r["theta"][-1].tolist() == [0.0, 0.0, 0.0]
