"""Oracle of the warm start: per-grain descriptors, the moment heuristic, the
local/global Legendre frame changes, training targets, the MLP (forward, MSE
gradient, Adam) and the scale search.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here is plain FP64 numpy written from the definitions:

* Section 5.6.2 seeds a fit from image moments: the centroid y'_i of grain G_i,
  the central second-moment matrix B'_i of its pixels, A'_i = B'_i^{-1} and the
  weight w'_i = sqrt(det A'_i) area(G_i) / pi, the ratio of the grain's area to
  that of the ellipse of B'_i as the paper describes it (area(G_i) = 4 |G_i| / n
  on [-1, 1]^2; the printed formula divides by |Omega|, which is the same ratio
  on a domain of unit area); the quadratic (x - y')^T A' (x - y') - w' is the
  anisotropic power-diagram score of Section 2.3.1 (eq. h-APD), rewritten in the
  Legendre basis with x^2 = (2 P_2(x) + 1) / 3 (Section 3.3).  At degree 1 the
  matrix is the identity and the common |x|^2 is dropped (it is a gauge term,
  Lemma 4.2).
* Frame changes substitute an affine map t = alpha x + beta into a Legendre
  series: each P_a is expanded into monomials (numpy's leg2poly), (alpha x +
  beta)^k is expanded binomially, and the result is taken back to the Legendre
  basis (poly2leg).
* The descriptor of grain i (32 numbers): log(N |G_i| / n), B'_i / r_i^2 (three
  entries), the 27 local Legendre indicator moments mean_{x in G_i} P_a(u_1)
  P_b(u_2) for 1 <= a + b <= 6 in the graded order, and log(N) / 10; the local
  coordinate is u = (x - y'_i) / r_i with r_i = 2 sqrt(lambda_max(B'_i)) (at
  least one pixel width 2 / max(H, W)).
* Training target of grain i from a fitted theta: with lambda > 0 and shift g the
  least-squares fit of theta_i ~ lambda theta'_i + g over grains (g is a common
  shift, a gauge, and lambda the free scale of Proposition 4.8),
  Delta_i = (theta_i - g) / lambda - theta'_i, written in grain i's local frame.
* MLP: 32 -> 256 -> 256 -> K, exact GELU z Phi(z), mean-squared-error loss over
  all B x K outputs, Adam (Kingma and Ba 2015).
* Warm start: theta_hat_i = theta'_i + (network output for grain i taken back to
  the global frame), then theta = s* theta_hat where s* maximises the concave
  one-dimensional restriction s -> Phi(s theta_hat) (Proposition 4.4), found by
  bracketing in log2(s) and a golden-section search.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import erf

DESC_DIM = 32
FRAME_DIM = 8
WIDTH = 256
MOMENT_DEGREE = 6


def _graded(d):
    """(a, b) pairs of total degree <= d in the library's order."""
    out = []
    for k in range(d + 1):
        for b in range(k + 1):
            out.append((k - b, b))
    return out


def _coords(H, W):
    x1 = (2.0 * np.arange(W) + 1.0 - W) / W
    x2 = (2.0 * np.arange(H) + 1.0 - H) / H
    return x1, x2


def grain_frames(labels, H, W, N):
    """Per grain (y'1, y'2, r, B11, B12, B22, |G_i|, 0); empty grains (0, 0, 1, 0...)."""
    lab = np.asarray(labels).reshape(H, W)
    fr = np.zeros((N, FRAME_DIM))
    fr[:, 2] = 1.0
    x1, x2 = _coords(H, W)
    rmin = 2.0 / max(H, W)
    for i in range(N):
        rr, cc = np.nonzero(lab == i)
        if rr.size == 0:
            continue
        X1, X2 = x1[cc], x2[rr]
        y1, y2 = X1.mean(), X2.mean()
        B11 = np.mean((X1 - y1) ** 2)
        B12 = np.mean((X1 - y1) * (X2 - y2))
        B22 = np.mean((X2 - y2) ** 2)
        lmax = np.linalg.eigvalsh(np.array([[B11, B12], [B12, B22]]))[-1]
        r = max(2.0 * math.sqrt(max(lmax, 0.0)), rmin)
        fr[i] = (y1, y2, r, B11, B12, B22, rr.size, 0.0)
    return fr


def descriptors(labels, H, W, N, frames=None):
    """N x 32 descriptors (FP64) of every grain; zeros for empty grains."""
    fr = grain_frames(labels, H, W, N) if frames is None else frames
    lab = np.asarray(labels).reshape(H, W)
    x1, x2 = _coords(H, W)
    n = H * W
    out = np.zeros((N, DESC_DIM))
    pairs = [p for p in _graded(MOMENT_DEGREE) if p != (0, 0)]
    for i in range(N):
        cnt = fr[i, 6]
        if cnt == 0:
            continue
        rr, cc = np.nonzero(lab == i)
        y1, y2, r = fr[i, 0], fr[i, 1], fr[i, 2]
        u1 = (x1[cc] - y1) / r
        u2 = (x2[rr] - y2) / r
        out[i, 0] = math.log(cnt * N / n)
        out[i, 1:4] = fr[i, 3:6] / (r * r)
        for q, (a, b) in enumerate(pairs):
            Pa = npleg.legval(u1, np.eye(a + 1)[a])
            Pb = npleg.legval(u2, np.eye(b + 1)[b])
            out[i, 4 + q] = np.mean(Pa * Pb)
        out[i, 31] = math.log(N) / 10.0
    return out


def heuristic_quadratic(frames, d, n):
    """Per grain (A11, A12, A22, y1, y2, w) of the moment seed (Section 5.6.2)."""
    out = []
    for f in frames:
        y1, y2, B11, B12, B22, cnt = f[0], f[1], f[3], f[4], f[5], f[6]
        if cnt == 0:
            out.append(None)
            continue
        det = B11 * B22 - B12 * B12
        if d >= 2 and det > 1e-300:
            # eq. A-guess: the inverse of the 2 x 2 moment matrix (adjugate / det)
            A = np.array([[B22, -B12], [-B12, B11]]) / det
        else:
            A = np.eye(2)
        area = 4.0 * cnt / n            # area of G_i in x units ([-1, 1]^2 has area 4)
        detA = A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]
        w = math.sqrt(max(detA, 0.0)) * area / math.pi
        out.append((A, np.array([y1, y2]), w))
    return out


def heuristic_theta(frames, H, W, d):
    """N x K Legendre coefficients of the moment seed; zero rows for empty grains."""
    K = (d + 1) * (d + 2) // 2
    idx = {p: k for k, p in enumerate(_graded(d))}
    th = np.zeros((len(frames), K))
    for i, q in enumerate(heuristic_quadratic(frames, d, H * W)):
        if q is None:
            continue
        A, y, w = q
        if d == 1:
            # |x - y|^2 - w without the common |x|^2
            th[i, idx[(0, 0)]] = y @ y - w
            th[i, idx[(1, 0)]] = -2.0 * y[0]
            th[i, idx[(0, 1)]] = -2.0 * y[1]
            continue
        # x^T A x - 2 (A y).x + y^T A y - w in monomials, then x^2 = (2 P_2 + 1)/3
        Ay = A @ y
        th[i, idx[(0, 0)]] = y @ Ay - w + (A[0, 0] + A[1, 1]) / 3.0
        th[i, idx[(1, 0)]] = -2.0 * Ay[0]
        th[i, idx[(0, 1)]] = -2.0 * Ay[1]
        th[i, idx[(2, 0)]] = 2.0 * A[0, 0] / 3.0
        th[i, idx[(1, 1)]] = 2.0 * A[0, 1]
        th[i, idx[(0, 2)]] = 2.0 * A[1, 1] / 3.0
    return th


def affine_matrix(alpha, beta, d):
    """M[a, a'] = coefficient of P_a'(x) in P_a(alpha x + beta), a, a' <= d."""
    M = np.zeros((d + 1, d + 1))
    for a in range(d + 1):
        mono = npleg.leg2poly(np.eye(a + 1)[a])          # P_a(t) = sum_k mono[k] t^k
        sub = np.zeros(d + 1)
        for k, ck in enumerate(mono):                    # t^k = (alpha x + beta)^k
            for j in range(k + 1):
                sub[j] += ck * math.comb(k, j) * alpha ** j * beta ** (k - j)
        leg = npleg.poly2leg(sub[: a + 1])
        M[a, : leg.size] = leg
    return M


def change_frame(coef, d, al1, be1, al2, be2):
    """Coefficients in P_a(x1) P_b(x2) of sum_ab c_ab P_a(al1 x1 + be1) P_b(al2 x2 + be2)."""
    pairs = _graded(d)
    idx = {p: k for k, p in enumerate(pairs)}
    M1 = affine_matrix(al1, be1, d)
    M2 = affine_matrix(al2, be2, d)
    out = np.zeros(len(pairs))
    for k, (a, b) in enumerate(pairs):
        c = coef[k]
        if c == 0.0:
            continue
        for a2 in range(a + 1):
            for b2 in range(b + 1):
                out[idx[(a2, b2)]] += c * M1[a, a2] * M2[b, b2]
    return out


def to_local(coef_global, frame, d):
    """Global-frame coefficients re-expanded in u = (x - y') / r (x = y' + r u)."""
    y1, y2, r = frame[0], frame[1], frame[2]
    return change_frame(coef_global, d, r, y1, r, y2)


def to_global(coef_local, frame, d):
    """Local-frame coefficients re-expanded in x (u = x / r - y' / r)."""
    y1, y2, r = frame[0], frame[1], frame[2]
    return change_frame(coef_local, d, 1.0 / r, -y1 / r, 1.0 / r, -y2 / r)


def targets(theta_fit, theta_h, frames, d):
    """(N x K local-frame targets, lambda): least-squares scale and shift of the
    fitted theta onto the seed, residual in each grain's local frame."""
    tf = np.asarray(theta_fit, np.float64)
    th = np.asarray(theta_h, np.float64)
    a = tf - tf.mean(axis=0)
    b = th - th.mean(axis=0)
    num, den = float(np.sum(a * b)), float(np.sum(b * b))
    lam = num / den if (den > 0.0 and num > 0.0) else 1.0
    g = tf.mean(axis=0) - lam * th.mean(axis=0)
    delta = (tf - g) / lam - th
    out = np.zeros_like(delta)
    for i in range(delta.shape[0]):
        out[i] = to_local(delta[i], frames[i], d)
    return out, lam


def apply_correction(theta_h, local, frames, d):
    """theta_hat = theta' + correction taken back to the global frame."""
    out = np.array(theta_h, np.float64, copy=True)
    for i in range(out.shape[0]):
        out[i] += to_global(np.asarray(local[i], np.float64), frames[i], d)
    return out


# ---------------------------------------------------------------- the network
def mlp_sizes(k_out, d_in=DESC_DIM, width=WIDTH):
    return [(d_in, width), (width,), (width, width), (width,), (width, k_out), (k_out,)]


def mlp_num_params(k_out, d_in=DESC_DIM, width=WIDTH):
    return sum(int(np.prod(s)) for s in mlp_sizes(k_out, d_in, width))


def mlp_unpack(params, k_out, d_in=DESC_DIM, width=WIDTH):
    """Flat buffer [W1 (d_in x width), b1, W2, b2, W3 (width x K), b3] -> arrays."""
    p = np.asarray(params, np.float64).reshape(-1)
    out, o = [], 0
    for s in mlp_sizes(k_out, d_in, width):
        m = int(np.prod(s))
        out.append(p[o: o + m].reshape(s))
        o += m
    assert o == p.size
    return out


def mlp_init(k_out, rng, d_in=DESC_DIM, width=WIDTH):
    """He-style normal weights (std sqrt(2 / fan_in)), zero biases, FP32 values."""
    parts = []
    for s in mlp_sizes(k_out, d_in, width):
        if len(s) == 2:
            parts.append(rng.normal(size=s) * math.sqrt(2.0 / s[0]))
        else:
            parts.append(np.zeros(s))
    return np.concatenate([q.reshape(-1) for q in parts]).astype(np.float32)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def mlp_forward(params, x, k_out, keep=False):
    W1, b1, W2, b2, W3, b3 = mlp_unpack(params, k_out)
    x = np.asarray(x, np.float64)
    z1 = x @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    y = h2 @ W3 + b3
    if keep:
        return y, (x, z1, h1, z2, h2)
    return y


def mlp_loss_grad(params, x, t, k_out):
    """(loss, flat gradient) of mean((y - t)^2) over all batch x K outputs."""
    W1, b1, W2, b2, W3, b3 = mlp_unpack(params, k_out)
    y, (x, z1, h1, z2, h2) = mlp_forward(params, x, k_out, keep=True)
    t = np.asarray(t, np.float64)
    B = x.shape[0]
    r = y - t
    loss = float(np.sum(r * r)) / (B * k_out)
    dy = 2.0 * r / (B * k_out)
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3.T) * gelu_grad(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([q.reshape(-1) for q in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, g


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- scale search
GOLDEN = (math.sqrt(5.0) - 1.0) / 2.0
BRACKET_STEP = 2.0      # log2 step of the bracketing (a factor 4 in s)
BRACKET_MAX = 12        # bracketing evaluations at most
GOLDEN_ITERS = 6        # golden-section evaluations


def initial_scale(H, W, N, eps):
    """Starting scale of the search: about one logit unit per pixel across a
    boundary of a seed whose cells have N-typical size."""
    return eps * max(H, W) / (28.0 * math.sqrt(N))


def scale_search(phi_of_scale, s0):
    """Maximise the unimodal u -> phi(2^u) from u0 = log2(s0).  Returns (s*, phi*,
    evaluations).  Bracketing: step up by BRACKET_STEP while phi increases (down
    if the first step up does not increase it); then GOLDEN_ITERS golden-section
    steps inside the bracket; the best point evaluated is returned."""
    cache = {}

    def f(u):
        if u not in cache:
            v = float(phi_of_scale(2.0 ** u))
            cache[u] = v if v == v else -math.inf   # NaN ranks lowest
        return cache[u]

    u0 = math.log2(s0)
    a, b = u0, u0 + BRACKET_STEP
    fa, fb = f(a), f(b)
    if fb >= fa:
        step = BRACKET_STEP
        lo, mid, fmid = a, b, fb
    else:
        step = -BRACKET_STEP
        lo, mid, fmid = b, a, fa
    hi = mid + step
    n_br = 0
    while n_br < BRACKET_MAX:
        fh = f(hi)
        n_br += 1
        if not (fh > fmid):
            break
        lo, mid, fmid = mid, hi, fh
        hi = mid + step
    left, right = min(lo, hi), max(lo, hi)
    # golden section on [left, right]
    x1 = right - GOLDEN * (right - left)
    x2 = left + GOLDEN * (right - left)
    f1, f2 = f(x1), f(x2)
    for _ in range(GOLDEN_ITERS - 2):
        if f1 >= f2:
            right, x2, f2 = x2, x1, f1
            x1 = right - GOLDEN * (right - left)
            f1 = f(x1)
        else:
            left, x1, f1 = x1, x2, f2
            x2 = left + GOLDEN * (right - left)
            f2 = f(x2)
    best_u = max(cache, key=lambda u: (cache[u], -abs(u - u0)))
    return 2.0 ** best_u, cache[best_u], len(cache)
