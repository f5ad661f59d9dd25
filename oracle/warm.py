"""Oracle of the warm start: per-grain descriptors, the moment seed, training
targets, the MLP (forward, MSE gradient, Adam), the assembly of a start from
network outputs and the scale search.

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
* Grains without pixels get the row (C, 0, ..., 0), C = 1 + max_i sum_k |theta_ik|
  over the other grains: since |P_a| <= 1 on [-1, 1], their score exceeds every
  other score, so they win no pixel.
* The descriptor of grain i (32 numbers): log(N |G_i| / n), the 27 Legendre
  indicator moments mean_{x in G_i} P_a(x_1) P_b(x_2) for 1 <= a + b <= 6 in the
  graded order, N B'_i (three entries) and log(N) / 10.
* Training target of grain i from a fitted theta: theta_i minus the mean over the
  non-empty grains (a common shift is a gauge, Lemma 4.2), divided by the root
  mean square of those centred values (the scale of a fit is free, Proposition
  4.8).
* MLP: 32 -> 256 -> 256 -> K, exact GELU z Phi(z), mean-squared-error loss over
  all B x K outputs, Adam (Kingma and Ba 2015).
* Warm start: theta_hat = network outputs centred over the non-empty grains
  (or the moment seed), then theta = s* theta_hat where s* maximises the concave
  one-dimensional restriction s -> Phi(s theta_hat) (Proposition 4.4), found by
  bracketing in log2(s) and a golden-section search; theta = 0 if that is worse
  than Phi(0).
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
        out[i, 0] = math.log(cnt * N / n)
        for q, (a, b) in enumerate(pairs):
            Pa = npleg.legval(x1[cc], np.eye(a + 1)[a])
            Pb = npleg.legval(x2[rr], np.eye(b + 1)[b])
            out[i, 1 + q] = np.mean(Pa * Pb)
        out[i, 28:31] = N * fr[i, 3:6]
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
    return fix_empty(th, frames)


def fix_empty(theta, frames):
    """Rows of grains without pixels := (C, 0, ..., 0), C = 1 + max over the other
    grains of sum_k |theta_ik| (their score then exceeds every other on [-1, 1]^2)."""
    th = np.array(theta, np.float64, copy=True)
    live = np.asarray(frames)[:, 6] > 0
    if np.all(live):
        return th
    C = 1.0 + (np.max(np.sum(np.abs(th[live]), axis=1)) if np.any(live) else 0.0)
    th[~live] = 0.0
    th[~live, 0] = C
    return th


def targets(theta_fit, frames):
    """(N x K targets, rms): the fitted theta centred over the non-empty grains and
    divided by the root mean square of the centred values; zero rows for empty
    grains."""
    tf = np.asarray(theta_fit, np.float64)
    live = np.asarray(frames)[:, 6] > 0
    out = np.zeros_like(tf)
    if not np.any(live):
        return out, 1.0
    c = tf[live] - tf[live].mean(axis=0)
    ss = float(np.sum(c * c))
    rms = math.sqrt(ss / c.size) if ss > 0.0 else 1.0
    out[live] = c / rms
    return out, rms


def assemble(outputs, frames):
    """theta_hat from network outputs: centred over the non-empty grains, empty
    grains given the row that wins no pixel."""
    y = np.asarray(outputs, np.float64)
    live = np.asarray(frames)[:, 6] > 0
    th = y - (y[live].mean(axis=0) if np.any(live) else 0.0)
    return fix_empty(th, frames)


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
