"""Pins of the warm-start oracle (oracle/warm.py) against closed forms and
invariants that do not reuse its own arithmetic."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import synth
from oracle import warm


def leg_eval_2d(coef, d, X1, X2):
    """sum_ab c_ab P_a(X1) P_b(X2), each P evaluated directly (numpy legval)."""
    out = np.zeros_like(X1)
    k = 0
    for deg in range(d + 1):
        for b in range(deg + 1):
            a = deg - b
            out += coef[k] * npleg.legval(X1, np.eye(a + 1)[a]) * npleg.legval(X2, np.eye(b + 1)[b])
            k += 1
    return out


def test_rectangle_frame_closed_form():
    """A rectangular grain of w x h pixels: centroid at its middle, B' =
    diag((w^2 - 1)/12 (2/W)^2, (h^2 - 1)/12 (2/H)^2) (discrete uniform variance)."""
    H, W = 20, 30
    lab = np.ones((H, W), np.int32)
    r0, r1, c0, c1 = 3, 9, 5, 17     # 7 rows x 13 columns, off-centre
    lab[r0:r1 + 1, c0:c1 + 1] = 0
    fr = warm.grain_frames(lab.reshape(-1), H, W, 2)
    w, h = c1 - c0 + 1, r1 - r0 + 1
    y1 = (2 * (c0 + c1) / 2 + 1 - W) / W
    y2 = (2 * (r0 + r1) / 2 + 1 - H) / H
    assert fr[0, 0] == pytest.approx(y1, abs=1e-15)
    assert fr[0, 1] == pytest.approx(y2, abs=1e-15)
    assert fr[0, 3] == pytest.approx((w * w - 1) / 12 * (2 / W) ** 2, rel=1e-13)
    assert fr[0, 5] == pytest.approx((h * h - 1) / 12 * (2 / H) ** 2, rel=1e-13)
    assert abs(fr[0, 4]) <= 1e-16
    assert fr[0, 6] == w * h
    assert fr[0, 2] == pytest.approx(2 * math.sqrt(fr[0, 3]), rel=1e-13)   # wider than tall
    D = warm.descriptors(lab.reshape(-1), H, W, 2, fr)
    assert D[0, 0] == pytest.approx(math.log(w * h * 2 / (H * W)), rel=1e-14)
    # the degree-1 moments are the centroid; N B' follows the closed form
    assert D[0, 1] == pytest.approx(y1, abs=1e-14) and D[0, 2] == pytest.approx(y2, abs=1e-14)
    assert D[0, 28] == pytest.approx(2 * (w * w - 1) / 12 * (2 / W) ** 2, rel=1e-13)
    assert D[0, 31] == pytest.approx(math.log(2) / 10)


def test_centred_rectangle_odd_moments_vanish():
    """A grain symmetric about the domain centre: pixel centres come in exact
    +-x pairs, so every Legendre moment with an odd exponent is zero, and the
    even ones equal the product of the 1-D means (separable grain)."""
    H, W = 24, 30
    lab = np.ones((H, W), np.int32)
    lab[5:19, 8:22] = 0              # rows 5..18, columns 8..21: centred
    D = warm.descriptors(lab.reshape(-1), H, W, 2)
    pairs = [p for p in warm._graded(6) if p != (0, 0)]
    x1 = (2 * np.arange(8, 22) + 1 - W) / W
    x2 = (2 * np.arange(5, 19) + 1 - H) / H
    for q, (a, b) in enumerate(pairs):
        if a % 2 or b % 2:
            assert abs(D[0, 1 + q]) <= 1e-15
        else:
            ref = np.mean(npleg.legval(x1, np.eye(a + 1)[a])) * np.mean(npleg.legval(x2, np.eye(b + 1)[b]))
            assert D[0, 1 + q] == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_empty_grain_descriptor_is_zero():
    H, W = 6, 6
    lab = np.zeros(H * W, np.int32)
    lab[:18] = 2
    fr = warm.grain_frames(lab, H, W, 3)
    assert fr[1].tolist() == [0, 0, 1, 0, 0, 0, 0, 0]
    assert np.all(warm.descriptors(lab, H, W, 3, fr)[1] == 0)
    th = warm.heuristic_theta(fr, H, W, 2)
    assert np.all(th[1, 1:] == 0) and th[1, 0] == 1 + np.max(np.abs(th[[0, 2]]).sum(1))
    # the empty grain wins no pixel
    F, _, _ = oracle.assign(th, H, W, 2)
    assert not np.any(F == 1)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_heuristic_is_the_apd_score(d):
    """Section 5.6.2 and eq. h-APD: theta'_i . psi(x) equals
    (x - y')^T A' (x - y') - w' (d >= 2), |x - y'|^2 - w' - |x|^2 (d = 1), with
    A' = B'^{-1} and w' the grain-to-ellipse area ratio; evaluated through the
    (independently pinned) design matrix."""
    gm = synth.anisotropic_power_diagram(24, 28, 5, np.random.default_rng(11))
    fr = warm.grain_frames(gm.labels, gm.H, gm.W, gm.N)
    th = warm.heuristic_theta(fr, gm.H, gm.W, d)
    X = oracle.features(gm.H, gm.W, d)
    x1 = np.tile((2 * np.arange(gm.W) + 1 - gm.W) / gm.W, gm.H)
    x2 = np.repeat((2 * np.arange(gm.H) + 1 - gm.H) / gm.H, gm.W)
    n = gm.H * gm.W
    for i in range(gm.N):
        y1, y2, B11, B12, B22, cnt = fr[i, 0], fr[i, 1], fr[i, 3], fr[i, 4], fr[i, 5], fr[i, 6]
        if d >= 2:
            det = B11 * B22 - B12 * B12
            A11, A12, A22 = B22 / det, -B12 / det, B11 / det
        else:
            A11, A12, A22 = 1.0, 0.0, 1.0
        w = math.sqrt(A11 * A22 - A12 * A12) * (4.0 * cnt / n) / math.pi
        e1, e2 = x1 - y1, x2 - y2
        ref = A11 * e1 * e1 + 2 * A12 * e1 * e2 + A22 * e2 * e2 - w
        if d == 1:
            ref -= x1 * x1 + x2 * x2
        got = th[i] @ X
        assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_heuristic_disk_weight_is_squared_radius():
    """A disk grain of radius R: w' = area / pi ~ R^2 for d = 1 (the power radius)."""
    H = W = 200
    x = (2 * np.arange(W) + 1 - W) / W
    X1, X2 = np.meshgrid(x, x)
    R = 0.5
    lab = np.where(X1 ** 2 + X2 ** 2 <= R * R, 0, 1).astype(np.int32).reshape(-1)
    fr = warm.grain_frames(lab, H, W, 2)
    th = warm.heuristic_theta(fr, H, W, 1)
    w = fr[0, 0] ** 2 + fr[0, 1] ** 2 - th[0, 0]
    assert w == pytest.approx(R * R, rel=2e-3)
    # d = 2: A' = B'^{-1} = (4 / R^2) I for a uniform disk, and the zero level set
    # of the seed is the disk boundary (w' = 4 there)
    q = warm.heuristic_quadratic(fr, 2, H * W)[0]
    assert np.allclose(q[0], 4 / R ** 2 * np.eye(2), rtol=3e-3, atol=0.02)
    assert q[2] == pytest.approx(4.0, rel=3e-3)


def test_targets_are_gauge_and_scale_free():
    """Targets of a * theta + g (a > 0, g a common row) equal those of theta
    (Lemma 4.2: a common shift leaves the diagram; the scale is free), have zero
    mean and unit root mean square; assembling them back gives theta up to
    that shift and scale."""
    rng = np.random.default_rng(3)
    gm = synth.polynomial_diagram(32, 32, 6, 3, rng)
    fr = warm.grain_frames(gm.labels, gm.H, gm.W, gm.N)
    th = rng.normal(size=(gm.N, 10))
    t1, r1 = warm.targets(th, fr)
    t2, r2 = warm.targets(3.7 * th + rng.normal(size=10), fr)
    assert np.max(np.abs(t1 - t2)) <= 1e-12
    assert r2 == pytest.approx(3.7 * r1, rel=1e-12)
    assert np.max(np.abs(t1.mean(0))) <= 1e-14
    assert np.sqrt(np.mean(t1 ** 2)) == pytest.approx(1.0, rel=1e-12)
    back = warm.assemble(t1 * r1, fr)
    assert np.max(np.abs(back - (th - th.mean(0)))) <= 1e-12 * np.max(np.abs(th))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    K = 6
    p = warm.mlp_init(K, rng).astype(np.float64)
    x = rng.normal(size=(7, 32))
    t = rng.normal(size=(7, K))
    loss, g = warm.mlp_loss_grad(p, x, t, K)
    idx = rng.choice(p.size, 60, replace=False)
    # include biases of every layer
    idx = np.concatenate([idx, [32 * 256 + 3, 33 * 256 + 256 * 256 + 7, p.size - 1]])
    h = 1e-6
    for j in idx:
        e = np.zeros_like(p)
        e[j] = h
        fd = (warm.mlp_loss_grad(p + e, x, t, K)[0] - warm.mlp_loss_grad(p - e, x, t, K)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * (abs(fd) + 1e-4), (j, fd, g[j])


def test_mlp_shapes_and_gelu():
    assert warm.mlp_num_params(28) == 32 * 256 + 256 + 256 * 256 + 256 + 256 * 28 + 28
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    # GELU = z Phi(z), Phi the standard normal CDF (erfc form)
    Phi = 0.5 * np.array([math.erfc(-v / math.sqrt(2)) for v in z])
    assert np.allclose(warm.gelu(z), z * Phi, rtol=1e-14, atol=1e-16)
    h = 1e-6
    assert np.allclose(warm.gelu_grad(z), (warm.gelu(z + h) - warm.gelu(z - h)) / (2 * h), atol=1e-8)


def test_adam_first_step_is_signed_lr():
    """Bias correction makes Adam's first step -lr g / (|g| + eps') per entry."""
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = warm.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-5)


def test_mlp_learns_a_linear_map():
    """Adam on the MSE loss fits a small linear target (training loop sanity)."""
    rng = np.random.default_rng(1)
    K = 3
    p = warm.mlp_init(K, rng).astype(np.float64)
    x = rng.normal(size=(64, 32)) * 0.5
    Wt = rng.normal(size=(32, K)) * 0.2
    t = x @ Wt
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = warm.mlp_loss_grad(p, x, t, K)[0]
    for step in range(1, 201):
        loss, g = warm.mlp_loss_grad(p, x, t, K)
        p, m, v = warm.adam_step(p, g, m, v, step, 1e-3)
    assert loss < 0.05 * l0


def test_scale_search_finds_the_maximum_of_a_concave_profile():
    """Golden-section search of a unimodal profile in log2 s: the best point is
    within one final bracket of the true maximiser (here s* = 2^5.3)."""
    f = lambda s: -(math.log2(s) - 5.3) ** 2
    s, v, ne = warm.scale_search(f, 1.0)
    assert abs(math.log2(s) - 5.3) < 0.25
    assert ne <= 2 + 12 + 6
    # decreasing profile: the search goes down
    s2, _, _ = warm.scale_search(lambda s: -s, 1.0)
    assert s2 < 1.0
    # NaN ranks lowest
    s3, v3, _ = warm.scale_search(lambda s: float("nan") if s > 3 else -abs(math.log2(s)), 1.0)
    assert v3 == 0.0 and s3 == 1.0


def test_scale_search_on_the_objective_is_a_maximum_along_the_ray():
    """Proposition 4.4: s -> Phi(s theta) is concave, so the chosen scale beats
    its neighbours."""
    gm = synth.config_c1()
    fr = warm.grain_frames(gm.labels, gm.H, gm.W, gm.N)
    th = warm.heuristic_theta(fr, gm.H, gm.W, 1)
    phi = lambda s: oracle.objective_grad(s * th, gm.labels, gm.H, gm.W, 1, 1e-2, grad=False)[0]
    s, v, _ = warm.scale_search(phi, warm.initial_scale(gm.H, gm.W, gm.N, 1e-2))
    assert v > -math.log(gm.N)
    assert v >= phi(s * 1.3) and v >= phi(s / 1.3)
