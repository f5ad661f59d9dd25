"""GPU parity: libpd's HIP kernels against the FP64 oracle, element by element.

Tolerances: assignments and FP64 features bit-exact; FP64 objective relative
1e-10 and gradient 1e-10 of its largest entry; FP32 mode 2e-3 (the
reduced-precision bound), with the measured error printed.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def problem(pdl, labels, H, W, N, d, eps):
    return pdl.Problem(dev(labels, torch.int32), H, W, N, d, eps)


def rel_err(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def grad_err(g, ref):
    return float(np.max(np.abs(g - ref)) / max(np.max(np.abs(ref)), 1e-300))


# ------------------------------------------------------------------ features --

@pytest.mark.parametrize("H,W,d", [(1, 1, 1), (7, 5, 3), (37, 53, 8), (64, 64, 2), (129, 70, 6)])
def test_features_bit_exact(pd, orc, H, W, d):
    pdl, ctx = pd
    ref = orc.features(H, W, d)
    out = ctx.features(H, W, d, "fp64").cpu().numpy()
    assert np.array_equal(out, ref)
    out32 = ctx.features(H, W, d, "fp32").cpu().numpy()
    assert np.array_equal(out32, ref.astype(np.float32))
    bf = ctx.features(H, W, d, "bf16").cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    hi = bf[0].view(np.float32).astype(np.float64)
    lo = bf[1].view(np.float32).astype(np.float64)
    assert np.max(np.abs(hi + lo - ref)) <= 2.0 ** -16 * np.max(np.abs(ref))


# ------------------------------------------------------------------ assignment --

@pytest.mark.parametrize("H,W,N,d,seed", [(5, 3, 2, 1, 0), (33, 70, 65, 2, 1), (64, 64, 8, 1, 2),
                                          (40, 129, 130, 4, 3), (17, 200, 7, 8, 4),
                                          (3, 64, 300, 6, 5)])
def test_assign_bit_exact_random(pd, orc, H, W, N, d, seed):
    pdl, ctx = pd
    rng = np.random.default_rng(seed)
    th = synth.random_theta(N, d, rng, multi_index=orc.multi_index(d))
    lab = synth.random_labels(H, W, N, rng)
    ref, nc, _ = orc.assign(th, H, W, d, lab)
    outs, cnt = ctx.assign([problem(pdl, lab, H, W, N, d, 1.0)], [dev(th)])
    assert np.array_equal(outs[0].cpu().numpy(), ref)
    assert int(cnt[0]) == nc


def test_assign_ties_nan_and_generated_maps(pd, orc):
    pdl, ctx = pd
    H, W = 20, 30
    outs, _ = ctx.assign([problem(pdl, np.zeros(H * W), H, W, 4, 2, 1.0)], [dev(np.zeros((4, 6)))])
    assert torch.all(outs[0] == 0)
    th = np.zeros((3, 3))
    th[1, 0] = np.nan
    outs, cnt = ctx.assign([problem(pdl, np.zeros(H * W), H, W, 3, 1, 1.0)], [dev(th)])
    assert torch.all(outs[0] == -1) and int(cnt[0]) == 0
    gm = synth.config_c1()
    y, w = gm.sites, gm.weights
    th = np.stack([(y ** 2).sum(1) - w, -2 * y[:, 0], -2 * y[:, 1]], 1)
    ref, nc, _ = orc.assign(th, gm.H, gm.W, 1, gm.labels)
    outs, cnt = ctx.assign([problem(pdl, gm.labels, gm.H, gm.W, gm.N, 1, 1e-2)], [dev(th)])
    assert np.array_equal(outs[0].cpu().numpy(), ref) and int(cnt[0]) == nc
    # power-of-two scaling leaves F unchanged bit for bit (Lemma 4.1)
    outs2, _ = ctx.assign([problem(pdl, gm.labels, gm.H, gm.W, gm.N, 1, 1e-2)], [dev(th * 2.0**-9)])
    assert torch.equal(outs[0], outs2[0])


# ------------------------------------------------------------------ objective --

CASES = [  # H, W, N, d, eps, theta scale, seed
    (4, 5, 2, 1, 0.1, 1.0, 0),
    (31, 67, 9, 2, 0.05, 0.5, 1),
    (64, 64, 64, 3, 0.02, 0.3, 2),
    (50, 130, 65, 4, 1e-2, 0.2, 3),
    (23, 300, 130, 6, 1e-2, 0.1, 4),
    (9, 20, 5, 8, 0.5, 1.0, 5),
]


@pytest.mark.parametrize("H,W,N,d,eps,scale,seed", CASES)
def test_objective_grad_fp64(pd, orc, H, W, N, d, eps, scale, seed):
    pdl, ctx = pd
    rng = np.random.default_rng(seed)
    th = synth.random_theta(N, d, rng, scale=scale, multi_index=orc.multi_index(d))
    lab = synth.random_labels(H, W, N, rng)
    phi_ref, g_ref = orc.objective_grad(th, lab, H, W, d, eps)
    phi, grads = ctx.objective_grad([problem(pdl, lab, H, W, N, d, eps)], [dev(th)], "fp64")
    phi = float(phi[0])
    g = grads[0].cpu().numpy()
    assert rel_err(phi, phi_ref) <= 1e-10, (phi, phi_ref)
    assert grad_err(g, g_ref) <= 1e-10


@pytest.mark.parametrize("H,W,N,d,eps,scale,seed", CASES)
def test_objective_grad_fp32(pd, orc, H, W, N, d, eps, scale, seed):
    pdl, ctx = pd
    rng = np.random.default_rng(seed)
    th = synth.random_theta(N, d, rng, scale=scale, multi_index=orc.multi_index(d))
    lab = synth.random_labels(H, W, N, rng)
    phi_ref, g_ref = orc.objective_grad(th, lab, H, W, d, eps)
    phi, grads = ctx.objective_grad([problem(pdl, lab, H, W, N, d, eps)], [dev(th)], "fp32")
    ep, eg = rel_err(float(phi[0]), phi_ref), grad_err(grads[0].cpu().numpy(), g_ref)
    print(f"fp32 H={H} W={W} N={N} d={d}: phi rel {ep:.2e} grad rel {eg:.2e}")
    assert ep <= 2e-3 and eg <= 2e-3


def test_phi_zero_and_gradient_sum(pd, orc):
    """Phi(0) = -log N; sum_i grad_i = 0; gauge invariance (Lemma 4.2) on the GPU."""
    pdl, ctx = pd
    gm = synth.config_c2()
    H, W, N, d, eps = gm.H, gm.W, gm.N, 2, 1e-2
    p = problem(pdl, gm.labels, H, W, N, d, eps)
    phi, g = ctx.objective_grad([p], [dev(np.zeros((N, 6)))], "fp64")
    assert abs(float(phi[0]) + np.log(N)) <= 1e-13 * np.log(N)
    rng = np.random.default_rng(7)
    th = synth.random_theta(N, d, rng, scale=0.2, multi_index=orc.multi_index(d))
    phi1, g1 = ctx.objective_grad([p], [dev(th)], "fp64")
    phi2, g2 = ctx.objective_grad([p], [dev(th + rng.normal(size=6))], "fp64")
    g1 = g1[0].cpu().numpy()
    assert abs(float(phi1[0]) - float(phi2[0])) <= 1e-12 * abs(float(phi1[0]))
    assert np.max(np.abs(g1.sum(0))) <= 1e-11 * np.max(np.abs(g1))
    phi_ref, g_ref = orc.objective_grad(th, gm.labels, H, W, d, eps)
    assert rel_err(float(phi1[0]), phi_ref) <= 1e-10
    assert grad_err(g1, g_ref) <= 1e-10


def test_mid_fit_iterates_fp64_fp32(pd, orc):
    """Parity along an oracle L-BFGS trajectory of the c1 power-diagram map."""
    pdl, ctx = pd
    gm = synth.config_c1()
    H, W, N, d, eps = gm.H, gm.W, gm.N, 1, 1e-2
    obj = lambda t: orc.objective_grad(t, gm.labels, H, W, d, eps)
    its = []
    orc.lbfgs_fit(obj, np.zeros((N, 3)), max_iter=40, callback=lambda k, x, f, a: its.append(x.copy()))
    p = problem(pdl, gm.labels, H, W, N, d, eps)
    for th in its[::8]:
        phi_ref, g_ref = obj(th)
        phi, g = ctx.objective_grad([p], [dev(th)], "fp64")
        assert rel_err(float(phi[0]), phi_ref) <= 1e-10
        assert grad_err(g[0].cpu().numpy(), g_ref) <= 1e-10
        phi, g = ctx.objective_grad([p], [dev(th)], "fp32")
        assert rel_err(float(phi[0]), phi_ref) <= 2e-3
        assert grad_err(g[0].cpu().numpy(), g_ref) <= 2e-3


def test_batched_equals_single_and_deterministic(pd, orc):
    pdl, ctx = pd
    rng = np.random.default_rng(11)
    probs, ths = [], []
    for (H, W, N, d) in [(30, 40, 5, 1), (64, 100, 70, 3), (17, 257, 130, 2), (50, 50, 3, 5)]:
        lab = synth.random_labels(H, W, N, rng)
        probs.append(problem(pdl, lab, H, W, N, d, 0.05))
        ths.append(dev(synth.random_theta(N, d, rng, scale=0.3, multi_index=orc.multi_index(d))))
    for prec in ("fp64", "fp32"):
        phi_b, g_b = ctx.objective_grad(probs, ths, prec)
        phi_b2, g_b2 = ctx.objective_grad(probs, ths, prec)
        assert torch.equal(phi_b, phi_b2) and all(torch.equal(a, b) for a, b in zip(g_b, g_b2))
        for k, (p, t) in enumerate(zip(probs, ths)):
            phi_s, g_s = ctx.objective_grad([p], [t], prec)
            assert torch.equal(phi_s[0], phi_b[k]) and torch.equal(g_s[0], g_b[k])
    outs_b, cnt_b = ctx.assign(probs, ths)
    for k, (p, t) in enumerate(zip(probs, ths)):
        outs_s, cnt_s = ctx.assign([p], [t])
        assert torch.equal(outs_s[0], outs_b[k]) and int(cnt_s[0]) == int(cnt_b[k])


def test_objective_without_gradient(pd, orc):
    pdl, ctx = pd
    rng = np.random.default_rng(12)
    H, W, N, d = 40, 44, 12, 2
    lab = synth.random_labels(H, W, N, rng)
    th = synth.random_theta(N, d, rng, multi_index=orc.multi_index(d))
    phi, g = ctx.objective_grad([problem(pdl, lab, H, W, N, d, 0.1)], [dev(th)], "fp64", grad=False)
    assert g is None
    assert rel_err(float(phi[0]), orc.objective_grad(th, lab, H, W, d, 0.1, grad=False)[0]) <= 1e-10


# ------------------------------------------------------------------ errors ------

def test_invalid_arguments_rejected(pd):
    pdl, ctx = pd
    lab = dev(np.zeros(16), torch.int32)
    bad = [(1, 1, 0.1),              # N < 2
           (3, 0, 0.1),              # degree 0
           (3, 9, 0.1),              # degree > 8
           (3, 1, 0.0),              # eps = 0
           (3, 1, float("nan"))]     # eps not finite
    for N, d, eps in bad:
        p = pdl.Problem(lab, 4, 4, N, d, eps)
        th = dev(np.zeros((N, max(pdl.num_features(d), 1))))
        with pytest.raises(pdl.PdError) as e:
            ctx.objective_grad([p], [th], "fp64")
        assert e.value.status == 1
        with pytest.raises(pdl.PdError):
            ctx.assign([p], [th])


def test_validate_labels(pd):
    pdl, ctx = pd
    lab = np.zeros(100, np.int32)
    ctx.validate([problem(pdl, lab, 10, 10, 2, 1, 0.1)])
    lab[57] = 2
    with pytest.raises(pdl.PdError):
        ctx.validate([problem(pdl, lab, 10, 10, 2, 1, 0.1)])
    lab[57] = -1
    with pytest.raises(pdl.PdError):
        ctx.validate([problem(pdl, lab, 10, 10, 2, 1, 0.1)])


# ------------------------------------------------------------------ BF16 -------

BF16_CASES = [  # H, W, N, d, eps, theta scale, seed
    (4, 5, 2, 1, 0.1, 1.0, 0),
    (31, 67, 9, 2, 0.05, 0.5, 1),
    (64, 64, 64, 3, 0.02, 0.3, 2),
    (50, 130, 65, 4, 1e-2, 0.2, 3),
    (23, 300, 130, 6, 1e-2, 0.1, 4),
    (40, 41, 200, 5, 1e-3, 0.05, 5),
    (17, 33, 300, 4, 1e-3, 0.02, 6),
]


@pytest.mark.parametrize("H,W,N,d,eps,scale,seed", BF16_CASES)
def test_objective_grad_bf16(pd, orc, H, W, N, d, eps, scale, seed):
    """Matrix-core path (three-piece BF16 logits, two-piece gradient product,
    FP32 accumulation) against the FP64 oracle at the reduced-precision bound."""
    pdl, ctx = pd
    rng = np.random.default_rng(seed)
    th = synth.random_theta(N, d, rng, scale=scale, multi_index=orc.multi_index(d))
    lab = synth.random_labels(H, W, N, rng)
    phi_ref, g_ref = orc.objective_grad(th, lab, H, W, d, eps)
    phi, grads = ctx.objective_grad([problem(pdl, lab, H, W, N, d, eps)], [dev(th)], "bf16")
    ep, eg = rel_err(float(phi[0]), phi_ref), grad_err(grads[0].cpu().numpy(), g_ref)
    print(f"bf16 H={H} W={W} N={N} d={d} eps={eps}: phi rel {ep:.2e} grad rel {eg:.2e}")
    assert ep <= 2e-3 and eg <= 2e-3


def test_bf16_polynomial_map_eps_1e3(pd, orc):
    """A degree-4 polynomial-diagram map at eps = 1e-3 near its generating theta:
    logits of size ~1e3 with sharp boundaries."""
    pdl, ctx = pd
    rng = np.random.default_rng(21)
    gm = synth.polynomial_diagram(96, 160, 120, 4, rng)
    th = synth.coef_to_theta(gm.coef, orc.multi_index(4))
    th = th + rng.normal(size=th.shape) * 1e-4
    phi_ref, g_ref = orc.objective_grad(th, gm.labels, gm.H, gm.W, 4, 1e-3)
    p = problem(pdl, gm.labels, gm.H, gm.W, gm.N, 4, 1e-3)
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-3), ("bf16", 2e-3)):
        phi, g = ctx.objective_grad([p], [dev(th)], prec)
        ep, eg = rel_err(float(phi[0]), phi_ref), grad_err(g[0].cpu().numpy(), g_ref)
        print(f"{prec}: phi rel {ep:.2e} grad rel {eg:.2e}")
        assert ep <= tol and eg <= tol, prec


def test_bf16_batched_and_degree_limit(pd, orc):
    pdl, ctx = pd
    rng = np.random.default_rng(22)
    probs, ths, refs = [], [], []
    for (H, W, N, d) in [(30, 40, 5, 2), (64, 100, 70, 3), (17, 257, 130, 4)]:
        lab = synth.random_labels(H, W, N, rng)
        th = synth.random_theta(N, d, rng, scale=0.3, multi_index=orc.multi_index(d))
        probs.append(problem(pdl, lab, H, W, N, d, 0.05))
        ths.append(dev(th))
        refs.append(orc.objective_grad(th, lab, H, W, d, 0.05))
    phi, g = ctx.objective_grad(probs, ths, "bf16")
    for k, (pr, gr) in enumerate(refs):
        assert rel_err(float(phi[k]), pr) <= 2e-3 and grad_err(g[k].cpu().numpy(), gr) <= 2e-3
        phi_s, g_s = ctx.objective_grad([probs[k]], [ths[k]], "bf16")
        assert torch.equal(phi_s[0], phi[k]) and torch.equal(g_s[0], g[k])
    lab = np.zeros(100, np.int32)
    with pytest.raises(pdl.PdError) as e:
        ctx.objective_grad([problem(pdl, lab, 10, 10, 3, 7, 0.1)], [dev(np.zeros((3, 36)))], "bf16")
    assert e.value.status == 2
