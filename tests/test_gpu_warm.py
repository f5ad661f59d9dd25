"""GPU parity of the warm-start kernels (descriptors, moment seed, targets,
network forward / backward / Adam, scale search) against oracle/warm.py."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import warm

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def maps_for_warm():
    rng = np.random.default_rng(77)
    out = [(synth.config_c1(), 1, 1e-2),
           (synth.anisotropic_power_diagram(50, 70, 12, rng), 2, 1e-2),
           (synth.polynomial_diagram(64, 41, 15, 4, rng), 4, 1e-3),
           (synth.polynomial_diagram(33, 90, 9, 6, rng), 6, 1e-3)]
    # a map with an empty grain (label 3 unused) and a one-pixel grain
    lab = synth.random_labels(20, 24, 3, rng).reshape(20, 24)
    lab[5, 7] = 4
    gm = synth.GrainMap(20, 24, lab.reshape(-1).astype(np.int32), 5, "handmade", 1)
    out.append((gm, 3, 1e-2))
    return out


def problems(pdl, items):
    return [pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, d, eps)
            for gm, d, eps in items]


def test_descriptors_and_frames(pd):
    pdl, ctx = pd
    items = maps_for_warm()
    probs = problems(pdl, items)
    desc, frames = ctx.descriptors(probs, frames=True)
    desc2 = ctx.descriptors(probs)
    for (gm, d, eps), D, F, D2 in zip(items, desc, frames, desc2):
        fr = warm.grain_frames(gm.labels, gm.H, gm.W, gm.N)
        ref = warm.descriptors(gm.labels, gm.H, gm.W, gm.N, fr)
        F = F.cpu().numpy()
        assert np.array_equal(F[:, 6], fr[:, 6])                      # exact counts
        assert np.max(np.abs(F[:, :6] - fr[:, :6])) <= 1e-12 * np.max(np.abs(fr[:, :6]))
        got = D.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - ref)) <= 2e-6 * max(1.0, np.max(np.abs(ref)))
        assert torch.equal(D, D2)                                      # reproducible
        empty = fr[:, 6] == 0
        assert np.all(got[empty] == 0)


def test_heuristic_matches_oracle(pd):
    pdl, ctx = pd
    items = maps_for_warm()
    probs = problems(pdl, items)
    ths = ctx.heuristic(probs)
    for (gm, d, eps), th in zip(items, ths):
        fr = warm.grain_frames(gm.labels, gm.H, gm.W, gm.N)
        ref = warm.heuristic_theta(fr, gm.H, gm.W, d)
        got = th.cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_targets_match_oracle(pd):
    pdl, ctx = pd
    items = maps_for_warm()
    probs = problems(pdl, items)
    rng = np.random.default_rng(5)
    fits = [rng.normal(size=(gm.N, pdl.num_features(d))) * 3.0 + 0.7 for gm, d, eps in items]
    tg, lam = ctx.warm_targets(probs, [dev(f) for f in fits])
    lam = lam.cpu().numpy()
    for k, ((gm, d, eps), f) in enumerate(zip(items, fits)):
        fr = warm.grain_frames(gm.labels, gm.H, gm.W, gm.N)
        ref, rms = warm.targets(f, fr)
        assert abs(lam[k] - rms) <= 1e-12 * rms
        got = tg[k].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("batch,K", [(1, 3), (37, 6), (300, 15), (1000, 28)])
def test_mlp_forward_backward_match_oracle(pd, batch, K):
    """FP32 kernels against the FP64 oracle network: outputs, loss and every
    parameter gradient (checked with finite differences in the oracle pins)."""
    pdl, ctx = pd
    rng = np.random.default_rng(batch)
    p = warm.mlp_init(K, rng)
    x = rng.normal(size=(batch, 32)).astype(np.float32)
    t = rng.normal(size=(batch, K)).astype(np.float32)
    P, Xd, Td = dev(p), dev(x), dev(t)
    y = ctx.mlp_forward(P, Xd, K, "fp32").cpu().numpy()
    yref = warm.mlp_forward(p.astype(np.float64), x.astype(np.float64), K)
    assert np.max(np.abs(y - yref)) <= 1e-4 * max(1.0, np.max(np.abs(yref)))
    loss, g = ctx.mlp_backward(P, Xd, Td)
    lref, gref = warm.mlp_loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), K)
    assert abs(float(loss[0]) - lref) <= 1e-5 * lref
    g = g.cpu().numpy().astype(np.float64)
    # per parameter block: FP32 accumulation over the batch
    sizes = [int(np.prod(s)) for s in warm.mlp_sizes(K)]
    o = 0
    for sz in sizes:
        blk, rb = g[o:o + sz], gref[o:o + sz]
        assert np.max(np.abs(blk - rb)) <= 2e-4 * np.max(np.abs(rb)) + 1e-9, (o, sz)
        o += sz
    loss2, g2 = ctx.mlp_backward(P, Xd, Td)
    assert torch.equal(loss, loss2) and np.array_equal(g2.cpu().numpy(), g.astype(np.float32))


def test_mlp_bf16_inference(pd):
    """BF16 matrix-core inference: within bf16 rounding of the FP64 network."""
    pdl, ctx = pd
    rng = np.random.default_rng(9)
    for batch, K in ((5, 6), (333, 28), (64, 45)):
        p = warm.mlp_init(K, rng)
        x = rng.normal(size=(batch, 32)).astype(np.float32)
        y = ctx.mlp_forward(dev(p), dev(x), K, "bf16").cpu().numpy()
        yref = warm.mlp_forward(p.astype(np.float64), x.astype(np.float64), K)
        err = np.abs(y - yref)
        assert np.max(err) <= 4e-2 * np.max(np.abs(yref)), (batch, K, np.max(err))
        assert np.sqrt(np.mean(err ** 2)) <= 1e-2 * np.sqrt(np.mean(yref ** 2))


def test_adam_matches_oracle(pd):
    pdl, ctx = pd
    rng = np.random.default_rng(2)
    n = 10000
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    P, M, V = dev(p), dev(m), dev(v)
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        ctx.mlp_adam(P, dev(g), M, V, step, 1e-3)
        pr, mr, vr = warm.adam_step(pr, g.astype(np.float64), mr, vr, step, 1e-3)
    assert np.max(np.abs(P.cpu().numpy() - pr)) <= 1e-6
    assert np.max(np.abs(M.cpu().numpy() - mr)) <= 1e-6


def test_warm_start_heuristic_scale_matches_oracle(pd, orc):
    """Moment seed + scale search in FP64: the same bracketing / golden-section
    decisions as the oracle, hence the same scale."""
    pdl, ctx = pd
    items = maps_for_warm()[:3]
    probs = problems(pdl, items)
    ths, scales = ctx.warm_start(probs, None, "fp64")
    for (gm, d, eps), th, s in zip(items, ths, scales):
        fr = warm.grain_frames(gm.labels, gm.H, gm.W, gm.N)
        seed = warm.heuristic_theta(fr, gm.H, gm.W, d)
        phi = lambda sc: orc.objective_grad(sc * seed, gm.labels, gm.H, gm.W, d, eps, grad=False)[0]
        sref, vref, _ = warm.scale_search(phi, warm.initial_scale(gm.H, gm.W, gm.N, eps))
        assert s == pytest.approx(sref, rel=1e-12)
        assert np.max(np.abs(th.cpu().numpy() - sref * seed)) <= 1e-10 * np.max(np.abs(sref * seed))
        assert vref > -math.log(gm.N)


def test_warm_start_assembles_network_outputs(pd):
    """theta_hat = BF16 network outputs centred over the non-empty grains, empty
    grains on the row that wins no pixel; the returned start is s* theta_hat."""
    pdl, ctx = pd
    items = [it for it in maps_for_warm() if it[1] <= 6]
    rng = np.random.default_rng(31)
    nets = {}
    for gm, d, eps in items:
        nets.setdefault(d, dev(warm.mlp_init(pdl.num_features(d), rng) * 0.1))
    probs = problems(pdl, items)
    ths, scales = ctx.warm_start(probs, pdl.Mlp(nets), "fp32")
    desc = ctx.descriptors(probs)
    for (gm, d, eps), th, s, D in zip(items, ths, scales, desc):
        fr = warm.grain_frames(gm.labels, gm.H, gm.W, gm.N)
        y = ctx.mlp_forward(nets[d], D, pdl.num_features(d), "bf16").cpu().numpy()
        ref = warm.assemble(y.astype(np.float64), fr)
        got = th.cpu().numpy()
        if s == 0.0:
            assert np.all(got == 0)
        else:
            assert np.max(np.abs(got / s - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_warm_start_falls_back_to_zero(pd):
    """A network that predicts the reverse of a diagram (each grain's score rises
    towards its own centroid) makes every scale worse than theta = 0: the map falls
    back to the cold start."""
    pdl, ctx = pd
    gm = synth.config_c1()
    prob = problems(pdl, [(gm, 1, 1e-2)])
    K = 3
    p = torch.zeros(pdl.mlp_num_params(K), dtype=torch.float32)
    o2 = 33 * 256
    o3 = o2 + 257 * 256
    p[1 * 256 + 0] = 1.0            # hidden 0 <- mean x1 (centroid)
    p[2 * 256 + 1] = 1.0            # hidden 1 <- mean x2
    p[32 * 256 + 0] = 2.0           # biases keep GELU on its increasing branch
    p[32 * 256 + 1] = 2.0
    p[o2 + 0 * 256 + 0] = 1.0
    p[o2 + 1 * 256 + 1] = 1.0
    p[o3 + 0 * K + 1] = 1.0         # theta_i = (0, +y1, +y2) up to a common shift
    p[o3 + 1 * K + 2] = 1.0
    ths, scales = ctx.warm_start(prob, pdl.Mlp({1: p.cuda()}), "fp64")
    assert scales[0] == 0.0
    assert torch.all(ths[0] == 0)


def test_fit_from_heuristic_and_network(pd, orc):
    pdl, ctx = pd
    rng = np.random.default_rng(21)
    gm = synth.polynomial_diagram(96, 96, 20, 4, rng)
    prob = problems(pdl, [(gm, 4, 1e-3)])
    th = dev(np.zeros((gm.N, 15)))
    rep = ctx.fit(prob, [th], "fp32", init="heuristic", max_iter=1500, target_acc=0.99)[0]
    assert rep["status"] == "target"
    _, nc, _ = orc.assign(th.cpu().numpy(), gm.H, gm.W, 4, gm.labels)
    assert nc / gm.labels.size >= 0.99
    p = dev(warm.mlp_init(15, rng) * 0.01)
    th2 = dev(np.zeros((gm.N, 15)))
    rep2 = ctx.fit(prob, [th2], "fp32", init="mlp", mlp=pdl.Mlp({4: p}), max_iter=1500,
                   target_acc=0.99)[0]
    assert rep2["status"] == "target"
    assert rep2["seconds_to_target"] > 0
