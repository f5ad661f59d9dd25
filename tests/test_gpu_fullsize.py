"""Parity at the full sizes of the benchmarked workloads, in the launch
configurations bench.py times: the 256x256 c2 map after the benchmark's FP32 fit
steps, the 16-map c4-style batch under its autotuned tiles, and the 1024x1024
degree-4 c3 map (BF16 matrix cores, FP32, FP64), each against the FP64 oracle."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def rel(a, b):
    return abs(a - b) / abs(b)


def gerr(g, gr):
    return np.linalg.norm(g - gr) / np.linalg.norm(gr)


def check(ctx, orc, probs, maps, ths, prec, tol_phi, tol_g):
    phi, grads = ctx.objective_grad(probs, [dev(t) for t in ths], prec)
    outs, cnt = ctx.assign(probs, [dev(t) for t in ths])
    for k, (gm, p, th) in enumerate(zip(maps, probs, ths)):
        phi_ref, g_ref = orc.objective_grad(th, gm.labels, p.H, p.W, p.d, p.eps)
        assert rel(float(phi[k]), phi_ref) <= tol_phi, (k, prec)
        assert gerr(grads[k].cpu().numpy(), g_ref) <= tol_g, (k, prec)
        F, nc, _ = orc.assign(th, p.H, p.W, p.d, gm.labels)
        assert np.array_equal(outs[k].cpu().numpy(), F) and int(cnt[k]) == nc, k


def test_c2_after_benchmark_steps(pd, orc):
    pdl, ctx = pd
    gm = synth.config_c2()
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 2, 1e-2)
    th = torch.zeros((gm.N, 6), dtype=torch.float64, device="cuda")
    ctx.fit([p], [th], "fp32", init="zero", max_iter=300, target_acc=2.0)
    x = th.cpu().numpy()
    check(ctx, orc, [p], [gm], [x], "fp64", 1e-10, 1e-10)
    check(ctx, orc, [p], [gm], [x], "fp32", 2e-3, 2e-3)


def test_c4_batch_autotuned(orc):
    import paper_2605_20816_amd as pdl
    ctx = pdl.Context(0)
    maps = [synth.config_c4_map(j) for j in range(16)]
    probs = [pdl.Problem(dev(g.labels, torch.int32), g.H, g.W, g.N, g.meta["degree"],
                         g.meta["eps"]) for g in maps]
    zeros = [torch.zeros((p.N, pdl.num_features(p.d)), dtype=torch.float64, device="cuda")
             for p in probs]
    assert ctx.autotune(probs, zeros, "fp32") > 0
    assert ctx.autotune(probs, zeros, "bf16") > 0
    ctx.fit(probs, zeros, "fp32", init="zero", max_iter=30, target_acc=2.0, history=16,
            precondition=20)
    ths = [z.cpu().numpy() for z in zeros]
    check(ctx, orc, probs, maps, ths, "fp64", 1e-10, 1e-10)
    check(ctx, orc, probs, maps, ths, "fp32", 2e-3, 2e-3)
    check(ctx, orc, probs, maps, ths, "bf16", 2e-3, 2e-3)


def test_c3_full_map(pd, orc):
    pdl, ctx = pd
    gm = synth.config_c3()
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 4, 1e-3)
    th = torch.zeros((gm.N, 15), dtype=torch.float64, device="cuda")
    ctx.fit([p], [th], "fp32", init="zero", max_iter=20, target_acc=2.0)
    x = th.cpu().numpy()
    phi_ref, g_ref = orc.objective_grad(x, gm.labels, gm.H, gm.W, 4, 1e-3)
    F, nc, _ = orc.assign(x, gm.H, gm.W, 4, gm.labels)
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-3), ("bf16", 2e-3)):
        phi, g = ctx.objective_grad([p], [th], prec)
        assert rel(float(phi[0]), phi_ref) <= tol, prec
        assert gerr(g[0].cpu().numpy(), g_ref) <= tol, prec
    outs, cnt = ctx.assign([p], [th])
    assert np.array_equal(outs[0].cpu().numpy(), F) and int(cnt[0]) == nc
