"""Parity at the full sizes of the benchmarked workloads, in the launch
configurations bench.py times, against the FP64 oracle:

* the 256x256 c2 map after the fit steps of a run and at a fitted (>= 99%
  accuracy) iterate;
* the 16-map c4-style batch under its autotuned tiles, and all 64 maps of the
  c4 workload as one batch (row bands);
* the 1024x1024 degree-4 c3 map after 20 FP32 iterations and at a fitted
  iterate (row bands there: the oracle's cost);
* the 2048x2048 degree-6 c5 map (N = 4895) in row bands of 8 rows at the top,
  middle and bottom, after 20 FP32 iterations: FP64, FP32 (both gradient forms)
  and BF16, and the assignment of those rows bit for bit.

Gradients are compared entry by entry: max |g - g_ref| / max |g_ref|.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 2e-3, "bf16": 2e-3}


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def rel(a, b):
    return abs(a - b) / abs(b)


def gerr(g, gr):
    """Largest entry error relative to the largest reference entry."""
    return float(np.max(np.abs(g - gr)) / np.max(np.abs(gr)))


def check(ctx, orc, probs, maps, ths, prec, tol_phi, tol_g):
    phi, grads = ctx.objective_grad(probs, [dev(t) for t in ths], prec)
    outs, cnt = ctx.assign(probs, [dev(t) for t in ths])
    for k, (gm, p, th) in enumerate(zip(maps, probs, ths)):
        phi_ref, g_ref = orc.objective_grad(th, gm.labels, p.H, p.W, p.d, p.eps)
        ep, eg = rel(float(phi[k]), phi_ref), gerr(grads[k].cpu().numpy(), g_ref)
        print(f"{prec} map {k} ({p.H}x{p.W} N={p.N} d={p.d}): phi {ep:.1e} grad {eg:.1e}")
        assert ep <= tol_phi, (k, prec)
        assert eg <= tol_g, (k, prec)
        F, nc, _ = orc.assign(th, p.H, p.W, p.d, gm.labels)
        assert np.array_equal(outs[k].cpu().numpy(), F) and int(cnt[k]) == nc, k


def check_bands(ctx, orc, p, gm, th, bands, precs, fit_form=False):
    """Row bands of one map against the oracle's sums over the same rows."""
    n = p.H * p.W
    refs = {}
    for r0, r1 in bands:
        v, g = orc.objective_rows(th, gm.labels, p.H, p.W, p.d, p.eps, r0, r1)
        refs[(r0, r1)] = (v / n, -g / (p.eps * n))
    for prec in precs:
        for form in ((False, True) if fit_form and prec != "bf16" else (False,)):
            for r0, r1 in bands:
                phi, g = ctx.objective_grad_rows([p], [dev(th)], [(r0, r1)], prec,
                                                 onehot_precomputed=form)
                pr, gr = refs[(r0, r1)]
                ep, eg = rel(float(phi[0]), pr), gerr(g[0].cpu().numpy(), gr)
                print(f"{p.H}x{p.W} {prec}{' fit form' if form else ''} rows [{r0},{r1}): "
                      f"phi {ep:.1e} grad {eg:.1e}")
                assert ep <= TOL[prec] and eg <= TOL[prec], (prec, form, r0)
    outs, _ = ctx.assign([p], [dev(th)])
    F = outs[0].cpu().numpy()
    for r0, r1 in bands:
        Fb, _, nn = orc.assign_rows(th, p.H, p.W, p.d, r0, r1, gm.labels)
        assert nn == 0 and np.array_equal(F[r0 * p.W:r1 * p.W], Fb), r0


def test_c2_after_benchmark_steps_and_at_the_fit(pd, orc):
    pdl, ctx = pd
    gm = synth.config_c2()
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 2, 1e-2)
    th = torch.zeros((gm.N, 6), dtype=torch.float64, device="cuda")
    ctx.fit([p], [th], "fp32", init="zero", max_iter=300, target_acc=2.0)
    x = th.cpu().numpy()
    check(ctx, orc, [p], [gm], [x], "fp64", 1e-10, 1e-10)
    check(ctx, orc, [p], [gm], [x], "fp32", 2e-3, 2e-3)
    # a fitted iterate (>= 99% accuracy), where p - delta cancels most: the
    # preconditioned FP32 fit gets there in about 1600 iterations (the plain FP64
    # fit needs about 2700 on this noisy map)
    th = torch.zeros((gm.N, 6), dtype=torch.float64, device="cuda")
    rep = ctx.fit([p], [th], "fp32", init="zero", max_iter=4000, target_acc=0.99, history=16,
                  precondition=40, check_every=8)[0]
    print(f"c2 fit: {rep['iters']} iterations, acc {rep['acc']:.4f}")
    assert rep["status"] == "target"
    x = th.cpu().numpy()
    for prec in ("fp64", "fp32", "bf16"):
        check(ctx, orc, [p], [gm], [x], prec, TOL[prec], TOL[prec])
    check_bands(ctx, orc, p, gm, x, [(0, gm.H)], ("fp64", "fp32"), fit_form=True)


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
    ctx.close()


def test_c4_all_64_maps_in_one_batch(orc):
    """The whole 64-map c4 workload as one batch under autotuned tiles, after 30
    batched FP32 iterations: per map a band of 4 rows at the top and one in the
    middle (the oracle's cost), FP64/FP32 in both gradient forms and BF16, and
    those rows' assignment bit for bit."""
    import paper_2605_20816_amd as pdl
    ctx = pdl.Context(0)
    maps = [synth.config_c4_map(j) for j in range(64)]
    probs = [pdl.Problem(dev(g.labels, torch.int32), g.H, g.W, g.N, g.meta["degree"],
                         g.meta["eps"]) for g in maps]
    ths = [torch.zeros((p.N, pdl.num_features(p.d)), dtype=torch.float64, device="cuda")
           for p in probs]
    assert ctx.autotune(probs, ths, "fp32") > 0
    reps = ctx.fit(probs, ths, "fp32", init="zero", max_iter=30, target_acc=2.0, history=16,
                   precondition=20)
    assert all(r["iters"] > 0 for r in reps)
    xs = [t.cpu().numpy() for t in ths]
    for band_of in (lambda g: (0, 4), lambda g: (g.H // 2, g.H // 2 + 4)):
        bands = [band_of(g) for g in maps]
        refs = []
        for g, p, x, (r0, r1) in zip(maps, probs, xs, bands):
            v, gr = orc.objective_rows(x, g.labels, p.H, p.W, p.d, p.eps, r0, r1)
            n = p.H * p.W
            refs.append((v / n, -gr / (p.eps * n)))
        for prec, forms in (("fp64", (False, True)), ("fp32", (False, True)), ("bf16", (False,))):
            for form in forms:
                phi, gs = ctx.objective_grad_rows(probs, ths, bands, prec, onehot_precomputed=form)
                worst = 0.0
                for k, (pr, gr) in enumerate(refs):
                    ep, eg = rel(float(phi[k]), pr), gerr(gs[k].cpu().numpy(), gr)
                    worst = max(worst, ep, eg)
                    assert ep <= TOL[prec] and eg <= TOL[prec], (k, prec, form, bands[k])
                print(f"64 maps {prec}{' fit form' if form else ''} rows {bands[0]}..: worst {worst:.1e}")
        outs, _ = ctx.assign(probs, ths)
        for k, (g, p, x, (r0, r1)) in enumerate(zip(maps, probs, xs, bands)):
            Fb, _, nn = orc.assign_rows(x, p.H, p.W, p.d, r0, r1, g.labels)
            assert nn == 0 and np.array_equal(outs[k].cpu().numpy()[r0 * p.W:r1 * p.W], Fb), k
    ctx.close()


def test_c3_full_map(pd, orc):
    pdl, ctx = pd
    gm = synth.config_c3()
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 4, 1e-3)
    th = torch.zeros((gm.N, 15), dtype=torch.float64, device="cuda")
    ctx.fit([p], [th], "fp32", init="zero", max_iter=20, target_acc=2.0)
    x = th.cpu().numpy()
    phi_ref, g_ref = orc.objective_grad(x, gm.labels, gm.H, gm.W, 4, 1e-3)
    F, nc, _ = orc.assign(x, gm.H, gm.W, 4, gm.labels)
    for prec in ("fp64", "fp32", "bf16"):
        phi, g = ctx.objective_grad([p], [th], prec)
        ep, eg = rel(float(phi[0]), phi_ref), gerr(g[0].cpu().numpy(), g_ref)
        print(f"c3 {prec}: phi {ep:.1e} grad {eg:.1e}")
        assert ep <= TOL[prec] and eg <= TOL[prec], prec
    outs, cnt = ctx.assign([p], [th])
    assert np.array_equal(outs[0].cpu().numpy(), F) and int(cnt[0]) == nc


def test_c3_at_the_fit(pd, orc):
    """A fitted c3 iterate (FP32 fit with the diagonal preconditioner to 99%:
    about 2200 iterations with memory 32 and the diagonal refreshed every 10)."""
    pdl, ctx = pd
    gm = synth.config_c3()
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 4, 1e-3)
    th = torch.zeros((gm.N, 15), dtype=torch.float64, device="cuda")
    rep = ctx.fit([p], [th], "fp32", init="zero", max_iter=5000, target_acc=0.99,
                  history=32, precondition=10)[0]
    print(f"c3 fit: {rep['iters']} iterations, acc {rep['acc']:.4f}")
    assert rep["status"] == "target"
    bands = [(0, 8), (508, 516), (1016, 1024)]
    check_bands(ctx, orc, p, gm, th.cpu().numpy(), bands, ("fp64", "fp32", "bf16"), fit_form=True)


def test_c5_row_bands(pd, orc):
    """The 2048x2048 degree-6 map: bands of 8 rows after 20 FP32 iterations; the
    whole map's FP64 evaluation equals the sum of a partition into bands, and its
    gradient sums to zero over the grains (Lemma 4.2)."""
    pdl, ctx = pd
    gm = synth.config_c5()
    assert gm.N == 4895
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 6, 1e-3)
    th = torch.zeros((gm.N, 28), dtype=torch.float64, device="cuda")
    ctx.fit([p], [th], "fp32", init="zero", max_iter=20, target_acc=2.0)
    x = th.cpu().numpy()
    bands = [(0, 8), (1020, 1028), (2040, 2048)]
    check_bands(ctx, orc, p, gm, x, bands, ("fp64", "fp32", "bf16"), fit_form=True)
    phi, g = ctx.objective_grad([p], [th], "fp64")
    parts = [(0, 500), (500, 1024), (1024, 1025), (1025, 2048)]
    tp, tg = 0.0, 0.0
    for r in parts:
        ph, gb = ctx.objective_grad_rows([p], [th], [r], "fp64")
        tp += float(ph[0])
        tg = tg + gb[0]
    assert rel(tp, float(phi[0])) <= 1e-12
    assert gerr(tg.cpu().numpy(), g[0].cpu().numpy()) <= 1e-12
    gs = g[0].sum(dim=0).abs().max().item()
    assert gs <= 1e-10 * g[0].abs().max().item()
