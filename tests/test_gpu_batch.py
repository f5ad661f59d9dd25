"""Batched maps of uneven size, grain count and degree in single launches
(the 64-map workload's pattern at test sizes), and the autotuner."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.fixture(scope="module")
def batch():
    return synth.batch_maps(4040, 6, hw=(40, 161), grains=(10, 151))


def problems(pdl, maps):
    return [pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, gm.meta["degree"],
                        gm.meta["eps"]) for gm in maps]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-3), ("bf16", 2e-3)])
def test_batched_objective_matches_oracle(pd, orc, batch, prec, tol):
    pdl, ctx = pd
    probs = problems(pdl, batch)
    rng = np.random.default_rng(5)
    ths = []
    for gm in batch:
        d = gm.meta["degree"]
        th = synth.coef_to_theta(gm.coef, orc.multi_index(d)) if gm.coef is not None else \
            synth.random_theta(gm.N, d, rng, scale=0.2, multi_index=orc.multi_index(d))
        ths.append(th + rng.normal(size=th.shape) * 1e-3)
    phi, g = ctx.objective_grad(probs, [dev(t) for t in ths], prec)
    for k, gm in enumerate(batch):
        d, eps = gm.meta["degree"], gm.meta["eps"]
        pr, gr = orc.objective_grad(ths[k], gm.labels, gm.H, gm.W, d, eps)
        ep = abs(float(phi[k]) - pr) / abs(pr)
        eg = float(np.max(np.abs(g[k].cpu().numpy() - gr)) / np.max(np.abs(gr)))
        print(f"{prec} map {k} ({gm.H}x{gm.W} N={gm.N} d={d}): phi {ep:.1e} grad {eg:.1e}")
        assert ep <= tol and eg <= tol


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batched_fit_equals_individual_fits(pd, orc, batch, prec):
    """One pd_fit over the whole batch (one launch per kernel per step, converged
    maps gated off) gives each map exactly the result of fitting it alone."""
    pdl, ctx = pd
    probs = problems(pdl, batch)
    ths = [dev(np.zeros((gm.N, pdl.num_features(gm.meta["degree"])))) for gm in batch]
    reps = ctx.fit(probs, ths, prec, init="zero", max_iter=150, target_acc=0.95)
    for k, gm in enumerate(batch):
        t1 = dev(np.zeros((gm.N, pdl.num_features(gm.meta["degree"]))))
        r1 = ctx.fit([probs[k]], [t1], prec, init="zero", max_iter=150, target_acc=0.95)[0]
        assert torch.equal(t1, ths[k]), k
        assert (r1["iters"], r1["evals"], r1["status"]) == (reps[k]["iters"], reps[k]["evals"],
                                                           reps[k]["status"])
        _, nc, _ = orc.assign(ths[k].cpu().numpy(), gm.H, gm.W, gm.meta["degree"], gm.labels)
        assert nc == round(reps[k]["acc"] * gm.H * gm.W)


def test_autotune_picks_candidate_and_keeps_parity(orc, batch):
    import paper_2605_20816_amd as pdl
    ctx = pdl.Context(0)   # own context: the tuned choice stays local to it
    probs = problems(pdl, batch)
    rng = np.random.default_rng(6)
    ths = [synth.random_theta(gm.N, gm.meta["degree"], rng, scale=0.2,
                              multi_index=orc.multi_index(gm.meta["degree"])) for gm in batch]
    for prec in ("fp32", "bf16"):
        w = ctx.autotune(probs, [dev(t) for t in ths], prec)
        assert w in (1024, 2048, 4096, 8192, 16384, 32768, 65536)
        phi, g = ctx.objective_grad(probs, [dev(t) for t in ths], prec)
        for k, gm in enumerate(batch):
            pr, gr = orc.objective_grad(ths[k], gm.labels, gm.H, gm.W, gm.meta["degree"],
                                        gm.meta["eps"])
            assert abs(float(phi[k]) - pr) <= 2e-3 * abs(pr)
            assert np.max(np.abs(g[k].cpu().numpy() - gr)) <= 2e-3 * np.max(np.abs(gr))
    ctx.close()


def test_bf16_batch_mixing_degree_3_and_6(pd, orc):
    """A BF16 batch whose degree-3 map has N a multiple of 64 (its last grain is the
    last row of its parameter pieces) next to a degree-6 map: the matrix-core
    kernels run two 16-feature blocks for the whole batch, and the degree-3 map
    must read zero padding there.  Batched results equal single-map results bit
    for bit and match the oracle."""
    pdl, ctx = pd
    rng = np.random.default_rng(77)
    specs = [(48, 70, 128, 3, 1e-2), (53, 61, 70, 6, 1e-2), (40, 64, 64, 4, 1e-2)]
    probs, ths, labs = [], [], []
    for H, W, N, d, eps in specs:
        lab = synth.random_labels(H, W, N, rng)
        th = synth.random_theta(N, d, rng, scale=0.05, multi_index=orc.multi_index(d))
        labs.append(lab)
        ths.append(th)
        probs.append(pdl.Problem(dev(lab, torch.int32), H, W, N, d, eps))
    phi, g = ctx.objective_grad(probs, [dev(t) for t in ths], "bf16")
    for k, (H, W, N, d, eps) in enumerate(specs):
        p1, g1 = ctx.objective_grad([probs[k]], [dev(ths[k])], "bf16")
        assert float(p1[0]) == float(phi[k]) and torch.equal(g1[0], g[k]), k
        pr, gr = orc.objective_grad(ths[k], labs[k], H, W, d, eps)
        ep = abs(float(phi[k]) - pr) / abs(pr)
        eg = float(np.max(np.abs(g[k].cpu().numpy() - gr)) / np.max(np.abs(gr)))
        print(f"bf16 mixed batch map {k} (d={d}, N={N}): phi {ep:.1e} grad {eg:.1e}")
        assert ep <= 2e-3 and eg <= 2e-3
        assert np.isfinite(g[k].cpu().numpy()).all()
