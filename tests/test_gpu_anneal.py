"""GPU parity of the eps schedule of pd_fit (annealing with Err-aligned stopping)
against the oracle's annealed_fit: the same levels, budgets and iterates."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _oracle(orc, gm, d, eps, **kw):
    obj_e = lambda th, e: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, e)
    acc = lambda th: orc.assign(th, gm.H, gm.W, d, gm.labels)[1] / (gm.H * gm.W)
    return orc.annealed_fit(obj_e, np.zeros((gm.N, orc.num_features(d))), eps, accuracy=acc, **kw)


def test_levels_match_oracle(pd, orc):
    """Three levels of 5 iterations each (eps * 64, eps * 8, eps), target out of
    reach: the device fit takes the oracle's iterates level after level."""
    pdl, ctx = pd
    gm = synth.polynomial_diagram(40, 48, 9, 2, np.random.default_rng(41))
    d, eps = 2, 1e-3
    ref = _oracle(orc, gm, d, eps, stages=2, factor=8.0, stage_iters=5, target_acc=2.0,
                  max_iter=15)
    th = dev(np.zeros((gm.N, 6)))
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, d, eps)
    rep = ctx.fit([p], [th], "fp64", init="zero", max_iter=15, target_acc=2.0,
                  anneal=(2, 8.0, 5))[0]
    print("device", rep, "oracle levels", ref["levels"])
    assert [v["iters"] for v in ref["levels"]] == [5, 5, 5]
    assert rep["iters"] == ref["iters"] == 15
    assert rep["evals"] == ref["evals"]
    x = th.cpu().numpy()
    assert np.max(np.abs(x - ref["theta"])) <= 1e-7 * np.max(np.abs(ref["theta"]))
    assert abs(rep["phi"] - ref["phi"]) <= 1e-9 * abs(ref["phi"])
    assert rep["status"] == "budget"


def test_err_aligned_stop(pd, orc):
    """The c1 power-diagram map with a schedule (eps * 16, eps * 4, eps): the fit
    stops at the first iterate of any level with >= 99% accuracy, close to where
    the oracle stops; Phi is reported at the map's own eps."""
    pdl, ctx = pd
    gm = synth.config_c1()
    d, eps = 1, 1e-2
    ref = _oracle(orc, gm, d, eps, stages=2, factor=4.0, stage_iters=40, target_acc=0.99,
                  max_iter=2000)
    th = dev(np.zeros((gm.N, 3)))
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, d, eps)
    rep = ctx.fit([p], [th], "fp64", init="zero", max_iter=2000, target_acc=0.99,
                  anneal=(2, 4.0, 40))[0]
    print("device", rep, "oracle", ref["iters"], ref["levels"])
    assert ref["status"] == "target" and rep["status"] == "target"
    assert abs(rep["iters"] - ref["iters"]) <= 2
    x = th.cpu().numpy()
    _, nc, _ = orc.assign(x, gm.H, gm.W, d, gm.labels)
    assert nc / (gm.H * gm.W) == rep["acc"] >= 0.99
    phi = orc.objective_grad(x, gm.labels, gm.H, gm.W, d, eps, grad=False)[0]
    assert abs(rep["phi"] - phi) <= 1e-10 * abs(phi)
    assert rep["seconds_to_target"] > 0


def test_batched_annealing_equals_single(pd):
    """A map's annealed fit does not depend on its batch (the maps that stop at a
    level leave the later levels' batches)."""
    pdl, ctx = pd
    maps = [synth.polynomial_diagram(64, 80, 12, 2, np.random.default_rng(50 + k)) for k in range(3)]
    probs = [pdl.Problem(dev(g.labels, torch.int32), g.H, g.W, g.N, 2, 1e-3) for g in maps]
    ths = [dev(np.zeros((g.N, 6))) for g in maps]
    reps = ctx.fit(probs, ths, "fp64", init="zero", max_iter=300, target_acc=0.98,
                   anneal=(2, 8.0, 20))
    for k, g in enumerate(maps):
        t1 = dev(np.zeros((g.N, 6)))
        r1 = ctx.fit([probs[k]], [t1], "fp64", init="zero", max_iter=300, target_acc=0.98,
                     anneal=(2, 8.0, 20))[0]
        assert r1["iters"] == reps[k]["iters"] and r1["status"] == reps[k]["status"]
        assert torch.equal(t1, ths[k])
