"""Non-finite parameters: a NaN or an infinite entry of theta makes Phi and the
gradient non-finite in every precision (nothing is silently skipped: padded grains
carry a large finite logit, never -inf, so the only non-finite values in the
kernels come from theta), the assignment labels the affected pixels -1, and a
fit that meets such a point stops with the non-finite status."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_objective_with_a_non_finite_entry(pd, bad, prec):
    pdl, ctx = pd
    gm = synth.config_c1()
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 2, 1e-2)
    rng = np.random.default_rng(5)
    th = rng.normal(scale=0.3, size=(gm.N, 6))
    phi, g = ctx.objective_grad([p], [dev(th)], prec)
    assert np.isfinite(float(phi[0])) and torch.isfinite(g[0]).all()
    th[3, 2] = bad
    phi, g = ctx.objective_grad([p], [dev(th)], prec)
    assert not np.isfinite(float(phi[0]))
    assert not torch.isfinite(g[0]).all()


def test_points_objective_with_nan(pd):
    pdl, ctx = pd
    rng = np.random.default_rng(6)
    X, lab, N = synth.power_points(4000, 3, 20, rng)
    q = pdl.Points(dev(X), dev(lab), N, 2, 1e-2)
    K = pdl.points_num_features(3, 2)
    th = rng.normal(scale=0.1, size=(N, K))
    th[0, 0] = np.nan
    for prec in ("fp64", "fp32"):
        phi, g = ctx.points_objective_grad([q], [dev(th)], prec)
        assert np.isnan(float(phi[0])), prec


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_fit_from_a_nan_start_stops(pd, prec):
    pdl, ctx = pd
    gm = synth.config_c1()
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 1, 1e-2)
    th = np.zeros((gm.N, 3))
    th[2, 1] = np.nan
    t = dev(th)
    rep = ctx.fit([p], [t], prec, init="given", max_iter=50, target_acc=0.99)[0]
    assert rep["status"] == "nonfinite" and rep["iters"] == 0
    outs, cnt = ctx.assign([p], [t])
    assert torch.all(outs[0] == -1) and int(cnt[0]) == 0
