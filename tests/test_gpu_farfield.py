"""The far-field skip and the spatial grain order of fit-form evaluations.

A fit-form evaluation stores its grains' row coefficients in the Morton order of
their centroids and leaves out every chunk of a wave whose terms are all below
2^-96 (FP64) or 2^-48 (FP32) of the reference; at a fitted iterate of a map with
many grains most chunks go.  These tests compare that form, where it skips the
most, with the oracle and with the plain form (grain order, nothing skipped):
Phi and grad Phi of the whole map and of row bands, Hessian-vector products, and
fits that must equal the oracle's first iterates.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def gerr(g, gr):
    return float(np.max(np.abs(g - gr)) / np.max(np.abs(gr)))


@pytest.fixture(scope="module")
def fitted(pd):
    """A 256x288 degree-4 polynomial map with 1000 drawn grains (16 groups of 64)
    at an iterate of a seeded FP32 fit: the moment seed, then 120 iterations."""
    pdl, ctx = pd
    rng = np.random.default_rng(777)
    gm = synth.polynomial_diagram(256, 288, 1000, 4, rng)
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, 4, 1e-3)
    th = torch.zeros((gm.N, 15), dtype=torch.float64, device="cuda")
    rep = ctx.fit([p], [th], "fp32", init="heuristic", max_iter=120, target_acc=2.0, history=16)[0]
    print(f"fitted start: N={gm.N} acc {rep['acc']:.4f}")
    assert rep["acc"] > 0.9
    return gm, p, th.cpu().numpy()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-3)])
def test_fit_form_rows_match_oracle(pd, orc, fitted, prec, tol):
    pdl, ctx = pd
    gm, p, x = fitted
    n = p.H * p.W
    for r0, r1 in [(0, 7), (125, 132), (249, 256)]:
        v, g = orc.objective_rows(x, gm.labels, p.H, p.W, p.d, p.eps, r0, r1)
        pr, gr = v / n, -g / (p.eps * n)
        for form in (False, True):
            phi, gg = ctx.objective_grad_rows([p], [dev(x)], [(r0, r1)], prec, onehot_precomputed=form)
            ep = abs(float(phi[0]) - pr) / abs(pr)
            eg = gerr(gg[0].cpu().numpy(), gr)
            print(f"{prec} form {'fit' if form else 'plain'} rows [{r0},{r1}): phi {ep:.1e} grad {eg:.1e}")
            assert ep <= tol and eg <= tol


def test_fit_form_whole_map_matches_plain_form(pd, fitted):
    """The whole map in FP64: the fit form (sorted, skipping, indicator moments
    subtracted) against the plain form (grain order, nothing skipped, -r weights
    in the kernel).  The skipped mass is below 2^-96 per term; what separates the
    forms is the labelled grain's weight.  At this iterate the logits reach ~1e4
    (eps = 1e-3), so s - lse carries an absolute rounding of ~2e-12 in every
    pixel; the plain form takes p_G - 1 as -r (sums of the small terms), the fit
    form as p_G minus the indicator moments, which keeps that rounding: 1.7e-10
    of the largest entry over the 74k pixels of this map (each band of 7 rows is
    within 4e-11 of the oracle, above)."""
    pdl, ctx = pd
    gm, p, x = fitted
    a_phi, a_g = ctx.objective_grad_rows([p], [dev(x)], [(0, p.H)], "fp64", onehot_precomputed=True)
    b_phi, b_g = ctx.objective_grad_rows([p], [dev(x)], [(0, p.H)], "fp64", onehot_precomputed=False)
    assert abs(float(a_phi[0]) - float(b_phi[0])) <= 1e-12 * abs(float(b_phi[0]))
    assert gerr(a_g[0].cpu().numpy(), b_g[0].cpu().numpy()) <= 5e-10


def test_hessian_products_at_the_fitted_iterate(pd, orc, fitted):
    """Hessian-vector products (which skip like the gradient) against the
    variance form of eq. hess evaluated by the oracle's softmax."""
    pdl, ctx = pd
    gm, p, x = fitted
    rng = np.random.default_rng(9)
    v = rng.normal(size=x.shape)
    hv = ctx.hessian_vec([p], [dev(x)], [dev(v)], "fp64")[0].cpu().numpy()
    P = orc.softmax_probs(x, p.H, p.W, p.d, p.eps)
    X = orc.features(p.H, p.W, p.d)
    u = v @ X
    ub = (P * u).sum(0)
    ref = ((P * (u - ub)) @ X.T) / (p.eps * p.eps * p.H * p.W)
    err = gerr(hv, ref)
    print(f"hvp at the fitted iterate: {err:.1e}")
    assert err <= 1e-9


def test_fit_from_the_fitted_iterate_matches_oracle(pd, orc, fitted):
    """Five FP64 L-BFGS iterations from the fitted iterate (where the far field
    is skipped in every evaluation) follow the oracle's."""
    pdl, ctx = pd
    gm, p, x = fitted
    obj = lambda th: orc.objective_grad(th, gm.labels, p.H, p.W, p.d, p.eps)
    ref = orc.lbfgs_fit(obj, x - x[-1], target_acc=2.0, max_iter=5, history=10)
    th = dev(x)
    rep = ctx.fit([p], [th], "fp64", init="given", max_iter=5, target_acc=2.0, history=10)[0]
    y = th.cpu().numpy()
    err = np.max(np.abs(y - ref["theta"])) / np.max(np.abs(ref["theta"]))
    print(f"5 iterations from the fitted iterate: {rep['evals']} evaluations (oracle {ref['evals']}), {err:.1e}")
    assert rep["evals"] == ref["evals"]
    assert err <= 1e-7
