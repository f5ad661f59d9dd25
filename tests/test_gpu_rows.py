"""Row bands (pd_objective_grad_rows) and the fit's form of the gradient
(PD_EVAL_ONEHOT_PRECOMPUTED) against the FP64 oracle, element by element.

A band's phi is (1/n) sum over its rows of log p_G and its gradient
(1/(eps n)) sum over its rows of (p - delta) psi, n the whole map; the oracle's
objective_rows returns the same sums unscaled.  Tolerances: FP64 1e-10 (phi
relative, gradient max |diff| / max |ref|), FP32 / BF16 2e-3."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 2e-3, "bf16": 2e-3}


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def band_ref(orc, th, lab, H, W, d, eps, r0, r1):
    v, g = orc.objective_rows(th, lab, H, W, d, eps, r0, r1)
    n = H * W
    return v / n, -g / (eps * n)


def max_rel(g, ref):
    return float(np.max(np.abs(g - ref)) / max(np.max(np.abs(ref)), 1e-300))


@pytest.mark.parametrize("prec,d", [("fp64", 3), ("fp32", 3), ("bf16", 3), ("fp64", 6),
                                    ("bf16", 6)])
def test_bands_match_oracle_and_partition(pd, orc, prec, d):
    pdl, ctx = pd
    rng = np.random.default_rng(40 + d)
    H, W, N, eps = 37, 70, 70, 0.05
    th = synth.random_theta(N, d, rng, scale=0.3, multi_index=orc.multi_index(d))
    lab = synth.random_labels(H, W, N, rng)
    p = pdl.Problem(dev(lab, torch.int32), H, W, N, d, eps)
    bands = [(0, 5), (5, 6), (6, 37)]
    phi_f, g_f = ctx.objective_grad([p], [dev(th)], prec)
    tot_phi, tot_g = 0.0, 0.0
    for r0, r1 in bands:
        phi, g = ctx.objective_grad_rows([p], [dev(th)], [(r0, r1)], prec)
        pr, gr = band_ref(orc, th, lab, H, W, d, eps, r0, r1)
        ep = abs(float(phi[0]) - pr) / abs(pr)
        eg = max_rel(g[0].cpu().numpy(), gr)
        print(f"{prec} d={d} rows [{r0},{r1}): phi {ep:.1e} grad {eg:.1e}")
        assert ep <= TOL[prec] and eg <= TOL[prec]
        tot_phi += float(phi[0])
        tot_g = tot_g + g[0]
    # the bands of a partition add up to the whole map's evaluation
    sum_tol = 1e-12 if prec == "fp64" else 1e-5
    assert abs(tot_phi - float(phi_f[0])) <= sum_tol * abs(float(phi_f[0]))
    assert max_rel(tot_g.cpu().numpy(), g_f[0].cpu().numpy()) <= sum_tol
    # an empty band
    phi, g = ctx.objective_grad_rows([p], [dev(th)], [(10, 10)], prec)
    assert float(phi[0]) == 0.0 and not torch.any(g[0] != 0)
    # rows (0, H) is pd_objective_grad, bit for bit
    phi, g = ctx.objective_grad_rows([p], [dev(th)], [(0, H)], prec)
    assert float(phi[0]) == float(phi_f[0]) and torch.equal(g[0], g_f[0])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_fit_form_of_the_gradient_matches_oracle(pd, orc, prec):
    """The gradient the fit evaluates: indicator moments once per call, subtracted
    in FP64 by the reduction (FP64 / FP32), on a batch and on a band."""
    pdl, ctx = pd
    rng = np.random.default_rng(50)
    maps = synth.batch_maps(4141, 3, hw=(40, 161), grains=(10, 151))
    probs, ths = [], []
    for gm in maps:
        d = gm.meta["degree"]
        th = synth.coef_to_theta(gm.coef, orc.multi_index(d)) if gm.coef is not None else \
            synth.random_theta(gm.N, d, rng, scale=0.2, multi_index=orc.multi_index(d))
        ths.append(th + rng.normal(size=th.shape) * 1e-3)
        probs.append(pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, d, gm.meta["eps"]))
    rows = [(0, gm.H) for gm in maps]
    rows[1] = (3, maps[1].H - 2)
    phi, g = ctx.objective_grad_rows(probs, [dev(t) for t in ths], rows, prec,
                                     onehot_precomputed=True)
    for k, gm in enumerate(maps):
        d, eps = gm.meta["degree"], gm.meta["eps"]
        pr, gr = band_ref(orc, ths[k], gm.labels, gm.H, gm.W, d, eps, *rows[k])
        ep = abs(float(phi[k]) - pr) / abs(pr)
        eg = max_rel(g[k].cpu().numpy(), gr)
        print(f"fit form {prec} map {k} d={d} rows {rows[k]}: phi {ep:.1e} grad {eg:.1e}")
        assert ep <= TOL[prec] and eg <= TOL[prec]


def test_invalid_rows_are_rejected(pd):
    pdl, ctx = pd
    H, W, N, d = 8, 9, 3, 1
    p = pdl.Problem(torch.zeros(H * W, dtype=torch.int32, device="cuda"), H, W, N, d, 0.1)
    th = torch.zeros((N, 3), dtype=torch.float64, device="cuda")
    for rows in ((3, 2), (-1, 4), (0, 9)):
        with pytest.raises(pdl.PdError) as e:
            ctx.objective_grad_rows([p], [th], [rows], "fp64")
        assert e.value.status == 1
