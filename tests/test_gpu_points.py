"""Unstructured 2-D and 3-D point sets against the point-set oracle: Phi and
grad Phi (FP64 at 1e-10, FP32 at 2e-3, gradients entry by entry), the hard
assignment bit for bit, ragged sizes (point counts not a multiple of the
64-point wave, grain counts past one 64-grain group), the pixel centres of a map
against the grid path, a batch against single calls, and the argument checks."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def gerr(g, gr):
    return float(np.max(np.abs(g - gr)) / np.max(np.abs(gr)))


def make(pdl, n, D, N, d, eps, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    X, lab, Nn = synth.power_points(n, D, N, rng)
    K = pdl.points_num_features(D, d)
    th = rng.normal(size=(Nn, K)) * scale / np.sqrt(K)
    q = pdl.Points(dev(X), dev(lab, torch.int32), Nn, d, eps)
    return X, lab, th, q


CASES = [(3001, 2, 70, 1, 0.05), (2500, 2, 40, 4, 0.02), (1777, 2, 20, 7, 0.05),
         (3000, 3, 90, 1, 0.05), (2049, 3, 30, 2, 0.03), (1500, 3, 140, 4, 0.05)]


@pytest.mark.parametrize("n,D,N,d,eps", CASES)
def test_points_match_oracle(pd, orc, n, D, N, d, eps):
    pdl, ctx = pd
    X, lab, th, q = make(pdl, n, D, N, d, eps, seed=n + 7 * D + d)
    phi_ref, g_ref = orc.points.objective_grad(th, X, lab, d, eps)
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-3)):
        phi, g = ctx.points_objective_grad([q], [dev(th)], prec)
        ep = abs(float(phi[0]) - phi_ref) / abs(phi_ref)
        eg = gerr(g[0].cpu().numpy(), g_ref)
        print(f"{D}-D n={n} N={q.N} d={d} {prec}: phi {ep:.1e} grad {eg:.1e}")
        assert ep <= tol and eg <= tol
    F_ref, nc_ref = orc.points.assign(th, X, d, lab)
    outs, cnt = ctx.points_assign([q], [dev(th)])
    assert np.array_equal(outs[0].cpu().numpy(), F_ref) and int(cnt[0]) == nc_ref


def test_points_at_a_sharp_iterate(pd, orc):
    """Large logits (a scaled-up theta at eps = 1e-3), where most grains are far
    from each point and skipped."""
    pdl, ctx = pd
    X, lab, th, q = make(pdl, 4000, 3, 200, 3, 1e-3, seed=11, scale=5.0)
    phi_ref, g_ref = orc.points.objective_grad(th, X, lab, 3, 1e-3)
    phi, g = ctx.points_objective_grad([q], [dev(th)], "fp64")
    assert abs(float(phi[0]) - phi_ref) <= 1e-10 * abs(phi_ref)
    assert gerr(g[0].cpu().numpy(), g_ref) <= 1e-10


def test_pixel_centres_match_the_grid_path(pd, orc):
    pdl, ctx = pd
    gm = synth.config_c2()
    d, eps = 2, 1e-2
    c = np.array([orc.coord(j, gm.W) for j in range(gm.W)])
    r = np.array([orc.coord(i, gm.H) for i in range(gm.H)])
    X = np.stack([np.tile(c, gm.H), np.repeat(r, gm.W)], axis=1)
    rng = np.random.default_rng(2)
    th = rng.normal(size=(gm.N, 6)) * 0.05
    q = pdl.Points(dev(X), dev(gm.labels, torch.int32), gm.N, d, eps)
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, d, eps)
    a_phi, a_g = ctx.points_objective_grad([q], [dev(th)], "fp64")
    b_phi, b_g = ctx.objective_grad([p], [dev(th)], "fp64")
    assert abs(float(a_phi[0]) - float(b_phi[0])) <= 1e-12 * abs(float(b_phi[0]))
    assert gerr(a_g[0].cpu().numpy(), b_g[0].cpu().numpy()) <= 1e-11
    Fa, ca = ctx.points_assign([q], [dev(th)])
    Fb, cb = ctx.assign([p], [dev(th)])
    assert torch.equal(Fa[0], Fb[0]) and int(ca[0]) == int(cb[0])


def test_points_batch_equals_single(pd):
    pdl, ctx = pd
    sets = [make(pdl, 1000, 2, 30, 3, 0.05, seed=21), make(pdl, 1300, 3, 50, 2, 0.05, seed=22)]
    qs = [s[3] for s in sets]
    ths = [dev(s[2]) for s in sets]
    phi, g = ctx.points_objective_grad(qs, ths, "fp64")
    for k in range(2):
        p1, g1 = ctx.points_objective_grad([qs[k]], [ths[k]], "fp64")
        assert float(phi[k]) == float(p1[0]) and torch.equal(g[k], g1[0])


def test_points_errors(pd):
    pdl, ctx = pd
    X, lab, th, q = make(pdl, 100, 3, 5, 2, 0.1, seed=3)
    with pytest.raises(pdl.PdError):
        ctx.points_objective_grad([q], [dev(th)], "bf16")
    bad = pdl.Points(q.coords, q.labels, q.N, 5, 0.1)  # 3-D degree above 4
    with pytest.raises(pdl.PdError):
        ctx.points_objective_grad([bad], [torch.zeros((q.N, 56), dtype=torch.float64, device="cuda")], "fp64")
    bad = pdl.Points(q.coords, q.labels, q.N, 2, 0.0)
    with pytest.raises(pdl.PdError):
        ctx.points_objective_grad([bad], [dev(th)], "fp64")
