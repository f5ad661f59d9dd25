"""Hessian-vector products (eq. hess of Proposition 4.4) and the Newton-CG fit
against the oracle: the dense FP64 Hessian, the oracle's Newton-CG iteration,
and the unique gauge-fixed maximiser of Proposition 4.11."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _problem(pdl, gm, d, eps):
    return pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, d, eps)


def _dense_hv(orc, gm, d, eps, th, v):
    N, K = th.shape
    Hm = -orc.hessian(th, gm.labels, gm.H, gm.W, d, eps)  # Hessian of -Phi
    return (Hm @ v.reshape(-1)).reshape(N, K)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
@pytest.mark.parametrize("H,W,N,d", [(37, 53, 9, 2), (20, 70, 5, 3), (64, 65, 90, 1)])
def test_hessian_vec_matches_dense_hessian(pd, orc, prec, tol, H, W, N, d):
    """Several pixel tiles, a ragged last tile, a grain count past one 64-grain
    group (74 grains), degrees 1-3."""
    pdl, ctx = pd
    rng = np.random.default_rng(H * 1000 + W + N)
    gm = synth.anisotropic_power_diagram(H, W, N, rng) if d >= 2 else synth.power_diagram(H, W, N, rng)
    K = pdl.num_features(d)
    eps = 0.05
    N = gm.N  # grains that own a pixel
    th = rng.normal(size=(N, K)) * 0.1
    v = rng.normal(size=(N, K))
    out = ctx.hessian_vec([_problem(pdl, gm, d, eps)], [dev(th)], [dev(v)], prec)[0].cpu().numpy()
    ref = _dense_hv(orc, gm, d, eps, th, v)
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    print(prec, H, W, N, d, err)
    assert err <= tol
    # v . H v = (1 / (eps^2 n)) sum_x Var_p(u) >= 0
    assert float(np.sum(v * out)) >= 0.0


def test_hessian_vec_batch_and_gauge(pd, orc):
    """A batch of maps of different degree gives each map's own product; the
    gauge direction (the same vector for every grain) is in the null space."""
    pdl, ctx = pd
    rng = np.random.default_rng(3)
    maps = [(synth.power_diagram(40, 33, 6, rng), 1), (synth.anisotropic_power_diagram(31, 45, 8, rng), 2)]
    probs, ths, vs = [], [], []
    for gm, d in maps:
        K = pdl.num_features(d)
        probs.append(_problem(pdl, gm, d, 0.03))
        ths.append(rng.normal(size=(gm.N, K)) * 0.1)
        vs.append(rng.normal(size=(gm.N, K)))
    out = ctx.hessian_vec(probs, [dev(t) for t in ths], [dev(v) for v in vs], "fp64")
    for (gm, d), th, v, o in zip(maps, ths, vs, out):
        alone = ctx.hessian_vec([_problem(pdl, gm, d, 0.03)], [dev(th)], [dev(v)], "fp64")[0]
        assert torch.equal(o, alone)
        ref = _dense_hv(orc, gm, d, 0.03, th, v)
        assert np.max(np.abs(o.cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
        c = np.tile(rng.normal(size=(1, th.shape[1])), (gm.N, 1))
        z = ctx.hessian_vec([_problem(pdl, gm, d, 0.03)], [dev(th)], [dev(c)], "fp64")[0].cpu().numpy()
        assert np.max(np.abs(z)) <= 1e-12 * np.max(np.abs(ref)) * max(1.0, np.max(np.abs(c)))


def test_hessian_vec_errors(pd):
    pdl, ctx = pd
    rng = np.random.default_rng(0)
    gm = synth.power_diagram(16, 16, 3, rng)
    p = _problem(pdl, gm, 1, 0.1)
    th = torch.zeros((gm.N, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(pdl.PdError):
        ctx.hessian_vec([p], [th], [th], "bf16")


def _oracle_newton(orc, gm, d, eps, th0, **kw):
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    hv = lambda th, v: _dense_hv(orc, gm, d, eps, th, v)
    acc = lambda th: orc.assign(th, gm.H, gm.W, d, gm.labels)[1] / gm.labels.size
    return orc.newton_cg_fit(obj, hv, th0, accuracy=acc, **kw)


def test_newton_cg_follows_the_oracle(pd, orc):
    """The device Newton-CG takes the oracle's iterations: the same number of
    iterations, evaluations and products, and the same points.  The first
    iterates agree to 1e-10; the last ones of this run (condition number about
    2.5e4 on the gauge subspace, 15 CG steps) amplify rounding: the oracle
    itself moves by 1.4e-4 at the end when its products are perturbed by 1e-15
    relative noise, so the end point is compared at 1e-3."""
    pdl, ctx = pd
    rng = np.random.default_rng(21)
    gm, d, eps = synth.power_diagram(48, 56, 7, rng), 1, 2e-2
    K = pdl.num_features(d)
    th0 = rng.normal(size=(gm.N, K)) * 0.05
    for mi, tol in [(1, 1e-10), (4, 1e-10), (8, 1e-9), (60, 1e-3)]:
        ref = _oracle_newton(orc, gm, d, eps, th0, max_iter=mi, cg_max=15, target_acc=0.995)
        th = dev(th0)
        rep = ctx.fit_newton_cg([_problem(pdl, gm, d, eps)], [th], "fp64", max_iter=mi, cg_max=15,
                                target_acc=0.995)[0]
        x = th.cpu().numpy()
        err = np.max(np.abs(x - ref["theta"])) / max(1.0, np.max(np.abs(ref["theta"])))
        print(mi, rep, ref["status"], ref["iters"], ref["evals"], ref["hvps"], ref["acc"], err)
        assert rep["status"] == ref["status"]
        assert (rep["iters"], rep["evals"], rep["hvps"]) == (ref["iters"], ref["evals"], ref["hvps"])
        assert np.all(x[-1] == 0.0)
        assert err <= tol
        assert abs(rep["phi"] - ref["phi"]) <= 10 * tol * abs(ref["phi"])
        if mi < 60:
            assert rep["status"] == "budget" and rep["acc"] == ref["acc"]
    assert ref["status"] == "target" and rep["acc"] >= 0.995


def test_newton_cg_reaches_the_unique_maximiser(pd, orc):
    """Proposition 4.11: random labels (no exact reconstruction); the device
    Newton-CG stops on the gradient test at the maximiser that the dense damped
    Newton solve of the oracle finds."""
    pdl, ctx = pd
    rng = np.random.default_rng(12)
    H, W, N, d, eps = 7, 9, 4, 2, 0.3
    lab = synth.random_labels(H, W, N, rng)
    K = pdl.num_features(d)
    obj = lambda th: orc.objective_grad(th, lab, H, W, d, eps)
    ref = orc.newton_fit(np.zeros((N, K)), obj, lambda th: orc.hessian(th, lab, H, W, d, eps))
    th = torch.zeros((N, K), dtype=torch.float64, device="cuda")
    p = pdl.Problem(dev(lab, torch.int32), H, W, N, d, eps)
    rep = ctx.fit_newton_cg([p], [th], "fp64", max_iter=60, cg_max=40, target_acc=2.0, gtol=1e-11)[0]
    print(rep)
    assert rep["status"] == "gtol"
    assert np.max(np.abs(th.cpu().numpy() - ref)) <= 1e-8 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_newton_cg_batch_is_independent(pd, prec):
    """Maps of a batch stop on their own and end where they end alone."""
    pdl, ctx = pd
    rng = np.random.default_rng(8)
    maps = [(synth.power_diagram(64, 64, 12, rng), 1, 1e-2),
            (synth.anisotropic_power_diagram(50, 70, 9, rng), 2, 1e-2)]
    probs = [_problem(pdl, gm, d, eps) for gm, d, eps in maps]
    th0 = [np.zeros((gm.N, pdl.num_features(d))) for gm, d, _ in maps]
    both = [dev(t) for t in th0]
    reps = ctx.fit_newton_cg(probs, both, prec, max_iter=80, cg_max=20, target_acc=0.99)
    for k, (gm, d, eps) in enumerate(maps):
        alone = dev(th0[k])
        r1 = ctx.fit_newton_cg([probs[k]], [alone], prec, max_iter=80, cg_max=20, target_acc=0.99)[0]
        print(prec, k, reps[k], r1)
        assert reps[k]["status"] == "target" and reps[k]["acc"] >= 0.99
        assert (reps[k]["iters"], reps[k]["evals"], reps[k]["hvps"]) == (r1["iters"], r1["evals"], r1["hvps"])
        assert torch.equal(both[k], alone)


def test_newton_cg_start_at_target_and_errors(pd):
    pdl, ctx = pd
    rng = np.random.default_rng(4)
    gm = synth.power_diagram(32, 32, 4, rng)
    p = _problem(pdl, gm, 1, 1e-2)
    th = torch.zeros((gm.N, 3), dtype=torch.float64, device="cuda")
    rep = ctx.fit_newton_cg([p], [th], "fp64", target_acc=0.0)[0]
    assert rep["status"] == "target" and rep["iters"] == 0 and rep["evals"] == 1 and rep["hvps"] == 0
    with pytest.raises(pdl.PdError):
        ctx.fit_newton_cg([p], [th], "bf16")
    with pytest.raises(pdl.PdError):
        ctx.fit_newton_cg([p], [th], "fp64", cg_max=0)
