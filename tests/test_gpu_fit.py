"""GPU parity of the device L-BFGS driver (pd_fit) against the oracle's L-BFGS."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def problem(pdl, gm, d, eps):
    return pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, d, eps)


def oracle_fit(orc, gm, d, eps, **kw):
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    acc = lambda th: orc.assign(th, gm.H, gm.W, d, gm.labels)[1] / (gm.H * gm.W)
    return orc.lbfgs_fit(obj, np.zeros((gm.N, orc.num_features(d))), accuracy=acc, **kw)


@pytest.mark.parametrize("iters", [1, 3, 8])
def test_first_iterates_match_oracle(pd, orc, iters):
    """Same state machine, same arithmetic up to summation order: the first
    iterates agree to ~1e-9 and the evaluation counts are identical."""
    pdl, ctx = pd
    gm = synth.config_c1()
    ref = oracle_fit(orc, gm, 1, 1e-2, target_acc=2.0, max_iter=iters)
    th = dev(np.zeros((gm.N, 3)))
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "fp64", init="zero", max_iter=iters,
                  target_acc=2.0)[0]
    assert rep["iters"] == ref["iters"] == iters
    assert rep["evals"] == ref["evals"]
    x = th.cpu().numpy()
    assert np.max(np.abs(x - ref["theta"])) <= 1e-8 * np.max(np.abs(ref["theta"]))
    assert abs(rep["phi"] - ref["phi"]) <= 1e-10 * abs(ref["phi"])
    assert x[-1].tolist() == [0.0, 0.0, 0.0]


def test_trace_follows_the_oracle_records(pd, orc):
    """The per-iteration metrics ring of pd_fit: the first 8 FP64 iterates of the
    c1 map against the oracle's records (Phi, accepted step, evaluation count,
    accuracy), the gradient norm at the last iterate against the oracle's
    gradient there, and rows of iterates not reached left as they were."""
    pdl, ctx = pd
    gm = synth.config_c1()
    ref = oracle_fit(orc, gm, 1, 1e-2, target_acc=2.0, max_iter=8)
    tr = torch.full((12, pdl.TRACE_FIELDS), -7.0, dtype=torch.float64, device="cuda")
    th = dev(np.zeros((gm.N, 3)))
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "fp64", init="zero", max_iter=8,
                  target_acc=2.0, trace=[tr])[0]
    T = tr.cpu().numpy()
    assert rep["iters"] == 8 and np.all(T[8:] == -7.0)
    recs = ref["records"]
    assert T[:8, 0].tolist() == list(range(1, 9))
    assert T[:8, 1].tolist() == list(1 + np.cumsum([r["evals"] for r in recs]))
    assert T[7, 1] == rep["evals"]
    for k, r in enumerate(recs):
        assert abs(T[k, 2] - r["phi"]) <= 1e-10 * abs(r["phi"]), k
        assert abs(T[k, 4] - r["t"]) <= 1e-7 * abs(r["t"]), k
        assert abs(T[k, 5] - r["acc"]) <= 2.0 / (gm.H * gm.W), k
    assert T[7, 2] == rep["phi"] and T[7, 5] == rep["acc"]
    _, g = orc.objective_grad(th.cpu().numpy(), gm.labels, gm.H, gm.W, 1, 1e-2)
    gi = np.max(np.abs(g[:-1]))  # the fit's gauge: the last grain's row is fixed
    assert abs(T[7, 3] - gi) <= 1e-9 * gi


def test_trace_ring_over_an_eps_schedule(pd):
    """Eight iterations over three levels of an eps schedule into a ring of 4:
    iterates 5..8 remain, numbered across the levels, in rows (k - 1) % 4."""
    pdl, ctx = pd
    gm = synth.config_c1()
    tr = torch.zeros((4, pdl.TRACE_FIELDS), dtype=torch.float64, device="cuda")
    th = dev(np.zeros((gm.N, 3)))
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "fp64", init="zero", max_iter=8,
                  target_acc=2.0, anneal=(2, 4.0, 3), trace=[tr])[0]
    T = tr.cpu().numpy()
    assert rep["iters"] == 8
    for k in range(5, 9):
        assert T[(k - 1) % 4, 0] == k
    ev = [T[(k - 1) % 4, 1] for k in range(5, 9)]
    assert all(a < b for a, b in zip(ev, ev[1:])) and ev[-1] == rep["evals"]
    assert np.all(T[:, 4] > 0) and np.all(T[:, 3] >= 0)


def test_power_diagram_fit_reaches_99(pd, orc):
    """Section 5.4 protocol on the 64x64 N = 8 power-diagram map: theta = 0,
    eps = 1e-2, FP64 L-BFGS to >= 99% pixel accuracy; the same iteration count as
    the oracle (trajectories agree), accuracy recomputed by the oracle."""
    pdl, ctx = pd
    gm = synth.config_c1()
    ref = oracle_fit(orc, gm, 1, 1e-2, target_acc=0.99, max_iter=2000)
    th = dev(np.zeros((gm.N, 3)))
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "fp64", init="zero", max_iter=2000,
                  target_acc=0.99)[0]
    assert rep["status"] == "target" and rep["acc"] >= 0.99
    _, nc, _ = orc.assign(th.cpu().numpy(), gm.H, gm.W, 1, gm.labels)
    assert nc / (gm.H * gm.W) == rep["acc"]
    assert abs(rep["iters"] - ref["iters"]) <= 2, (rep["iters"], ref["iters"])
    assert rep["seconds_to_target"] > 0


def test_fp32_fit_reaches_99(pd, orc):
    pdl, ctx = pd
    gm = synth.config_c1()
    th = dev(np.zeros((gm.N, 3)))
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "fp32", init="zero", max_iter=2000,
                  target_acc=0.99)[0]
    assert rep["status"] == "target"
    _, nc, _ = orc.assign(th.cpu().numpy(), gm.H, gm.W, 1, gm.labels)
    assert nc / (gm.H * gm.W) >= 0.99
    assert nc / (gm.H * gm.W) == rep["acc"]


@pytest.mark.parametrize("d,eps,iters", [(6, 1e-3, 25), (4, 1e-3, 60), (3, 1e-2, 40)])
def test_bf16_fit_accuracy_is_the_canonical_one(pd, orc, d, eps, iters):
    """The accuracy a BF16 fit reports is certified inside the matrix-core
    objective (chunk maxima of the matrix-core logits, the best chunk again in
    FP64, the undecided pixels by the canonical arg-min): it is exactly the
    oracle's count at the returned iterate, early in the fit (many close logits)
    and later."""
    pdl, ctx = pd
    gm = poly_map(70 + d, 96, 80, 40, d)
    K = pdl.num_features(d)
    th = dev(np.zeros((gm.N, K)))
    rep = ctx.fit([problem(pdl, gm, d, eps)], [th], "bf16", init="zero", max_iter=iters,
                  target_acc=2.0)[0]
    _, nc, _ = orc.assign(th.cpu().numpy(), gm.H, gm.W, d, gm.labels)
    print(f"d={d} eps={eps}: {rep['iters']} iterations, accuracy {rep['acc']:.4f}")
    assert rep["iters"] > 0
    assert nc / (gm.H * gm.W) == rep["acc"]


def test_nonseparable_fit_matches_newton(pd, orc):
    """Proposition 4.11: unique gauge-fixed maximiser, found by the device fit and
    by the oracle's dense Newton solve."""
    pdl, ctx = pd
    rng = np.random.default_rng(10)
    H, W, N, d, eps = 8, 9, 3, 2, 0.5
    lab = synth.random_labels(H, W, N, rng)
    obj = lambda th: orc.objective_grad(th, lab, H, W, d, eps)
    hes = lambda th: orc.hessian(th, lab, H, W, d, eps)
    xn = orc.newton_fit(np.zeros((N, 6)), obj, hes)
    th = dev(np.zeros((N, 6)))
    rep = ctx.fit([pdl.Problem(dev(lab, torch.int32), H, W, N, d, eps)], [th], "fp64",
                  init="zero", max_iter=500, target_acc=2.0, gtol=1e-12)[0]
    assert rep["status"] in ("gtol", "linesearch", "budget")
    x = th.cpu().numpy()
    assert np.max(np.abs(x - xn)) <= 1e-6 * np.max(np.abs(xn))


def test_batched_fit_equals_single(pd, orc):
    pdl, ctx = pd
    rng = np.random.default_rng(3)
    maps = [synth.config_c1(), synth.power_diagram(40, 56, 6, rng),
            synth.anisotropic_power_diagram(48, 48, 9, rng)]
    degs = [1, 1, 2]
    probs = [problem(pdl, gm, d, 1e-2) for gm, d in zip(maps, degs)]
    ths = [dev(np.zeros((gm.N, pdl.num_features(d)))) for gm, d in zip(maps, degs)]
    reps = ctx.fit(probs, ths, "fp64", init="zero", max_iter=300, target_acc=0.99)
    for k, (p, gm, d) in enumerate(zip(probs, maps, degs)):
        t1 = dev(np.zeros((gm.N, pdl.num_features(d))))
        r1 = ctx.fit([p], [t1], "fp64", init="zero", max_iter=300, target_acc=0.99)[0]
        assert torch.equal(t1, ths[k])
        assert (r1["iters"], r1["evals"], r1["status"]) == (reps[k]["iters"], reps[k]["evals"],
                                                           reps[k]["status"])


def test_centered_gauge_and_given_start(pd, orc):
    pdl, ctx = pd
    gm = synth.config_c1()
    rng = np.random.default_rng(4)
    th0 = rng.normal(size=(gm.N, 3)) * 0.01
    th = dev(th0)
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "fp64", gauge="centered", init="given",
                  max_iter=200, target_acc=0.99)[0]
    x = th.cpu().numpy()
    assert np.max(np.abs(x.sum(0))) <= 1e-12 * np.max(np.abs(x)) * gm.N
    assert rep["status"] == "target"


def test_zero_budget_returns_start(pd, orc):
    pdl, ctx = pd
    gm = synth.config_c1()
    th = dev(np.zeros((gm.N, 3)))
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "fp64", init="zero", max_iter=0,
                  target_acc=0.99)[0]
    assert rep["iters"] == 0 and rep["status"] == "budget"
    assert abs(rep["phi"] + np.log(gm.N)) < 1e-12
    assert torch.all(th == 0)


def test_bf16_fit_reaches_99(pd, orc):
    """The matrix-core evaluation drives the same device L-BFGS to >= 99% on the
    power-diagram map (accuracy recomputed by the oracle in FP64)."""
    pdl, ctx = pd
    gm = synth.config_c1()
    th = dev(np.zeros((gm.N, 3)))
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "bf16", init="zero", max_iter=2000,
                  target_acc=0.99)[0]
    assert rep["status"] == "target"
    _, nc, _ = orc.assign(th.cpu().numpy(), gm.H, gm.W, 1, gm.labels)
    assert nc / (gm.H * gm.W) >= 0.99
    assert nc / (gm.H * gm.W) == rep["acc"]


@pytest.mark.parametrize("d,eps,iters", [(6, 1e-3, 25), (4, 1e-3, 60), (3, 1e-2, 40)])
def test_bf16_fit_accuracy_is_the_canonical_one(pd, orc, d, eps, iters):
    """The accuracy a BF16 fit reports is certified inside the matrix-core
    objective (chunk maxima of the matrix-core logits, the best chunk again in
    FP64, the undecided pixels by the canonical arg-min): it is exactly the
    oracle's count at the returned iterate, early in the fit (many close logits)
    and later."""
    pdl, ctx = pd
    gm = poly_map(70 + d, 96, 80, 40, d)
    K = pdl.num_features(d)
    th = dev(np.zeros((gm.N, K)))
    rep = ctx.fit([problem(pdl, gm, d, eps)], [th], "bf16", init="zero", max_iter=iters,
                  target_acc=2.0)[0]
    _, nc, _ = orc.assign(th.cpu().numpy(), gm.H, gm.W, d, gm.labels)
    print(f"d={d} eps={eps}: {rep['iters']} iterations, accuracy {rep['acc']:.4f}")
    assert rep["iters"] > 0
    assert nc / (gm.H * gm.W) == rep["acc"]


def test_bf16_fit_accuracy_with_large_coefficients(pd, orc):
    """A start with large coefficients (sum |thc| ~ 1e6 at eps = 1e-3): the
    matrix-core bound then exceeds the logit gaps at most pixels, the FP64 pass
    over the row coefficients decides them, and the reported accuracy is still
    exactly the oracle's count at the returned iterate."""
    pdl, ctx = pd
    d, eps = 4, 1e-3
    gm = poly_map(91, 96, 80, 40, d)
    K = pdl.num_features(d)
    th0 = np.random.default_rng(92).normal(scale=30.0, size=(gm.N, K))
    th = dev(th0)
    rep = ctx.fit([problem(pdl, gm, d, eps)], [th], "bf16", init="given", max_iter=3,
                  target_acc=2.0)[0]
    _, nc, _ = orc.assign(th.cpu().numpy(), gm.H, gm.W, d, gm.labels)
    print(f"large start: {rep['iters']} iterations, accuracy {rep['acc']:.4f}")
    assert nc / (gm.H * gm.W) == rep["acc"]


def test_given_start_is_moved_into_the_gauge(pd, orc):
    """Lemma 4.2: a given start enters the gauge theta_{N-1} = 0 by the common
    shift -theta_{N-1}, which leaves Phi unchanged (not by zeroing the row)."""
    pdl, ctx = pd
    gm = synth.config_c1()
    rng = np.random.default_rng(8)
    th0 = rng.normal(size=(gm.N, 3)) * 0.05
    th = dev(th0)
    rep = ctx.fit([problem(pdl, gm, 1, 1e-2)], [th], "fp64", init="given", max_iter=0,
                  target_acc=2.0)[0]
    x = th.cpu().numpy()
    assert np.array_equal(x, th0 - th0[-1])
    phi_ref, _ = orc.objective_grad(th0, gm.labels, gm.H, gm.W, 1, 1e-2)
    assert abs(rep["phi"] - phi_ref) <= 1e-12 * abs(phi_ref)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
def test_hessian_diag_matches_oracle(pd, orc, prec, tol):
    """Diagonal of eq. hess (sum_x p (1 - p) psi^2 / (eps^2 n)) against the oracle."""
    pdl, ctx = pd
    rng = np.random.default_rng(41)
    cases = [(23, 70, 9, 2, 0.05), (40, 33, 70, 3, 0.02), (17, 19, 5, 6, 0.3)]
    probs, ths, refs = [], [], []
    for H, W, N, d, eps in cases:
        lab = synth.random_labels(H, W, N, rng)
        th = synth.random_theta(N, d, rng, scale=0.2, multi_index=orc.multi_index(d))
        probs.append(pdl.Problem(dev(lab, torch.int32), H, W, N, d, eps))
        ths.append(dev(th))
        refs.append(orc.hessian_diag(th, lab, H, W, d, eps))
    out = ctx.hessian_diag(probs, ths, prec)
    for D, ref in zip(out, refs):
        D = D.cpu().numpy()
        assert np.all(D >= 0)
        assert np.max(np.abs(D - ref)) <= tol * np.max(ref)


def poly_map(seed=3, H=64, W=64, N=16, d=3):
    return synth.polynomial_diagram(H, W, N, d, np.random.default_rng(seed))


@pytest.mark.parametrize("iters", [1, 4, 12])
def test_preconditioned_iterates_match_oracle(pd, orc, iters):
    """Diagonal preconditioner refreshed every 5 iterations: the same state machine
    as the oracle's, so the first iterates agree (12 crosses two refreshes)."""
    pdl, ctx = pd
    gm = poly_map()
    d, eps = 3, 1e-3
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    pre = lambda th: orc.hessian_diag(th, gm.labels, gm.H, gm.W, d, eps)
    ref = orc.lbfgs_fit(obj, np.zeros((gm.N, 10)), target_acc=2.0, max_iter=iters,
                        precondition=pre, diag_every=5)
    th = dev(np.zeros((gm.N, 10)))
    rep = ctx.fit([problem(pdl, gm, d, eps)], [th], "fp64", init="zero", max_iter=iters,
                  target_acc=2.0, precondition=5)[0]
    assert rep["iters"] == ref["iters"] == iters
    assert rep["evals"] == ref["evals"]
    x = th.cpu().numpy()
    assert np.max(np.abs(x - ref["theta"])) <= 1e-7 * np.max(np.abs(ref["theta"]))
    assert np.all(x[-1] == 0)


@pytest.mark.parametrize("N,side", [(20, 64), (40, 64), (90, 96)])
@pytest.mark.parametrize("pre", [0, 5])
def test_single_block_iterates_match_oracle(pd, orc, N, side, pre):
    """One block per map (N K < 1024): N K = 200, 400 and 900 at d = 3 put up to
    4, 8 and 16 elements on each lane of the per-wave dot products of the
    memory; 12 iterations fill the memory past the number of waves, and with the
    preconditioner cross two refreshes.  Same state machine as the oracle's."""
    pdl, ctx = pd
    gm = poly_map(11, side, side, N, 3)
    d, eps = 3, 1e-3
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    kw = {}
    if pre:
        kw = dict(precondition=lambda th: orc.hessian_diag(th, gm.labels, gm.H, gm.W, d, eps),
                  diag_every=pre)
    iters = 12
    ref = orc.lbfgs_fit(obj, np.zeros((gm.N, 10)), target_acc=2.0, max_iter=iters, **kw)
    th = dev(np.zeros((gm.N, 10)))
    rep = ctx.fit([problem(pdl, gm, d, eps)], [th], "fp64", init="zero", max_iter=iters,
                  target_acc=2.0, precondition=pre)[0]
    assert rep["iters"] == ref["iters"] == iters
    assert rep["evals"] == ref["evals"]
    x = th.cpu().numpy()
    assert np.max(np.abs(x - ref["theta"])) <= 1e-7 * np.max(np.abs(ref["theta"]))
    assert abs(rep["phi"] - ref["phi"]) <= 1e-9 * abs(ref["phi"])
    assert np.all(x[-1] == 0)


def test_preconditioned_fit_needs_fewer_iterations(pd, orc):
    pdl, ctx = pd
    gm = poly_map(5, 128, 128, 40, 4)
    p = problem(pdl, gm, 4, 1e-3)
    th0 = dev(np.zeros((gm.N, 15)))
    r0 = ctx.fit([p], [th0], "fp32", init="zero", max_iter=2000, target_acc=0.99)[0]
    th1 = dev(np.zeros((gm.N, 15)))
    r1 = ctx.fit([p], [th1], "fp32", init="zero", max_iter=2000, target_acc=0.99,
                 precondition=10)[0]
    assert r0["status"] == r1["status"] == "target"
    _, nc, _ = orc.assign(th1.cpu().numpy(), gm.H, gm.W, 4, gm.labels)
    assert nc / gm.labels.size >= 0.99
    print(f"\niterations to 99%: plain {r0['iters']}, preconditioned {r1['iters']}")
    assert r1["iters"] < r0["iters"]


def test_bf16_preconditioned_fit_needs_fewer_iterations(pd, orc):
    """BF16 evaluation with the diagonal preconditioner (its Hessian diagonal
    from an FP32 evaluation at the refresh iterates): reaches 99% in fewer
    iterations than the BF16 fit without it, and the result passes the oracle's
    assignment."""
    pdl, ctx = pd
    gm = poly_map(5, 128, 128, 40, 4)
    p = problem(pdl, gm, 4, 1e-3)
    th0 = dev(np.zeros((gm.N, 15)))
    r0 = ctx.fit([p], [th0], "bf16", init="zero", max_iter=2000, target_acc=0.99)[0]
    th1 = dev(np.zeros((gm.N, 15)))
    r1 = ctx.fit([p], [th1], "bf16", init="zero", max_iter=2000, target_acc=0.99,
                 precondition=10)[0]
    assert r0["status"] == r1["status"] == "target"
    _, nc, _ = orc.assign(th1.cpu().numpy(), gm.H, gm.W, 4, gm.labels)
    assert nc / gm.labels.size >= 0.99
    print(f"\nBF16 iterations to 99%: plain {r0['iters']}, preconditioned {r1['iters']}")
    assert r1["iters"] < r0["iters"]


def test_preconditioned_batched_equals_single(pd):
    pdl, ctx = pd
    rng = np.random.default_rng(9)
    maps = [(poly_map(), 3), (synth.anisotropic_power_diagram(40, 52, 12, rng), 2)]
    probs = [problem(pdl, gm, d, 1e-2) for gm, d in maps]
    ths = [dev(np.zeros((gm.N, pdl.num_features(d)))) for gm, d in maps]
    reps = ctx.fit(probs, ths, "fp32", init="zero", max_iter=150, target_acc=0.99, precondition=10)
    for k, (p, (gm, d)) in enumerate(zip(probs, maps)):
        t1 = dev(np.zeros((gm.N, pdl.num_features(d))))
        r1 = ctx.fit([p], [t1], "fp32", init="zero", max_iter=150, target_acc=0.99,
                     precondition=10)[0]
        assert torch.equal(t1, ths[k])
        assert (r1["iters"], r1["evals"]) == (reps[k]["iters"], reps[k]["evals"])


def test_preconditioner_argument_checks(pd):
    pdl, ctx = pd
    gm = synth.config_c1()
    p = problem(pdl, gm, 1, 1e-2)
    th = dev(np.zeros((gm.N, 3)))
    for kw, status in ((dict(gauge="centered"), "UNSUPPORTED"), (dict(precondition=-1), "INVALID_ARG")):
        args = dict(prec="fp32", init="zero", max_iter=5, precondition=10)
        args.update(kw)
        prec = args.pop("prec")
        with pytest.raises(pdl.PdError, match=status):
            ctx.fit([p], [th], prec, **args)


@pytest.fixture
def split_path():
    """Every map takes the multi-block path of an accepted step (the dot
    products and the direction on several blocks, from per-block partials)."""
    import os
    old = os.environ.get("PD_FIT_SPLIT_MIN")
    os.environ["PD_FIT_SPLIT_MIN"] = "1"
    yield
    if old is None:
        del os.environ["PD_FIT_SPLIT_MIN"]
    else:
        os.environ["PD_FIT_SPLIT_MIN"] = old


@pytest.mark.parametrize("iters,pre", [(1, 0), (8, 0), (4, 5), (12, 5)])
def test_split_path_iterates_match_oracle(pd, orc, split_path, iters, pre):
    """N K = 1300 (three 512-element chunks): the multi-block path runs the same
    state machine as the oracle's L-BFGS (with the preconditioner, 12 iterations
    cross two refreshes)."""
    pdl, ctx = pd
    gm = poly_map(7, 96, 96, 130, 3)
    d, eps = 3, 1e-3
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    kw = {}
    if pre:
        kw = dict(precondition=lambda th: orc.hessian_diag(th, gm.labels, gm.H, gm.W, d, eps),
                  diag_every=pre)
    ref = orc.lbfgs_fit(obj, np.zeros((gm.N, 10)), target_acc=2.0, max_iter=iters, **kw)
    th = dev(np.zeros((gm.N, 10)))
    rep = ctx.fit([problem(pdl, gm, d, eps)], [th], "fp64", init="zero", max_iter=iters,
                  target_acc=2.0, precondition=pre)[0]
    assert rep["iters"] == ref["iters"] == iters
    assert rep["evals"] == ref["evals"]
    x = th.cpu().numpy()
    assert np.max(np.abs(x - ref["theta"])) <= 1e-7 * np.max(np.abs(ref["theta"]))
    assert abs(rep["phi"] - ref["phi"]) <= 1e-9 * abs(ref["phi"])


@pytest.mark.parametrize("case", ["single-block", "multi-block-preconditioned"])
def test_resumed_fit_follows_the_uninterrupted_one(pd, orc, case):
    """k0 iterations with the L-BFGS state written out, then k1 more resumed from
    it: the iterate, Phi and the evaluation count of the uninterrupted run (the
    oracle's L-BFGS, which takes every direction by the two-loop recursion), the
    iteration count continued in the state's header and in the trace.  The
    multi-block map (N K = 1300) refreshes its preconditioner at iterations 5
    and 10, before and after the resume."""
    pdl, ctx = pd
    if case == "single-block":
        gm, d, eps, pre, k0, k1, m = synth.config_c1(), 1, 1e-2, 0, 3, 5, 10
    else:
        gm, d, eps, pre, k0, k1, m = poly_map(7, 96, 96, 130, 3), 3, 1e-3, 5, 6, 6, 10
    K = pdl.num_features(d)
    obj = lambda th: orc.objective_grad(th, gm.labels, gm.H, gm.W, d, eps)
    kw = {}
    if pre:
        kw = dict(precondition=lambda th: orc.hessian_diag(th, gm.labels, gm.H, gm.W, d, eps),
                  diag_every=pre)
    ref = orc.lbfgs_fit(obj, np.zeros((gm.N, K)), target_acc=2.0, max_iter=k0 + k1, history=m, **kw)
    prob = problem(pdl, gm, d, eps)
    st = torch.full((pdl.fit_state_size(gm.N, d, m),), np.nan, dtype=torch.float64, device="cuda")
    th = dev(np.zeros((gm.N, K)))
    r0 = ctx.fit([prob], [th], "fp64", init="zero", max_iter=k0, target_acc=2.0, history=m,
                 precondition=pre, state=[st])[0]
    h = st[:16].cpu().numpy()
    assert r0["iters"] == k0 and h[6] == k0 and h[3] == m and h[1] == gm.N and h[2] == K
    tr = torch.zeros((k0 + k1, pdl.TRACE_FIELDS), dtype=torch.float64, device="cuda")
    r1 = ctx.fit([prob], [th], "fp64", init="given", max_iter=k1, target_acc=2.0, history=m,
                 precondition=pre, state=[st], resume=True, trace=[tr])[0]
    assert r1["iters"] == k1 and st[6].item() == k0 + k1
    T = tr.cpu().numpy()
    assert T[k0:, 0].tolist() == list(range(k0 + 1, k0 + k1 + 1))  # numbering continues
    assert r0["evals"] + r1["evals"] - 1 == ref["evals"]  # the resume re-evaluates its start
    x = th.cpu().numpy()
    err = np.max(np.abs(x - ref["theta"])) / np.max(np.abs(ref["theta"]))
    print(f"{case}: resumed after {k0} of {k0 + k1} iterations, {err:.1e} from the oracle")
    assert err <= 1e-7
    assert abs(r1["phi"] - ref["phi"]) <= 1e-9 * abs(ref["phi"])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_resumed_reduced_precision_fit_follows_the_uninterrupted_one(pd, prec):
    """The same split of a fit in FP32 and BF16 evaluations (k0 = 4, k1 = 6 on a
    degree-3 map with the preconditioner every 3 iterations): against the
    uninterrupted fit in the same precision, whose evaluations are deterministic,
    the resumed iterate differs only by the rounding of the first direction."""
    pdl, ctx = pd
    gm, d, eps, m = poly_map(3, 64, 64, 16, 3), 3, 1e-3, 8
    K = pdl.num_features(d)
    prob = problem(pdl, gm, d, eps)
    kw = dict(target_acc=2.0, history=m, precondition=3)
    ta = dev(np.zeros((gm.N, K)))
    ra = ctx.fit([prob], [ta], prec, init="zero", max_iter=10, **kw)[0]
    st = torch.zeros((pdl.fit_state_size(gm.N, d, m),), dtype=torch.float64, device="cuda")
    tb = dev(np.zeros((gm.N, K)))
    r0 = ctx.fit([prob], [tb], prec, init="zero", max_iter=4, state=[st], **kw)[0]
    r1 = ctx.fit([prob], [tb], prec, init="given", max_iter=6, state=[st], resume=True, **kw)[0]
    assert ra["iters"] == 10 and r0["iters"] + r1["iters"] == 10
    assert r0["evals"] + r1["evals"] - 1 == ra["evals"]
    a, b = ta.cpu().numpy(), tb.cpu().numpy()
    err = np.max(np.abs(a - b)) / np.max(np.abs(a))
    print(f"{prec}: resumed after 4 of 10 iterations, {err:.1e} from the uninterrupted fit")
    assert err <= 1e-9


def test_resume_argument_checks(pd):
    pdl, ctx = pd
    gm = synth.config_c1()
    prob = problem(pdl, gm, 1, 1e-2)
    th = dev(np.zeros((gm.N, 3)))
    st = torch.zeros((pdl.fit_state_size(gm.N, 1, 10),), dtype=torch.float64, device="cuda")
    with pytest.raises(pdl.PdError):  # nothing written there yet
        ctx.fit([prob], [th], "fp64", init="given", max_iter=2, state=[st], resume=True)
    with pytest.raises(pdl.PdError):  # resume without a state
        ctx.fit([prob], [th], "fp64", init="given", max_iter=2, resume=True)
    ctx.fit([prob], [th], "fp64", init="zero", max_iter=2, target_acc=2.0, state=[st])
    with pytest.raises(pdl.PdError):  # another preconditioner than the state's
        ctx.fit([prob], [th], "fp64", init="given", max_iter=2, history=10, precondition=3,
                state=[st], resume=True)
    with pytest.raises(pdl.PdError):  # a resume starts from the given iterate
        ctx.fit([prob], [th], "fp64", init="zero", max_iter=2, state=[st], resume=True)
    with pytest.raises(pdl.PdError):  # not across an eps schedule
        ctx.fit([prob], [th], "fp64", init="given", max_iter=2, anneal=(1, 2.0, 1), state=[st])
    r = ctx.fit([prob], [th], "fp64", init="given", max_iter=0, target_acc=2.0, state=[st], resume=True)[0]
    assert r["iters"] == 0 and st[6].item() == 2


def test_split_path_batch_reaches_99(pd, orc, split_path):
    """A batch where every map takes the multi-block path reaches 99% like the
    single-block path, and the accuracy the fit reports is the oracle's."""
    pdl, ctx = pd
    maps = [(poly_map(), 3), (poly_map(5, 128, 128, 40, 4), 4)]
    probs = [problem(pdl, gm, d, 1e-3) for gm, d in maps]
    ths = [dev(np.zeros((gm.N, pdl.num_features(d)))) for gm, d in maps]
    reps = ctx.fit(probs, ths, "fp32", init="zero", max_iter=2000, target_acc=0.99, history=16,
                   precondition=10, check_every=4)
    for (gm, d), r, t in zip(maps, reps, ths):
        assert r["status"] == "target"
        _, nc, _ = orc.assign(t.cpu().numpy(), gm.H, gm.W, d, gm.labels)
        assert nc / gm.labels.size == r["acc"] and r["acc"] >= 0.99


def test_split_path_batched_equals_single(pd, split_path):
    """On the multi-block path too, a map's fit does not depend on its batch:
    the chunking and every partial sum are the map's own."""
    pdl, ctx = pd
    maps = [(poly_map(7, 96, 96, 130, 3), 3), (poly_map(), 3)]
    probs = [problem(pdl, gm, d, 1e-3) for gm, d in maps]
    ths = [dev(np.zeros((gm.N, pdl.num_features(d)))) for gm, d in maps]
    reps = ctx.fit(probs, ths, "fp32", init="zero", max_iter=60, target_acc=2.0, history=16,
                   precondition=10)
    for k, (p, (gm, d)) in enumerate(zip(probs, maps)):
        t1 = dev(np.zeros((gm.N, pdl.num_features(d))))
        r1 = ctx.fit([p], [t1], "fp32", init="zero", max_iter=60, target_acc=2.0, history=16,
                     precondition=10)[0]
        assert torch.equal(t1, ths[k])
        assert (r1["iters"], r1["evals"]) == (reps[k]["iters"], reps[k]["evals"])
