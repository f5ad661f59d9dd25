"""Benchmark of the polynomial-diagram fitting hot path on one MI355X.

Workload (default): the 2048x2048 random degree-6 polynomial diagram (N = 5000
drawn, 4895 non-empty grains), fitted at degree d = 6 (K = 28) with eps = 1e-3,
in FP64 (the paper's arithmetic).  One step = one L-BFGS iteration of the device
fit: the objective + gradient evaluations of its line search over all
4895 x 4194304 pixel-grain pairs, the gauge projection, the memory update and
two-loop recursion, and the hard assignment with its accuracy check.  The steps
are timed from a non-trivial start (theta after 20 FP32 iterations from 0) by the
device clock inside pd_fit, from the decision on the first evaluation to the last
accepted iterate, so the fit's set-up (tables, indicator moments, graph capture)
is not in the figure.  The metric is pixel-grain pairs of L + grad L evaluated per
second over those steps.  Early in a fit every pair is evaluated; later most
pairs are far field and skipped (to rounding), so the same steps are also timed
from a ~95% iterate and reported apart, in dense-equivalent pairs per second.

Printed: one JSON line with the metric, the same steps in FP32 and BF16 with
their error against the FP64 oracle on a band of rows, a live roofline of the
dominant kernel (per-stage HIP-event timing on the library's stream), the CPU
oracle timed on a band of rows of the same map, time-to-99% pixel accuracy
of the plain method (FP64, theta = 0, one map at a time) against the accelerated
one (all maps in one batched fit, reduced precision, longer L-BFGS memory, with
and without the learned warm start) on a batch of c4-style maps, and on the c5
map the time to the accuracy that the plain method reaches in 100 iterations.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense): FP64 vector 78.6 TFLOP/s, FP32 vector 157.3 TFLOP/s.
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}


def flops_per_pair(stage: str, d: int) -> int:
    """Algorithmic flops per (pixel, grain) pair of one evaluation stage, with the
    logit evaluated through the row factorisation (d FMAs) and an FMA counted as
    2 flops, the exponential as 1:
      lse : logit 2d + max 1 + subtract 1 + exp 1 + add 1        = 2d + 4
      grad: logit 2d + subtract 1 + exp 1 + accumulate 2d + 1    = 4d + 3
    """
    return 2 * d + 4 if stage == "lse" else 4 * d + 3


def measured_peaks(pdl, ctx) -> dict:
    """The unit rates of pd_probe_peak (flop/s; exponentials/s for exp2 and
    fp32_fma4_exp2, which runs four FMAs per exponential)."""
    return {k: ctx.probe_peak(k) for k in pdl.Context.PEAK_KINDS}


def traffic_from_profile(kernel: str):
    """HBM bytes per launch of `kernel` from profiles/traffic_<kernel>.md (FETCH_SIZE
    and WRITE_SIZE per dispatch, each scaled by its copy-kernel calibration
    factor), or None if the summary is missing or was taken on other source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", txt, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    for name, sha in rec["sources"].items():
        src = os.path.join(ROOT, "paper_2605_20816_amd", "csrc", name)
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != sha:
            return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"])


def time_to_99(pdl, ctx, n_maps, with_net, torch, synth):
    """Plain (FP64, theta = 0, history 10, one map per call) against accelerated
    (one batched call with autotuned tiles; reduced precision; longer memory; the
    diagonal preconditioner; accuracy checked every 8 iterations; with and
    without the learned warm start) fits of c4-style maps
    to 99% pixel accuracy.  Times are from each fit call's start to the iterate
    that reaches 99% (for the batch: the last of the maps the plain method also
    brings to 99%)."""
    from paper_2605_20816_amd import warm_train as wt
    maps = [synth.config_c4_map(j) for j in range(n_maps)]
    probs = [pdl.Problem(torch.as_tensor(g.labels).cuda(), g.H, g.W, g.N, g.meta["degree"],
                         g.meta["eps"]) for g in maps]

    def zeros(pp):
        return [torch.zeros((p.N, pdl.num_features(p.d)), dtype=torch.float64, device="cuda")
                for p in pp]

    plain, plain_total = [], []
    for p in probs:
        r = ctx.fit([p], zeros([p]), "fp64", init="zero", history=10, max_iter=2000,
                    target_acc=0.99)[0]
        plain.append(r["seconds_to_target"])
        plain_total.append(r["seconds_total"])
    nets = None
    train_s = None
    if with_net:
        # networks per degree, trained on plain fits of other maps of the same kinds
        t0 = time.perf_counter()
        nets = {}
        for d in sorted({p.d for p in probs}):
            tm = [g for g in synth.batch_maps(70000 + 100 * d, 24, hw=(128, 257), grains=(20, 201),
                                              degrees=(d,))]
            tp = [pdl.Problem(torch.as_tensor(g.labels).cuda(), g.H, g.W, g.N, d, g.meta["eps"])
                  for g in tm]
            th, _ = wt.plain_fits(ctx, tp, "fp32", 2000)
            X, T = wt.training_rows(ctx, tp, th)
            nets[d], _ = wt.train(ctx, X, T, steps=2000, lr=1e-3)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
    out = {"workload": f"{n_maps} c4-style maps (seeds 404..{403 + n_maps}): sides 128..768, "
                       f"N 20..500, d 2..4, eps 1e-2 (d=2) / 1e-3",
           "plain": "FP64, theta0=0, L-BFGS memory 10, one map per pd_fit call",
           "target_acc": 0.99, "budget_iters": 2000}
    # accelerated: one batched call; tiles autotuned for the batch; longer memory;
    # the diagonal preconditioner (refreshed every 40 iterations); accuracy checked
    # every 8 iterations (settings chosen on c4-style maps 16..31, not the 16 timed here)
    tune_s = {}
    for prec in ("fp32", "bf16"):
        t0 = time.perf_counter()
        waves = ctx.autotune(probs, zeros(probs), prec)
        tune_s[prec] = time.perf_counter() - t0
        out[f"autotuned_waves_per_map_{prec}"] = waves
    out["autotune_seconds_included"] = tune_s
    fast = dict(history=16, precondition=40, check_every=8)
    variants = [("accelerated_fp32", "fp32", "zero", None, fast),
                ("accelerated_bf16", "bf16", "zero", None, fast)]
    if with_net:
        variants.append(("accelerated_fp32_mlp", "fp32", "mlp", pdl.Mlp(nets), fast))
        variants.append(("accelerated_bf16_mlp", "bf16", "mlp", pdl.Mlp(nets), fast))
    for name, prec, init, mlp, kw in variants:
        reps = ctx.fit(probs, zeros(probs), prec, init=init, mlp=mlp, max_iter=2000,
                       target_acc=0.99, **kw)
        both = [k for k in range(n_maps) if plain[k] > 0 and reps[k]["seconds_to_target"] > 0]
        t_plain = sum(plain[k] for k in both)
        t_acc = (max(reps[k]["seconds_to_target"] for k in both) + tune_s[prec]) if both else None
        # the whole workload: a map that misses 99% is charged its whole fit
        # (the budget), in both runs
        t_plain_all = sum(plain[k] if plain[k] > 0 else plain_total[k] for k in range(n_maps))
        t_acc_all = max(r["seconds_to_target"] if r["seconds_to_target"] > 0 else r["seconds_total"]
                        for r in reps) + tune_s[prec]
        out[name] = {"settings": dict(prec=prec, init=init, **kw),
                     "maps_at_99": len(both), "plain_seconds": t_plain, "seconds": t_acc,
                     "speedup": (t_plain / t_acc) if t_acc else None,
                     "plain_maps_at_99": sum(t > 0 for t in plain),
                     "maps_at_99_this_mode": sum(r["seconds_to_target"] > 0 for r in reps),
                     "speedup_all_maps_misses_at_budget": t_plain_all / t_acc_all}
    if train_s is not None:
        out["network_training_seconds_excluded"] = train_s
    return out


def c5_equal_accuracy(pdl, ctx, prob, torch, synth, plain_iters, with_net):
    """The c5 map at equal pixel accuracy: the plain method (FP64, theta = 0,
    L-BFGS memory 10) for `plain_iters` iterations sets the accuracy; each
    accelerated fit (reduced precision, memory 16, a warm start) stops at the
    first accepted iterate that reaches it.  99% is out of reach of every fit of
    this map within minutes (from the moment seed an FP32 fit reaches 95.5% in 150
    iterations and 96.2% in 1200), so the comparison is made at the accuracy the
    plain fit reaches.  Times are from each call's start (set-up and warm start
    included; the network's training excluded)."""
    from paper_2605_20816_amd import warm_train as wt
    K = pdl.num_features(prob.d)

    def z():
        return torch.zeros((prob.N, K), dtype=torch.float64, device="cuda")

    rp = ctx.fit([prob], [z()], "fp64", init="zero", history=10, max_iter=plain_iters,
                 target_acc=2.0)[0]
    acc_p, t_p = rp["acc"], rp["seconds_total"]
    out = {"plain": {"settings": "FP64, theta0=0, L-BFGS memory 10", "iters": rp["iters"],
                     "acc": acc_p, "seconds": t_p}}
    variants = [("fp32_cold", "fp32", "zero", {}), ("fp32_seed", "fp32", "heuristic", {}),
                ("bf16_seed", "bf16", "heuristic", {})]
    if with_net:
        # a network for degree 6, trained on plain fits of 256x256 degree-6 maps
        t0 = time.perf_counter()
        tm = [synth.training_map(k) for k in range(48)]
        tp = [pdl.Problem(torch.as_tensor(g.labels).cuda(), g.H, g.W, g.N, 6, g.meta["eps"])
              for g in tm]
        th, _ = wt.plain_fits(ctx, tp, "fp32", 2000)
        X, T = wt.training_rows(ctx, tp, th)
        net, _ = wt.train(ctx, X, T, steps=2000, lr=1e-3)
        torch.cuda.synchronize()
        out["network_training_seconds_excluded"] = time.perf_counter() - t0
        mlp = pdl.Mlp({6: net})
        variants += [("bf16_mlp", "bf16", "mlp", {"mlp": mlp}), ("fp32_mlp", "fp32", "mlp", {"mlp": mlp})]
    for name, prec, init, kw in variants:
        r = ctx.fit([prob], [z()], prec, init=init, history=16, max_iter=4 * plain_iters,
                    target_acc=acc_p, check_every=2, **kw)[0]
        t = r["seconds_to_target"]
        out[name] = {"settings": dict(prec=prec, init=init, history=16), "status": r["status"],
                     "iters": r["iters"], "acc": r["acc"], "seconds": t if t > 0 else None,
                     "speedup": (t_p / t) if t > 0 else None}
    return out


def points_throughput(pdl, ctx, torch, synth, n=262144, N=2000, d=4):
    """Unstructured 3-D points (uniform in [-1, 1]^3, labelled by a random power
    diagram of N sites), degree d (K = 35 at d = 4): one call of
    pd_points_objective_grad (features, objective, gradient, reductions), timed
    with events over 5 calls after one warm-up, FP64 and FP32.  Algorithmic flops per pair as
    for the grid with K-FMA logits: objective 2K + 4, gradient 4K + 3."""
    rng = np.random.default_rng(2025)
    X, lab, Nn = synth.power_points(n, 3, N, rng)
    K = pdl.points_num_features(3, d)
    th = torch.as_tensor(rng.normal(size=(Nn, K)) * 0.05 / np.sqrt(K)).cuda()
    q = pdl.Points(torch.as_tensor(X).cuda(), torch.as_tensor(lab).cuda(), Nn, d, 1e-2)
    pairs = n * Nn
    out = {"workload": f"{n} points in [-1,1]^3, {Nn} grains (random power diagram), d={d} (K={K}), "
                       "eps=1e-2", "pairs": pairs}
    for prec in ("fp64", "fp32"):
        ctx.points_objective_grad([q], [th], prec)
        torch.cuda.synchronize()
        # the library launches on torch's current stream, so its events bracket
        # exactly the five calls' kernels
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            ctx.points_objective_grad([q], [th], prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        fl = (2 * K + 4 + 4 * K + 3) * pairs
        out[prec] = {"ms_per_evaluation": ms, "pairs_per_s": pairs / (ms * 1e-3),
                     "tflops": fl / (ms * 1e-3) / 1e12,
                     "frac": fl / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec]}
    return out


def roofline_at_scale(pdl, ctx, torch, synth, n_maps=16):
    """The evaluation kernels at scale: the c4-style batch (about 6e8 pairs per
    evaluation), FP32, with its autotuned tiles, at theta after 20 batched FP32
    iterations from 0 (at theta = 0 every grain ties and the certified objective
    hands every pixel to the canonical pass); flops per pair as in flops_per_pair
    with each map's own degree."""
    maps = [synth.config_c4_map(j) for j in range(n_maps)]
    probs = [pdl.Problem(torch.as_tensor(g.labels).cuda(), g.H, g.W, g.N, g.meta["degree"],
                         g.meta["eps"]) for g in maps]
    ths = [torch.zeros((p.N, pdl.num_features(p.d)), dtype=torch.float64, device="cuda")
           for p in probs]
    ctx.autotune(probs, ths, "fp32")
    ctx.fit(probs, ths, "fp32", init="zero", max_iter=20, target_acc=2.0, history=16)
    st = ctx.profile_eval(probs, ths, "fp32", reps=10)
    out = {"workload": f"{n_maps} c4-style maps, FP32, theta after 20 FP32 iterations, autotuned tiles",
           "pairs": int(sum(p.H * p.W * p.N for p in probs)),
           "stage_ms": {k: round(v, 4) for k, v in st.items()}}
    for stage in ("lse", "grad"):
        fl = sum(flops_per_pair(stage, p.d) * p.H * p.W * p.N for p in probs)
        ach = fl / (st[stage] * 1e-3) / 1e12
        out[f"k_{stage}"] = {"achieved_tflops": round(ach, 2), "frac": round(ach / PEAK_TFLOPS["fp32"], 4),
                             "frac_of_nonpacked_fp32": round(ach / (PEAK_TFLOPS["fp32"] / 2), 4)}
    return out


def fit_steps(ctx, prob, th0, prec, steps, torch):
    """`steps` L-BFGS iterations from th0 (a copy); returns (ms per step, evaluations
    in the window, the report) from the device-clock window of the report."""
    th = th0.clone()
    torch.cuda.synchronize()
    rep = ctx.fit([prob], [th], prec, init="given", max_iter=steps, target_acc=2.0)[0]
    torch.cuda.synchronize()
    if rep["iters"] < 1 or rep["seconds_iterating"] <= 0:
        raise RuntimeError(f"fit made no timed step: {rep}")
    return rep["seconds_iterating"] / rep["iters"] * 1e3, rep["evals_iterating"], rep, th


def band_errors(ctx, orc_rows, prob, th, prec, band, torch):
    """Errors of Phi and grad Phi over a band of rows against the oracle's sums
    over the same rows (phi relative; gradient max |diff| / max |ref|)."""
    v, g = orc_rows
    n = prob.H * prob.W
    pr, gr = v / n, -g / (prob.eps * n)
    phi, gg = ctx.objective_grad_rows([prob], [th], [band], prec)
    gd = gg[0].cpu().numpy()
    return {"phi_rel": abs(float(phi[0]) - pr) / abs(pr),
            "grad_max_rel": float(np.max(np.abs(gd - gr)) / np.max(np.abs(gr)))}


def summarize_trace(path: str, top: int = 30) -> str:
    """Markdown summary of a rocprofv3 --kernel-trace CSV: per kernel, the number
    of launches and their average duration, and the same over the working
    launches only.  A fit captures several steps per graph, and a map that has
    stopped leaves its later steps as gated launches that return at once; those
    (under 2% of the kernel's longest launch) are counted apart, so the working
    average is the one to compare with a live per-launch timing."""
    import csv
    durs = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            d = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
            durs.setdefault(row["Kernel_Name"], []).append(d)
    lines = ["| kernel | launches | avg us (all) | working launches | avg us (working) | total ms |",
             "|---|---|---|---|---|---|"]
    for name, ds in sorted(durs.items(), key=lambda kv: -sum(kv[1]))[:top]:
        mx = max(ds)
        work = [d for d in ds if d >= 0.02 * mx]
        lines.append(f"| `{name}` | {len(ds)} | {sum(ds) / len(ds) / 1e3:.2f} | {len(work)} | "
                     f"{sum(work) / len(work) / 1e3:.2f} | {sum(ds) / 1e6:.2f} |")
    return "\n".join(lines)


def summarize_counters(path: str) -> str:
    """Markdown summary of a rocprofv3 --pmc counter CSV: per kernel and counter,
    the dispatches and the average counter value per dispatch over the working
    dispatches (those whose counter sum is at least 2% of the kernel's largest:
    gated launches of a stopped map read almost nothing)."""
    import csv
    vals = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            key = (row["Kernel_Name"], row["Counter_Name"])
            vals.setdefault(key, {}).setdefault(row["Dispatch_Id"], 0.0)
            vals[key][row["Dispatch_Id"]] += float(row["Counter_Value"])
    lines = ["| kernel | counter | dispatches | working | avg per working dispatch |",
             "|---|---|---|---|---|"]
    for (name, ctr), per in sorted(vals.items(), key=lambda kv: -sum(kv[1].values()))[:40]:
        v = list(per.values())
        mx = max(v) if v else 0.0
        work = [x for x in v if x >= 0.02 * mx] or v
        lines.append(f"| `{name}` | {ctr} | {len(v)} | {len(work)} | {sum(work) / len(work):.6g} |")
    return "\n".join(lines)


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--summarize-trace":
        print(summarize_trace(sys.argv[2]))
        return
    if len(sys.argv) == 3 and sys.argv[1] == "--summarize-counters":
        print(summarize_counters(sys.argv[2]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed L-BFGS iterations")
    ap.add_argument("--warmup", type=int, default=5, help="untimed iterations first")
    ap.add_argument("--start-iters", type=int, default=20,
                    help="FP32 iterations from theta = 0 that give the start of the timed steps")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--late-steps", type=int, default=20,
                    help="steps timed again from a ~95%% iterate, where far-field skipping "
                         "acts (0 skips it)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--t99-maps", type=int, default=16,
                    help="c4-style maps in the time-to-99%% comparison (0 skips it)")
    ap.add_argument("--c5-plain-iters", type=int, default=100,
                    help="iterations of the plain FP64 c5 fit that set the accuracy of the "
                         "equal-accuracy comparison (0 skips it)")
    ap.add_argument("--points", type=int, default=1,
                    help="also time the unstructured 3-D point-set path (0 skips it)")
    ap.add_argument("--no-net", action="store_true",
                    help="skip the learned warm start in the time-to-99%% comparison")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a plain copy of known size "
                         "that calibrates hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the pixel-sharded design is described in DESIGN.md); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2605_20816_amd as pdl
    import synth

    if args.copy_probe:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = pdl.Context(0)
    gm = synth.config_c5()
    d, eps = gm.meta["degree"], gm.meta["eps"]
    H, W, N = gm.H, gm.W, gm.N
    K = pdl.num_features(d)
    prob = pdl.Problem(torch.as_tensor(gm.labels).cuda(), H, W, N, d, eps)
    pairs = H * W * N
    print(f"bench: {H}x{W} N={N} d={d} loaded", file=sys.stderr, flush=True)

    th0 = torch.zeros((N, K), dtype=torch.float64, device="cuda")
    ctx.fit([prob], [th0], "fp32", init="zero", max_iter=args.start_iters, target_acc=2.0)

    steps = {}
    for prec in [args.prec] + [q for q in ("fp64", "fp32", "bf16") if q != args.prec]:
        if args.warmup:
            fit_steps(ctx, prob, th0, prec, args.warmup, torch)
        ms, evals, rep, th_end = fit_steps(ctx, prob, th0, prec, args.steps, torch)
        steps[prec] = dict(ms=ms, evals=evals, rep=rep, th=th_end)
        print(f"bench: {prec} {ms:.3f} ms/step ({evals} evaluations in {rep['iters']} steps)",
              file=sys.stderr, flush=True)
    main_s = steps[args.prec]
    value = main_s["evals"] * pairs / (main_s["ms"] * 1e-3 * main_s["rep"]["iters"])

    # the same steps later in a fit, where most pixel-grain pairs are far field:
    # from the moment seed plus 150 FP32 iterations (about 95% accuracy)
    late = None
    if args.late_steps:
        th1 = torch.zeros((N, K), dtype=torch.float64, device="cuda")
        r1 = ctx.fit([prob], [th1], "fp32", init="heuristic", max_iter=150, target_acc=2.0,
                     history=16)[0]
        late = {"start": "moment seed + 150 FP32 L-BFGS iterations", "start_acc": r1["acc"]}
        for prec in ("fp64", "fp32", "bf16"):
            ms, ev, rep, _ = fit_steps(ctx, prob, th1, prec, args.late_steps, torch)
            late[prec] = {"ms_per_step": ms, "dense_pairs_per_s": ev * pairs / (ms * 1e-3 * rep["iters"]),
                          "evals": ev, "iters": rep["iters"]}
            print(f"bench: late {prec} {ms:.3f} ms/step", file=sys.stderr, flush=True)

    # errors against the FP64 oracle over a band of rows at the start theta
    band = (1020, 1028)
    import oracle
    oracle.build(force=False)
    x0 = th0.cpu().numpy()
    orc_band = oracle.objective_rows(x0, gm.labels, H, W, d, eps, *band)
    errs = {q: band_errors(ctx, orc_band, prob, th0, q, band, torch) for q in ("fp64", "fp32", "bf16")}
    F_band, nc_band, _ = oracle.assign_rows(x0, H, W, d, *band, gm.labels)
    outs, _ = ctx.assign([prob], [th0])
    assign_exact = bool(np.array_equal(outs[0].cpu().numpy()[band[0] * W:band[1] * W], F_band))

    # live roofline of the dominant kernel, at the start theta
    st = ctx.profile_eval([prob], [th0], args.prec, reps=5)
    dom = max(("lse", "grad"), key=lambda k: st[k])
    fl = flops_per_pair(dom, d) * pairs
    achieved = fl / (st[dom] * 1e-3) / 1e12
    peak = PEAK_TFLOPS["fp64" if args.prec == "fp64" else "fp32"]
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": traffic_from_profile(f"k_{dom}"), "kernel": f"k_{dom}",
            "ms_per_launch": round(st[dom], 5), "flops_per_pair": flops_per_pair(dom, d),
            "pairs_per_launch": pairs,
            "stage_ms": {k: round(v, 5) for k, v in st.items()},
            "measured_peaks": {k: float(f"{v:.4g}") for k, v in measured_peaks(pdl, ctx).items()}}

    t99 = time_to_99(pdl, ctx, args.t99_maps, not args.no_net, torch, synth) if args.t99_maps else None
    at_scale = roofline_at_scale(pdl, ctx, torch, synth) if args.t99_maps else None
    c5eq = (c5_equal_accuracy(pdl, ctx, prob, torch, synth, args.c5_plain_iters, not args.no_net)
            if args.c5_plain_iters else None)
    pts = points_throughput(pdl, ctx, torch, synth) if args.points else None

    cpu = None
    if not args.no_cpu:
        # the oracle over bands of 16 rows of the same map at the same theta, for
        # about 10 s of host time
        rows_done, r0, t0 = 0, 0, time.perf_counter()
        while time.perf_counter() - t0 < 10.0 and r0 < H:
            oracle.objective_rows(x0, gm.labels, H, W, d, eps, r0, min(r0 + 16, H))
            rows_done += min(16, H - r0)
            r0 += 16
        cs = time.perf_counter() - t0
        cpu = {"value": rows_done * W * N / cs, "unit": "pairs/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"FP64 L + grad L over rows 0..{rows_done - 1} ({rows_done} of {H} rows, "
                         f"{rows_done * W * N:.3g} pairs) of the same map at the same theta"}

    other = {}
    for q in ("fp64", "fp32", "bf16"):
        if q == args.prec:
            continue
        o = steps[q]
        other[q] = {"value": o["evals"] * pairs / (o["ms"] * 1e-3 * o["rep"]["iters"]),
                    "ms_per_step": o["ms"], "err_vs_oracle_rows_1020_1028": errs[q],
                    "acc_after_steps": o["rep"]["acc"],
                    "acc_after_steps_fp64": steps["fp64"]["rep"]["acc"]}
    rep = main_s["rep"]
    out = {
        "metric": "pixel-grain evals/s for L+grad L (device L-BFGS fit step)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_s["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{H}x{W} random degree-6 polynomial diagram, N=5000 drawn "
                               f"({N} non-empty), fit at d=6 (K=28), eps=1e-3, from theta after "
                               f"{args.start_iters} FP32 L-BFGS iterations",
                   "pixels": H * W, "grains": N, "degree": d, "evals": rep["evals_iterating"],
                   "iters": rep["iters"], "parallelism": "single GPU"},
        "err_vs_oracle_rows_1020_1028": errs[args.prec],
        "assign_rows_1020_1028_bit_exact": assign_exact,
        "other_precision": other,
        "steps_at_a_late_iterate": late,
        "roofline": roof,
        "roofline_at_scale": at_scale,
        "cpu_baseline": cpu,
        "time_to_99": t99,
        "c5_equal_accuracy": c5eq,
        "points_3d": pts,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
