"""Benchmark of the polynomial-diagram fitting hot path on one MI355X.

Workload (default): the 256x256 anisotropic-power-diagram map with N = 100
grains (90 non-empty), 1% boundary noise, fitted at degree d = 2 (K = 6) with
eps = 1e-2 from theta = 0.  One step = one L-BFGS iteration of the device fit
(objective + gradient evaluations of the line search, gauge projection, memory
update, two-loop recursion, hard assignment and accuracy check).  The metric is
pixel-grain pairs of L + grad L evaluated per second over the timed steps.

Printed: one JSON line with the metric, a live roofline of the dominant kernel
(per-stage HIP-event timing on the library's stream; HBM traffic from the
committed rocprofv3 counter summary when it was taken on the current kernel
source), the CPU oracle timed on a bounded sample, and time-to-99% pixel
accuracy of the plain method (FP64, theta = 0, one map at a time) against the
accelerated one (all maps in one batched fit, reduced precision, longer L-BFGS
memory, with and without the learned warm start) on a batch of c4-style maps.
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


def valu_per_pair(stage: str, d: int):
    """Vector instructions per (pixel, grain) pair in the FP32 inner loops as
    compiled for gfx950 (counted in the assembly; one of them the exponential):
      k_lse,  8 grains per pass: 40 + 8 d (8 d FMAs, 8 moves of the first row
              coefficient into a vector register -- one scalar operand per
              instruction --, 4 max3, 9 subtract + 9 exp + 1 multiply for the
              running rescale, 8 adds)                     -> 5 + d per pair,
              of which 9/8 exponentials
      k_grad, per pixel column: d FMAs logit, 1 subtract, 1 exp, 1 add, d FMAs
              accumulate                                   -> 2 d + 3, 1 exp
    """
    if stage == "lse":
        return 5 + d, 9 / 8
    return 2 * d + 3, 1.0


def issue_ceiling(stage: str, d: int, peaks: dict) -> float:
    """Pairs/s that the vector issue rate allows: every instruction takes one FMA
    slot except the exponential, which takes fma_rate / exp_rate slots (measured:
    the two do not overlap)."""
    n, n_exp = valu_per_pair(stage, d)
    fma_rate = peaks["fp32_fma"] / 2  # FMAs per second over all lanes
    exp_cost = fma_rate / peaks["exp2"]
    return fma_rate / (n + n_exp * (exp_cost - 1.0))


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

    plain = []
    for p in probs:
        r = ctx.fit([p], zeros([p]), "fp64", init="zero", history=10, max_iter=2000,
                    target_acc=0.99)[0]
        plain.append(r["seconds_to_target"])
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
        out[name] = {"settings": dict(prec=prec, init=init, **kw),
                     "maps_at_99": len(both), "plain_seconds": t_plain, "seconds": t_acc,
                     "speedup": (t_plain / t_acc) if t_acc else None,
                     "plain_maps_at_99": sum(t > 0 for t in plain),
                     "maps_at_99_this_mode": sum(r["seconds_to_target"] > 0 for r in reps)}
    if train_s is not None:
        out["network_training_seconds_excluded"] = train_s
    return out


def roofline_at_scale(pdl, ctx, torch, synth, peaks, n_maps=16):
    """The evaluation kernels at scale: the c4-style batch (about 6e8 pairs per
    evaluation) at theta = 0, FP32, with its autotuned tiles; flops per pair as in
    flops_per_pair with each map's own degree."""
    maps = [synth.config_c4_map(j) for j in range(n_maps)]
    probs = [pdl.Problem(torch.as_tensor(g.labels).cuda(), g.H, g.W, g.N, g.meta["degree"],
                         g.meta["eps"]) for g in maps]
    ths = [torch.zeros((p.N, pdl.num_features(p.d)), dtype=torch.float64, device="cuda")
           for p in probs]
    ctx.autotune(probs, ths, "fp32")
    st = ctx.profile_eval(probs, ths, "fp32", reps=10)
    out = {"workload": f"{n_maps} c4-style maps, FP32, theta = 0, autotuned tiles",
           "pairs": int(sum(p.H * p.W * p.N for p in probs)),
           "stage_ms": {k: round(v, 4) for k, v in st.items()}}
    for stage in ("lse", "grad"):
        fl = sum(flops_per_pair(stage, p.d) * p.H * p.W * p.N for p in probs)
        ach = fl / (st[stage] * 1e-3) / 1e12
        # issue-bound time of the batch: each map's pairs at its own degree's ceiling
        t_min = sum(p.H * p.W * p.N / issue_ceiling(stage, p.d, peaks) for p in probs)
        out[f"k_{stage}"] = {"achieved_tflops": round(ach, 2), "frac": round(ach / PEAK_TFLOPS["fp32"], 4),
                             "frac_of_nonpacked_fp32": round(ach / (PEAK_TFLOPS["fp32"] / 2), 4),
                             "frac_of_issue_ceiling": round(t_min / (st[stage] * 1e-3), 4)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 2000 steps: the paper's iteration budget, and long enough (~0.1 s) that the
    # per-call set-up of pd_fit and the GPU's clock state do not move the rate
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--t99-maps", type=int, default=16,
                    help="c4-style maps in the time-to-99%% comparison (0 skips it)")
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
    gm = synth.config_c2()
    d, eps = 2, 1e-2
    H, W, N = gm.H, gm.W, gm.N
    K = pdl.num_features(d)
    prob = pdl.Problem(torch.as_tensor(gm.labels).cuda(), H, W, N, d, eps)
    pairs = H * W * N

    def run_fit(iters, prec):
        th = torch.zeros((N, K), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = ctx.fit([prob], [th], prec, init="zero", max_iter=iters, target_acc=2.0)[0]
        torch.cuda.synchronize()
        return time.perf_counter() - t0, rep, th

    run_fit(args.warmup, args.prec)
    secs, rep, th = run_fit(args.steps, args.prec)
    value = rep["evals"] * pairs / secs
    other = "fp64" if args.prec == "fp32" else "fp32"
    run_fit(args.warmup, other)
    secs_o, rep_o, _ = run_fit(args.steps, other)

    peaks = measured_peaks(pdl, ctx)
    # live roofline of the dominant kernel, at the fitted parameters
    st = ctx.profile_eval([prob], [th], args.prec, reps=50)
    dom = max(("lse", "grad"), key=lambda s: st[s])
    fl = flops_per_pair(dom, d) * pairs
    achieved = fl / (st[dom] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[args.prec],
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[args.prec], 4),
            "traffic": traffic_from_profile(f"k_{dom}"), "kernel": f"k_{dom}",
            "ms_per_launch": round(st[dom], 5), "flops_per_pair": flops_per_pair(dom, d),
            "frac_of_nonpacked": round(achieved / (PEAK_TFLOPS[args.prec] / (2 if args.prec == "fp32" else 1)), 4),
            "stage_ms": {k: round(v, 5) for k, v in st.items()},
            "measured_peaks": {k: float(f"{v:.4g}") for k, v in peaks.items()}}
    if args.prec == "fp32":
        roof["frac_of_issue_ceiling"] = round(
            pairs / issue_ceiling(dom, d, peaks) / (st[dom] * 1e-3), 4)
    t99 = time_to_99(pdl, ctx, args.t99_maps, not args.no_net, torch, synth) if args.t99_maps else None
    at_scale = roofline_at_scale(pdl, ctx, torch, synth, peaks) if args.t99_maps else None

    cpu = None
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        th0 = th.cpu().numpy()
        n_eval, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 10.0:
            oracle.objective_grad(th0, gm.labels, H, W, d, eps)
            n_eval += 1
        cs = time.perf_counter() - t0
        cpu = {"value": n_eval * pairs / cs, "unit": "pairs/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{n_eval} full FP64 L+grad L evaluations of the 256x256 N={N} d=2 map"}

    out = {
        "metric": "pixel-grain evals/s for L+grad L (device L-BFGS fit step)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "256x256 anisotropic power diagram, N=100 (90 non-empty), "
                               "1% boundary noise, d=2 (K=6), eps=1e-2, theta0=0",
                   "pixels": H * W, "grains": N, "degree": d, "evals": rep["evals"],
                   "iters": rep["iters"], "parallelism": "single GPU"},
        "other_precision": {"dtype": "f32" if other == "fp32" else "f64",
                            "value": rep_o["evals"] * pairs / secs_o,
                            "ms_per_step": secs_o / args.steps * 1e3},
        "roofline": roof,
        "roofline_at_scale": at_scale,
        "cpu_baseline": cpu,
        "time_to_99": t99,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
