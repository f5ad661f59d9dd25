"""Benchmark of the polynomial-diagram fitting hot path on one MI355X.

Workload (default): the 256x256 anisotropic-power-diagram map with N = 100
grains (90 non-empty), 1% boundary noise, fitted at degree d = 2 (K = 6) with
eps = 1e-2 from theta = 0.  One step = one L-BFGS iteration of the device fit
(objective + gradient evaluations of the line search, gauge projection, memory
update, two-loop recursion, hard assignment and accuracy check).  The metric is
pixel-grain pairs of L + grad L evaluated per second over the timed steps.

Printed: one JSON line with the metric, a live roofline of the dominant kernel
(per-stage HIP-event timing on the library's stream), the CPU oracle timed on a
bounded sample, and time-to-99% of the 64x64 power-diagram fit.
"""
from __future__ import annotations

import argparse
import json
import os
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the pixel-sharded design is described in DESIGN.md); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2605_20816_amd as pdl
    import synth

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

    # live roofline of the dominant kernel, at the fitted parameters
    st = ctx.profile_eval([prob], [th], args.prec, reps=50)
    dom = max(("lse", "grad"), key=lambda s: st[s])
    fl = flops_per_pair(dom, d) * pairs
    achieved = fl / (st[dom] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[args.prec],
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[args.prec], 4),
            "traffic": None, "kernel": f"k_{dom}", "ms_per_launch": round(st[dom], 5),
            "flops_per_pair": flops_per_pair(dom, d),
            "stage_ms": {k: round(v, 5) for k, v in st.items()}}

    # time to 99% on the 64x64 N = 8 power-diagram map (FP64 plain fit from zero)
    c1 = synth.config_c1()
    p1 = pdl.Problem(torch.as_tensor(c1.labels).cuda(), c1.H, c1.W, c1.N, 1, 1e-2)
    ctx.fit([p1], [torch.zeros((c1.N, 3), dtype=torch.float64, device="cuda")], "fp64",
            init="zero", max_iter=2000, target_acc=0.99)
    r1 = ctx.fit([p1], [torch.zeros((c1.N, 3), dtype=torch.float64, device="cuda")], "fp64",
                 init="zero", max_iter=2000, target_acc=0.99)[0]
    t99 = {"workload": "64x64 power diagram, N=8, d=1, eps=1e-2, FP64, theta0=0",
           "seconds": r1["seconds_to_target"], "iters": r1["iters"], "evals": r1["evals"],
           "acc": r1["acc"]}

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
        obj = lambda t: oracle.objective_grad(t, c1.labels, c1.H, c1.W, 1, 1e-2)
        acc = lambda t: oracle.assign(t, c1.H, c1.W, 1, c1.labels)[1] / (c1.H * c1.W)
        t0 = time.perf_counter()
        ro = oracle.lbfgs_fit(obj, np.zeros((c1.N, 3)), accuracy=acc, target_acc=0.99)
        t99["cpu_oracle_seconds"] = time.perf_counter() - t0
        t99["cpu_oracle_iters"] = ro["iters"]

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
        "cpu_baseline": cpu,
        "time_to_99": t99,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
