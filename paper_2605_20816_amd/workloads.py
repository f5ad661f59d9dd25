"""Named workloads for profiling the library under rocprofv3.

    python -m paper_2605_20816_amd.workloads <name> [--reps R]

  c3_eval   1024x1024 degree-4 polynomial map (N = 974), eps = 1e-3: R objective +
            gradient evaluations in each precision (FP64, FP32, BF16) at theta
            after 20 FP32 L-BFGS iterations.
  c5_eval   2048x2048 degree-6 polynomial map (N = 4895), eps = 1e-3: the same at
            theta = 0 (FP32 and BF16).
  c4_fit    the first 16 maps of the 64-map c4 batch: one batched FP32 fit
            (tiles autotuned for the batch, memory 16, diagonal preconditioner
            refreshed every 40 iterations, accuracy checked every 8 iterations)
            to 99% pixel accuracy or 2000 iterations.

The maps are the repository's seeded synthetic grain maps (module `synth`).
"""
from __future__ import annotations

import argparse
import os
import sys
import time


def _maps():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    return synth


def main():
    ap = argparse.ArgumentParser(description="profiling workloads")
    ap.add_argument("name", choices=["c3_eval", "c5_eval", "c4_fit"])
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    import torch

    from . import Context, Problem, num_features
    synth = _maps()
    ctx = Context(0)
    t0 = time.perf_counter()
    if a.name in ("c3_eval", "c5_eval"):
        gm = synth.config_c3() if a.name == "c3_eval" else synth.config_c5()
        d = gm.meta["degree"]
        p = Problem(torch.as_tensor(gm.labels).cuda(), gm.H, gm.W, gm.N, d, gm.meta["eps"])
        th = torch.zeros((gm.N, num_features(d)), dtype=torch.float64, device="cuda")
        if a.name == "c3_eval":
            ctx.fit([p], [th], "fp32", init="zero", max_iter=20, target_acc=2.0)
        precs = ("fp64", "fp32", "bf16") if a.name == "c3_eval" else ("fp32", "bf16")
        for prec in precs:
            for _ in range(a.reps):
                phi, _ = ctx.objective_grad([p], [th], prec)
            torch.cuda.synchronize()
            print(f"{a.name} {prec}: Phi = {float(phi[0]):.6f}", flush=True)
    else:
        maps = [synth.config_c4_map(j) for j in range(16)]
        probs = [Problem(torch.as_tensor(g.labels).cuda(), g.H, g.W, g.N, g.meta["degree"],
                         g.meta["eps"]) for g in maps]
        zeros = lambda: [torch.zeros((q.N, num_features(q.d)), dtype=torch.float64,
                                     device="cuda") for q in probs]
        ctx.autotune(probs, zeros(), "fp32")
        reps = ctx.fit(probs, zeros(), "fp32", init="zero", history=16, precondition=40,
                       check_every=8, max_iter=2000, target_acc=0.99)
        torch.cuda.synchronize()
        print(f"c4_fit: {sum(r['status'] == 'target' for r in reps)} of 16 maps at 99%, "
              f"longest time to 99% {max(r['seconds_to_target'] for r in reps):.3f} s", flush=True)
    print(f"done in {time.perf_counter() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
