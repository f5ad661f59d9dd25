"""Training of the warm-start networks on fits produced by the plain method.

The pipeline, every numeric step of which runs in libpd's kernels:

1. plain fits: ``Context.fit`` from theta = 0 on each training map (batched);
2. per-grain descriptors (``Context.descriptors``) and local-frame targets
   (``Context.warm_targets``: the fitted theta matched to the moment seed of
   Section 5.6.2 by a common scale and shift, residual in the grain's frame);
3. the network 32 -> 256 -> 256 -> K trained by Adam on the mean squared error
   (``Context.mlp_backward`` + ``Context.mlp_adam``); the minibatch rows are
   drawn with torch's generator (data plumbing only);
4. ``save`` / ``load`` of the parameters (numpy ``.npz``, no pickled objects).

A fit then uses the network through ``Context.fit(..., init="mlp", mlp=Mlp({d:
params}))``.  ``python -m paper_2605_20816_amd.warm_train --help`` trains on the
repository's synthetic polynomial diagrams.
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np
import torch

from . import Context, Mlp, Problem, mlp_num_params, num_features


def plain_fits(ctx: Context, probs, prec="fp64", max_iter=2000, target_acc=0.99, history=10,
               batch=64):
    """Cold-start fits (theta = 0) of every map, `batch` maps per pd_fit call.
    Returns (thetas, reports)."""
    thetas, reps = [], []
    for k in range(0, len(probs), batch):
        pp = probs[k:k + batch]
        th = [torch.zeros((p.N, num_features(p.d)), dtype=torch.float64,
                          device=p.labels.device) for p in pp]
        reps += ctx.fit(pp, th, prec, init="zero", max_iter=max_iter, target_acc=target_acc,
                        history=history)
        thetas += th
    return thetas, reps


def training_rows(ctx: Context, probs, thetas):
    """(X, T): descriptors and local-frame targets of every non-empty grain, as
    float32 device tensors (rows x 32, rows x K); all maps must share one degree."""
    degs = {p.d for p in probs}
    if len(degs) != 1:
        raise ValueError("training rows of one degree at a time")
    desc, frames = ctx.descriptors(probs, frames=True)
    targets, _ = ctx.warm_targets(probs, thetas)
    X, T = [], []
    for D, F, Tg in zip(desc, frames, targets):
        keep = F[:, 6] > 0
        X.append(D[keep])
        T.append(Tg[keep])
    return torch.cat(X).contiguous(), torch.cat(T).contiguous()


def init_params(k_out: int, seed: int = 0, device="cuda"):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, in the library's
    layout [W1, b1, W2, b2, W3, b3] (input-major weights)."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    for fan_in, fan_out in ((32, 256), (256, 256), (256, k_out)):
        parts.append(torch.randn(fan_in * fan_out, generator=g, dtype=torch.float32) *
                     math.sqrt(2.0 / fan_in))
        parts.append(torch.zeros(fan_out, dtype=torch.float32))
    p = torch.cat(parts).to(device)
    assert p.numel() == mlp_num_params(k_out)
    return p


def train(ctx: Context, X, T, steps=2000, lr=1e-3, batch=4096, seed=0, params=None,
          log_every=0):
    """Adam on mean((net(X) - T)^2) with minibatches of `batch` rows.  Returns
    (params, losses per step as a numpy array)."""
    K = int(T.shape[1])
    p = init_params(K, seed, X.device) if params is None else params.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    grad = torch.empty_like(p)
    rows = X.shape[0]
    g = torch.Generator(device=X.device).manual_seed(seed + 1)
    losses = torch.empty(steps, dtype=torch.float64, device=X.device)
    for step in range(1, steps + 1):
        if rows > batch:
            idx = torch.randint(0, rows, (batch,), generator=g, device=X.device)
            xb, tb = X.index_select(0, idx).contiguous(), T.index_select(0, idx).contiguous()
        else:
            xb, tb = X, T
        ctx.mlp_backward(p, xb, tb, loss_out=losses[step - 1:step], grad_out=grad)
        ctx.mlp_adam(p, grad, m, v, step, lr)
        if log_every and step % log_every == 0:
            print(f"step {step}: loss {float(losses[step - 1]):.4e}", flush=True)
    return p, losses.cpu().numpy()


def evaluate(ctx: Context, params, X, T):
    """Mean squared error of the FP32 network on (X, T)."""
    y = ctx.mlp_forward(params, X, int(T.shape[1]), "fp32")
    return float(((y - T) ** 2).mean())


def save(path: str, nets: dict):
    """nets: {degree: params tensor}."""
    np.savez(path, **{f"degree_{d}": p.detach().cpu().numpy() for d, p in nets.items()})


def load(path: str, device="cuda") -> Mlp:
    with np.load(path, allow_pickle=False) as z:
        nets = {int(k.split("_")[1]): torch.from_numpy(z[k]).to(device) for k in z.files}
    return Mlp(nets)


def _main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--maps", type=int, default=2000, help="training maps")
    ap.add_argument("--size", type=int, default=256, help="map side")
    ap.add_argument("--degree", type=int, default=6)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--prec", default="fp64", help="precision of the plain fits")
    ap.add_argument("--max-iter", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="warm_mlp.npz")
    a = ap.parse_args()
    import synth   # the repository's synthetic grain maps
    ctx = Context(0)
    t0 = time.time()
    X, T = [], []
    for k0 in range(0, a.maps, 64):
        gms = [synth.training_map(k, H=a.size, W=a.size, D=a.degree)
               for k in range(k0, min(a.maps, k0 + 64))]
        probs = [Problem(torch.as_tensor(g.labels).cuda(), g.H, g.W, g.N, a.degree, a.eps)
                 for g in gms]
        th, reps = plain_fits(ctx, probs, a.prec, a.max_iter)
        x, t = training_rows(ctx, probs, th)
        X.append(x)
        T.append(t)
        print(f"maps {k0 + len(gms)}/{a.maps}: {sum(r['status'] == 'target' for r in reps)} "
              f"reached the target, {time.time() - t0:.1f} s", flush=True)
    X, T = torch.cat(X), torch.cat(T)
    p, losses = train(ctx, X, T, a.steps, a.lr, log_every=max(1, a.steps // 10))
    save(a.out, {a.degree: p})
    print(f"{X.shape[0]} grains, final loss {losses[-1]:.4e}, saved {a.out}")


if __name__ == "__main__":
    _main()
