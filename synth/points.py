"""Seeded unstructured point sets in 2-D and 3-D labelled by a random power
diagram (nearest site in the power distance |x - y_i|^2 - w_i, first index on
ties).  Input generation only: nothing of the method is computed here."""
from __future__ import annotations

import numpy as np


def power_points(n: int, D: int, N: int, rng, wmax: float = 0.02):
    """n points uniform in [-1, 1]^D, N sites uniform, weights U[0, wmax]; grains
    that own no point are dropped and the labels compacted.  Returns (X (n x D)
    float64, labels int32, number of non-empty grains)."""
    X = rng.uniform(-1.0, 1.0, size=(n, D))
    y = rng.uniform(-1.0, 1.0, size=(N, D))
    w = rng.uniform(0.0, wmax, size=N)
    lab = np.empty(n, np.int64)
    for s in range(0, n, 65536):
        xb = X[s:s + 65536]
        d2 = ((xb[:, None, :] - y[None, :, :]) ** 2).sum(-1) - w[None, :]
        lab[s:s + 65536] = np.argmin(d2, axis=1)
    keep = np.unique(lab)
    remap = np.full(N, -1, np.int64)
    remap[keep] = np.arange(keep.size)
    return X, remap[lab].astype(np.int32), int(keep.size)
