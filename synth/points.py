"""Seeded unstructured point sets in 2-D and 3-D labelled by a random power
diagram (nearest site in the power distance |x - y_i|^2 - w_i, evaluated as
(|y_i|^2 - w_i) - 2 x.y_i, first index on ties).  Input generation only: nothing
of the method is computed here."""
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
    c = (y * y).sum(1) - w  # |x - y|^2 - w = |x|^2 - 2 x.y + (|y|^2 - w)
    for s in range(0, n, 16384):
        xb = X[s:s + 16384]
        lab[s:s + 16384] = np.argmin(c[None, :] - 2.0 * (xb @ y.T), axis=1)
    keep = np.unique(lab)
    remap = np.full(N, -1, np.int64)
    remap[keep] = np.arange(keep.size)
    return X, remap[lab].astype(np.int32), int(keep.size)
