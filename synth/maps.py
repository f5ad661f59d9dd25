"""Seeded synthetic grain maps for the polynomial-diagram workloads.

Recipes (all with ``numpy.random.default_rng(seed)``, draws in the order
sites, weights, matrices, coefficients, noise):

* power diagram (Section 2.3.1): sites uniform in [-1,1]^2, weights uniform in
  [0, wmax]; pixel x goes to the cell minimising |x - y_i|^2 - w_i.
* anisotropic power diagram (eq. L-APD): A_i = R(phi) diag(l1, l2) R(phi)^T with
  l log-uniform in [lmin, lmax] and phi uniform in [0, pi); score
  (x - y_i).A_i(x - y_i) - w_i.
* random polynomial diagram of degree D: the power-diagram part
  (|y_i|^2 - w_i) - 2 y_i.x plus sigma * xi, xi_{i,(a,b)} ~ N(0, 1/(a+b+1)^2) on
  the Legendre products P_a(x1) P_b(x2), a + b <= D; h = 2/sqrt(N) (the typical
  site spacing), weights uniform in [0, h^2/8], sigma = h^2/16 (chosen so that
  at least 95% of the cells are non-empty at N = 1000, D = 4 and N = 250, D = 6).
* boundary noise: a pixel is on a boundary when a 4-neighbour has another
  label; round(frac * #boundary) of them, drawn without replacement, take a
  label drawn uniformly from their distinct differing 4-neighbour labels.

Ties in the labelling go to the smallest index (numpy argmin).  Labels of empty
cells are compacted away; ``keep`` lists the surviving original indices.
Pixel (r, c) of an H x W map sits at ((2c+1-W)/W, (2r+1-H)/H).
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as npleg


@dataclass
class GrainMap:
    H: int
    W: int
    labels: np.ndarray            # int32, H*W, row-major, values 0..N-1
    N: int
    kind: str
    degree_truth: int             # degree of the generating diagram
    coef: np.ndarray | None = None  # N x (D+1) x (D+1) Legendre coefficients C[i,a,b]
    sites: np.ndarray | None = None
    weights: np.ndarray | None = None
    aniso: np.ndarray | None = None   # N x 2 x 2
    keep: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


def axis_centres(length: int) -> np.ndarray:
    return (2.0 * np.arange(length) + 1.0 - length) / length


def _compact(labels, N):
    present = np.zeros(N, bool)
    present[np.unique(labels)] = True
    keep = np.nonzero(present)[0]
    remap = -np.ones(N, np.int64)
    remap[keep] = np.arange(keep.size)
    return remap[labels].astype(np.int32), keep


def _argmin_rows(H, W, score_row):
    """Row by row, the first index of the smallest score (N x W scores per row).
    Large rows use torch's multi-threaded CPU argmin (same first-index rule)."""
    out = np.empty((H, W), np.int32)
    try:
        import torch
    except ImportError:          # pragma: no cover - torch is part of this image
        torch = None
    for r in range(H):
        S = score_row(r)
        if torch is not None and S.size >= 1 << 20:
            out[r] = torch.from_numpy(np.ascontiguousarray(S)).argmin(dim=0).numpy()
        else:
            out[r] = np.argmin(S, axis=0)
    return out.reshape(-1)


def power_diagram(H, W, N, rng, wmax=0.05):
    y = rng.uniform(-1.0, 1.0, size=(N, 2))
    w = rng.uniform(0.0, wmax, size=N)
    xs, ys = axis_centres(W), axis_centres(H)

    def row(r):
        d2 = (xs[None, :] - y[:, 0:1]) ** 2 + (ys[r] - y[:, 1:2]) ** 2
        return d2 - w[:, None]

    lab = _argmin_rows(H, W, row)
    lab, keep = _compact(lab, N)
    return GrainMap(H, W, lab, keep.size, "pd", 1, sites=y[keep], weights=w[keep], keep=keep)


def rotation_spd(rng, N, lmin, lmax):
    lam = np.exp(rng.uniform(np.log(lmin), np.log(lmax), size=(N, 2)))
    phi = rng.uniform(0.0, np.pi, size=N)
    c, s = np.cos(phi), np.sin(phi)
    R = np.stack([np.stack([c, -s], -1), np.stack([s, c], -1)], -2)
    return R @ (lam[:, :, None] * np.transpose(R, (0, 2, 1)))


def anisotropic_power_diagram(H, W, N, rng, wmax=0.02, lmin=0.5, lmax=2.0):
    y = rng.uniform(-1.0, 1.0, size=(N, 2))
    w = rng.uniform(0.0, wmax, size=N)
    A = rotation_spd(rng, N, lmin, lmax)
    xs, ys = axis_centres(W), axis_centres(H)

    def row(r):
        dx = xs[None, :] - y[:, 0:1]
        dy = ys[r] - y[:, 1:2]
        return (A[:, 0, 0:1] * dx * dx + 2.0 * A[:, 0, 1:2] * dx * dy
                + A[:, 1, 1:2] * dy * dy - w[:, None])

    lab = _argmin_rows(H, W, row)
    lab, keep = _compact(lab, N)
    return GrainMap(H, W, lab, keep.size, "apd", 2, sites=y[keep], weights=w[keep],
                    aniso=A[keep], keep=keep)


def _polynomial_parts(H, W, N, D, rng):
    """Draws of a random polynomial diagram and its per-row score function."""
    h = 2.0 / np.sqrt(N)
    y = rng.uniform(-1.0, 1.0, size=(N, 2))
    w = rng.uniform(0.0, 0.125 * h * h, size=N)
    C = np.zeros((N, D + 1, D + 1))
    C[:, 0, 0] = (y ** 2).sum(1) - w
    C[:, 1, 0] = -2.0 * y[:, 0]
    C[:, 0, 1] = -2.0 * y[:, 1]
    sigma = 0.0625 * h * h
    for k in range(D + 1):
        for b in range(k + 1):
            a = k - b
            C[:, a, b] += sigma * rng.normal(0.0, 1.0 / (k + 1), size=N)
    Vx = npleg.legvander(axis_centres(W), D)     # W x (D+1)
    Vy = npleg.legvander(axis_centres(H), D)     # H x (D+1)

    def row(r):
        ca = C @ Vy[r]                           # N x (D+1) over a
        return ca @ Vx.T                         # N x W

    return C, y, w, sigma, h, row


def polynomial_diagram(H, W, N, D, rng, cache=None):
    """Random polynomial diagram of degree D.  With ``cache`` (a path), the
    uncompacted arg-min labels are read from that file when it holds this map
    (same H, W, N, D and the same coefficients), and written to it otherwise."""
    C, y, w, sigma, h, row = _polynomial_parts(H, W, N, D, rng)
    raw = _cached_labels(cache, H, W, N, D, C) if cache else None
    if raw is None:
        raw = _argmin_rows(H, W, row)
        if cache:
            _store_labels(cache, H, W, N, D, C, raw)
    lab, keep = _compact(raw, N)
    return GrainMap(H, W, lab, keep.size, "poly", D, coef=C[keep], sites=y[keep],
                    weights=w[keep], keep=keep, meta=dict(sigma=sigma, h=h))


def _coef_digest(C):
    return hashlib.sha256(np.ascontiguousarray(C, dtype=np.float64).tobytes()).hexdigest()


def _cached_labels(path, H, W, N, D, C):
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        if (tuple(int(v) for v in z["shape"]) != (H, W, N, D)
                or str(z["coef_sha256"]) != _coef_digest(C)):
            return None
        return z["raw"].astype(np.int32).reshape(-1)


def _store_labels(path, H, W, N, D, C, raw):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    dt = np.int16 if N <= 32767 else np.int32
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, raw=raw.astype(dt), shape=np.array([H, W, N, D]),
                        coef_sha256=np.array(_coef_digest(C)))
    os.replace(tmp, path)


def boundary_noise(gm: GrainMap, frac, rng):
    H, W = gm.H, gm.W
    L = gm.labels.reshape(H, W)
    nbrs = []
    for dr, dc in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        sh = np.full((H, W), -1, np.int64)
        rs = slice(max(dr, 0), H + min(dr, 0))
        rd = slice(max(-dr, 0), H + min(-dr, 0))
        cs = slice(max(dc, 0), W + min(dc, 0))
        cd = slice(max(-dc, 0), W + min(-dc, 0))
        sh[rd, cd] = L[rs, cs]
        nbrs.append(sh)
    nb = np.stack(nbrs, -1)                      # H x W x 4
    differs = (nb >= 0) & (nb != L[:, :, None])
    boundary = np.nonzero(differs.any(-1).reshape(-1))[0]
    n_pick = int(round(frac * boundary.size))
    pick = rng.choice(boundary, size=n_pick, replace=False) if n_pick else np.zeros(0, np.int64)
    flat = gm.labels.copy()
    nbf = nb.reshape(-1, 4)
    dif = differs.reshape(-1, 4)
    for j in np.sort(pick):
        cands = np.unique(nbf[j][dif[j]])
        flat[j] = cands[rng.integers(cands.size)]
    gm.labels = flat.astype(np.int32)
    gm.meta["noise_pixels"] = int(n_pick)
    gm.meta["boundary_pixels"] = int(boundary.size)
    return gm


# ---------------------------------------------------------------------------
# The named workloads.

def config_c1(seed=101):
    """64x64 power diagram, N = 8, weights in [0, 0.05]; fit at d = 1, eps = 1e-2."""
    rng = np.random.default_rng(seed)
    gm = power_diagram(64, 64, 8, rng, wmax=0.05)
    gm.meta.update(degree=1, eps=1e-2)
    return gm


def config_c2(seed=202, H=256, W=256, N=100):
    """256x256 anisotropic power diagram, N = 100, 1% boundary noise; d = 2."""
    rng = np.random.default_rng(seed)
    gm = anisotropic_power_diagram(H, W, N, rng, wmax=0.02)
    gm = boundary_noise(gm, 0.01, rng)
    gm.meta.update(degree=2, eps=1e-2)
    return gm


def config_c3(seed=303, H=1024, W=1024, N=1000, D=4):
    """1024x1024 random degree-4 polynomial diagram, N = 1000; d = 4, eps = 1e-3."""
    rng = np.random.default_rng(seed)
    gm = polynomial_diagram(H, W, N, D, rng)
    gm.meta.update(degree=D, eps=1e-3)
    return gm


def config_c4_shapes(seed=404, n_maps=64):
    """Sizes of the 64-map batch: (H, W, N, d) per map, drawn from seed 404 + j."""
    out = []
    for j in range(n_maps):
        rng = np.random.default_rng(seed + j)
        H, W = (int(v) for v in rng.integers(128, 769, size=2))
        N = int(rng.integers(20, 501))
        d = int(rng.integers(2, 5))
        out.append((H, W, N, d))
    return out


def config_c4_map(j, seed=404):
    rng = np.random.default_rng(seed + j)
    H, W = (int(v) for v in rng.integers(128, 769, size=2))
    N = int(rng.integers(20, 501))
    d = int(rng.integers(2, 5))
    if d == 2:
        gm = anisotropic_power_diagram(H, W, N, rng, wmax=0.02)
        gm = boundary_noise(gm, 0.01, rng)
    else:
        gm = polynomial_diagram(H, W, N, d, rng)
    gm.meta.update(degree=d, eps=1e-3 if d > 2 else 1e-2)
    return gm


CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cache")


def config_c5(seed=505, H=2048, W=2048, N=5000, D=6, use_cache=True):
    """2048x2048 random degree-6 polynomial diagram, N = 5000; d = 6.  The arg-min
    labels (about 90 s of CPU work) are kept in synth/cache/, keyed by the
    diagram's coefficients; tests regenerate sampled rows to check the file."""
    rng = np.random.default_rng(seed)
    cache = None
    if use_cache:
        cache = os.path.join(CACHE_DIR, f"poly_{H}x{W}_N{N}_D{D}_seed{seed}.npz")
    gm = polynomial_diagram(H, W, N, D, rng, cache=cache)
    gm.meta.update(degree=D, eps=1e-3)
    return gm


def config_c5_rows(rows, seed=505, H=2048, W=2048, N=5000, D=6):
    """Uncompacted arg-min labels of the given rows of the c5 map, computed
    directly (no cache): a check of the cached file."""
    rng = np.random.default_rng(seed)
    _, _, _, _, _, row = _polynomial_parts(H, W, N, D, rng)
    return np.stack([np.argmin(row(r), axis=0).astype(np.int32) for r in rows])


def training_map(k, base=10000, H=256, W=256, D=6):
    """Warm-start training map k: 256x256 degree-6 polynomial diagram with
    N uniform in 50..150 (seed base + k)."""
    rng = np.random.default_rng(base + k)
    N = int(rng.integers(50, 151))
    gm = polynomial_diagram(H, W, N, D, rng)
    gm.meta.update(degree=D, eps=1e-3)
    return gm


def random_theta(N, d, rng, scale=1.0, multi_index=None):
    """N x K_d parameters with entries N(0, (scale/(a+b+1))^2); multi_index gives the
    exponent pairs (a, b) in the caller's feature order."""
    a, b = multi_index
    k = np.asarray(a) + np.asarray(b)
    return rng.normal(0.0, 1.0, size=(N, k.size)) * (scale / (k + 1.0))[None, :]


def random_labels(H, W, N, rng):
    """Labels uniform in 0..N-1 (a non-separable map for small tests)."""
    return rng.integers(0, N, size=H * W).astype(np.int32)


def coef_to_theta(coef, multi_index):
    """Gather a coefficient array C[i, a, b] into N x K columns in the given
    exponent order (zero where (a, b) lies outside C)."""
    a, b = multi_index
    N, Da, Db = coef.shape
    out = np.zeros((N, len(a)))
    for k, (aa, bb) in enumerate(zip(a, b)):
        if aa < Da and bb < Db:
            out[:, k] = coef[:, aa, bb]
    return out


def batch_maps(seed, n_maps, hw=(128, 769), grains=(20, 501), degrees=(2, 3, 4)):
    """Maps drawn like the 64-map batch (sizes, grain counts and degrees uniform
    over the given ranges; APD + boundary noise at d = 2, random polynomial
    diagrams of degree d otherwise), one seed per map (seed + j)."""
    out = []
    for j in range(n_maps):
        rng = np.random.default_rng(seed + j)
        H, W = (int(v) for v in rng.integers(hw[0], hw[1], size=2))
        N = int(rng.integers(grains[0], grains[1]))
        d = int(rng.choice(np.asarray(degrees)))
        if d == 2:
            gm = anisotropic_power_diagram(H, W, N, rng, wmax=0.02)
            gm = boundary_noise(gm, 0.01, rng)
        else:
            gm = polynomial_diagram(H, W, N, d, rng)
        gm.meta.update(degree=d, eps=1e-3 if d > 2 else 1e-2)
        out.append(gm)
    return out
