"""Seeded synthetic stereo MRFs (input recipe only, no BP arithmetic).

Recipe (every draw comes from ``numpy.random.default_rng(seed)`` in the order
written here, so a seed fixes the arrays bit for bit):

1. Left texture ``L ~ U[0, 255)`` of shape (H, W), float64.
2. Integer disparity map ``D`` on the left grid, one of two variants:

   * ``"rectangles"``: a background value ``U{0..M-1}``, then four
     rectangles, each with height ``U{H//8..H//2}``, width ``U{W//8..W//2}``,
     a uniformly placed top-left corner and its own value ``U{0..M-1}``;
     later rectangles overwrite earlier ones.
   * ``"slanted"``: eight seed points uniform in the image, Voronoi regions
     (nearest seed, ties to the lower index), a plane per region
     ``d_k + a_k (r - r_k) + b_k (c - c_k)`` with ``d_k ~ U[0, M-1]`` and
     ``a_k, b_k ~ U[-0.15, 0.15]``, clipped to ``[0, M-1]`` and rounded.

3. Right image: ``R ~ U[0, 255)`` fills disocclusions; for each disparity
   ``d = 0 .. M-1`` in ascending order the left pixels with ``D == d`` are
   pasted at ``R[r, c - d]`` (when ``c - d >= 0``), so nearer surfaces win;
   then ``R += N(0, sigma^2)``.
4. Unary (Sec. 6 form, without the unary truncation):
   ``g[r, c, x] = exp(-beta * |L[r, c] - R[r, max(c - x, 0)]|)``, computed in
   float64 and stored as float32.  The FP32 array is what both the GPU and the
   oracle consume (the oracle upcasts it).

Ground truth labels are ``D`` itself.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class GridConfig:
    """One synthetic workload: grid size, label count, potential and unary parameters."""

    name: str
    H: int          # rows
    W: int          # columns
    M: int          # labels (disparities)
    T: int          # truncation: f = exp(-alpha*|d|) for |d| <= T, fbar beyond
    alpha: float    # smoothness weight
    beta: float     # unary weight
    sigma: float    # right-image noise
    variant: str    # "rectangles" or "slanted"
    seed: int
    iters: int      # iterations the workload runs
    ckpt_every: int = 0  # checkpoint interval for the differentiation workload

    @property
    def fbar(self) -> float:
        return math.exp(-self.alpha * self.T)

    @property
    def n_pixels(self) -> int:
        return self.H * self.W

    @property
    def n_directed_edges(self) -> int:
        return 2 * (self.H * (self.W - 1) + self.W * (self.H - 1))


CONFIGS = {
    # 16x16, M=16, T=2: the small case every path is checked on in full.
    "stereo16": GridConfig("stereo16", 16, 16, 16, 2, 1.0, 0.05, 4.0, "rectangles", 0, 10),
    # Tsukuba-sized 288x384 (rows x cols), M=16, T=2.
    "stereo288x384": GridConfig("stereo288x384", 288, 384, 16, 2, 1.0, 0.05, 4.0,
                                "rectangles", 1, 50),
    # 480x640 (rows x cols), M=64, T=4, alpha=0.5: the throughput workload.
    "stereo480x640": GridConfig("stereo480x640", 480, 640, 64, 4, 0.5, 0.03, 6.0,
                                "slanted", 2, 100),
    # 256x256, M=32, T=3: forward + adjoint of 30 unrolled iterations.
    "stereo256grad": GridConfig("stereo256grad", 256, 256, 32, 3, 1.0, 0.05, 4.0,
                                "rectangles", 4, 30, ckpt_every=5),
    # Paper-shaped context run: 144x192 (Sec. 6 resized Tsukuba), 10 sweeps.
    "stereo144x192": GridConfig("stereo144x192", 144, 192, 16, 2, 1.0, 0.05, 4.0,
                                "rectangles", 5, 10),
}


def _disparity_rectangles(rng, H, W, M):
    D = np.full((H, W), int(rng.integers(0, M)), dtype=np.int64)
    for _ in range(4):
        h = int(rng.integers(H // 8, H // 2 + 1))
        w = int(rng.integers(W // 8, W // 2 + 1))
        r0 = int(rng.integers(0, H - h + 1))
        c0 = int(rng.integers(0, W - w + 1))
        D[r0:r0 + h, c0:c0 + w] = int(rng.integers(0, M))
    return D


def _disparity_slanted(rng, H, W, M, n_regions=8):
    rs = rng.uniform(0, H, n_regions)
    cs = rng.uniform(0, W, n_regions)
    d0 = rng.uniform(0, M - 1, n_regions)
    a = rng.uniform(-0.15, 0.15, n_regions)
    b = rng.uniform(-0.15, 0.15, n_regions)
    rr, cc = np.mgrid[0:H, 0:W].astype(np.float64)
    dist = (rr[..., None] - rs) ** 2 + (cc[..., None] - cs) ** 2
    k = np.argmin(dist, axis=-1)  # first minimum: ties go to the lower index
    D = d0[k] + a[k] * (rr - rs[k]) + b[k] * (cc - cs[k])
    return np.rint(np.clip(D, 0, M - 1)).astype(np.int64)


def make_stereo(H, W, M, beta, sigma, variant, seed):
    """Return ``(g32, D, L, R)`` for one seeded synthetic stereo pair.

    ``seed`` may be an int or a sequence accepted by ``default_rng``.
    """
    rng = np.random.default_rng(seed)
    L = rng.uniform(0.0, 255.0, (H, W))
    if variant == "rectangles":
        D = _disparity_rectangles(rng, H, W, M)
    elif variant == "slanted":
        D = _disparity_slanted(rng, H, W, M)
    else:
        raise ValueError(f"unknown disparity variant {variant!r}")
    R = rng.uniform(0.0, 255.0, (H, W))
    cols = np.arange(W)
    for d in range(M):
        rr, cc = np.nonzero(D == d)
        keep = cc - d >= 0
        R[rr[keep], cc[keep] - d] = L[rr[keep], cc[keep]]
    R = R + rng.normal(0.0, sigma, (H, W))
    src = np.maximum(cols[:, None] - np.arange(M)[None, :], 0)  # [W, M]
    g = np.exp(-beta * np.abs(L[:, :, None] - R[:, src]))
    return g.astype(np.float32), D, L, R


def make_config(cfg: GridConfig):
    """Unary (float32, [H, W, M]) and ground-truth labels (int64, [H, W]) of a config."""
    g32, D, _, _ = make_stereo(cfg.H, cfg.W, cfg.M, cfg.beta, cfg.sigma, cfg.variant, cfg.seed)
    return g32, D


@dataclass(frozen=True)
class BatchInstance:
    H: int
    W: int
    M: int
    T: int
    alpha: float
    index: int
    beta: float = 0.05
    sigma: float = 4.0
    variant: str = "rectangles"

    @property
    def fbar(self) -> float:
        return math.exp(-self.alpha * self.T)

    @property
    def seed(self):
        return [3, self.index]


def make_batch_configs(n=32, seed=3, hw_range=(64, 512), labels=(16, 32, 64, 128),
                       t_range=(1, 8), alpha_range=(0.3, 1.5)):
    """The batched workload: ``n`` independent grids of uneven size, M and T.

    Per instance, in this order: (H, W) ~ U{lo..hi}^2, M ~ choice(labels),
    T ~ U{t_lo..t_hi}, alpha ~ U[a_lo, a_hi); the instance's images come from
    ``default_rng([seed, j])``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        H, W = (int(v) for v in rng.integers(hw_range[0], hw_range[1] + 1, 2))
        M = int(rng.choice(list(labels)))
        T = int(rng.integers(t_range[0], t_range[1] + 1))
        T = min(T, M - 1)
        alpha = float(rng.uniform(alpha_range[0], alpha_range[1]))
        out.append(BatchInstance(H, W, M, T, alpha, j))
    return out


def make_batch_instance(inst: BatchInstance):
    g32, D, _, _ = make_stereo(inst.H, inst.W, inst.M, inst.beta, inst.sigma, inst.variant,
                               inst.seed)
    return g32, D


def random_unary(H, W, M, seed, low=1e-3, high=1.0):
    """Plain seeded random unary in [low, high) (float32), for shape sweeps and edge cases."""
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, (H, W, M)).astype(np.float32)


def sha256_of(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
