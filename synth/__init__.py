"""Seeded synthetic inputs for SegSALSA-STR (arXiv 1504.07028).

This module only draws random numbers and builds input arrays.  It holds none
of the method's arithmetic: both the FP64 CPU oracle and the GPU tests and
benchmark take their inputs from here, and nothing here depends on either.

The paper evaluates on an AVIRIS hyperspectral scene whose class likelihoods
come from a trained classifier (Sec. 4).  Neither the scene nor the classifier
is available, so the generator stands in for them with class-probability
fields of the same shapes: a Voronoi ground-truth map, Gaussian logits with a
bonus on the true class, optional outlier pixels with uniform logits, softmax
over the classes.  The patch multipliers follow the Gaussian weighting of the
patch-based Jacobian (Sec. 3, eq. (4)).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "voronoi_labels",
    "synthetic_logits",
    "softmax_fp64",
    "gaussian_patch_multipliers",
    "make_image",
    "batch_shapes",
    "make_batch",
    "random_state",
]


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: image shape, classes, patch and solver parameters."""

    name: str
    H: int
    W: int
    K: int
    M: int                # patch radius: patch is (2M+1) x (2M+1)
    patch_sigma: float    # Gaussian bandwidth of the patch weights
    schatten_p: float
    lam: float
    mu: float
    iters: int
    seed: int
    logit_sigma: float
    bonus: float
    outlier_frac: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return (2 * self.M + 1) ** 2

    @property
    def n(self) -> int:
        return self.H * self.W


# The five workloads.  Shapes of the second and third follow the paper's
# Indian-Pines subscene (145 x 145, 16 classes) and a 610 x 340, 9-class scene.
WORKLOADS = {
    "plain_64x64_k4": Workload("plain_64x64_k4", 64, 64, 4, 1, 1.0, 1.0, 1.0, 1.0, 100,
                               seed=1, logit_sigma=1.0, bonus=1.5),
    "pines_145x145_k16": Workload("pines_145x145_k16", 145, 145, 16, 2, 1.5, 1.0, 2.0, 2.0, 300,
                                  seed=2, logit_sigma=1.0, bonus=1.0),
    "scene_610x340_k9": Workload("scene_610x340_k9", 610, 340, 9, 2, 1.5, 1.0, 1.5, 1.5, 500,
                                 seed=3, logit_sigma=1.5, bonus=1.0, outlier_frac=0.05),
    "large_2048x2048_k16": Workload("large_2048x2048_k16", 2048, 2048, 16, 2, 1.5, 1.0, 1.5, 1.5, 500,
                                    seed=4, logit_sigma=1.5, bonus=1.0, outlier_frac=0.05),
    "diff_256x256_k8": Workload("diff_256x256_k8", 256, 256, 8, 1, 1.0, 1.0, 1.0, 1.0, 50,
                                seed=6, logit_sigma=1.0, bonus=1.5),
}

# Batched workload: 64 images, sides uniform in [96, 512] (non-square),
# K uniform in {4, 8, 9, 16}, 3x3 patch, 200 rounds.
BATCH = dict(name="batch64_96to512", count=64, side_lo=96, side_hi=512, K_choices=(4, 8, 9, 16),
             M=1, patch_sigma=1.0, schatten_p=1.0, lam=1.5, mu=1.5, iters=200, seed=5,
             logit_sigma=1.5, bonus=1.0, outlier_frac=0.05, image_seed_base=1000)


def voronoi_labels(rng: np.random.Generator, H: int, W: int, K: int) -> np.ndarray:
    """Ground-truth map: K uniform seeds, nearest seed (non-periodic Euclidean), lowest seed on ties."""
    ys = rng.uniform(0.0, H, size=K)
    xs = rng.uniform(0.0, W, size=K)
    r = np.arange(H, dtype=np.float64)[:, None] + 0.5
    c = np.arange(W, dtype=np.float64)[None, :] + 0.5
    best = np.full((H, W), np.inf)
    lab = np.zeros((H, W), dtype=np.int32)
    for s in range(K):
        d = (r - ys[s]) ** 2 + (c - xs[s]) ** 2
        take = d < best          # strict: the lowest seed index wins ties
        best = np.where(take, d, best)
        lab = np.where(take, s, lab)
    return lab


def synthetic_logits(rng: np.random.Generator, labels: np.ndarray, K: int, logit_sigma: float,
                     bonus: float, outlier_frac: float) -> np.ndarray:
    """Gaussian logits [K][H][W] with a bonus on the true class; outlier pixels get U(-3, 3) logits."""
    H, W = labels.shape
    logits = rng.normal(0.0, logit_sigma, size=(K, H, W))
    onehot = (np.arange(K)[:, None, None] == labels[None]).astype(np.float64)
    logits = logits + bonus * onehot
    if outlier_frac > 0.0:
        mask = rng.uniform(0.0, 1.0, size=(H, W)) < outlier_frac
        fresh = rng.uniform(-3.0, 3.0, size=(K, H, W))
        logits = np.where(mask[None], fresh, logits)
    return logits


def softmax_fp64(logits: np.ndarray) -> np.ndarray:
    """Max-subtracted softmax over the class axis (axis 0), in FP64 (input preparation only)."""
    x = np.asarray(logits, dtype=np.float64)
    e = np.exp(x - x.max(axis=0, keepdims=True))
    return e / e.sum(axis=0, keepdims=True)


def gaussian_patch_multipliers(M: int, sigma: float) -> np.ndarray:
    """Patch multipliers c_j, j row-major over (dy, dx) in [-M, M]^2 with dy outer.

    The Gaussian weights w = exp(-(dy^2+dx^2)/(2 sigma^2)) are normalised to sum 1
    and c_j = sqrt(w_j), so the structure tensor is the Gaussian-weighted sum of
    gradient outer products and a 1x1 patch gives c = 1.
    """
    d = np.arange(-M, M + 1, dtype=np.float64)
    dy, dx = np.meshgrid(d, d, indexing="ij")
    w = np.exp(-(dy ** 2 + dx ** 2) / (2.0 * sigma * sigma)).reshape(-1)
    w = w / w.sum()
    return np.sqrt(w)


def make_image(H: int, W: int, K: int, seed: int, logit_sigma: float, bonus: float,
               outlier_frac: float = 0.0):
    """Return (probabilities [K][H][W] FP64, logits [K][H][W] FP64, labels [H][W] int32)."""
    rng = np.random.default_rng(seed)
    labels = voronoi_labels(rng, H, W, K)
    logits = synthetic_logits(rng, labels, K, logit_sigma, bonus, outlier_frac)
    return softmax_fp64(logits), logits, labels


def make_workload(wl: Workload):
    """Inputs for a named workload: dict with probs, logits, labels, weights."""
    probs, logits, labels = make_image(wl.H, wl.W, wl.K, wl.seed, wl.logit_sigma, wl.bonus,
                                       wl.outlier_frac)
    return dict(probs=probs, logits=logits, labels=labels,
                weights=gaussian_patch_multipliers(wl.M, wl.patch_sigma))


def batch_shapes(count: int = BATCH["count"], seed: int = BATCH["seed"], lo: int = BATCH["side_lo"],
                 hi: int = BATCH["side_hi"], K_choices=BATCH["K_choices"]):
    """(H, W, K) per image of the batched workload: sides U{lo..hi}, W != H, K from K_choices."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(count):
        H = int(rng.integers(lo, hi + 1))
        W = int(rng.integers(lo, hi + 1))
        while W == H:
            W = int(rng.integers(lo, hi + 1))
        K = int(K_choices[int(rng.integers(0, len(K_choices)))])
        shapes.append((H, W, K))
    return shapes


def make_batch(shapes=None, base_seed: int = BATCH["image_seed_base"], logit_sigma=BATCH["logit_sigma"],
               bonus=BATCH["bonus"], outlier_frac=BATCH["outlier_frac"]):
    """List of (probs, logits, labels) per image; image i draws from seed base_seed + i."""
    if shapes is None:
        shapes = batch_shapes()
    return [make_image(H, W, K, base_seed + i, logit_sigma, bonus, outlier_frac)
            for i, (H, W, K) in enumerate(shapes)]


def random_state(K: int, H: int, W: int, L: int, seed: int, scale: float = 0.1):
    """A random solver state (z, d1, d3, d4, d2) for single-round checks (d2 is [L][2][K][H][W])."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(0.0, 1.0, size=(K, H, W))
    z = z / z.sum(axis=0, keepdims=True)
    d1 = scale * rng.standard_normal((K, H, W))
    d3 = scale * rng.standard_normal((K, H, W))
    d4 = scale * rng.standard_normal((K, H, W))
    d2 = scale * rng.standard_normal((L, 2, K, H, W))
    return z, d1, d3, d4, d2

