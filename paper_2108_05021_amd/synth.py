"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module draws random images and nothing else: it holds none of the
filter's arithmetic, imports neither the GPU binding nor the oracle, and only
depends on numpy/scipy.  The paper's own images (natural photographs, an MRI
volume) are not available; these piecewise-constant-plus-noise images stand in
for them, with the structure the filter is designed for (flat regions separated
by straight edges and corners, Sec. I-E and III-E).

Recipes (all FP32 output, noise i.i.d. N(0, sigma^2) added after painting, no
clipping):
  rectangles(H, W, n, ...)  background 0.5, n axis-aligned rectangles with
                            top-left uniform, sides uniform in {16..128}
                            clipped to the image, painted in order, levels
                            uniform in [0, 1].
  voronoi(H, W, K, ...)     K uniform sites, each pixel takes the level of its
                            nearest site (K random convex polygons), levels
                            uniform in [0, 1] per region and channel.
  voronoi3d(D, H, W, K, ...) the same in a volume (K random convex polyhedra),
                            standing in for the paper's MRI volume.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rectangles", "voronoi", "workload_single", "workload_rgb", "workload_batched",
    "workload_precision", "workload_grad", "voronoi3d", "workload_volume", "integer_image",
    "dyadic_rectangles",
]


def rectangles(H: int, W: int, n: int, sigma: float, rng, C: int = 1) -> np.ndarray:
    """(C, H, W) float32 rectangles on a 0.5 background plus Gaussian noise."""
    img = np.full((C, H, W), 0.5, np.float64)
    for _ in range(n):
        x0 = int(rng.integers(0, W))
        y0 = int(rng.integers(0, H))
        w = int(rng.integers(16, 129))
        h = int(rng.integers(16, 129))
        lev = rng.uniform(0.0, 1.0, size=C)
        img[:, y0:min(H, y0 + h), x0:min(W, x0 + w)] = lev[:, None, None]
    img += rng.normal(0.0, sigma, size=img.shape)
    return img.astype(np.float32)


def _voronoi_labels(H: int, W: int, K: int, rng) -> np.ndarray:
    from scipy.spatial import cKDTree

    sites = np.stack([rng.uniform(0, H, K), rng.uniform(0, W, K)], axis=1)
    tree = cKDTree(sites)
    lab = np.empty((H, W), np.int32)
    xs = np.arange(W, dtype=np.float64) + 0.5
    step = max(1, (1 << 22) // max(W, 1))
    for y0 in range(0, H, step):
        y1 = min(H, y0 + step)
        yy, xx = np.meshgrid(np.arange(y0, y1, dtype=np.float64) + 0.5, xs, indexing="ij")
        _, idx = tree.query(np.stack([yy.ravel(), xx.ravel()], axis=1), workers=-1)
        lab[y0:y1] = idx.reshape(y1 - y0, W)
    return lab


def voronoi(H: int, W: int, K: int, sigma: float, rng, C: int = 1) -> np.ndarray:
    """(C, H, W) float32 Voronoi piecewise-constant image plus Gaussian noise."""
    lab = _voronoi_labels(H, W, K, rng)
    levels = rng.uniform(0.0, 1.0, size=(C, K))
    out = np.empty((C, H, W), np.float32)
    for c in range(C):
        plane = levels[c][lab].astype(np.float32)
        plane += rng.normal(0.0, sigma, size=(H, W)).astype(np.float32)
        out[c] = plane
    return out


def voronoi3d(D: int, H: int, W: int, K: int, sigma: float, rng) -> np.ndarray:
    """(D, H, W) float32 Voronoi piecewise-constant volume plus Gaussian noise."""
    from scipy.spatial import cKDTree

    sites = np.stack([rng.uniform(0, D, K), rng.uniform(0, H, K), rng.uniform(0, W, K)], axis=1)
    tree = cKDTree(sites)
    levels = rng.uniform(0.0, 1.0, size=K)
    out = np.empty((D, H, W), np.float32)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64) + 0.5, np.arange(W, dtype=np.float64) + 0.5,
                         indexing="ij")
    step = max(1, (1 << 22) // max(H * W, 1))
    for z0 in range(0, D, step):
        z1 = min(D, z0 + step)
        zz = np.repeat(np.arange(z0, z1, dtype=np.float64) + 0.5, H * W)
        pts = np.stack([zz, np.tile(yy.ravel(), z1 - z0), np.tile(xx.ravel(), z1 - z0)], axis=1)
        _, idx = tree.query(pts, workers=-1)
        out[z0:z1] = levels[idx].reshape(z1 - z0, H, W)
    out += rng.normal(0.0, sigma, size=out.shape).astype(np.float32)
    return out


# ---------------------------------------------------------------- workloads

def workload_single(seed: int = 1) -> np.ndarray:
    """256x256x1: 12 rectangles on 0.5, sigma 0.05 (filtered with r=2, T=10)."""
    return rectangles(256, 256, 12, 0.05, np.random.default_rng(seed))


def workload_rgb(seed: int = 2, H: int = 2048, W: int = 2048) -> np.ndarray:
    """3x2048x2048: Voronoi K=64, sigma 0.03 (r in {2,5,10}, T=30)."""
    return voronoi(H, W, 64, 0.03, np.random.default_rng(seed), C=3)


def workload_batched(seed: int = 3, n: int = 256, hw_range=(64, 1024)):
    """List of n dicts {img (C,H,W) f32, r, T}: H, W uniform in hw_range,
    C in {1,3}, Voronoi K=16, sigma 0.05, r in {1,2,4,8}, T uniform in {5..30}."""
    children = np.random.SeedSequence(seed).spawn(n)
    items = []
    for ss in children:
        rng = np.random.default_rng(ss)
        H = int(rng.integers(hw_range[0], hw_range[1] + 1))
        W = int(rng.integers(hw_range[0], hw_range[1] + 1))
        C = int(rng.choice([1, 3]))
        r = int(rng.choice([1, 2, 4, 8]))
        T = int(rng.integers(5, 31))
        items.append({"img": voronoi(H, W, 16, 0.05, rng, C=C), "r": r, "T": T})
    return items


def workload_precision(seed: int = 4, H: int = 8192, W: int = 8192) -> np.ndarray:
    """1x8192x8192 FP32: Voronoi K=256, sigma 0.02 (stored as BF16/FP16, r=16, T=20)."""
    return voronoi(H, W, 256, 0.02, np.random.default_rng(seed), C=1)


def workload_grad(seed: int = 5, N: int = 32, C: int = 3, H: int = 512, W: int = 512,
                  weight_seed: int = 50):
    """(x, w): x (N,C,H,W) Voronoi K=64 per image, sigma 0.05; w ~ N(0,1)
    (loss = sum(w * filter(x)), r=3, T=10)."""
    rng = np.random.default_rng(seed)
    x = np.stack([voronoi(H, W, 64, 0.05, rng, C=C) for _ in range(N)])
    w = np.random.default_rng(weight_seed).normal(0.0, 1.0, size=x.shape).astype(np.float32)
    return x, w


def workload_volume(seed: int = 6, D: int = 256, H: int = 256, W: int = 256) -> np.ndarray:
    """256^3 FP32 volume: Voronoi K=64, sigma 0.05 (r in {1,2,3}, T=10)."""
    return voronoi3d(D, H, W, 64, 0.05, np.random.default_rng(seed))


# ------------------------------------------------------- test-only helpers

def integer_image(H: int, W: int, rng, hi: int = 255, C: int = 1) -> np.ndarray:
    """(C,H,W) integer-valued float32 image, values uniform in {0..hi}."""
    return rng.integers(0, hi + 1, size=(C, H, W)).astype(np.float32)


def dyadic_rectangles(H: int, W: int, n: int, rng, denom: int = 64) -> np.ndarray:
    """(H,W) float32 noise-free rectangles with levels that are multiples of
    1/denom (exactly representable, so window sums are exact)."""
    img = np.full((H, W), 32.0 / denom, np.float32)
    for _ in range(n):
        x0 = int(rng.integers(0, W))
        y0 = int(rng.integers(0, H))
        w = int(rng.integers(1, W + 1))
        h = int(rng.integers(1, H + 1))
        img[y0:y0 + h, x0:x0 + w] = float(rng.integers(0, denom + 1)) / denom
    return img
