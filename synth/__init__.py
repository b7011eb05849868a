"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module only draws random inputs (points, partitions, landmark samples);
it holds none of the clustering arithmetic.  Every generator uses numpy's
PCG64 ``default_rng(seed)``, draws in float64 and rounds the points once to
float32, so the oracle and the GPU library consume bit-identical coordinates.

The paper evaluates on 2-D random points, manifold/subspace sets, 62-D face
contour features and >150-D calligraphy features (Section 5).  Those datasets
are not available here; the families below stand in for their shapes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Points:
    X: np.ndarray          # (n, d) float32, C-contiguous
    labels: np.ndarray     # (n,) int64 ground-truth component
    seed: int


def _f32(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x.astype(np.float32))


def gaussian_2d(n: int = 1000, k: int = 10, seed: int = 1001, std: float = 0.5,
                box: float = 10.0) -> Points:
    """2-D mixture: k centres uniform in [0,box]^2, equal weights, isotropic std.

    Stands in for the paper's randomly selected 2-D point sets (Section 5)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, box, size=(k, 2))
    lab = rng.integers(0, k, size=n)
    x = centres[lab] + rng.normal(0.0, std, size=(n, 2))
    return Points(_f32(x), lab.astype(np.int64), seed)


def gaussian_mixture(n: int = 20000, d: int = 64, k: int = 50, seed: int = 2001,
                     centre_std: float = 4.0, std: float = 1.0, alpha: float = 2.0,
                     clip: float | None = None) -> Points:
    """d-D mixture: centres N(0, centre_std^2 I), weights Dirichlet(alpha), std.

    Stands in for the 62-D face-contour features (Section 5), scaled up."""
    rng = np.random.default_rng(seed)
    centres = rng.normal(0.0, centre_std, size=(k, d))
    w = rng.dirichlet(np.full(k, alpha))
    lab = rng.choice(k, size=n, p=w)
    x = centres[lab] + rng.normal(0.0, std, size=(n, d))
    if clip is not None:
        x = np.clip(x, -clip, clip)
    return Points(_f32(x), lab.astype(np.int64), seed)


def subspaces(n: int = 40000, d: int = 100, n_sub: int = 20, dim: int = 5,
              noise: float = 0.05, seed: int = 3001) -> Points:
    """Union of n_sub random dim-dimensional linear subspaces of R^d.

    Stands in for the manifold/subspace sets of Section 5."""
    rng = np.random.default_rng(seed)
    bases = [np.linalg.qr(rng.normal(size=(d, dim)))[0] for _ in range(n_sub)]
    lab = rng.integers(0, n_sub, size=n)
    coef = rng.normal(size=(n, dim))
    x = np.empty((n, d))
    for j in range(n_sub):
        m = lab == j
        x[m] = coef[m] @ bases[j].T
    x += rng.normal(0.0, noise, size=(n, d))
    return Points(_f32(x), lab.astype(np.int64), seed)


def image_features(n: int = 200000, d: int = 128, k: int = 20, seed: int = 4001) -> Points:
    """Image-sized feature vectors: 20-component mixture, std 1, clipped to [-3,3].

    Stands in for the calligraphy contour features (Section 5)."""
    return gaussian_mixture(n=n, d=d, k=k, seed=seed, centre_std=1.0, std=1.0, clip=3.0)


def random_partition(n: int, parts: int = 8, lo: int = 3000, hi: int = 7000,
                     seed: int = 3001) -> tuple[np.ndarray, np.ndarray]:
    """Random uneven partition: sizes drawn in [lo,hi], normalised to sum n.

    Returns (perm int64 (n,), offsets int64 (parts+1,)); the members of part j
    are perm[offsets[j]:offsets[j+1]].  Remainders go to the largest
    fractional parts, lowest part first on ties."""
    rng = np.random.default_rng(seed + 7919)
    u = rng.uniform(lo, hi, size=parts)
    exact = n * u / u.sum()
    sizes = np.floor(exact).astype(np.int64)
    rem = int(n - sizes.sum())
    frac = exact - sizes
    order = sorted(range(parts), key=lambda j: (-frac[j], j))
    for j in order[:rem]:
        sizes[j] += 1
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    perm = rng.permutation(n).astype(np.int64)
    return perm, offsets


def landmarks(n: int, count: int, seed: int) -> np.ndarray:
    """Uniform sample of `count` distinct indices (Algorithm 3, Step 1), sorted."""
    rng = np.random.default_rng(seed + 104729)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def batch_instances(count: int = 512, n_lo: int = 100, n_hi: int = 2000,
                    k_lo: int = 2, k_hi: int = 20, seed0: int = 3101) -> list[Points]:
    """Independent 2-D mixture instances of uneven sizes (one per seed)."""
    out = []
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        n = int(rng.integers(n_lo, n_hi + 1))
        k = int(rng.integers(k_lo, k_hi + 1))
        out.append(gaussian_2d(n=n, k=k, seed=seed0 + j))
    return out


# --------------------------------------------------------------------------
# Inputs for the warm-start network (parameters, feature batches)
# --------------------------------------------------------------------------
MLP_SHAPES = ((16, 128), (128,), (128, 128), (128,), (128, 2), (2,))


def mlp_params(seed: int, bias_std: float = 0.1) -> np.ndarray:
    """Flat FP32 parameter vector (W1, b1, W2, b2, W3, b3, row-major): weights
    uniform in +-1/sqrt(fan_in), biases N(0, bias_std^2)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            b = 1.0 / np.sqrt(shape[0])
            parts.append(rng.uniform(-b, b, size=shape).ravel())
        else:
            parts.append(rng.normal(0.0, bias_std, size=shape))
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def mlp_batch(count: int, seed: int):
    """Feature-like inputs (count x 16), targets (count x 2) and point weights
    summing to 1, all FP32."""
    rng = np.random.default_rng(seed)
    F = rng.normal(0.0, 1.5, size=(count, 16))
    F[:, :12] = -np.abs(F[:, :12])          # similarities are mostly negative
    F[:, 14] = rng.uniform(0.0, 1.0, count)
    F[:, 15] = rng.uniform(0.6, 1.1, count)
    T = rng.normal(0.0, 2.0, size=(count, 2))
    w = rng.uniform(0.5, 1.5, count)
    w /= w.sum()
    return _f32(F), _f32(T), _f32(w)
