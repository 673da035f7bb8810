"""Seeded synthetic point sets for the FAMST workloads.

This module only draws random inputs; it holds none of the method's
arithmetic and is shared by the GPU path's tests and benchmark and by the
CPU oracle's tests.  Every generator uses ``numpy.random.default_rng`` with
the draw order fixed as written, so a (name, n, seed) triple always yields
the same float32 array.

The paper evaluates on public datasets (its Table 1) that are not available
here; these generators stand in for them with the shapes and value
distributions of the five workloads the implementation is measured on:

* ``blobs``      -- Gaussian mixture of isotropic clusters (make_blobs-like,
                    the paper's synthetic "Blobs" family, Sec. 5.1).
* ``gamma_int``  -- nonnegative integer-valued features in [0, 255] from a
                    clipped gamma law with per-cluster mean offsets (an
                    image-descriptor-like distribution).
* ``lowrank``    -- rank-32 Gaussian latent mapped to 960 dimensions plus
                    noise, rows L2-normalised (embedding-like data).
* ``vmf``        -- unit-norm rows from a mixture around random unit centres.
* ``clouds``     -- a batch of uneven-size Gaussian-mixture point clouds.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "blobs", "gamma_int", "lowrank", "vmf", "clouds", "subsample", "WORKLOADS",
]


def blobs(n: int = 10_000, d: int = 32, n_clusters: int = 10, sigma: float = 1.0,
          box: float = 10.0, seed: int = 0) -> np.ndarray:
    """Equal-weight mixture of ``n_clusters`` isotropic Gaussians.

    centers ~ U(-box, box)^(n_clusters x d); labels are ``arange`` repeated so
    every cluster gets n // n_clusters points (the remainder goes to the first
    clusters); X = centers[labels] + N(0, sigma^2).
    """
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-box, box, size=(n_clusters, d))
    labels = np.arange(n) % n_clusters
    labels = np.sort(labels, kind="stable")
    X = centers[labels] + sigma * rng.standard_normal(size=(n, d))
    return np.ascontiguousarray(X, dtype=np.float32)


def gamma_int(n: int = 1_000_000, d: int = 128, n_clusters: int = 200,
              shape: float = 0.5, scale: float = 40.0, seed: int = 0,
              chunk: int = 131_072) -> np.ndarray:
    """Integer-valued features in [0, 255].

    off ~ Gamma(shape, scale)^(n_clusters x d); lab ~ U{0..n_clusters-1}^n;
    X = clip(rint(off[lab] + Gamma(shape, scale)^(n x d)), 0, 255).
    The per-point gamma draws are taken in row chunks (same stream order).
    """
    rng = np.random.default_rng(seed)
    off = rng.gamma(shape, scale, size=(n_clusters, d))
    lab = rng.integers(0, n_clusters, size=n)
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        g = rng.gamma(shape, scale, size=(e - s, d))
        X[s:e] = np.clip(np.rint(off[lab[s:e]] + g), 0, 255)
    return X


def lowrank(n: int = 500_000, d: int = 960, rank: int = 32, noise: float = 0.1,
            seed: int = 0, chunk: int = 65_536) -> np.ndarray:
    """Z A + noise with Z ~ N(0,1)^(n x rank), A ~ N(0,1)^(rank x d), rows
    L2-normalised."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal(size=(rank, d))
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        Z = rng.standard_normal(size=(e - s, rank))
        Y = Z @ A + noise * rng.standard_normal(size=(e - s, d))
        Y /= np.linalg.norm(Y, axis=1, keepdims=True)
        X[s:e] = Y
    return X


def vmf(n: int = 4_000_000, d: int = 96, n_clusters: int = 1000, sigma: float = 0.2,
        seed: int = 0, chunk: int = 262_144) -> np.ndarray:
    """Unit-norm rows: normalise(c[lab] + sigma N(0,1)) with unit centres c."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(size=(n_clusters, d))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    lab = rng.integers(0, n_clusters, size=n)
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        Y = c[lab[s:e]] + sigma * rng.standard_normal(size=(e - s, d))
        Y /= np.linalg.norm(Y, axis=1, keepdims=True)
        X[s:e] = Y
    return X


def clouds(n_clouds: int = 256, lo: int = 512, hi: int = 8192, d: int = 64,
           n_clusters: int = 5, box: float = 5.0, seed: int = 0,
           sizes: np.ndarray | None = None):
    """A batch of point clouds concatenated row-wise.

    sizes ~ U{lo..hi}^n_clouds (unless given); per cloud: centers ~
    U(-box, box)^(n_clusters x d), lab ~ U{0..n_clusters-1}, X = c[lab] +
    N(0,1).  Returns (X [sum n_i, d] float32, offs int64 [n_clouds + 1]).
    """
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = rng.integers(lo, hi + 1, size=n_clouds)
    sizes = np.asarray(sizes, dtype=np.int64)
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    X = np.empty((int(offs[-1]), d), dtype=np.float32)
    for b, m in enumerate(sizes):
        c = rng.uniform(-box, box, size=(n_clusters, d))
        lab = rng.integers(0, n_clusters, size=int(m))
        X[offs[b]:offs[b + 1]] = c[lab] + rng.standard_normal(size=(int(m), d))
    return X, offs


def subsample(n_total: int, m: int, seed: int = 1) -> np.ndarray:
    """Sorted index sample of size m without replacement."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=m, replace=False))


# name -> (generator, kwargs, k, lambda) for the five measured workloads
WORKLOADS = {
    "blobs-10k-d32": (blobs, dict(n=10_000, d=32), 10, 5),
    "gamma-int-1m-d128": (gamma_int, dict(n=1_000_000, d=128), 20, 10),
    "lowrank-500k-d960": (lowrank, dict(n=500_000, d=960), 20, 10),
    "vmf-4m-d96": (vmf, dict(n=4_000_000, d=96), 16, 8),
}
