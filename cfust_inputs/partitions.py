"""Seeded starting partitions of a data set for the restarts of the
initialisation (Sec. 3.3, Algorithm 1, which draws a fresh partition of the
data for every start).  They are inputs of the initialiser on both sides, like the lattice
design; how a partition is found is not part of the CFUST method.

  random_partitions  uniform labels in [0, g)
  kmeans_partitions  Lloyd's k-means from k-means++ seeds (one per start), at most `iters` rounds
"""
from __future__ import annotations

import numpy as np


def random_partitions(n: int, g: int, nstarts: int, seed: int) -> np.ndarray:
    """int32 [nstarts][n] uniform labels."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, g, size=(nstarts, n)).astype(np.int32)


def _kmeans_once(y: np.ndarray, g: int, rng: np.random.Generator, iters: int) -> np.ndarray:
    n = y.shape[0]
    centers = np.empty((g, y.shape[1]))
    centers[0] = y[rng.integers(n)]
    d2 = ((y - centers[0]) ** 2).sum(1)
    for k in range(1, g):                      # k-means++ seeding
        tot = d2.sum()
        idx = rng.choice(n, p=d2 / tot) if tot > 0 else rng.integers(n)
        centers[k] = y[idx]
        d2 = np.minimum(d2, ((y - centers[k]) ** 2).sum(1))
    lab = np.zeros(n, dtype=np.int64)
    for _ in range(iters):
        dist = ((y[:, None, :] - centers[None, :, :]) ** 2).sum(2)
        new = dist.argmin(1)                   # ties -> lowest index
        if np.array_equal(new, lab) and _ > 0:
            break
        lab = new
        for k in range(g):
            sel = lab == k
            if sel.any():
                centers[k] = y[sel].mean(0)
    return lab.astype(np.int32)


def kmeans_partitions(y: np.ndarray, g: int, nstarts: int, seed: int, iters: int = 25) -> np.ndarray:
    """int32 [nstarts][n] k-means labels, one seeded k-means++ start each.
    y: [n][p]."""
    rng = np.random.default_rng(seed)
    y = np.asarray(y, dtype=np.float64)
    return np.stack([_kmeans_once(y, g, rng, iters) for _ in range(nstarts)])
