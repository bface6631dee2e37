"""Quasi-Monte Carlo design: rank-1 lattice generating vector and random shifts.

The multivariate t probabilities T_m of the CFUST density (Sec. 2, eq. 4) and of
the E-step weights (Sec. 3.1, eq. 13) are estimated by separation of variables
on a randomly shifted rank-1 lattice.  The paper does not say how T_q is
computed; the lattice rule is this project's reading.  Both the oracle and the
HIP path receive the generating vector ``z`` and the shifts as inputs, so
neither side generates them.

Point k of shift s in lattice dimension j is, on both sides,
    t = frac(k * z[j] / N + shift[s, j]),   x = 1 - |2 t - 1|   (tent / baker map)
The design below only chooses ``z`` (Korobov form, searched with the weighted
P_2 figure of merit) and draws the shifts from a seeded generator.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np

MAX_LATTICE_DIM = 8  # an m-variate integral uses m-1 lattice coordinates (m with its moments); m <= 8


@dataclass(frozen=True)
class QmcDesign:
    N: int                 # lattice points per shift
    S: int                 # number of random shifts
    z: np.ndarray          # int32 [MAX_LATTICE_DIM] generating vector
    shifts: np.ndarray     # float64 [S][MAX_LATTICE_DIM], each in [0,1)
    seed: int


def _p2_weighted(N: int, zs: np.ndarray, gamma: np.ndarray) -> np.ndarray:
    """Weighted P_2 criterion for many candidate vectors at once.

    zs: int64 [C][s] candidate vectors.  Returns float64 [C].
    P_2 = -1 + (1/N) sum_k prod_j (1 + gamma_j 2 pi^2 B_2({k z_j / N})),
    B_2(x) = x^2 - x + 1/6 (Bernoulli polynomial of degree 2).
    """
    k = np.arange(N, dtype=np.int64)
    out = np.empty(zs.shape[0])
    for c in range(zs.shape[0]):
        x = ((k[:, None] * zs[c][None, :]) % N) / N
        b2 = x * x - x + 1.0 / 6.0
        out[c] = -1.0 + np.prod(1.0 + gamma[None, :] * 2.0 * np.pi ** 2 * b2, axis=1).mean()
    return out


@functools.lru_cache(maxsize=32)
def _korobov_cached(N: int, dim: int) -> tuple:
    gamma = 1.0 / (np.arange(1, dim + 1, dtype=np.float64) ** 2)
    cands = np.arange(3, max(N // 2, 4), 2, dtype=np.int64)  # odd a: gcd(a, 2^k) = 1
    if N & (N - 1):
        cands = np.array([a for a in range(2, max(N // 2, 3)) if np.gcd(a, N) == 1], dtype=np.int64)
    if cands.size == 0:
        return tuple([1] * dim)
    # Thin the candidate set for very large N to keep the search around a second.
    if cands.size * N * dim > 4e8:
        step = int(np.ceil(cands.size * N * dim / 4e8))
        cands = cands[::step]
    vecs = np.empty((cands.size, dim), dtype=np.int64)
    vecs[:, 0] = 1
    for j in range(1, dim):
        vecs[:, j] = (vecs[:, j - 1] * cands) % N
    best = int(np.argmin(_p2_weighted(N, vecs, gamma)))
    return tuple(int(v) for v in vecs[best])


def korobov_vector(N: int, dim: int = MAX_LATTICE_DIM) -> np.ndarray:
    """Korobov generating vector (1, a, a^2, ... mod N) minimising weighted P_2."""
    if N < 2:
        raise ValueError("lattice needs N >= 2")
    return np.asarray(_korobov_cached(int(N), int(dim)), dtype=np.int32)


def make_design(N: int, S: int, seed: int = 20160607) -> QmcDesign:
    """Design with ``S`` shifts drawn from numpy's PCG64 stream of ``seed``."""
    if S < 1:
        raise ValueError("need at least one shift")
    rng = np.random.default_rng(seed)
    shifts = rng.random((S, MAX_LATTICE_DIM))
    return QmcDesign(N=int(N), S=int(S), z=korobov_vector(N), shifts=shifts, seed=int(seed))
