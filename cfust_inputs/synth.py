"""Seeded synthetic CFUST data drawn from the four-level hierarchy (Sec. 3, eq. 6).

    Z_j ~ Mult_g(1, pi)
    W_j | z_hj = 1 ~ gamma(nu_h / 2, rate nu_h / 2)
    U_j | w_j ~ HN_q(0, I_q / w_j)                 (half-normal: |N(0, I/w)|)
    Y_j | u_j, w_j ~ N_p(mu_h + Delta_h u_j, Sigma_h / w_j)

Parameter layouts (float64, row-major) are those of the library boundary:
pi[g], mu[g][p], Sigma[g][p][p], Delta[g][p][q], nu[g].  Data y is [n][p];
``Dataset.y_soa`` gives the [p][n] layout the library reads.

The workload recipes (sizes, distributions) are the five synthetic stand-ins
described in the design notes; the paper's own data sets (flow cytometry,
Iris, KDD-Cup Protein) are not used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Params:
    pi: np.ndarray      # [g]
    mu: np.ndarray      # [g][p]
    Sigma: np.ndarray   # [g][p][p]
    Delta: np.ndarray   # [g][p][q]
    nu: np.ndarray      # [g]

    @property
    def g(self) -> int:
        return int(self.pi.shape[0])

    @property
    def p(self) -> int:
        return int(self.mu.shape[1])

    @property
    def q(self) -> int:
        return int(self.Delta.shape[2])

    def copy(self) -> "Params":
        return Params(*(np.array(a, dtype=np.float64, copy=True) for a in
                        (self.pi, self.mu, self.Sigma, self.Delta, self.nu)))

    def permuted(self, perm) -> "Params":
        perm = np.asarray(perm)
        return Params(self.pi[perm].copy(), self.mu[perm].copy(), self.Sigma[perm].copy(),
                      self.Delta[perm].copy(), self.nu[perm].copy())


@dataclass
class Dataset:
    y: np.ndarray            # [n][p] float64
    labels: np.ndarray       # [n] int32 true component
    params: Params           # the Psi the data were drawn from
    meta: dict = field(default_factory=dict)

    @property
    def y_soa(self) -> np.ndarray:
        return np.ascontiguousarray(self.y.T)


def random_spd(rng: np.random.Generator, p: int, df: int = 6, unit_diag: bool = True) -> np.ndarray:
    """Wishart(df, I_p) draw, optionally scaled to unit diagonal.

    For p > df - 2 the degrees of freedom are raised to p + 2 so that the draw
    is nonsingular (the workload recipe asks for 6 at p <= 4).
    """
    df = max(int(df), p + 2)
    x = rng.standard_normal((p, df))
    w = x @ x.T
    if unit_diag:
        d = 1.0 / np.sqrt(np.diag(w))
        w = w * d[:, None] * d[None, :]
    return 0.5 * (w + w.T)


def draw_params(rng: np.random.Generator, p: int, q: int, g: int, *, pi=None, nu=None,
                sigma: str = "aat", delta_range: float = 3.0, mu_range: float = 5.0,
                nu_range=(3.0, 15.0)) -> Params:
    """Draw Psi.  ``sigma`` = 'aat' gives A A^T + I with A ~ N(0,1); 'wishart'
    gives a Wishart(6) draw scaled to unit diagonal."""
    if pi is None:
        pi = rng.dirichlet(2.0 * np.ones(g))
    pi = np.asarray(pi, dtype=np.float64)
    mu = rng.uniform(-mu_range, mu_range, size=(g, p))
    Sig = np.empty((g, p, p))
    for h in range(g):
        if sigma == "aat":
            a = rng.standard_normal((p, p))
            Sig[h] = a @ a.T + np.eye(p)
        else:
            Sig[h] = random_spd(rng, p)
    Del = rng.uniform(-delta_range, delta_range, size=(g, p, q))
    if nu is None:
        nu = rng.uniform(nu_range[0], nu_range[1], size=g)
    return Params(pi, mu, Sig, Del, np.asarray(nu, dtype=np.float64))


def sample_hierarchy(rng: np.random.Generator, params: Params, n: int):
    """Draw n observations from eq. (6).  Returns (y [n][p], labels [n])."""
    g, p, q = params.g, params.p, params.q
    lab = rng.choice(g, size=n, p=params.pi / params.pi.sum())
    y = np.empty((n, p))
    for h in range(g):
        idx = np.nonzero(lab == h)[0]
        m = idx.size
        if m == 0:
            continue
        nu = params.nu[h]
        # W ~ Gamma(nu/2, rate nu/2); nu = infinity (the normal limit) is W = 1
        w = np.ones(m) if np.isinf(nu) else rng.gamma(shape=nu / 2.0, scale=2.0 / nu, size=m)
        u = np.abs(rng.standard_normal((m, q))) / np.sqrt(w)[:, None]
        L = np.linalg.cholesky(params.Sigma[h])
        e = (rng.standard_normal((m, p)) @ L.T) / np.sqrt(w)[:, None]
        y[idx] = params.mu[h][None, :] + u @ params.Delta[h].T + e
    return y, lab.astype(np.int32)


def _affine_to_box(y: np.ndarray, params: Params, lo_hi=(0.0, 1024.0)):
    """Per-coordinate min-max map of y onto [lo, hi], applied to Psi as well."""
    lo, hi = lo_hi
    mn, mx = y.min(axis=0), y.max(axis=0)
    s = (hi - lo) / (mx - mn)
    y2 = (y - mn[None, :]) * s[None, :] + lo
    P = params.copy()
    P.mu = (P.mu - mn[None, :]) * s[None, :] + lo
    P.Sigma = P.Sigma * s[None, :, None] * s[None, None, :]
    P.Delta = P.Delta * s[None, :, None]
    return y2, P


def _wl_small(seed: int, n: int = 1000) -> Dataset:
    rng = np.random.default_rng(seed)
    P = draw_params(rng, 2, 2, 2, pi=[0.4, 0.6], nu=[4.0, 8.0], sigma="aat")
    y, lab = sample_hierarchy(rng, P, n)
    return Dataset(y, lab, P, dict(workload="cfust_n1000_p2_q2_g2", N=1024, S=4, iters=20))


def _wl_p4(seed: int, n: int = 20000) -> Dataset:
    rng = np.random.default_rng(seed)
    P = draw_params(rng, 4, 4, 3, sigma="wishart", nu_range=(3.0, 15.0))
    y, lab = sample_hierarchy(rng, P, n)
    return Dataset(y, lab, P, dict(workload="cfust_n20000_p4_q4_g3", N=4096, S=8))


def _wl_cyto(seed: int, n: int = 1_000_000) -> Dataset:
    rng = np.random.default_rng(seed)
    p = q = 8
    g = 5
    P = draw_params(rng, p, q, g, sigma="wishart", delta_range=4.0, nu_range=(3.0, 10.0))
    # well separated: component means 4 * sigma_max apart along the axes
    smax = max(np.sqrt(np.linalg.eigvalsh(P.Sigma[h] + P.Delta[h] @ P.Delta[h].T).max())
               for h in range(g))
    P.mu = np.zeros((g, p))
    for h in range(g):
        P.mu[h, h] = 4.0 * smax
    y, lab = sample_hierarchy(rng, P, n)
    y, P = _affine_to_box(y, P)
    return Dataset(y, lab, P, dict(workload="cfust_n1e6_p8_q8_g5_box1024", N=8192, S=8, iters=50))


def batch_specs(seed: int, nfits: int = 64, n_lo: float = 5e3, n_hi: float = 2e5):
    """Uneven fits for the batched-restart workload: (n, p, q, g, Params)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nfits):
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        p = int(rng.integers(3, 9))
        g = int(rng.integers(2, 7))
        if g == 2:
            P = draw_params(rng, p, p, g, pi=[0.4, 0.6], nu=[4.0, 8.0], sigma="aat")
        else:
            P = draw_params(rng, p, p, g, sigma="aat", nu_range=(4.0, 8.0))
        out.append((n, p, p, g, P))
    return out


def _wl_batch(seed: int, nfits: int = 64, n_lo: float = 5e3, n_hi: float = 2e5):
    specs = batch_specs(seed, nfits, n_lo, n_hi)
    rng = np.random.default_rng(seed + 1)
    sets = []
    for (n, p, q, g, P) in specs:
        y, lab = sample_hierarchy(rng, P, n)
        sets.append(Dataset(y, lab, P, dict(workload="batched_fit", N=1024, S=4)))
    return sets


def restart_params(seed: int, nstarts: int = 64):
    """Starting parameter sets for restarts on the n = 1000, p = q = 2, g = 2
    data: each drawn like that workload's own parameters (weights 0.4/0.6,
    nu = 4, 8, mu ~ U[-5, 5]^2, Sigma = A A^T + I, Delta ~ U[-3, 3])."""
    rng = np.random.default_rng(seed)
    return [draw_params(rng, 2, 2, 2, pi=[0.4, 0.6], nu=[4.0, 8.0], sigma="aat") for _ in range(nstarts)]


WORKLOADS = {
    "cfust_n1000_p2_q2_g2": _wl_small,
    "cfust_n20000_p4_q4_g3": _wl_p4,
    "cfust_n1e6_p8_q8_g5_box1024": _wl_cyto,
}


def workload(name: str, seed: int = 1606, **kw):
    if name == "batched_fit":
        return _wl_batch(seed, **kw)
    return WORKLOADS[name](seed, **kw)


def draw_mvt_problems(rng: np.random.Generator, m: int, batch: int, nmat: int = 4,
                      lim=(-3.0, 3.0), dof=(2.0, 30.0)):
    """Random T_m(b; 0, R, nu) problems: limits b [batch][m], lower Cholesky
    factors L [nmat][m][m] of unit-diagonal SPD matrices, mat_idx [batch], nu [batch]."""
    L = np.zeros((nmat, m, m))
    for i in range(nmat):
        L[i] = np.linalg.cholesky(random_spd(rng, m))
    b = rng.uniform(lim[0], lim[1], size=(batch, m))
    idx = rng.integers(0, nmat, size=batch).astype(np.int32)
    nu = rng.uniform(dof[0], dof[1], size=batch)
    return b, L, idx, nu
