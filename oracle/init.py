"""Initialisation of the EM algorithm (Sec. 3.3, eq. 23, Algorithm 1) --
TEST INFRASTRUCTURE ONLY (plain numpy, FP64).

For a partition of the data and a value alpha in (0, 1), every cluster h
gives, from its sample mean ybar, sample covariance S (divisor n_h - 1) and
s* = diag(S), the starting values of eq. (23):
    delta_i = sign(m3_i) sqrt(pi (1 - alpha) s*_i / (pi - 2)),
    Sigma   = S - (1 - alpha) diag(s*)        (on the skewed coordinates),
    mu      = ybar - sqrt(2/pi) delta,
with m3_i the third central sample moment of coordinate i (sign 0 taken
as +), Delta[:, l] = delta_l e_l for l < q (the first q coordinates skewed;
q = p gives Delta = diag(delta)), nu = nu0 and pi_h = n_h / n.  A candidate
is invalid when a cluster has n_h < p + 1 or a Sigma that is not positive
definite.  Algorithm 1 evaluates the log-likelihood of every (start, alpha)
candidate and keeps the first largest.
"""
from __future__ import annotations

import numpy as np

from cfust_inputs.synth import Params


def cluster_stats(y, labels, g):
    """Per cluster: (n_h, ybar [p], S [p][p] with divisor n_h - 1, m3 [p])."""
    y = np.asarray(y, dtype=np.float64)
    out = []
    for h in range(g):
        yh = y[labels == h]
        nh = yh.shape[0]
        if nh == 0:
            out.append((0, np.zeros(y.shape[1]), np.zeros((y.shape[1],) * 2), np.zeros(y.shape[1])))
            continue
        ybar = yh.mean(0)
        r = yh - ybar
        S = r.T @ r / (nh - 1) if nh > 1 else np.zeros((y.shape[1],) * 2)
        m3 = (r ** 3).mean(0)
        out.append((nh, ybar, S, m3))
    return out


def candidate(y, labels, g, q, alpha, nu0=10.0):
    """Params of eq. (23) for one partition and alpha; returns (Params, valid)."""
    n, p = np.asarray(y).shape
    stats = cluster_stats(y, labels, g)
    pi = np.zeros(g); mu = np.zeros((g, p)); Sig = np.zeros((g, p, p)); Del = np.zeros((g, p, q))
    valid = True
    for h, (nh, ybar, S, m3) in enumerate(stats):
        pi[h] = nh / n
        sstar = np.diag(S).copy()
        sign = np.where(m3 < 0, -1.0, 1.0)
        delta = np.zeros(p)
        delta[:q] = sign[:q] * np.sqrt(np.pi * (1.0 - alpha) * sstar[:q] / (np.pi - 2.0))
        Sh = S.copy()
        for i in range(q):
            Sh[i, i] -= (1.0 - alpha) * sstar[i]
        mu[h] = ybar - np.sqrt(2.0 / np.pi) * delta
        Sig[h] = Sh
        for l in range(q):
            Del[h, l, l] = delta[l]
        if nh < p + 1:
            valid = False
        else:
            try:
                np.linalg.cholesky(Sh)
            except np.linalg.LinAlgError:
                valid = False
    return Params(pi, mu, Sig, Del, np.full(g, float(nu0))), valid


def initialise(y, labels, g, q, alphas, design, nu0=10.0):
    """Algorithm 1 over the starts labels [nstarts][n] and the alpha grid.
    Returns (best Params, loglik [nstarts][nalpha] with -inf for invalid
    candidates, best flat index start * nalpha + a)."""
    import oracle
    nstarts, nal = len(labels), len(alphas)
    ll = np.full((nstarts, nal), -np.inf)
    cands = []
    for s in range(nstarts):
        for a, alpha in enumerate(alphas):
            P, ok = candidate(y, labels[s], g, q, alpha, nu0)
            cands.append(P)
            if ok:
                ll[s, a] = oracle.loglik(y, P, design)
    best = int(np.argmax(ll.ravel()))
    return cands[best], ll, best
