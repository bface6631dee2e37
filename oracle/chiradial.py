"""Chi-radial separation-of-variables estimate of T_m(b; 0, L L^T, nu) --
TEST INFRASTRUCTURE ONLY (numpy + scipy's normal and chi-square functions).

An alternative to the t-SOV lattice rule of the library (Genz's sequential
conditional t form, with the first factor exact).  A multivariate t vector is
a normal vector divided by sqrt(W / nu), W ~ chi-square(nu), so

    T_m(b; 0, R, nu) = E_W[ Phi_m(b sqrt(W / nu); 0, R) ],

and with W = F^{-1}_{chi2(nu)}(x_0) the remaining normal probability is
separated in the usual way: for i = 0 .. m-1,
    u_i = (b_i r - sum_{j<i} L_ij y_j) / L_ii,   e_i = Phi(u_i),
    y_i = Phi^{-1}(x_{i+1} e_i)  (i < m-1),
with r = sqrt(W / nu); the integrand is prod_i e_i over the lattice point
x in [0,1)^m.  It needs one lattice coordinate more than the t form (the
radial one) and no first factor in closed form, but each conditional law is
the normal, so each factor is a normal CDF and quantile.

The lattice points, shifts and tent transform are those of the oracle's t
rule (coordinate j of point k of shift s: t = frac(k z_j / N + shift_sj),
x = 1 - |2t - 1| clamped to [2^-24, 1 - 2^-24]).  Not on the product path:
kept to measure it against the t rule at equal lattice size.
"""
from __future__ import annotations

import numpy as np
from scipy import stats


def lattice_points(design, m: int) -> list:
    """Per shift: the N x m tent-transformed lattice points."""
    N = int(design.N)
    k = np.arange(N, dtype=np.int64)[:, None]
    z = np.asarray(design.z, dtype=np.int64)[None, :m]
    out = []
    for s in range(int(design.S)):
        t = np.mod((k * z) % N / N + np.asarray(design.shifts)[s][None, :m], 1.0)
        out.append(np.clip(1.0 - np.abs(2.0 * t - 1.0), 2.0 ** -24, 1.0 - 2.0 ** -24))
    return out


def mvt_chiradial(b, L, nu, design):
    """T_m(b; 0, L L^T, nu) by the chi-radial rule.  Returns (estimate, stderr)
    with the estimate the mean of the per-shift means and stderr their
    standard deviation over sqrt(S)."""
    b = np.asarray(b, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    m = b.shape[0]
    means = []
    for X in lattice_points(design, m):
        r = np.sqrt(stats.chi2.ppf(X[:, 0], nu) / nu)
        f = np.ones(X.shape[0])
        y = np.zeros((X.shape[0], m))
        for i in range(m):
            u = (b[i] * r - y[:, :i] @ L[i, :i]) / L[i, i]
            e = stats.norm.cdf(u)
            f = f * e
            if i < m - 1:
                y[:, i] = stats.norm.ppf(X[:, i + 1] * e)
        means.append(f.mean())
    means = np.array(means)
    se = means.std(ddof=1) / np.sqrt(len(means)) if len(means) > 1 else float("nan")
    return float(means.mean()), float(se)
