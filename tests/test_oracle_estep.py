"""Pins of the oracle E-step (Sec. 3.1, eqs. 7-17; density eq. 4; eq. 27).

References are independent of the closed forms the oracle uses:
  * direct numerical integration of the hierarchy (Sec. 3, eq. 6) over the
    latent (u, w) gives f(y), E[W|y], E[W U|y], E[W U U^T|y];
  * Delta = 0 reduces the CFUST component to the multivariate t (Sec. 2),
    whose density (scipy) and E-step quantities are textbook closed forms;
  * structural facts from Sec. 4.1: sum_h tau_hj = 1 and per-component
    independence (permuting components permutes every output).
"""
import numpy as np
import pytest
from scipy import special as sp, stats

from cfust_inputs import Params, draw_params, make_design, sample_hierarchy

DES = make_design(4096, 8, seed=21)
SMALL = make_design(256, 4, seed=22)


def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def hierarchy_moments(y, mu, Sig, Del, nu, nw=500, ns=40):
    """f(y), E[W|y], E[WU|y], E[WUU^T|y] by quadrature of eq. (6).

    w = exp(v), trapezoid in v; u = s / sqrt(w), tensor Gauss-Legendre in s on a
    box that covers the truncated Gaussian in s with a wide margin."""
    p, q = Del.shape
    Si = np.linalg.inv(Sig)
    ldS = np.linalg.slogdet(Sig)[1]
    v = np.linspace(-30.0, 9.0, nw)
    dv = v[1] - v[0]
    # box for s: the s-law given w is Gaussian with mean sqrt(w) c, cov Lambda
    Lam = np.linalg.inv(np.eye(q) + Del.T @ Si @ Del)
    c = Lam @ Del.T @ Si @ (y - mu)
    F = 0.0
    EW = 0.0
    EWU = np.zeros(q)
    EWUU = np.zeros((q, q))
    for vk in v:
        w = np.exp(vk)
        nodes, wts = [], []
        for i in range(q):
            hi = max(0.0, np.sqrt(w) * c[i]) + 14.0 * np.sqrt(Lam[i, i])
            xs, ws = _gl(ns, 0.0, hi)
            nodes.append(xs)
            wts.append(ws)
        grids = np.meshgrid(*nodes, indexing="ij")
        S = np.stack([gg.ravel() for gg in grids], axis=1)          # [K][q]
        W = np.prod(np.meshgrid(*wts, indexing="ij"), axis=0).ravel()
        U = S / np.sqrt(w)
        r = (y - mu)[None, :] - U @ Del.T
        qf = np.einsum("ki,ij,kj->k", r, Si, r)
        # N_p(y; mu + Delta u, Sigma/w) * 2^q N_q(s; 0, I)   (du = ds / w^{q/2})
        logk = (0.5 * p * np.log(w) - 0.5 * p * np.log(2 * np.pi) - 0.5 * ldS - 0.5 * w * qf
                + q * np.log(2.0) - 0.5 * q * np.log(2 * np.pi) - 0.5 * (S * S).sum(1))
        # gamma(nu/2, rate nu/2) density of w, times dw = w dv
        logg = (0.5 * nu * np.log(0.5 * nu) - sp.gammaln(0.5 * nu) + (0.5 * nu - 1) * np.log(w)
                - 0.5 * nu * w + np.log(w))
        val = np.exp(logk + logg) * W * dv
        F += val.sum()
        EW += (w * val).sum()
        EWU += (w * val[:, None] * U).sum(0)
        EWUU += np.einsum("k,ki,kj->ij", w * val, U, U)
    return F, EW / F, EWU / F, EWUU / F


@pytest.mark.parametrize("p,q,seed", [(2, 2, 1), (3, 2, 2), (2, 1, 3), (3, 3, 4)])
def test_estep_vs_hierarchy_quadrature(orc, p, q, seed):
    rng = np.random.default_rng(seed)
    P = draw_params(rng, p, q, 1, pi=[1.0], nu=[rng.uniform(3.0, 9.0)], sigma="aat", delta_range=2.0)
    y, _ = sample_hierarchy(rng, P, 3)
    es = orc.estep(y, P, DES)
    for j in range(y.shape[0]):
        F, EW, EWU, EWUU = hierarchy_moments(y[j], P.mu[0], P.Sigma[0], P.Delta[0], P.nu[0],
                                             ns=40 if q < 3 else 26)
        assert abs(es.logf_obs[j] - np.log(F)) < 2e-5
        assert abs(es.w[0, j] / EW - 1) < 2e-5
        np.testing.assert_allclose(es.e2[0, :, j], EWU, rtol=2e-4, atol=2e-5 * np.abs(EWU).max())
        iu = np.triu_indices(q)
        np.testing.assert_allclose(es.e3[0, :, j], EWUU[iu], rtol=2e-4, atol=2e-5 * np.abs(EWUU).max())
        assert es.tau[0, j] == 1.0


def test_estep_delta_zero_is_t_mixture(orc):
    rng = np.random.default_rng(8)
    p, q, g = 3, 2, 2
    P = draw_params(rng, p, q, g, sigma="aat")
    P.Delta[:] = 0.0
    y, _ = sample_hierarchy(rng, P, 16)
    es = orc.estep(y, P, DES)
    for h in range(g):
        nu = P.nu[h]
        lt = stats.multivariate_t(loc=P.mu[h], shape=P.Sigma[h], df=nu).logpdf(y)
        np.testing.assert_allclose(es.logf_comp[h], lt, atol=3e-6)
        r = y - P.mu[h]
        d = np.einsum("ki,ij,kj->k", r, np.linalg.inv(P.Sigma[h]), r)
        wex = (nu + p) / (nu + d)
        np.testing.assert_allclose(es.w[h], wex, rtol=1e-5)
        np.testing.assert_allclose(es.e1[h], sp.digamma((nu + p) / 2) - np.log((nu + d) / 2), rtol=1e-5,
                                   atol=1e-6)
        nus = nu + p + 2
        s = (nu + d) / nus
        EU = np.sqrt(s) * np.sqrt(nus / np.pi) * np.exp(sp.gammaln((nus - 1) / 2) - sp.gammaln(nus / 2))
        np.testing.assert_allclose(es.e2[h, 0], wex * EU, rtol=1e-4)
        np.testing.assert_allclose(es.e2[h, 1], wex * EU, rtol=1e-4)
        np.testing.assert_allclose(es.e3[h, 0], wex * s * nus / (nus - 2), rtol=1e-4)   # (0,0)
        np.testing.assert_allclose(es.e3[h, 1], wex * s * nus / (nus - 2) * 2 / np.pi, rtol=1e-4)  # (0,1)
    # tau of a t mixture
    lp = np.log(P.pi)[:, None] + es.logf_comp
    np.testing.assert_allclose(es.tau, np.exp(lp - np.logaddexp.reduce(lp, axis=0)), rtol=1e-12)


def test_estep_tau_sums_to_one_and_loglik(orc):
    rng = np.random.default_rng(10)
    P = draw_params(rng, 3, 3, 3, sigma="wishart")
    y, _ = sample_hierarchy(rng, P, 60)
    es = orc.estep(y, P, SMALL)
    np.testing.assert_allclose(es.tau.sum(0), 1.0, atol=1e-13)
    lp = np.log(P.pi)[:, None] + es.logf_comp
    np.testing.assert_allclose(es.logf_obs, np.logaddexp.reduce(lp, axis=0), atol=1e-12)
    assert abs(es.loglik - es.logf_obs.sum()) < 1e-9


def test_estep_component_permutation_equivariance(orc):
    rng = np.random.default_rng(12)
    P = draw_params(rng, 3, 3, 3, sigma="aat")
    y, _ = sample_hierarchy(rng, P, 30)
    a = orc.estep(y, P, SMALL)
    perm = [2, 0, 1]
    b = orc.estep(y, P.permuted(perm), SMALL)
    for name in ["logf_comp", "w", "e1", "e2", "e3"]:
        np.testing.assert_array_equal(getattr(b, name), getattr(a, name)[perm])
    np.testing.assert_allclose(b.tau, a.tau[perm], atol=1e-15)
    np.testing.assert_allclose(b.logf_obs, a.logf_obs, atol=1e-13)


def test_estep_row_subset_matches_full(orc):
    rng = np.random.default_rng(13)
    P = draw_params(rng, 2, 2, 2, sigma="aat")
    y, _ = sample_hierarchy(rng, P, 25)
    full = orc.estep(y, P, SMALL)
    rows = np.array([3, 17, 0, 24])
    sub = orc.estep(y, P, SMALL, rows=rows)
    np.testing.assert_array_equal(sub.w, full.w[:, rows])
    np.testing.assert_array_equal(sub.e3, full.e3[:, :, rows])
    np.testing.assert_array_equal(sub.tau, full.tau[:, rows])
