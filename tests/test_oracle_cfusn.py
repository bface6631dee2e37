"""The normal limit of the CFUST family (CFUSN, nu = infinity per component,
Table 1) in the oracle: pins against closed forms and against the t model at
very large nu.

  * the univariate laws: Phi and Phi^-1 (scipy);
  * T_m at nu = infinity: bivariate and trivariate normal orthant
    probabilities 1/4 + asin(rho)/(2 pi), 1/8 + sum asin(rho_ik)/(4 pi);
  * q = 1 (the restricted skew normal): density 2 phi_p(y; mu, Omega)
    Phi(c / sqrt(Lambda)) and the truncated normal moments of U | y in closed
    form;
  * Delta = 0: a normal mixture (scipy's multivariate normal), tau included;
  * q = 2: E[U | y], E[U U^T | y] by 2-D quadrature of the truncated normal;
  * the limit itself: the t model at nu = 1e8 gives the same E-step (w -> 1,
    e1 -> 0) and M-step to within O(d^2 / nu), and the M-step keeps nu
    infinite.
"""
import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
from cfust_inputs import make_design
from cfust_inputs.synth import draw_params, sample_hierarchy

INF = float("inf")
DES = make_design(4096, 8, seed=11)


def test_univariate_normal_laws():
    x = np.array([-30.0, -8.0, -1.3, 0.0, 0.7, 5.0])
    np.testing.assert_allclose(oracle.tcdf(x, INF), stats.norm.cdf(x), rtol=1e-12, atol=0)
    p = np.array([1e-300, 1e-20, 0.01, 0.3, 0.5, 0.9, 1 - 1e-12])
    np.testing.assert_allclose(oracle.tinv(p, INF), stats.norm.ppf(p), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(oracle.t1pdf(1.3, 2.0, INF), stats.norm.pdf(1.3, scale=np.sqrt(2.0)), rtol=1e-14)


@pytest.mark.parametrize("rho", [-0.7, 0.1, 0.6])
def test_bivariate_normal_orthant(rho):
    L = np.linalg.cholesky(np.array([[1.0, rho], [rho, 1.0]]))
    est, se = oracle.mvt(np.zeros(2), L, INF, DES)
    assert abs(est - (0.25 + np.arcsin(rho) / (2 * np.pi))) < max(6 * se, 1e-9)


def test_trivariate_normal_orthant():
    R = np.array([[1.0, 0.3, -0.2], [0.3, 1.0, 0.5], [-0.2, 0.5, 1.0]])
    est, se = oracle.mvt(np.zeros(3), np.linalg.cholesky(R), INF, DES)
    ref = 0.125 + (np.arcsin(0.3) + np.arcsin(-0.2) + np.arcsin(0.5)) / (4 * np.pi)
    assert abs(est - ref) < max(6 * se, 1e-6), (est, ref, se)


def _normal_params(rng, p, q, g, **kw):
    P = draw_params(rng, p, q, g, sigma="aat", **kw)
    P.nu[:] = INF
    return P


def test_q1_restricted_skew_normal_closed_form():
    rng = np.random.default_rng(3)
    p, g = 3, 2
    P = _normal_params(rng, p, 1, g)
    y, _ = sample_hierarchy(rng, P, 40)
    es = oracle.estep(y, P, DES)
    for h in range(g):
        d = P.Delta[h][:, 0]
        Om = P.Sigma[h] + np.outer(d, d)
        Oi = np.linalg.inv(Om)
        c = (y - P.mu[h]) @ Oi @ d
        lam = 1.0 - d @ Oi @ d
        z = c / np.sqrt(lam)
        lf = np.log(2.0) + stats.multivariate_normal(P.mu[h], Om).logpdf(y) + stats.norm.logcdf(z)
        np.testing.assert_allclose(es.logf_comp[h], lf, rtol=0, atol=1e-10)
        mills = np.exp(stats.norm.logpdf(z) - stats.norm.logcdf(z))
        eu = c + np.sqrt(lam) * mills
        euu = lam + c * c + c * np.sqrt(lam) * mills
        sel = es.tau[h] > 1e-12
        np.testing.assert_allclose(es.w[h][sel], 1.0, rtol=0, atol=0)
        np.testing.assert_allclose(es.e1[h][sel], 0.0, rtol=0, atol=0)
        np.testing.assert_allclose(es.e2[h, 0][sel], eu[sel], rtol=1e-9)
        np.testing.assert_allclose(es.e3[h, 0][sel], euu[sel], rtol=1e-9)


def test_delta_zero_is_normal_mixture():
    rng = np.random.default_rng(4)
    p, q, g = 3, 2, 3
    P = _normal_params(rng, p, q, g)
    P.Delta[:] = 0.0
    y, _ = sample_hierarchy(rng, P, 30)
    es = oracle.estep(y, P, DES)
    lc = np.stack([stats.multivariate_normal(P.mu[h], P.Sigma[h]).logpdf(y) for h in range(g)])
    np.testing.assert_allclose(es.logf_comp, lc, rtol=0, atol=1e-10)
    lp = np.log(P.pi)[:, None] + lc
    np.testing.assert_allclose(es.tau, np.exp(lp - special.logsumexp(lp, axis=0)), rtol=1e-10)


def test_q2_moments_by_quadrature():
    rng = np.random.default_rng(5)
    p, q = 2, 2
    P = _normal_params(rng, p, q, 1, pi=[1.0])
    y, _ = sample_hierarchy(rng, P, 3)
    es = oracle.estep(y, P, make_design(16384, 8, seed=12))
    D = P.Delta[0]
    Om = P.Sigma[0] + D @ D.T
    Oi = np.linalg.inv(Om)
    Lam = np.eye(q) - D.T @ Oi @ D
    for j in range(3):
        c = D.T @ Oi @ (y[j] - P.mu[0])
        dens = stats.multivariate_normal(c, Lam)
        f = lambda u2, u1, k: dens.pdf([u1, u2]) * k(u1, u2)
        hi = c + 12 * np.sqrt(np.diag(Lam))
        I = lambda k: integrate.dblquad(lambda u2, u1: f(u2, u1, k), 0, hi[0], 0, hi[1], epsabs=1e-13)[0]
        Z = I(lambda a, b: 1.0)
        EU = [I(lambda a, b: a) / Z, I(lambda a, b: b) / Z]
        EUU = [I(lambda a, b: a * a) / Z, I(lambda a, b: a * b) / Z, I(lambda a, b: b * b) / Z]
        np.testing.assert_allclose(es.e2[0, :, j], EU, rtol=2e-5, atol=1e-8)
        np.testing.assert_allclose(es.e3[0, :, j], EUU, rtol=2e-5, atol=1e-8)


def test_large_nu_t_model_converges_to_the_limit():
    rng = np.random.default_rng(6)
    p, q, g = 3, 2, 2
    P = _normal_params(rng, p, q, g)
    y, _ = sample_hierarchy(rng, P, 25)
    Pt = P.copy()
    Pt.nu[:] = 1e8
    en, et = oracle.estep(y, P, DES), oracle.estep(y, Pt, DES)
    np.testing.assert_allclose(et.logf_comp, en.logf_comp, rtol=0, atol=1e-5)
    np.testing.assert_allclose(et.w, en.w, rtol=0, atol=1e-5)
    np.testing.assert_allclose(et.e1, en.e1, rtol=0, atol=1e-5)
    np.testing.assert_allclose(et.e2, en.e2, rtol=1e-4, atol=1e-5)
    np.testing.assert_allclose(et.e3, en.e3, rtol=1e-4, atol=1e-5)
    # M-step: nu stays infinite; the other blocks match the t model's with nu held
    Mn, _ = oracle.mstep(y, en, P)
    Mt, _ = oracle.mstep(y, et, Pt)
    assert np.all(np.isinf(Mn.nu))
    for a, b in ((Mn.pi, Mt.pi), (Mn.mu, Mt.mu), (Mn.Sigma, Mt.Sigma), (Mn.Delta, Mt.Delta)):
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5)
