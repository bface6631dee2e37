"""Pins of the oracle's multivariate t CDF T_m (used in Sec. 2 eq. 4 and Sec. 3.1
eq. 13) and of its truncated-t moments (the moments of Sec. 3.1 eqs. 16-17).

Every reference here is independent of the oracle's formulas: closed-form
orthant probabilities of elliptical laws, direct numerical quadrature of the
t density, Monte Carlo draws of the t law, and half-t closed forms.
"""
import numpy as np
import pytest
from scipy import integrate, special as sp, stats

from cfust_inputs import make_design, random_spd

BIG = make_design(4096, 8, seed=11)
MED = make_design(1024, 8, seed=12)


def _tdens(z, Rinv, logdetR, nu):
    m = z.shape[-1]
    qf = np.einsum("...i,ij,...j->...", z, Rinv, z)
    return np.exp(sp.gammaln((nu + m) / 2) - sp.gammaln(nu / 2) - 0.5 * m * np.log(nu * np.pi)
                  - 0.5 * logdetR - 0.5 * (nu + m) * np.log1p(qf / nu))


def test_mvt_m1_is_univariate(orc):
    for nu in [1.3, 5.0, 40.0]:
        for b in [-7.0, -0.2, 0.0, 3.3]:
            v, se = orc.mvt([b], [[1.7]], nu, MED)
            assert se == 0.0
            assert abs(v - float(orc.tcdf(b / 1.7, nu))) < 1e-15


@pytest.mark.parametrize("rho", [-0.85, -0.3, 0.0, 0.45, 0.9])
@pytest.mark.parametrize("nu", [2.5, 9.0])
def test_mvt_orthant_m2(orc, rho, nu):
    L = np.linalg.cholesky(np.array([[1.0, rho], [rho, 1.0]]))
    v, se = orc.mvt([0.0, 0.0], L, nu, BIG)
    exact = 0.25 + np.arcsin(rho) / (2 * np.pi)
    assert abs(v - exact) < 5 * se + 2e-6


def test_mvt_orthant_m3(orc):
    rng = np.random.default_rng(5)
    for nu in [3.0, 12.0]:
        R = random_spd(rng, 3)
        v, se = orc.mvt(np.zeros(3), np.linalg.cholesky(R), nu, BIG)
        exact = 0.125 + (np.arcsin(R[0, 1]) + np.arcsin(R[0, 2]) + np.arcsin(R[1, 2])) / (4 * np.pi)
        assert abs(v - exact) < 5 * se + 2e-5


@pytest.mark.parametrize("m", [2, 3, 5, 8])
def test_mvt_equicorrelated_orthant(orc, m):
    R = 0.5 * np.eye(m) + 0.5
    v, se = orc.mvt(np.zeros(m), np.linalg.cholesky(R), 4.5, MED)
    assert abs(v - 1.0 / (m + 1)) < 5 * se + 2e-5


@pytest.mark.parametrize("case", range(4))
def test_mvt_m2_vs_quadrature(orc, case):
    rng = np.random.default_rng(100 + case)
    R = random_spd(rng, 2) * rng.uniform(0.5, 3.0)
    b = rng.uniform(-2.5, 2.0, 2)
    nu = rng.uniform(1.5, 20.0)
    Ri = np.linalg.inv(R)
    ld = np.log(np.linalg.det(R))
    f = lambda z2, z1: float(_tdens(np.array([z1, z2]), Ri, ld, nu))
    ref, err = integrate.dblquad(f, -np.inf, b[0], -np.inf, b[1], epsabs=1e-11, epsrel=1e-10)
    v, se = orc.mvt(b, np.linalg.cholesky(R), nu, BIG)
    assert abs(v - ref) < 6 * se + 1e-8, (v, ref, se)


def test_mvt_m4_vs_scipy_multivariate_t(orc):
    rng = np.random.default_rng(7)
    R = random_spd(rng, 4)
    b = np.array([0.4, -0.3, 1.1, 0.2])
    nu = 6.5
    ref = stats.multivariate_t(loc=np.zeros(4), shape=R, df=nu).cdf(b, maxpts=4_000_000,
                                                                     random_state=1)
    v, se = orc.mvt(b, np.linalg.cholesky(R), nu, BIG)
    assert abs(v - ref) < 5e-5


def test_mvt_marginal_consistency(orc):
    rng = np.random.default_rng(9)
    R = random_spd(rng, 4)
    b = np.array([60.0, 0.3, -0.4, 0.8])   # first limit at +infinity in effect
    nu = 7.0
    v, se = orc.mvt(b, np.linalg.cholesky(R), nu, BIG)
    v3, se3 = orc.mvt(b[1:], np.linalg.cholesky(R[1:, 1:]), nu, BIG)
    assert abs(v - v3) < 5 * (se + se3) + 1e-6


# -- truncated moments ---------------------------------------------------------

@pytest.mark.parametrize("a,s,nu", [(-1.3, 1.0, 5.0), (0.7, 2.5, 3.5), (2.0, 0.4, 11.0), (-4.0, 1.0, 2.8)])
def test_tmoments_m1_vs_quadrature(orc, a, s, nu):
    M0, M1, M2, T2 = orc.tmoments([a], [[s]], nu, MED)
    dens = lambda z: stats.t.pdf(z, nu, scale=np.sqrt(s))
    r0 = integrate.quad(dens, -np.inf, a, epsabs=1e-14, epsrel=1e-12)[0]
    r1 = integrate.quad(lambda z: z * dens(z), -np.inf, a, epsabs=1e-14, epsrel=1e-12)[0]
    r2 = integrate.quad(lambda z: z * z * dens(z), -np.inf, a, epsabs=1e-14, epsrel=1e-12)[0]
    assert abs(M0 - r0) < 1e-12
    assert abs(M1[0] - r1) < 1e-9 * max(1, abs(r1))
    assert abs(M2[0, 0] - r2) < 1e-8 * max(1, abs(r2))


@pytest.mark.parametrize("case", range(3))
def test_tmoments_m2_vs_quadrature(orc, case):
    rng = np.random.default_rng(200 + case)
    R = random_spd(rng, 2) * rng.uniform(0.5, 2.0)
    a = rng.uniform(-1.5, 1.5, 2)
    nu = rng.uniform(4.0, 15.0)
    Ri, ld = np.linalg.inv(R), np.log(np.linalg.det(R))

    def q(fn):
        return integrate.dblquad(lambda z2, z1: fn(z1, z2) * float(_tdens(np.array([z1, z2]), Ri, ld, nu)),
                                 -np.inf, a[0], -np.inf, a[1], epsabs=1e-10, epsrel=1e-9)[0]

    M0, M1, M2, T2 = orc.tmoments(a, R, nu, BIG)
    ref1 = np.array([q(lambda x, y: x), q(lambda x, y: y)])
    ref2 = np.array([[q(lambda x, y: x * x), q(lambda x, y: x * y)],
                     [q(lambda x, y: x * y), q(lambda x, y: y * y)]])
    np.testing.assert_allclose(M1, ref1, atol=2e-7)
    np.testing.assert_allclose(M2, ref2, atol=2e-6)
    np.testing.assert_allclose(M2, M2.T, atol=2e-6)


def test_tmoments_m3_vs_monte_carlo(orc):
    rng = np.random.default_rng(31)
    R = random_spd(rng, 3) * 1.5
    a = np.array([0.5, -0.2, 0.9])
    nu = 8.0
    M0, M1, M2, T2 = orc.tmoments(a, R, nu, BIG)
    nd = 4_000_000
    Lr = np.linalg.cholesky(R)
    draws = []
    for chunk in range(4):
        x = rng.standard_normal((nd // 4, 3)) @ Lr.T
        w = rng.chisquare(nu, nd // 4) / nu
        z = x / np.sqrt(w)[:, None]
        draws.append(z[np.all(z <= a, axis=1)])
    z = np.concatenate(draws)
    p = z.shape[0] / nd
    e1 = z.sum(0) / nd
    e2 = (z[:, :, None] * z[:, None, :]).sum(0) / nd
    se1 = z.std(0) * np.sqrt(p) / np.sqrt(nd) + 1e-12
    assert abs(M0 - p) < 5 * np.sqrt(p * (1 - p) / nd)
    assert np.all(np.abs(M1 - e1) < 6 * se1 + 1e-4)
    se2 = np.sqrt(((z[:, :, None] * z[:, None, :]) ** 2).sum(0) / nd / nd)
    assert np.all(np.abs(M2 - e2) < 6 * se2 + 1e-4)


def test_tmoments_half_t_closed_forms(orc):
    """a = 0, R = sigma^2 I: the truncated law is a half-t; its moments are
    E[Z_i | Z<=0] = -sigma sqrt(nu/pi) G((nu-1)/2)/G(nu/2), E[Z_i^2|.] = sigma^2 nu/(nu-2),
    E[Z_i Z_k|.] = sigma^2 nu/(nu-2) 2/pi."""
    m, s2, nu = 3, 2.2, 6.5
    M0, M1, M2, T2 = orc.tmoments(np.zeros(m), s2 * np.eye(m), nu, BIG)
    assert abs(M0 - 0.125) < 2e-6
    sig = np.sqrt(s2)
    e1 = -sig * np.sqrt(nu / np.pi) * np.exp(sp.gammaln((nu - 1) / 2) - sp.gammaln(nu / 2))
    np.testing.assert_allclose(M1 / M0, e1, rtol=2e-5)
    ref = s2 * nu / (nu - 2) * (2 / np.pi) * np.ones((m, m))
    np.fill_diagonal(ref, s2 * nu / (nu - 2))
    np.testing.assert_allclose(M2 / M0, ref, rtol=3e-5)
