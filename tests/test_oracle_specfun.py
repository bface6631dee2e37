"""Pins of the oracle's special functions against third-party and closed forms.

The univariate t CDF/quantile, the incomplete beta and the digamma function
feed every T_m evaluation (Sec. 2 eq. 4, Sec. 3.1 eq. 13) and e1 (eq. 15).
scipy.special is an independent implementation; the integer-dof t CDFs are
closed forms.
"""
import numpy as np
import pytest
from scipy import special as sp
from scipy import integrate, stats

NUS = [0.5, 1.0, 2.3, 4.0, 10.7, 30.0, 150.0]


def test_tcdf_vs_scipy(orc):
    t = np.concatenate([-np.logspace(-6, 3, 40), [0.0], np.logspace(-6, 3, 40)])
    for nu in NUS:
        ref = sp.stdtr(nu, t)
        got = orc.tcdf(t, nu)
        lo = t < 0
        # lower tail relative, upper half absolute
        np.testing.assert_allclose(got[lo], ref[lo], rtol=2e-12, atol=0)
        np.testing.assert_allclose(got[~lo], ref[~lo], rtol=0, atol=1.5e-14)


def test_tcdf_integer_dof_closed_forms(orc):
    t = np.linspace(-40, 40, 161)
    # nu = 1 (Cauchy) and nu = 2 have elementary CDFs
    np.testing.assert_allclose(orc.tcdf(t, 1.0), 0.5 + np.arctan(t) / np.pi, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(orc.tcdf(t, 2.0), 0.5 + t / (2.0 * np.sqrt(2.0 + t * t)), rtol=1e-13, atol=1e-16)
    # nu = 3: 1/2 + (1/pi)[ t/(sqrt3 (1+t^2/3)) + atan(t/sqrt3) ]
    r = t / np.sqrt(3.0)
    np.testing.assert_allclose(orc.tcdf(t, 3.0), 0.5 + (r / (1 + r * r) + np.arctan(r)) / np.pi,
                               rtol=1e-12, atol=1e-16)


def test_tcdf_symmetry(orc):
    t = np.linspace(0.01, 20, 50)
    for nu in NUS:
        np.testing.assert_allclose(orc.tcdf(-t, nu) + orc.tcdf(t, nu), 1.0, atol=2e-16 * 8)


def test_tinv_vs_scipy_and_roundtrip(orc):
    p = np.concatenate([np.logspace(-250, -1, 40), [0.3, 0.5, 0.7], 1 - np.logspace(-15, -1, 20)])
    for nu in NUS[1:]:
        y = orc.tinv(p, nu)
        # scipy's quantile clamps at 1e100 and loses digits in the far tail;
        # compare where it is reliable, and pin the rest by the round trip.
        ref = sp.stdtrit(nu, p)
        fin = (p > 1e-40) & (np.abs(ref) < 1e90)
        np.testing.assert_allclose(y[fin], ref[fin], rtol=1e-9, atol=1e-15)
        back = orc.tcdf(y, nu)
        lo = p < 0.5
        np.testing.assert_allclose(back[lo], p[lo], rtol=1e-12)
        np.testing.assert_allclose(back[~lo], p[~lo], rtol=0, atol=4e-16)


def test_betai_vs_scipy(orc):
    rng = np.random.default_rng(3)
    a = rng.uniform(0.2, 60, 200)
    b = rng.uniform(0.2, 60, 200)
    x = rng.uniform(0, 1, 200)
    np.testing.assert_allclose(orc.betai(a, b, x), sp.betainc(a, b, x), rtol=1e-11, atol=1e-300)


def test_digamma_vs_scipy(orc):
    x = np.concatenate([np.linspace(0.05, 3, 30), np.logspace(0.5, 6, 30)])
    np.testing.assert_allclose(orc.digamma(x), sp.digamma(x), rtol=1e-13, atol=1e-14)


def test_t1pdf_normalised_and_vs_scipy(orc):
    for nu in [1.5, 4.0, 17.0]:
        for s in [0.3, 1.0, 7.0]:
            val, _ = integrate.quad(lambda x: orc.tcdf(0, 1) * 0 + float(orc.t1pdf(x, s, nu)), -np.inf, np.inf)
            assert abs(val - 1.0) < 1e-8
            x = np.linspace(-9, 9, 19)
            np.testing.assert_allclose(orc.t1pdf(x, s, nu), stats.t.pdf(x, nu, scale=np.sqrt(s)), rtol=1e-12)
