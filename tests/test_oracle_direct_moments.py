"""The direct SOV moment estimator (every coordinate of the lattice point
drawn; P, M1, M2 = lattice means of f, f z, f z z^T) in the oracle: pins,
and a quick check of the measurement that decides against it.

Pins: P is the standard SOV estimate bit for bit (same points, same
weights); m = 1 against the closed form of the truncated t mean and second
moment; both estimators converge to the same moments.  Measurement (quick
form, m = 3): at equal lattice size the gradient-identity route is far more
accurate, because the direct weights f z z^T inherit the heavy t tails while
the identity route integrates smooth lower-dimensional CDFs.  At q = 8, where
the direct estimator needs 12x fewer instructions per pair and lattice point,
tests/sov_rules_measure.py finds it still less accurate at 16x the points."""
import numpy as np
from scipy import stats

import oracle
from cfust_inputs import make_design

L3 = np.linalg.cholesky(np.array([[1.0, 0.5, 0.2], [0.5, 1.0, 0.3], [0.2, 0.3, 1.0]]))
B3 = np.array([0.3, -0.2, 0.5])


def test_probability_equals_standard_estimate():
    d = make_design(1024, 4, seed=3)
    P, _, _ = oracle.mvt_moments(B3, L3, 7.0, d)
    assert P == oracle.mvt(B3, L3, 7.0, d)[0]


def test_univariate_closed_form():
    nu, a = 6.0, 0.4
    d = make_design(4096, 8, seed=5)
    P, M1, M2 = oracle.mvt_moments(np.array([a]), np.array([[1.0]]), nu, d)
    t = stats.t.pdf(a, nu)
    m1 = -(nu + a * a) / (nu - 1.0) * t
    m2 = nu / (nu - 2.0) * stats.t.cdf(a * np.sqrt((nu - 2.0) / nu), nu - 2.0) + a * m1
    assert abs(P - stats.t.cdf(a, nu)) < 1e-13
    assert abs(M1[0] - m1) < 2e-3 * abs(m1)
    assert abs(M2[0, 0] - m2) < 2e-3 * abs(m2)


def test_converges_to_identity_moments_but_slower():
    R = L3 @ L3.T
    err_d, err_i = [], []
    ref = None
    for N, S in [(65536, 16), (1024, 8), (16384, 8)]:
        d = make_design(N, S, seed=3)
        _, M1, M2 = oracle.mvt_moments(B3, L3, 7.0, d)
        _, m1, m2, _ = oracle.tmoments(B3, R, 7.0, d)
        if ref is None:
            ref = m2                 # identity route on the largest lattice
            np.testing.assert_allclose(M2, ref, rtol=2e-4, atol=2e-4)
            np.testing.assert_allclose(M1, m1, rtol=2e-4, atol=2e-5)
            continue
        err_d.append(np.abs(M2 - ref).max())
        err_i.append(np.abs(m2 - ref).max())
    # more points help the direct estimator, and at both sizes the identity
    # route is at least 100 times closer to the reference
    assert err_d[1] < err_d[0]
    assert all(e_i * 100 < e_d for e_i, e_d in zip(err_i, err_d)), (err_i, err_d)
