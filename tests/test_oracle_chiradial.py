"""The chi-radial SOV rule (oracle/chiradial.py): pins, and a quick check of
the measurement that decides against it for the library.

Pins: m = 1 against the univariate t CDF; m = 2 orthant probabilities
against 1/4 + asin(rho) / (2 pi); m = 3 against the oracle's t rule within
their standard errors.  Measurement (quick form): at equal lattice size the
chi-radial standard error is far above the t rule's at m = 2 (the t rule
integrates one lattice dimension there, the chi-radial rule two) and above it
at m = 3, 4.  The full measurement (tests/sov_rules_measure.py: m = 2..8, 20
problems per m, three lattice sizes) finds its standard error 1.1-13x the t
rule's at every m, against 0.72-0.85x the t rule's issue slots per point in
the FP32 kernels: slower at equal accuracy for every m."""
import numpy as np
from scipy import stats

import oracle
from oracle.chiradial import mvt_chiradial
from cfust_inputs import make_design


def _corr(rng, m):
    A = rng.standard_normal((m, m + 2))
    R = A @ A.T
    d = np.sqrt(np.diag(R))
    return R / np.outer(d, d)


def test_univariate_is_the_t_cdf():
    d = make_design(1024, 8, seed=4)
    for b, nu in [(-1.3, 5.0), (0.4, 12.0), (2.2, 3.5)]:
        est, se = mvt_chiradial(np.array([b]), np.array([[1.7]]), nu, d)
        ref = stats.t.cdf(b / 1.7, nu)
        assert abs(est - ref) < max(6 * se, 1e-6), (b, nu, est, ref, se)


def test_bivariate_orthant():
    d = make_design(2048, 8, seed=5)
    for rho in (-0.6, 0.2, 0.8):
        L = np.linalg.cholesky(np.array([[1.0, rho], [rho, 1.0]]))
        est, se = mvt_chiradial(np.zeros(2), L, 7.0, d)
        ref = 0.25 + np.arcsin(rho) / (2 * np.pi)
        assert abs(est - ref) < max(6 * se, 2e-5), (rho, est, ref, se)


def test_trivariate_agrees_with_t_rule():
    rng = np.random.default_rng(6)
    d = make_design(4096, 8, seed=7)
    for _ in range(3):
        L = np.linalg.cholesky(_corr(rng, 3))
        b = rng.uniform(-1.0, 2.0, 3)
        nu = rng.uniform(5.0, 15.0)
        ec, sc = mvt_chiradial(b, L, nu, d)
        et, st = oracle.mvt(b, L, nu, d)
        assert abs(ec - et) < 6 * np.hypot(sc, st) + 1e-7, (ec, et, sc, st)


def test_t_rule_is_more_accurate_at_equal_lattice_size():
    rng = np.random.default_rng(1)
    d = make_design(1024, 8, seed=1606)
    ratios = {2: [], 3: [], 4: []}
    for trial in range(12):
        m = (2, 3, 4)[trial % 3]
        L = np.linalg.cholesky(_corr(rng, m))
        b = rng.uniform(-1.5, 2.5, m)
        nu = rng.uniform(7.0, 20.0)
        _, sc = mvt_chiradial(b, L, nu, d)
        _, st = oracle.mvt(b, L, nu, d)
        ratios[m].append(sc / max(st, 1e-300))
    med = {m: float(np.median(v)) for m, v in ratios.items()}
    print("median stderr ratio chi-radial / t rule:", med)
    assert med[2] > 10.0
    assert med[3] > 1.0 and med[4] > 1.0
