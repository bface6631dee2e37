"""Pins of the oracle's initialiser (Sec. 3.3, eq. 23, Algorithm 1).

Eq. (23) inverts the first two moments of the skew-normal limit of the model
(nu -> infinity): E[Y] = mu + sqrt(2/pi) Delta 1, Var[Y] = Sigma + (1 - 2/pi)
Delta Delta^T.  The pin draws a large sample from that model with the
starting values and checks that its mean and covariance are the cluster's
sample mean and covariance -- the model is simulated, the formula is not
retyped."""
import numpy as np

from oracle import init as oinit
from cfust_inputs import make_design, workload, kmeans_partitions


def _skewed_cluster(rng, n, p):
    A = rng.standard_normal((p, p)) * 0.15
    e = rng.standard_normal((n, p)) @ (np.eye(p) + A).T
    skew = np.zeros(p)
    skew[0], skew[1] = 2.0, -1.5
    return 3.0 + e + np.abs(rng.standard_normal((n, 1))) * skew


def _simulate_skew_normal(rng, P, h, n):
    q = P.Delta.shape[2]
    u = np.abs(rng.standard_normal((n, q)))
    e = rng.standard_normal((n, P.mu.shape[1])) @ np.linalg.cholesky(P.Sigma[h]).T
    return P.mu[h] + u @ P.Delta[h].T + e


def test_starting_values_reproduce_cluster_moments():
    rng = np.random.default_rng(4)
    for q in (3, 2):
        y = _skewed_cluster(rng, 5000, 3)
        lab = np.zeros(5000, dtype=np.int32)
        for alpha in (0.6, 0.9):
            P, ok = oinit.candidate(y, lab, 1, q, alpha)
            assert ok
            sim = _simulate_skew_normal(rng, P, 0, 400000)
            S = np.cov(y.T)
            np.testing.assert_allclose(sim.mean(0), y.mean(0), atol=0.02)
            np.testing.assert_allclose(np.cov(sim.T), S, atol=0.03 * np.abs(S).max())


def test_delta_sign_follows_third_moment():
    rng = np.random.default_rng(5)
    y = _skewed_cluster(rng, 4000, 3)
    P, _ = oinit.candidate(y, np.zeros(4000, dtype=np.int32), 1, 3, 0.5)
    d = np.diag(P.Delta[0])
    assert d[0] > 0 and d[1] < 0


def test_invalid_when_sigma_not_positive_definite():
    rng = np.random.default_rng(6)
    C = np.array([[1.0, 0.85], [0.85, 1.0]])
    y = rng.standard_normal((3000, 2)) @ np.linalg.cholesky(C).T
    lab = np.zeros(3000, dtype=np.int32)
    assert not oinit.candidate(y, lab, 1, 2, 0.1)[1]      # S - 0.9 diag(S) is indefinite
    assert oinit.candidate(y, lab, 1, 2, 0.9)[1]
    # a cluster with fewer than p + 1 points
    lab2 = np.zeros(3000, dtype=np.int32); lab2[:2] = 1
    assert not oinit.candidate(y, lab2, 2, 2, 0.9)[1]


def test_algorithm1_keeps_the_best_start():
    ds = workload("cfust_n1000_p2_q2_g2")
    y = ds.y[:300]
    labels = kmeans_partitions(y, 2, 3, seed=11)
    alphas = [0.1, 0.5, 0.9]
    best, ll, k = oinit.initialise(y, labels, 2, 2, alphas, make_design(256, 2, seed=1))
    assert ll.shape == (3, 3)
    assert np.isfinite(ll).any()
    assert k == int(np.argmax(ll.ravel()))
    s, a = divmod(k, 3)
    P, _ = oinit.candidate(y, labels[s], 2, 2, alphas[a])
    np.testing.assert_array_equal(best.mu, P.mu)
