"""Pins of the oracle M-step (Sec. 3.2, eqs. 18-22) and of the EM iteration.

The M-step updates are closed-form maximisers of the expected complete-data
log-likelihood Q of the hierarchy (Sec. 3, eq. 6).  Q is written here from the
hierarchy itself (normal, half-normal and gamma log-densities with the E-step
expectations substituted), independently of the update formulas; each
conditional-maximisation step must be a stationary point of Q in its own
block (mu with Delta^(k); Delta with mu^(k+1); Sigma with both new; nu).
The stationary point in nu pins the reading of the sign in eq. (22).
"""
import numpy as np
import pytest
from scipy import special as sp

from cfust_inputs import Params, draw_params, make_design, sample_hierarchy

DES = make_design(256, 4, seed=31)


def _unpack_e3(e3col, q):
    M = np.zeros((q, q))
    iu = np.triu_indices(q)
    M[iu] = e3col
    return M + np.triu(M, 1).T


def q_function(y, tau, w, e1, e2, e3, mu, Sig, Del, nu):
    """Terms of Q for one component that depend on (mu, Sigma, Delta, nu)."""
    n, p = y.shape
    q = Del.shape[1]
    Si = np.linalg.inv(Sig)
    ld = np.linalg.slogdet(Sig)[1]
    r = y - mu
    quad = np.einsum("ji,ik,jk->j", r, Si, r)
    cross = np.einsum("ji,ik,kl,lj->j", r, Si, Del, e2)
    E3 = np.stack([_unpack_e3(e3[:, j], q) for j in range(n)])
    tr = np.einsum("ab,bc,jcd,ad->j", Si, Del, E3, Del)
    qn = -0.5 * ld - 0.5 * (w * quad - 2 * cross + tr)
    qnu = 0.5 * nu * np.log(0.5 * nu) - sp.gammaln(0.5 * nu) + 0.5 * nu * (e1 - w)
    return float((tau * (qn + qnu)).sum())


def _grad(f, x, eps):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp = x.copy(); xp[i] += eps
        xm = x.copy(); xm[i] -= eps
        g[i] = (f(xp) - f(xm)) / (2 * eps)
    return g


@pytest.fixture(scope="module")
def em_case(orc):
    rng = np.random.default_rng(41)
    P = draw_params(rng, 3, 2, 2, sigma="aat", delta_range=2.0)
    y, _ = sample_hierarchy(rng, P, 150)
    P0 = P.copy()
    P0.mu += 0.3 * rng.standard_normal(P0.mu.shape)
    P0.Delta *= 0.8
    P0.nu = np.array([6.0, 9.0])
    es = orc.estep(y, P0, DES)
    P1, frozen = orc.mstep(y, es, P0)
    return y, P0, es, P1, frozen


def test_mstep_pi(em_case):
    y, P0, es, P1, frozen = em_case
    assert frozen == 0
    np.testing.assert_allclose(P1.pi, es.tau.sum(1) / y.shape[0], rtol=1e-14)
    assert abs(P1.pi.sum() - 1) < 1e-13


def test_mstep_blocks_are_stationary_points_of_Q(em_case):
    y, P0, es, P1, _ = em_case
    q = P0.q
    for h in range(P0.g):
        args = (y, es.tau[h], es.w[h], es.e1[h], es.e2[h], es.e3[h])
        scale = es.tau[h].sum()
        # mu block with Delta^(k), Sigma^(k)
        g = _grad(lambda m: q_function(*args, m, P0.Sigma[h], P0.Delta[h], P0.nu[h]), P1.mu[h], 1e-5)
        assert np.abs(g).max() < 1e-6 * scale
        # Delta block with mu^(k+1)
        g = _grad(lambda D: q_function(*args, P1.mu[h], P0.Sigma[h], D, P0.nu[h]), P1.Delta[h], 1e-5)
        assert np.abs(g).max() < 1e-6 * scale
        # Sigma block with mu^(k+1), Delta^(k+1) (symmetric perturbations)
        S1 = P1.Sigma[h]
        for a in range(S1.shape[0]):
            for b in range(a, S1.shape[0]):
                E = np.zeros_like(S1); E[a, b] = E[b, a] = 1.0
                f = lambda t: q_function(*args, P1.mu[h], S1 + t * E, P1.Delta[h], P0.nu[h])
                d = (f(1e-6) - f(-1e-6)) / 2e-6
                assert abs(d) < 1e-5 * scale
        # nu: dQ/dnu = 0 at the update (eq. 22 with "+")
        f = lambda v: q_function(*args, P1.mu[h], P1.Sigma[h], P1.Delta[h], v)
        nu1 = P1.nu[h]
        assert 1.0 < nu1 < 200.0
        d = (f(nu1 + 1e-6) - f(nu1 - 1e-6)) / 2e-6
        assert abs(d) < 1e-6 * scale
        # and the printed sign would have no root: its left side stays positive
        m = (es.tau[h] * (es.e1[h] - es.w[h])).sum() / scale
        assert m < -1.0
        for v in np.logspace(-2, 6, 50):
            assert np.log(v / 2) - sp.digamma(v / 2) + 1 - m > 0


def test_mstep_frozen_component(orc):
    rng = np.random.default_rng(43)
    P = draw_params(rng, 2, 2, 2, sigma="aat")
    y, _ = sample_hierarchy(rng, P, 40)
    es = orc.estep(y, P, DES)
    es.tau[1] = 1e-6
    es.tau[0] = 1 - 1e-6
    P1, frozen = orc.mstep(y, es, P)
    assert frozen == 2
    np.testing.assert_array_equal(P1.mu[1], P.mu[1])
    np.testing.assert_array_equal(P1.Sigma[1], P.Sigma[1])
    np.testing.assert_array_equal(P1.Delta[1], P.Delta[1])
    assert P1.nu[1] == P.nu[1]
    assert abs(P1.pi[1] - 1e-6) < 1e-18


def test_em_loglik_nondecreasing(orc):
    """EM on a small C1-shaped problem: l^(k+1) >= l^(k) up to the QMC noise of
    the log-likelihood (measured as the spread of l under two shift sets)."""
    rng = np.random.default_rng(47)
    P = draw_params(rng, 2, 2, 2, pi=[0.4, 0.6], nu=[4.0, 8.0], sigma="aat")
    y, _ = sample_hierarchy(rng, P, 200)
    cur = P.copy()
    cur.mu += 0.5
    cur.Delta *= 0.6
    cur.nu = np.array([10.0, 10.0])
    alt = make_design(256, 4, seed=32)
    noise = abs(orc.loglik(y, cur, DES) - orc.loglik(y, cur, alt))
    ll = []
    for it in range(6):
        es = orc.estep(y, cur, DES)
        ll.append(es.loglik)
        cur, _ = orc.mstep(y, es, cur)
    for a, b in zip(ll, ll[1:]):
        assert b >= a - 3 * noise - 1e-9 * abs(a), (ll, noise)
    assert ll[-1] > ll[0]
