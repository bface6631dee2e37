"""GPU tests of the initialiser (Sec. 3.3, eq. 23, Algorithm 1) and of
log-likelihood-only batches, against the oracle (oracle/init.py) and the
single-fit log-likelihood call."""
import numpy as np
import pytest
import torch

from oracle import init as oinit
from cfust_inputs import make_design, workload, kmeans_partitions, random_partitions
from cfust_inputs.synth import draw_params, sample_hierarchy

pytestmark = pytest.mark.gpu

ALPHAS = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9]


@pytest.fixture(scope="module")
def cf():
    import paper_1606_02054_amd as cf
    assert torch.cuda.is_available()
    cf.default_handle()
    return cf


def _loglik_only(cf, y, P, prec):
    n = y.shape[1]
    es = cf.EStepResult(None, torch.zeros(n, dtype=torch.float64, device="cuda"),
                        torch.zeros(1, dtype=torch.float64, device="cuda"), None, None, None, None,
                        torch.zeros((P.g, n), dtype=torch.float64, device="cuda"), None, None, prec)
    return es


@pytest.mark.parametrize("precision", [0, 1])
def test_density_only_batch_equals_loglik(cf, precision):
    print(f"density-only batch, precision {precision}", flush=True)
    rng = np.random.default_rng(21)
    qmc = cf.device_qmc(make_design(512, 4, seed=3), precision)
    fits, ref = [], []
    for (n, p, q, g) in [(200, 2, 2, 2), (131, 3, 1, 2), (333, 4, 4, 3), (90, 5, 3, 2)]:
        P = draw_params(rng, p, q, g, sigma="aat", nu_range=(4.0, 8.0))
        y = torch.tensor(np.ascontiguousarray(sample_hierarchy(rng, P, n)[0].T)).cuda()
        dp = cf.device_params(P)
        fits.append((y, dp, _loglik_only(cf, y, dp, precision)))
        lo = torch.zeros(n, dtype=torch.float64, device="cuda")
        ref.append((cf.cfust_loglik(y, dp, qmc, logf_obs=lo)[0], lo))
    B = cf.Batch(fits, qmc)
    B.estep()
    torch.cuda.synchronize()
    for k, ((_, _, es), (ll, lo)) in enumerate(zip(fits, ref)):
        assert torch.equal(es.loglik, ll), k
        assert torch.equal(es.logf_obs, lo), k
    with pytest.raises(RuntimeError):
        B.mstep()
    B.close()


def _compare_init(cf, y, g, q, labels, prec, design):
    yt = torch.tensor(np.ascontiguousarray(y.T)).cuda()
    lt = torch.tensor(labels).cuda()
    qmc = cf.device_qmc(design, prec)
    best, ll, k = cf.initialise(yt, g, q, lt, qmc, alphas=ALPHAS)
    torch.cuda.synchronize()
    obest, oll, ok = oinit.initialise(y, labels, g, q, ALPHAS, design)
    ll = ll.cpu().numpy()
    assert np.array_equal(np.isfinite(ll), np.isfinite(oll))
    fin = np.isfinite(oll)
    n = y.shape[0]
    tol = (1e-6 if prec == 0 else 1e-4) * n
    assert np.abs(ll[fin] - oll[fin]).max() <= tol, np.abs(ll[fin] - oll[fin]).max()
    assert k == ok
    for f in ("pi", "mu", "Sigma", "Delta", "nu"):
        np.testing.assert_allclose(getattr(best, f).cpu().numpy(), getattr(obest, f), rtol=1e-10, atol=1e-10)
    return ll


def test_init_vs_oracle_fp64(cf):
    print("initialiser vs oracle, n=300 p=q=2 g=2", flush=True)
    ds = workload("cfust_n1000_p2_q2_g2")
    y = ds.y[:300]
    labels = np.concatenate([kmeans_partitions(y, 2, 3, seed=11), random_partitions(300, 2, 1, seed=12)])
    ll = _compare_init(cf, y, 2, 2, labels, 0, make_design(256, 2, seed=1))
    assert np.isfinite(ll).sum() >= 9


def test_init_vs_oracle_q_below_p(cf):
    print("initialiser vs oracle, n=400 p=3 q=2 g=3", flush=True)
    rng = np.random.default_rng(31)
    P = draw_params(rng, 3, 2, 3, sigma="aat", nu_range=(4.0, 8.0))
    y = sample_hierarchy(rng, P, 400)[0]
    labels = kmeans_partitions(y, 3, 2, seed=13)
    _compare_init(cf, y, 3, 2, labels, 0, make_design(256, 2, seed=2))


def test_init_mixed_picks_the_best_loglik(cf):
    """Mixed precision on the n=20000, p=q=4, g=3 data: every valid
    candidate's value equals the single-fit log-likelihood of its parameters;
    the winner is the first largest."""
    print("initialiser, mixed, n=20000", flush=True)
    ds = workload("cfust_n20000_p4_q4_g3")
    y = torch.tensor(ds.y_soa).cuda()
    labels = torch.tensor(kmeans_partitions(ds.y, 3, 4, seed=5)).cuda()
    qmc = cf.device_qmc(make_design(1024, 4, seed=1606), cf.CFUST_MIXED)
    best, ll, k = cf.initialise(y, 3, 4, labels, qmc, alphas=ALPHAS)
    llc = ll.cpu().numpy().ravel()
    assert k == int(np.argmax(llc)) and np.isfinite(llc[k])
    ref = float(cf.cfust_loglik(y, best, qmc)[0].cpu()[0])
    assert ref == llc[k]
    # candidate parameters for that index, from the oracle's eq. (23)
    s, a = divmod(k, len(ALPHAS))
    P, ok = oinit.candidate(ds.y, labels.cpu().numpy()[s], 3, 4, ALPHAS[a])
    assert ok
    np.testing.assert_allclose(best.Sigma.cpu().numpy(), P.Sigma, rtol=1e-9, atol=1e-9)
